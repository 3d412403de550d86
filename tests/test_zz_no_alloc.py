"""nb_step_static (the stepping entry point with its launch scratch in a static device
array, for callers that cannot allocate) against nb_step, bit for bit, through the C-ABI:
two calls in a row on different models, the second smaller than the first, so that the
second call finds the first call's words in the shared array; a batch; and a status error
raised and cleared through the static array."""
import ctypes as C
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def nb():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    import paper_1912_10596_amd as nb
    nb.lib()
    return nb


def _pair(nb, d, steps):
    a = nb.Model(d)
    b = nb.Model(d)
    nb._check(nb.lib().nb_step(a.h, steps), "nb_step")
    nb._check(nb.lib().nb_step_static(b.h, steps), "nb_step_static")
    assert a.step_index() == b.step_index() == min(steps, d["n_steps"])
    return a, b


def test_static_scratch_equals_workspace_scratch_two_calls(nb):
    big = workloads.small_params(n_flavor=3, n_energy=130, n_u=7, n_steps=20, r_start_km=10.0,
                                 r_end_km=11.0)
    small = workloads.small_params(n_flavor=2, n_energy=37, n_u=5, n_steps=15)
    for d, steps in ((big, 20), (small, 15)):
        _say(f"static scratch: {d['n_flavor']}f {d['n_energy']}x{d['n_u']}, {steps} steps")
        a, b = _pair(nb, d, steps)
        np.testing.assert_array_equal(a.get_state().cpu().numpy(), b.get_state().cpu().numpy())
        np.testing.assert_array_equal(a.pee().cpu().numpy(), b.pee().cpu().numpy())


def test_static_scratch_packed_row_tails(nb):
    """A three-flavour model with one row per wavefront and a short last pass (130 energies,
    16 rows in two blocks): the stepper's packed-row-tail variant through both entry points."""
    d = workloads.small_params(n_flavor=3, n_energy=130, n_u=8, n_steps=12, r_start_km=10.0,
                               r_end_km=10.6)
    a, b = _pair(nb, d, 12)
    np.testing.assert_array_equal(a.get_state().cpu().numpy(), b.get_state().cpu().numpy())


def test_static_scratch_split_calls_and_batch(nb):
    ds = []
    for d in workloads.batch_256(5):
        d = dict(d, n_energy=20 + d["n_energy"] % 90, n_u=2 + d["n_u"] % 7, n_steps=12,
                 r_start_km=10.0, r_end_km=11.0)
        ds.append(d)
    a = nb.Model(ds); a.run()
    b = nb.Model(ds)
    b.step_static(5)
    b.step_static(100)                   # clamped at r_end
    assert b.step_index() == 12
    np.testing.assert_array_equal(a.get_state().cpu().numpy(), b.get_state().cpu().numpy())


def test_static_scratch_reports_and_clears_errors(nb):
    import torch
    d = workloads.small_params(n_flavor=2, n_energy=20, n_u=3, n_steps=4)
    m = nb.Model(d)
    x = m.get_state()
    x[0, 5] = float("nan")
    m.set_state(x, 0)
    with pytest.raises(nb.NubulbError) as e:
        m.step_static(1)
    assert e.value.code == nb.NB_ENUMERIC
    m.reset()
    m.step_static(4)                     # the array was cleared: a clean run afterwards
    ref = nb.Model(d); ref.run()
    np.testing.assert_array_equal(m.pee().cpu().numpy(), ref.pee().cpu().numpy())
    assert torch.isfinite(m.pee()).all()
