"""GPU parity of the adaptive step-size control (nb_run_adaptive) against the oracle.

Every accept/reject decision is taken from the same reduced error estimate on both sides,
so the bar is the same as for fixed steps: identical step statistics and a bit-for-bit
identical final state.  Cases include runs whose first steps are rejected, step doubling
in vacuum, ragged row tails, several lane iterations per row, and the 200k-beam shape.
"""
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


def _case(name):
    if name == "2f-16x4-reject":
        return workloads.small_params(n_flavor=2, n_energy=16, n_u=4, n_steps=1, r_start_km=100.0,
                                      r_end_km=102.0, n0_cm3=1e32), 1e-5, 0.0
    if name == "3f-37x5-reject":
        return workloads.small_params(n_flavor=3, n_energy=37, n_u=5, n_steps=2, r_start_km=100.0,
                                      r_end_km=101.0, n0_cm3=1e32), 1e-5, 0.0
    if name == "2f-vacuum-doubling":
        return workloads.small_params(n_flavor=2, n_energy=40, n_u=3, n_steps=40, r_start_km=10.0,
                                      r_end_km=40.0, lum_erg_s=[0.0, 0.0, 0.0], n0_cm3=0.0), 1e-6, 0.0
    if name == "3f-129x3-capped":
        return workloads.small_params(n_flavor=3, n_energy=129, n_u=3, n_steps=8, r_start_km=200.0,
                                      r_end_km=204.0), 1e-6, 0.1
    if name == "2f-200k-shape":
        d = workloads.adjoint_200k_resolved()
        return dict(d, r_end_km=d["r_start_km"] + 1.0, n_steps=10), 1e-7, 0.0
    raise KeyError(name)


CASES = ["2f-16x4-reject", "3f-37x5-reject", "2f-vacuum-doubling", "3f-129x3-capped",
         "2f-200k-shape"]


@pytest.mark.parametrize("name", CASES)
def test_adaptive_bitwise_matches_oracle(nb, oracle, name):
    d, tol, hmax = _case(name)
    _say(f"adaptive case {name}: {2 * d['n_energy'] * d['n_u']} beams, tol {tol}")
    o = oracle.Model(d)
    so = o.run_adaptive(tol, h_max=hmax)
    m = nb.Model(d, adaptive=True)
    sg = m.run_adaptive(tol, h_max=hmax)
    _say(f"  oracle {so}  gpu {sg}")
    assert (sg["accepted"], sg["rejected"], sg["h_last"]) == (so["accepted"], so["rejected"], so["h_last"])
    assert sg["attempts"] == sg["accepted"] + sg["rejected"]
    assert m.step_index() == d["n_steps"]
    np.testing.assert_array_equal(m.get_state().cpu().numpy(), o.get_state())
    np.testing.assert_array_equal(m.pee().cpu().numpy(), o.pee().ravel())


def test_adaptive_repeat_after_reset_and_failures(nb):
    d, tol, hmax = _case("2f-16x4-reject")
    m = nb.Model(d, adaptive=True)
    s1 = m.run_adaptive(tol)
    p1 = m.pee().cpu().numpy()
    with pytest.raises(nb.NubulbError) as e:
        m.run_adaptive(tol)                         # not at step 0
    assert e.value.code == nb.NB_EINVAL
    m.reset()
    with pytest.raises(nb.NubulbError) as e:
        m.run_adaptive(tol, max_attempts=s1["attempts"] - 1)
    assert e.value.code == nb.NB_ESTEP
    m.reset()
    s2 = m.run_adaptive(tol)
    assert s2 == s1
    np.testing.assert_array_equal(m.pee().cpu().numpy(), p1)
    with pytest.raises(nb.NubulbError) as e:
        nb.Model(d).run_adaptive(tol)               # created without adaptive = 1
    assert e.value.code == nb.NB_EINVAL
