"""GPU parity of the extended bulb model (azimuthal bins, four moments) against the oracle.

Same bar as the bulb model: bit-for-bit equal states and P_ee.  Cases cover both flavour
counts, even and odd bin counts, ragged row tails, states that break the axial symmetry
(so that the azimuthal moments J_sc and J_ss matter), and a prefix of the paper's own
benchmark shape (10 azimuthal x 100 energy bins, here with 1000 polar bins).
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


def _tilted_state(nf, nb_beams, seed):
    rng = np.random.default_rng(seed)
    if nf == 2:
        x = rng.normal(size=(3, nb_beams))
    else:
        x = rng.normal(size=(6, nb_beams))
    return x / np.linalg.norm(x, axis=0)


CASES = [
    ("2f-13x3x4-sym", dict(n_flavor=2, n_energy=13, n_u=3, n_phi=4, n_steps=20), False),
    ("2f-70x3x5-random", dict(n_flavor=2, n_energy=70, n_u=3, n_phi=5, n_steps=12), True),
    ("3f-37x3x6-sym", dict(n_flavor=3, n_energy=37, n_u=3, n_phi=6, n_steps=10), False),
    ("3f-37x2x3-random", dict(n_flavor=3, n_energy=37, n_u=2, n_phi=3, n_steps=8), True),
    ("3f-129x2x2-random", dict(n_flavor=3, n_energy=129, n_u=2, n_phi=2, n_steps=5), True),
]


@pytest.mark.parametrize("name,kw,random_state", CASES, ids=[c[0] for c in CASES])
def test_extended_bitwise_matches_oracle(nb, oracle, name, kw, random_state):
    import torch
    d = workloads.small_params(r_start_km=100.0, r_end_km=101.0, n0_cm3=1e32, **kw)
    o = oracle.Model(d)
    m = nb.Model(d)
    _say(f"extended case {name}: {m.nb} beams")
    assert m.nb == o.nb
    if random_state:
        x = _tilted_state(d["n_flavor"], m.nb, 41)
        o.set_state(x, 0)
        m.set_state(torch.as_tensor(x), 0)
        jm = o.moments4(d["r_start_km"])
        assert np.abs(jm[2:]).max() > 0.0
    o.run()
    m.run()
    np.testing.assert_array_equal(m.get_state().cpu().numpy(), o.get_state())
    np.testing.assert_array_equal(m.pee().cpu().numpy(), o.pee().ravel())


def test_extended_paper_shape_prefix(nb, oracle):
    """10 azimuthal x 100 energy x 1000 polar bins x 2 species (2M two-flavour beams), the
    shape of the paper's extended-model benchmark with 1000 of its 10k-30k polar bins:
    a 3-step prefix from a state with broken axial symmetry, against the oracle."""
    import torch
    d = workloads.base_params(n_flavor=2, n_energy=100, n_u=1000, n_phi=10, n_steps=3000,
                              r_end_km=310.0, n0_cm3=workloads.draw_n0())
    m = nb.Model(d)
    _say(f"extended paper-shape prefix: {m.nb} beams")
    o = oracle.Model(d)
    x = _tilted_state(2, m.nb, 43)
    o.set_state(x, 0)
    m.set_state(torch.as_tensor(x), 0)
    o.step(3)
    m.step(3)
    np.testing.assert_array_equal(m.get_state().cpu().numpy(), o.get_state())


def test_extended_equals_bulb_under_axial_symmetry_on_gpu(nb):
    """GPU version of the paper's consistency check: every azimuthal bin of an axially
    symmetric extended run follows the bulb model."""
    base = workloads.small_params(n_flavor=3, n_energy=37, n_u=4, n_steps=100, r_start_km=100.0,
                                  r_end_km=101.0, n0_cm3=1e32)
    b = nb.Model(base)
    b.run()
    pb = b.pee().cpu().numpy().reshape(2, 4, 37)
    e = nb.Model(dict(base, n_phi=4))
    e.run()
    pe = e.pee().cpu().numpy().reshape(2, 4, 4, 37)
    for p in range(4):
        np.testing.assert_allclose(pe[:, :, p, :], pb, atol=1e-11)
