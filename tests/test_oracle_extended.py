"""Pins of the oracle's extended bulb model (azimuthal bins, Sec. 2 with the replacements
of Eq. int-v, and the four moments of Eq. F).

The four-moment Hamiltonian is checked against the direct O(N^2) beam-pair sum with the
full 1 - v.v' (tests/physref.py), and the model against the paper's own consistency check:
with axial symmetry unbroken it must reproduce the bulb model.
"""
import numpy as np
import pytest

import workloads
from tests import physref as ref


def _herm(h9):
    H = np.zeros((3, 3), complex)
    H[0, 0], H[1, 1], H[2, 2] = h9[0], h9[1], h9[2]
    H[0, 1] = h9[3] + 1j * h9[4]; H[0, 2] = h9[5] + 1j * h9[6]; H[1, 2] = h9[7] + 1j * h9[8]
    H[1, 0], H[2, 0], H[2, 1] = np.conj(H[0, 1]), np.conj(H[0, 2]), np.conj(H[1, 2])
    return H


@pytest.mark.parametrize("nf", [2, 3])
def test_four_moment_hamiltonian_equals_brute_pair_sum(oracle, nf):
    """J0, J1, J_sc, J_ss factorise the extended H_nunu: equal to the direct pair sum over
    (angle, azimuth, energy) beams with the full 1 - v.v', for random states (odd n_phi, so
    no symmetry makes the azimuthal terms vanish)."""
    NE, NU, NP = 3, 3, 5
    d = workloads.small_params(n_flavor=nf, n_energy=NE, n_u=NU, n_steps=10, r_start_km=10.0,
                               r_end_km=20.0, n_phi=NP)
    m = oracle.Model(d)
    rng = np.random.default_rng(31)
    nb = 2 * NU * NP * NE
    if nf == 2:
        P = rng.normal(size=(3, nb)); P /= np.linalg.norm(P, axis=0)
        m.set_state(P, 0)
        rho = 0.5 * (np.eye(2)[None] + P[0][:, None, None] * np.array([[0, 1], [1, 0]])
                     + P[1][:, None, None] * np.array([[0, -1j], [1j, 0]])
                     + P[2][:, None, None] * np.array([[1, 0], [0, -1]]))
    else:
        psi = rng.normal(size=(6, nb)); psi /= np.linalg.norm(psi, axis=0)
        m.set_state(psi, 0)
        pv = (psi[0::2] + 1j * psi[1::2]).T
        rho = np.einsum("bi,bj->bij", pv, pv.conj())
    rho = rho.reshape(2, NU, NP, NE, nf, nf)
    r = 13.7
    jm = m.moments4(r)
    assert np.abs(jm[2:]).max() > 1e-3 * np.abs(jm[:2]).max()   # azimuthal moments present
    H = m.hamiltonian4(r, jm).reshape(2, NU, NP, NE, -1)
    Hnn = ref.brute_h_nunu_ext(d, r, rho[0], rho[1])
    E, dE, u, du = ref.bins(d)
    lam = ref.sqrt2gf_km_cm3() * d["n0_cm3"] * (d["r_nu_km"] / r) ** 3
    for s in range(2):
        sg = 1 if s == 0 else -1
        for j in range(NU):
            for p in range(NP):
                for k in range(NE):
                    if nf == 2:
                        Ht = ref.hvac2(d, E[k]) + sg * np.diag([lam, 0]) + Hnn[s, j, p, k]
                        np.testing.assert_allclose(H[s, j, p, k], ref.bvec(Ht), rtol=1e-12,
                                                   atol=1e-12 * np.abs(Ht).max())
                    else:
                        Ht = ref.hvac3(d, E[k]) + sg * np.diag([lam, 0, 0]) + Hnn[s, j, p, k]
                        D = _herm(H[s, j, p, k]) - Ht
                        D -= np.trace(D) / 3 * np.eye(3)
                        assert np.abs(D).max() < 1e-12 * np.abs(Ht).max()


def test_phi_table_is_the_bin_midpoints(oracle):
    for NP in (4, 5, 10):
        d = workloads.small_params(n_flavor=2, n_energy=2, n_u=2, n_steps=1, n_phi=NP)
        t = oracle.Model(d).phi_table()
        phi = 2 * np.pi * (np.arange(NP) + 0.5) / NP
        np.testing.assert_allclose(t[0], np.cos(phi), atol=4e-16)
        np.testing.assert_allclose(t[1], np.sin(phi), atol=4e-16)
        if NP % 2 == 0:                       # exact antipodal pairs
            np.testing.assert_array_equal(t[:, NP // 2:], -t[:, :NP // 2])


@pytest.mark.parametrize("nf", [2, 3])
def test_extended_equals_bulb_under_axial_symmetry(oracle, nf):
    """The paper's consistency check: while axial symmetry is unbroken (every azimuthal bin
    in the same state, even n_phi) the azimuthal moments vanish exactly and every azimuthal
    bin follows the bulb model (up to the rounding of the fixed-point sums, whose weights
    differ by the factor 1/n_phi)."""
    base = workloads.small_params(n_flavor=nf, n_energy=8, n_u=4, n_steps=200, r_start_km=100.0,
                                  r_end_km=102.0, n0_cm3=1e32)
    b = oracle.Model(base)
    b.run()
    pb = b.pee()
    e = oracle.Model(dict(base, n_phi=6))
    e.step(100)
    jm = e.moments4(101.0)
    assert np.all(jm[2:] == 0.0)
    e.run()
    pe = e.pee()
    for p in range(6):
        np.testing.assert_allclose(pe[:, :, p, :], pb, atol=1e-11)


def test_broken_symmetry_couples_the_azimuthal_bins(oracle):
    """A state that differs between azimuthal bins produces azimuthal moments, and the bins
    then evolve differently (the spontaneous symmetry breaking the extended model is for)."""
    d = workloads.small_params(n_flavor=2, n_energy=6, n_u=3, n_steps=50, r_start_km=100.0,
                               r_end_km=101.0, n0_cm3=1e32, n_phi=4)
    m = oracle.Model(d)
    x = m.get_state().copy().reshape(3, 2, 3, 4, 6)
    x[0, :, :, 0, :] = 0.1                     # tilt azimuthal bin 0 only
    x[2, :, :, 0, :] = np.sqrt(1 - 0.01)
    m.set_state(x.reshape(3, -1), 0)
    jm = m.moments4(100.0)
    assert np.abs(jm[2:]).max() > 0.0
    m.run()
    pe = m.pee()
    assert np.abs(pe[:, :, 1, :] - pe[:, :, 2, :]).max() > 1e-8
