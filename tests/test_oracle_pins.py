"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: each checks it against a closed form, a
library routine (libm, SciPy expm / quadrature), a brute-force sum written from the
paper's equations (tests/physref.py), an invariant, or a hand-computed value.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import linalg
from scipy.spatial.transform import Rotation

import workloads
from tests import physref as ref

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- units (Sec. 2)
def _half_last_digit(s: str) -> float:
    """Half a unit in the last printed digit of a hand value written as a string."""
    mant, _, ex = s.partition("e")
    dec = len(mant.split(".")[1]) if "." in mant else 0
    return 0.5 * 10.0 ** (int(ex or 0) - dec) * 1.001


def _close(x, g: str):
    assert abs(x - float(g)) <= _half_last_digit(g), (x, g)


def test_units_against_hand_values(oracle):
    g = json.load(open(os.path.join(GOLD, "units.json")))
    # omega = dm^2/4E at dm^2 = 2.4e-3 eV^2, E = 10 MeV: one energy bin centred on 10 MeV
    d = workloads.base_params(n_energy=1, n_u=1, e_min_mev=9.5, e_max_mev=10.5,
                              dm2_ev2=[2.4e-3, 0.0], n0_cm3=1e33, n_steps=1)
    t = oracle.Model(d).tables()
    bx, bz = t["bv"][0]
    omega = 0.5 * math.hypot(bx, bz)            # |B_vac| = 2 omega
    _close(omega, g["omega_km_at_dm2_2.4e-3_E_10MeV"])
    _close(t["lam0"], g["lambda_km_at_n0_1e33"])
    f2, f3 = ref.fd_moments()
    _close(f3 / f2, g["mean_energy_over_T"])
    # nu-nu scale sqrt2 G_F N/(2 pi R^2 c) at R for each species, N = L/<E>
    for key, T in (("nue", 2.76), ("nuebar", 4.01), ("nux", 6.26)):
        N = 1e51 * ref.ERG_MEV / (T * f3 / f2)
        _close(t["kappa0"] * N, g[f"nunu_scale_km_{key}_L1e51_R10km"])


def test_spectrum_weights_against_quadrature(oracle):
    """Explicit-species weights / (kappa0 du dE N) are the normalised Fermi-Dirac spectra;
    their midpoint sums match the quadrature of f over [1, 50] MeV."""
    d = workloads.base_params(n_energy=2000, n_u=1, n_steps=1)
    m = oracle.Model(d, species4=1)
    t = m.tables()
    E, dE, u, du = ref.bins(d)
    f2, f3 = ref.fd_moments()
    from scipy import integrate
    for s, (a, T) in enumerate([(0, 2.76), (2, 6.26)]):   # nu_e and nu_x rows
        N = d["lum_erg_s"][a] * ref.ERG_MEV / (T * f3 / f2)
        f = t["w"][s] / (t["kappa0"] * du * dE * N)
        np.testing.assert_allclose(f, ref.spectrum(E, T), rtol=1e-12)
        exact = integrate.quad(lambda x: ref.spectrum(x, T), 1.0, 50.0, epsabs=1e-14)[0]
        assert np.sum(f) * dE == pytest.approx(exact, rel=1e-6)     # midpoint rule, O(dE^2)


# --------------------------------------------------------- primitives (Eq. U)
def test_sincos_against_libm(oracle):
    rng = np.random.default_rng(7)
    x = np.concatenate([np.linspace(-8, 8, 20001), rng.uniform(-1e3, 1e3, 20000),
                        rng.uniform(-4e6, 4e6, 20000), rng.uniform(-1e15, 1e15, 20000),
                        [0.0, -0.0, np.pi / 4, 1e-300, 2.0 ** 50 * 0.999]])
    s, c = oracle.sincos(x)
    assert np.max(np.abs(s - np.sin(x))) <= 2.3e-16
    assert np.max(np.abs(c - np.cos(x))) <= 2.3e-16


def test_rotation_against_scipy(oracle):
    rng = np.random.default_rng(3)
    for scale in (1e-9, 1e-3, 1.0, 30.0, 3e5):
        for _ in range(20):
            x = rng.normal(size=3) * scale
            p = rng.normal(size=3); p /= np.linalg.norm(p)
            want = Rotation.from_rotvec(x).apply(p)
            got = oracle.rotate(x, p)
            np.testing.assert_allclose(got, want, atol=4e-16 * max(1.0, scale) + 1e-15)
    # zero rotation is the identity
    np.testing.assert_array_equal(oracle.rotate(np.zeros(3), np.array([0.3, 0.4, 0.5])),
                                  [0.3, 0.4, 0.5])


def _herm(k9):
    H = np.diag(k9[:3]).astype(complex)
    for t, (a, b) in enumerate([(0, 1), (0, 2), (1, 2)]):
        H[a, b] = k9[3 + 2 * t] + 1j * k9[4 + 2 * t]
        H[b, a] = np.conj(H[a, b])
    return H


def _rho(psi6):
    p = psi6[0::2] + 1j * psi6[1::2]
    return np.outer(p, p.conj())


@pytest.mark.parametrize("kind", ["random", "degenerate", "matter", "tiny", "diag"])
def test_exp3_against_expm(oracle, kind):
    """exp(-iK) psi (up to a global phase) against SciPy's expm, incl. degenerate spectra."""
    rng = np.random.default_rng(11)
    for scale in (1e-4, 0.3, 5.0, 2e3, 3e6):
        for _ in range(10):
            if kind == "random":
                k9 = rng.normal(size=9) * scale
            elif kind == "degenerate":     # eigenvalues (a, a, b) in a random basis
                Q, _ = np.linalg.qr(rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3)))
                a = rng.normal() * scale
                H = Q @ np.diag([a, a, -2 * a + 0.1 * scale]) @ Q.conj().T
                k9 = np.array([H[0, 0].real, H[1, 1].real, H[2, 2].real, H[0, 1].real,
                               H[0, 1].imag, H[0, 2].real, H[0, 2].imag, H[1, 2].real,
                               H[1, 2].imag])
            elif kind == "matter":         # large e-e entry, small mixing (MSW-like)
                k9 = np.zeros(9); k9[0] = scale
                k9[3:] = rng.normal(size=6) * 0.1
                k9[1:3] = rng.normal(size=2) * 0.05
            elif kind == "tiny":
                k9 = rng.normal(size=9) * 1e-12
            else:
                k9 = np.zeros(9); k9[:3] = rng.normal(size=3) * scale
            psi = rng.normal(size=6); psi /= np.linalg.norm(psi)
            got = oracle.exp3_apply(k9, psi)
            U = linalg.expm(-1j * _herm(k9))
            pv = psi[0::2] + 1j * psi[1::2]
            want = np.outer(U @ pv, (U @ pv).conj())
            kn = np.abs(k9).max()
            np.testing.assert_allclose(_rho(got), want, atol=3e-15 * max(1.0, kn) + 1e-14)
    # K = 0 is the identity
    psi = np.array([0.6, 0.0, 0.0, 0.8, 0.0, 0.0])
    np.testing.assert_array_equal(oracle.exp3_apply(np.zeros(9), psi), psi)


def test_exp3_state_along_isolated_eigenvector(oracle):
    """psi (almost) along the eigenvector of the largest-magnitude eigenvalue, where the plane
    component P psi is tiny: against expm for |P psi| from 1e-2 down to 1e-17 and 0 (a
    diagonal K with a flavour eigenstate), so the plane angle taken from P psi stays harmless."""
    rng = np.random.default_rng(13)
    for scale in (0.3, 50.0, 3e4):
        for _ in range(6):
            k9 = rng.normal(size=9) * scale
            H = _herm(k9)
            ev, V = np.linalg.eigh(H - np.trace(H) / 3 * np.eye(3))
            i1 = int(np.argmax(np.abs(ev)))
            v1 = V[:, i1]
            pl = V[:, [i for i in range(3) if i != i1]] @ (rng.normal(size=2) + 1j * rng.normal(size=2))
            pl /= np.linalg.norm(pl)
            for dlt in (1e-2, 1e-6, 1e-10, 1e-14, 1e-17):
                pv = v1 + dlt * pl
                pv /= np.linalg.norm(pv)
                psi = np.empty(6); psi[0::2] = pv.real; psi[1::2] = pv.imag
                got = oracle.exp3_apply(k9, psi)
                U = linalg.expm(-1j * H)
                want = np.outer(U @ pv, (U @ pv).conj())
                np.testing.assert_allclose(_rho(got), want, atol=3e-15 * max(1.0, scale * 3) + 1e-14)
    k9 = np.zeros(9); k9[:3] = [3.0, -1.0, 0.5]
    for e in range(3):
        psi = np.zeros(6); psi[2 * e] = 1.0
        got = oracle.exp3_apply(k9, psi)
        assert np.isfinite(got).all()
        np.testing.assert_allclose(_rho(got), _rho(psi), atol=1e-15)


def test_exp3_magnitude_range(oracle):
    """The unnormalised form's range: |K0| from just above its lower end (1e-29: every
    intermediate about |K0|^10 stays normal) to 1e9, first-order exact at the small end
    (psi' = psi - i K psi) and against expm above; below the end (1e-31) K0 counts as zero."""
    rng = np.random.default_rng(12)
    for scale in (1e-29, 1e-20, 1e9):
        for _ in range(10):
            k9 = rng.normal(size=9) * scale
            psi = rng.normal(size=6); psi /= np.linalg.norm(psi)
            got = oracle.exp3_apply(k9, psi)
            assert np.isfinite(got).all()
            pv = psi[0::2] + 1j * psi[1::2]
            U = linalg.expm(-1j * _herm(k9))
            want = np.outer(U @ pv, (U @ pv).conj())
            np.testing.assert_allclose(_rho(got), want, atol=3e-15 * max(1.0, scale * 3) + 1e-14)
            if scale < 1e-19:
                # global phase fixed by the first entry: psi' = (1 - i K0) psi to O(K^2)
                H = _herm(k9)
                H0 = H - np.trace(H) / 3 * np.eye(3)
                lin = pv - 1j * (H0 @ pv)
                g = got[0::2] + 1j * got[1::2]
                ph = (g @ lin.conj()) / abs(g @ lin.conj())
                np.testing.assert_allclose(g / ph, lin, rtol=0, atol=1e-15)
    k9 = rng.normal(size=9) * 1e-31
    psi = rng.normal(size=6); psi /= np.linalg.norm(psi)
    np.testing.assert_array_equal(oracle.exp3_apply(k9, psi), psi)


def test_fixed_point_sum_exact_and_order_free(oracle):
    rng = np.random.default_rng(5)
    v = rng.normal(size=2000) * 10.0 ** rng.uniform(-8, 3, size=2000)
    e = 40
    got = oracle.fixed_sum(v, e)
    exact = sum(Fraction(int(math.trunc(Fraction(x) * 2 ** e)), 2 ** e) for x in v.tolist())
    assert abs(Fraction(got) - exact) <= abs(exact) * Fraction(1, 2 ** 52)
    for _ in range(3):
        assert oracle.fixed_sum(rng.permutation(v), e) == got      # bitwise, any order
    assert got == pytest.approx(math.fsum(v), abs=len(v) * 2.0 ** -e)


def test_fix_round_is_round_half_even_of_exact_product(oracle):
    """Every beam contribution is the exact product v * ws rounded once to the nearest
    integer, ties to even, over the whole range the fixed point allows (|v ws| <= 2^51):
    against Python's exact rationals.  Includes exact ties and values just either side."""
    rng = np.random.default_rng(17)
    n = 20000
    v = rng.uniform(-2.0, 2.0, n) * 10.0 ** rng.uniform(-6, 0, n)
    ws = rng.uniform(-1.0, 1.0, n) * 2.0 ** rng.uniform(0, 50, n)
    ties_v = np.array([0.5, 1.5, -2.5, 0.75, 1.25, -0.25, 1.0, -1.0])
    ties_w = np.array([1.0, 1.0, 1.0, 2.0, 2.0, 2.0, 2.0 ** 50 + 0.5, 2.0 ** 50 + 0.5])
    near_v = np.array([0.5, 0.5, -0.5, -0.5])
    near_w = np.array([1.0 + 2.0 ** -52, 1.0 - 2.0 ** -53, 1.0 + 2.0 ** -52, 1.0 - 2.0 ** -53])
    edge_v = np.array([1.0, -1.0, 1.9999999999999998])
    edge_w = np.array([2.0 ** 51, 2.0 ** 51, 2.0 ** 50])
    v = np.concatenate([v, ties_v, near_v, edge_v])
    ws = np.concatenate([ws, ties_w, near_w, edge_w])
    got = oracle.fix_round(v, ws)
    want = [round(Fraction(a) * Fraction(b)) for a, b in zip(v.tolist(), ws.tolist())]
    assert got.tolist() == want                     # Python's round() is half-to-even


# ------------------------------------------------- closed forms (Sec. 2, Eq. U)
def _vacuum_case(nf, n_u=3, ne=6, steps=400, **kw):
    args = dict(n_flavor=nf, n_energy=ne, n_u=n_u, n_steps=steps, r_start_km=10.0,
                r_end_km=40.0, lum_erg_s=[0.0, 0.0, 0.0], n0_cm3=0.0)
    args.update(kw)
    return workloads.small_params(**args)


@pytest.mark.parametrize("nf", [2, 3])
def test_vacuum_oscillation_closed_form(oracle, nf):
    """No matter, no neutrinos: P_ee = 1 - sum 4|U_ei U_ej|^2 sin^2(dm_ij^2 L/4E) along the
    beam's path length L (2 flavours: 1 - sin^2 2theta sin^2(dm^2 L/4E))."""
    d = _vacuum_case(nf)
    m = oracle.Model(d); m.run()
    pee = m.pee()
    E, dE, u, du = ref.bins(d)
    L = ref.path_length(d["r_end_km"], d["r_start_km"], d["r_nu_km"], u)[:, None]
    if nf == 2:
        w = ref.omega_km(d["dm2_ev2"][0], E)[None, :]
        want = 1.0 - np.sin(2 * d["theta"][0]) ** 2 * np.sin(w * L) ** 2
    else:
        U = ref.pmns(*d["theta"])
        m2 = [0.0, d["dm2_ev2"][0], d["dm2_ev2"][1]]
        want = np.ones((len(u), len(E)))
        for i in range(3):
            for j in range(i + 1, 3):
                ph = (m2[j] - m2[i]) / (4.0 * E * 1e6) / ref.HBARC_EV_KM
                want -= 4 * U[0, i] ** 2 * U[0, j] ** 2 * np.sin(ph[None, :] * L) ** 2
    for s in range(2):       # antineutrinos: same vacuum Hamiltonian (real mixing)
        np.testing.assert_allclose(pee[s], want, atol=2e-10)


@pytest.mark.parametrize("nf", [2, 3])
def test_msw_constant_density_closed_form(oracle, nf):
    """Constant n_e: the textbook matter solution (2f: sin^2 2theta_m, dm^2_m with
    A -> -A for antineutrinos; 3f: expm of the constant Hamiltonian)."""
    d = _vacuum_case(nf, ne_power=0, n0_cm3=2.0e28, steps=400)
    m = oracle.Model(d); m.run()
    pee = m.pee()
    E, dE, u, du = ref.bins(d)
    lam = ref.sqrt2gf_km_cm3() * d["n0_cm3"]
    L = ref.path_length(d["r_end_km"], d["r_start_km"], d["r_nu_km"], u)
    for s, sign in ((0, 1.0), (1, -1.0)):
        for k, e in enumerate(E):
            if nf == 2:
                th = d["theta"][0]
                w = ref.omega_km(d["dm2_ev2"][0], e)
                A = sign * lam / (2 * w)
                s22m = np.sin(2 * th) ** 2 / ((np.cos(2 * th) - A) ** 2 + np.sin(2 * th) ** 2)
                wm = w * np.sqrt((np.cos(2 * th) - A) ** 2 + np.sin(2 * th) ** 2)
                want = 1 - s22m * np.sin(wm * L) ** 2
            else:
                H = ref.hvac3(d, e) + sign * np.diag([lam, 0, 0])
                want = np.array([abs(ref.expm_apply(H, l, np.array([1, 0, 0]))[0]) ** 2
                                 for l in L])
            np.testing.assert_allclose(pee[s, :, k], want, atol=2e-10)


# -------------------------------------------------- H_nunu (Eqs. Hnu and F)
@pytest.mark.parametrize("nf", [2, 3])
@pytest.mark.parametrize("xbar", [False, True])
def test_factored_hamiltonian_equals_brute_pair_sum(oracle, nf, xbar):
    """J0/J1 factorisation = direct O(N^2) beam-pair sum of Eq. Hnu with every initial
    flavour explicit; also pins weights, the d cos(theta') Jacobian and the antineutrino
    conjugation (xbar: anti-nu_x with its own luminosity and temperature)."""
    kw = dict(lum_xbar_erg_s=2.3e51, temp_xbar_mev=5.1) if xbar else {}
    d = workloads.small_params(n_flavor=nf, n_energy=3, n_u=4, n_steps=10,
                               r_start_km=10.0, r_end_km=20.0, **kw)
    m = oracle.Model(d)
    rng = np.random.default_rng(21)
    NE, NU, nb = 3, 4, 2 * 3 * 4
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
    rho = rho.reshape(2, NU, NE, nf, nf)
    r = 13.7
    j0, j1 = m.moments(r)
    H = m.hamiltonian(r, j0, j1).reshape(2, NU, NE, -1)
    Hnn = ref.brute_h_nunu(d, r, rho[0], rho[1])
    E, dE, u, du = ref.bins(d)
    lam = ref.sqrt2gf_km_cm3() * d["n0_cm3"] * (d["r_nu_km"] / r) ** 3
    for s in range(2):
        sg = 1 if s == 0 else -1
        for j in range(NU):
            for k in range(NE):
                if nf == 2:
                    Ht = ref.hvac2(d, E[k]) + sg * np.diag([lam, 0]) + Hnn[s, j, k]
                    np.testing.assert_allclose(H[s, j, k], ref.bvec(Ht), rtol=1e-12,
                                               atol=1e-12 * np.abs(Ht).max())
                else:
                    Ht = ref.hvac3(d, E[k]) + sg * np.diag([lam, 0, 0]) + Hnn[s, j, k]
                    Ho = _herm(H[s, j, k])
                    # equal up to a multiple of the identity
                    D = Ho - Ht
                    D -= np.trace(D) / 3 * np.eye(3)
                    assert np.abs(D).max() <= 1e-12 * np.abs(Ht).max()


# ----------------------------------------------------- invariants, reductions
@pytest.mark.parametrize("nf,bound", [(2, 1e-13), (3, 5e-13)])
def test_norm_conserved_without_renormalisation(oracle, nf, bound):
    """Trace and purity of every beam over 1000 steps (4000 exponentials) with the
    renormalisation switched off.  The 2x2 rotation is unitary to the last ulp.  The 3x3
    exponential does not normalise anything: the plane angle th = sqrt(|(K0 - hm) P psi|^2 /
    |P psi|^2) is rounded, and cos(th) and sin(th)/th come from that rounded value, so an
    application moves |psi| by about one ulp of 1 (1.1e-16 on average over random K, 2e-15
    at worst), and 4000 of them stay below 4000 x 1.1e-16 = 4.4e-13 (the production path
    renormalises)."""
    d = workloads.small_params(n_flavor=nf, n_energy=7, n_u=3, n_steps=1000, renorm=0,
                               r_start_km=60.0, r_end_km=70.0)
    m = oracle.Model(d); m.run()
    x = m.get_state()
    nrm = np.sqrt(np.sum(x * x, axis=0))
    assert np.max(np.abs(nrm - 1.0)) <= bound


def _tilted_nunu_only(oracle, steps, jac=True):
    d = workloads.small_params(n_flavor=2, n_energy=6, n_u=5, n_steps=steps, renorm=1,
                               r_start_km=30.0, r_end_km=60.0, dm2_ev2=[0.0, 0.0],
                               n0_cm3=0.0, lum_erg_s=[1e49, 1e49, 1e49])
    m = oracle.Model(d)
    rng = np.random.default_rng(9)
    P = rng.normal(size=(3, m.nb)) + np.array([[0.0], [0.0], [2.0]])
    P /= np.linalg.norm(P, axis=0)
    m.set_state(P, 0)
    _, D0 = m.moments(d["r_start_km"])
    m.run()
    _, D1 = m.moments(d["r_end_km"])
    return np.linalg.norm(D1 - D0) / np.linalg.norm(D0)


def test_flux_weighted_polarisation_invariant(oracle):
    """Pure nu-nu evolution conserves D = sum_b g_b P~_b (Eq. Hnu's kernel is symmetric
    once the d cos(theta') Jacobian is in); the integrator keeps it to O(h^4)."""
    e1 = _tilted_nunu_only(oracle, 200)
    e2 = _tilted_nunu_only(oracle, 400)
    e3 = _tilted_nunu_only(oracle, 800)
    assert e3 < 2e-7
    assert e1 / e2 > 12 and e2 / e3 > 12


def test_single_angle_equals_one_angle_bin(oracle):
    d = workloads.small_params(n_flavor=2, n_energy=9, n_u=1, n_steps=60)
    m = oracle.Model(d); m.run()
    sa = oracle.single_angle_run(d)
    np.testing.assert_allclose(m.pee()[:, 0, :], sa, atol=1e-12)


@pytest.mark.parametrize("nf", [2, 3])
@pytest.mark.parametrize("xbar", [False, True])
def test_two_tracked_species_equal_explicit_species(oracle, nf, xbar):
    """Tracking every initially populated flavour explicitly (the paper's four particles;
    six for three flavours) gives the electron-born results of the two tracked species, and
    each heavy-flavour-born state is the complement fixed by unitarity (sum over the flavours
    of the same particle type = I).  With xbar the anti-nu_x spectrum differs from nu_x."""
    kw = dict(lum_xbar_erg_s=2.3e51, temp_xbar_mev=5.1) if xbar else {}
    d = workloads.small_params(n_flavor=nf, n_energy=5, n_u=3, n_steps=40, **kw)
    a = oracle.Model(d); a.run()
    b = oracle.Model(d, species4=1); b.run()
    pa, pb = a.pee(), b.pee()
    np.testing.assert_allclose(pa[0], pb[0], atol=1e-11)        # nu_e-born
    np.testing.assert_allclose(pa[1], pb[nf], atol=1e-11)       # anti-nu_e-born
    # P_ee summed over the born flavours of one particle type is 1 (columns of a unitary)
    np.testing.assert_allclose(pb[:nf].sum(axis=0), 1.0, atol=1e-11)
    np.testing.assert_allclose(pb[nf:].sum(axis=0), 1.0, atol=1e-11)
    if xbar:
        c = oracle.Model(workloads.small_params(n_flavor=nf, n_energy=5, n_u=3, n_steps=40))
        c.run()
        assert np.abs(c.pee() - pa).max() > 1e-8                # the anti-nu_x spectrum matters


# ------------------------------------------------------------------ integrator
def _err_at(oracle, steps, integrator=0, ref_steps=3200):
    """Non-stiff setting (h |H| < 1) with O(1) flavour conversion."""
    base = dict(n_flavor=2, n_energy=5, n_u=3, r_start_km=60.0, r_end_km=64.0,
                lum_erg_s=[1e50, 6e49, 3e49], n0_cm3=1e30, theta=[0.5, 0.0, 0.0])
    d = workloads.small_params(n_steps=steps, **base)
    m = oracle.Model(d, integrator=integrator); m.run()
    r = oracle.Model(workloads.small_params(n_steps=ref_steps, **base)); r.run()
    assert np.max(np.abs(r.pee() - 1.0)) > 0.3           # the case is not trivial
    return np.max(np.abs(m.pee() - r.pee()))


def test_rkmk4_fourth_order(oracle):
    e = [_err_at(oracle, n) for n in (50, 100, 200)]
    assert e[0] / e[1] > 12 and e[1] / e[2] > 12
    assert e[2] < 3e-6


def test_plain_rk4_agrees_on_nonstiff(oracle):
    ea = _err_at(oracle, 100, integrator=1)
    eb = _err_at(oracle, 200, integrator=1)
    assert ea / eb > 12 and eb < 3e-5


def test_plain_rk4_fails_on_stiff_bulb(oracle):
    """At the neutrinosphere the matter and nu-nu terms are ~1e5-1e6 km^-1 against a
    0.1 km step: the explicit RK4 stability bound is violated by orders of magnitude."""
    d = workloads.two_flavor_small()
    d["renorm"] = 0
    m = oracle.Model(d, integrator=1)
    with pytest.raises(oracle.OracleError):
        m.step(40)


# ------------------------------------------------------------------ determinism
def test_thread_count_and_restart_are_bitwise(oracle):
    d = workloads.small_params(n_flavor=3, n_energy=11, n_u=4, n_steps=12)
    outs = []
    for t in (1, 2, 8):
        oracle.set_threads(t)
        m = oracle.Model(d); m.run(); outs.append(m.get_state())
    oracle.set_threads(0)
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])
    m = oracle.Model(d); m.step(5)
    x = m.get_state()
    m2 = oracle.Model(d); m2.set_state(x, 5); m2.step(7)
    np.testing.assert_array_equal(m2.get_state(), outs[0])


@pytest.mark.parametrize("nf", [2, 3])
def test_one_step_equals_definition(oracle, nf):
    """One oracle RKMK4 step from a random state against the method written out with dense
    matrices and SciPy's expm: stage generators K_i = (h / cos theta(r_i)) H(r_i, Y_i) with
    H = H_vac + lam E_ee + H_nunu (antineutrinos: H_vac - lam E_ee - H_nunu^*, H_nunu by the
    brute-force pair sum over the stage state Y_i), Y2 = e^{-i K1/2} psi,
    Y3 = e^{-i (K2/2 + i[K1,K2]/8)} psi, Y4 = e^{-i K3} psi and
    psi' = e^{-i Theta} psi with Theta = (K1 + 2 K2 + 2 K3 + K4)/6 + i[K1,K4]/12.  This pins
    the oracle's restated arithmetic (generators from per-row constants, commutators by
    bilinearity, the eigen-split exponential, fixed-point moments) against the definitions."""
    NE, NU = 3, 4
    d = workloads.small_params(n_flavor=nf, n_energy=NE, n_u=NU, n_steps=100, r_start_km=100.0,
                               r_end_km=101.0, n0_cm3=1e32)
    m = oracle.Model(d)
    rng = np.random.default_rng(29)
    nb = 2 * NU * NE
    if nf == 2:
        P = rng.normal(size=(3, nb)); P /= np.linalg.norm(P, axis=0)
        m.set_state(P, 0)
        sig = [np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]])]
        rho0 = 0.5 * (np.eye(2)[None] + sum(P[i][:, None, None] * sig[i] for i in range(3)))
    else:
        psi = rng.normal(size=(6, nb)); psi /= np.linalg.norm(psi, axis=0)
        m.set_state(psi, 0)
        pv = (psi[0::2] + 1j * psi[1::2]).T
        rho0 = np.einsum("bi,bj->bij", pv, pv.conj())
    rho0 = rho0.reshape(2, NU, NE, nf, nf)
    E, dE, u, du = ref.bins(d)
    R, h = d["r_nu_km"], (d["r_end_km"] - d["r_start_km"]) / d["n_steps"]
    r0, rm, r1 = d["r_start_km"], d["r_start_km"] + 0.5 * h, d["r_start_km"] + h
    hvac = ref.hvac2 if nf == 2 else ref.hvac3
    e_ee = np.zeros((nf, nf)); e_ee[0, 0] = 1.0

    def gens(r, rho):
        lam = ref.sqrt2gf_km_cm3() * d["n0_cm3"] * (R / r) ** 3
        Hnn = ref.brute_h_nunu(d, r, rho[0], rho[1])
        K = np.zeros((2, NU, NE, nf, nf), complex)
        for s in range(2):
            sg = 1 if s == 0 else -1
            for j in range(NU):
                c = np.sqrt(1.0 - u[j] * (R / r) ** 2)
                for k in range(NE):
                    K[s, j, k] = (h / c) * (hvac(d, E[k]) + sg * lam * e_ee + Hnn[s, j, k])
        return K

    def evolve(G, rho):
        U = np.array([[[linalg.expm(-1j * G[s, j, k]) for k in range(NE)] for j in range(NU)]
                      for s in range(2)])
        return U @ rho @ np.conj(np.swapaxes(U, -1, -2))

    def icomm(A, B):
        return 1j * (A @ B - B @ A)

    K1 = gens(r0, rho0)
    K2 = gens(rm, evolve(0.5 * K1, rho0))
    K3 = gens(rm, evolve(0.5 * K2 + icomm(K1, K2) / 8.0, rho0))
    K4 = gens(r1, evolve(K3, rho0))
    want = evolve((K1 + 2.0 * K2 + 2.0 * K3 + K4) / 6.0 + icomm(K1, K4) / 12.0, rho0)
    m.step(1)
    x = m.get_state()
    if nf == 2:
        got = 0.5 * (np.eye(2)[None] + sum(x[i][:, None, None] * sig[i] for i in range(3)))
    else:
        gv = (x[0::2] + 1j * x[1::2]).T
        got = np.einsum("bi,bj->bij", gv, gv.conj())
    got = got.reshape(2, NU, NE, nf, nf)
    kmax = max(np.abs(K1).max(), np.abs(K4).max())
    assert kmax > 1e-3                      # the step actually rotates the states
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)
