"""The two-flavour Bloch-vector form (oracle/bloch2.py) and the dot-product test of the
oracle's reverse-mode adjoint.

Forward mode by complex-step differentiation of the Bloch form gives J v, the directional
derivative of every beam's final P_ee; the adjoint gives J^T w.  The dot-product identity
<J v, w> = <v, J^T w> must hold to rounding for any v, w.  The Bloch form itself is pinned
to the plain mode (an independent C implementation with density matrices and a Jacobi
exponential) and to central differences of itself.
"""
import numpy as np
import pytest

import workloads
from oracle.bloch2 import Bloch2, default_x


def _case(**kw):
    args = dict(n_flavor=2, n_energy=13, n_u=4, n_steps=60, r_start_km=60.0, r_end_km=80.0,
                n0_cm3=1e31, lum_erg_s=[3e50, 2e50, 1e50], theta=[0.5, 0.0, 0.0])
    args.update(kw)
    return workloads.small_params(**args)


CASES = {
    "fd104": _case(),
    "ragged630": _case(n_energy=35, n_u=9, n_steps=40, r_end_km=75.0),
    # strong self-interaction with conversion across the spectrum (P_ee spread 0.95),
    # resolved by its step (the two C modes agree to 3e-14)
    "dense_nunu": _case(n_energy=16, n_u=5, n_steps=200, r_start_km=60.0, r_end_km=70.0,
                        lum_erg_s=[2e51, 1.5e51, 1e51]),
}


@pytest.mark.parametrize("name", list(CASES))
def test_bloch_form_matches_plain_mode(oracle, name):
    d = CASES[name]
    b = Bloch2(d)
    P = b.run(d["n_steps"])
    o = oracle.PlainModel(d)
    o.run()
    np.testing.assert_allclose(b.pee(P), o.pee().reshape(-1), rtol=0, atol=1e-12)
    s = oracle.Model(d)
    s.run()
    np.testing.assert_allclose(P, s.get_state(), rtol=0, atol=2e-12)


def test_bloch_form_without_self_interaction_is_a_rotation(oracle):
    """No self-interaction and no matter: the stage generators of a beam are parallel, the
    commutators vanish and the step integrates the path length l = int dr / c(r) =
    sqrt(r^2 - u R^2) between the ends, so P_ee follows the vacuum two-flavour formula
    1 - sin^2 2t sin^2(dm^2 l / 4E) up to the quadrature error of the step."""
    d = _case(lum_erg_s=[0.0, 0.0, 0.0], n0_cm3=0.0, n_u=1, n_steps=200)
    b = Bloch2(d)
    P = b.run(d["n_steps"])
    # with n_u = 1, u = 1/2: c(r) varies, l = int dr / c(r) = sqrt(r^2 - u R^2) |_r0^r1
    R, u = d["r_nu_km"], 0.5
    l = np.sqrt(d["r_end_km"] ** 2 - u * R * R) - np.sqrt(d["r_start_km"] ** 2 - u * R * R)
    om = abs(d["dm2_ev2"][0]) / (4.0 * b.E * 1.0e6) / 1.973269804e-10
    want = 1.0 - np.sin(2 * d["theta"][0]) ** 2 * np.sin(om * l) ** 2
    pee = b.pee(P).reshape(2, 1, -1)
    np.testing.assert_allclose(pee[0, 0], want, atol=1e-9)
    np.testing.assert_allclose(pee[1, 0], want, atol=1e-9)


@pytest.mark.parametrize("name", ["fd104", "dense_nunu"])
def test_complex_step_agrees_with_central_differences(name):
    d = CASES[name]
    b = Bloch2(d)
    x0 = default_x(d)
    rng = np.random.default_rng(5)
    w = rng.uniform(-1, 1, b.nb)
    for i in range(5):
        dx = np.zeros(5)
        dx[i] = x0[i] if i != 3 else 1.0
        jv, _ = b.jvp(d["n_steps"], dx=dx)
        hh = 1e-6
        xp = x0 + hh * dx
        xm = x0 - hh * dx
        fd = (b.pee(b.run(d["n_steps"], x=xp)) - b.pee(b.run(d["n_steps"], x=xm))) / (2 * hh)
        num, ref = float(w @ jv), float(w @ fd)
        assert abs(num - ref) <= 1e-6 * max(abs(ref), 1e-300) + 1e-12, (i, num, ref)


def _dot_test(adjoint_fn, d, seed):
    """<J dx, w> against <dx, J^T w> for the parameters, and <J_s u, w> against
    <u, state_bar> for the start state; returns the worst relative mismatch."""
    b = Bloch2(d)
    rng = np.random.default_rng(seed)
    w = rng.uniform(-1.0, 1.0, b.nb) / b.nb
    grad, sbar = adjoint_fn(d, w)
    x0 = default_x(d)
    worst = 0.0
    for trial in range(3):
        v = rng.uniform(-1.0, 1.0, 5)
        dx = v * np.where(np.arange(5) == 3, 1.0, x0)     # relative directions (theta absolute)
        u = rng.uniform(-1.0, 1.0, (3, b.nb))
        jv, _ = b.jvp(d["n_steps"], dx=dx)
        ju, _ = b.jvp(d["n_steps"], dstate=u)
        lhs_p, rhs_p = float(w @ jv), float(dx @ grad)
        lhs_s, rhs_s = float(w @ ju), float((u * sbar).sum())
        for lhs, rhs, scale in ((lhs_p, rhs_p, np.abs(dx * grad).sum()),
                                (lhs_s, rhs_s, np.abs(u * sbar).sum())):
            worst = max(worst, abs(lhs - rhs) / scale)
    return worst


def _oracle_adjoint(oracle):
    def fn(d, w):
        _, g, sb = oracle.Model(d).adjoint(ckpt=16, dl_dpee=w, want_state_bar=True)
        return g, sb
    return fn


@pytest.mark.parametrize("name", list(CASES))
def test_oracle_adjoint_dot_product(oracle, name):
    worst = _dot_test(_oracle_adjoint(oracle), CASES[name], seed=11)
    assert worst <= 1e-10, worst
