"""Pins of the oracle's reverse-mode adjoint (two flavours).

The adjoint is checked against central finite differences of the oracle's own forward
integration (a different computation: no derivative code is involved), against the closed
form of the vacuum derivative, and against properties every adjoint has (linearity in
the cotangent, independence of the checkpoint period).
"""
import copy

import numpy as np
import pytest

import workloads
from tests import physref as ref

PARAMS = [("lum_erg_s", 0), ("lum_erg_s", 1), ("lum_erg_s", 2), ("theta", 0), ("n0_cm3", None)]


def _case(**kw):
    """Resolved two-flavour case in which every parameter moves the final P_ee by a
    sizeable fraction (an MSW region crossed by the path and a nu-nu term of the same
    size), so that central differences resolve the gradient far below 1e-6."""
    args = dict(n_flavor=2, n_energy=13, n_u=4, n_steps=60, r_start_km=60.0, r_end_km=80.0,
                n0_cm3=1e31, lum_erg_s=[3e50, 2e50, 1e50], theta=[0.5, 0.0, 0.0])
    args.update(kw)
    return workloads.small_params(**args)


def _cotangent(nb, seed=1):
    return np.random.default_rng(seed).uniform(-1.0, 1.0, nb) / nb


def _loss(oracle, d, c, state=None):
    o = oracle.Model(d)
    if state is not None:
        o.set_state(state, 0)
    o.run()
    return float(c @ o.pee().reshape(-1))


def _shift(d, key, j, delta):
    q = copy.deepcopy(d)
    if j is None:
        q[key] = q[key] + delta
    else:
        q[key][j] = q[key][j] + delta
    return q


def test_adjoint_matches_central_differences(oracle):
    """dL/d{L_e, L_ebar, L_x, theta_v, n0} against central differences with a step of
    1e-6 of each parameter's value."""
    d = _case()
    m = oracle.Model(d)
    c = _cotangent(m.nb)
    L, g = m.adjoint(7, c)
    assert L == pytest.approx(_loss(oracle, d, c), rel=1e-14)
    for i, (key, j) in enumerate(PARAMS):
        v = d[key] if j is None else d[key][j]
        h = 1e-6 * abs(v)
        fd = (_loss(oracle, _shift(d, key, j, h), c) - _loss(oracle, _shift(d, key, j, -h), c)) / (2 * h)
        assert abs(g[i] * v) > 1e-4, (key, j)          # the case must actually be sensitive
        assert g[i] == pytest.approx(fd, rel=1e-6), (key, j, g[i], fd)


def test_adjoint_of_initial_state_matches_central_differences(oracle):
    """The state cotangent that reaches r_start (through every stage rotation, the
    moment broadcasts and the renormalisations) against differences of the initial
    Bloch vectors of a few beams.  The step is 1e-4: along P_z of an initial eigenstate
    the renormalisation removes most of the change, the derivative is small and a smaller
    step is dominated by rounding of the loss."""
    d = _case(n_steps=30, r_end_km=70.0)
    m = oracle.Model(d)
    c = _cotangent(m.nb, seed=2)
    x0 = m.get_state().copy()
    _, _, sbar = m.adjoint(4, c, want_state_bar=True)
    h = 1e-4
    for b in (0, 17, m.nb - 1):
        for comp in range(3):
            xp = x0.copy(); xp[comp, b] += h
            xm = x0.copy(); xm[comp, b] -= h
            fd = (_loss(oracle, d, c, xp) - _loss(oracle, d, c, xm)) / (2 * h)
            assert sbar[comp, b] == pytest.approx(fd, rel=2e-6, abs=2e-12), (b, comp)


def test_adjoint_vacuum_mixing_angle_closed_form(oracle):
    """No matter, no neutrinos: P_ee = 1 - sin^2(2 theta) sin^2(omega L), so
    dP_ee/dtheta = -2 sin(4 theta) sin^2(omega L) for every beam.  (Away from the
    neutrinosphere the step's quadrature of the path length is exact to rounding.)"""
    d = workloads.small_params(n_flavor=2, n_energy=6, n_u=3, n_steps=300, r_start_km=60.0,
                               r_end_km=90.0, lum_erg_s=[0.0, 0.0, 0.0], n0_cm3=0.0,
                               theta=[0.3, 0.0, 0.0])
    m = oracle.Model(d)
    c = _cotangent(m.nb, seed=3)
    _, g = m.adjoint(64, c)
    E, dE, u, du = ref.bins(d)
    Lp = ref.path_length(d["r_end_km"], d["r_start_km"], d["r_nu_km"], u)[:, None]
    w = ref.omega_km(d["dm2_ev2"][0], E)[None, :]
    dp = -2.0 * np.sin(4 * d["theta"][0]) * np.sin(w * Lp) ** 2      # [u][E]
    want = float(c @ np.concatenate([dp.reshape(-1), dp.reshape(-1)]))
    assert g[3] == pytest.approx(want, rel=1e-9, abs=1e-13)


def test_adjoint_independent_of_checkpoint_period(oracle):
    """Recomputed segments are the same arithmetic: every period gives the same bits, and
    the model is left at r_end with the state of a plain forward run."""
    d = _case(n_steps=23, r_end_km=70.0)
    fwd = oracle.Model(d); fwd.run()
    res = []
    for k in (1, 5, 23, 64):
        m = oracle.Model(d)
        L, g, sb = m.adjoint(k, None, want_state_bar=True)
        assert m.step_index() == d["n_steps"]
        np.testing.assert_array_equal(m.get_state(), fwd.get_state())
        res.append((L, g, sb))
    for L, g, sb in res[1:]:
        assert L == res[0][0]
        np.testing.assert_array_equal(g, res[0][1])
        np.testing.assert_array_equal(sb, res[0][2])


def test_adjoint_default_loss_and_linearity(oracle):
    """The default loss is the energy-integrated, angle-averaged P_ee of both species
    (cotangent dE/N_u), and gradients are linear in the cotangent."""
    d = _case(n_steps=20, r_end_km=66.0)
    nb = oracle.Model(d).nb
    dE = (d["e_max_mev"] - d["e_min_mev"]) / d["n_energy"]
    L0, g0 = oracle.Model(d).adjoint(8)
    L1, g1 = oracle.Model(d).adjoint(8, np.full(nb, dE / d["n_u"]))
    assert L0 == L1
    np.testing.assert_array_equal(g0, g1)
    ca, cb = _cotangent(nb, 4), _cotangent(nb, 5)
    _, ga = oracle.Model(d).adjoint(8, ca)
    _, gb = oracle.Model(d).adjoint(8, cb)
    _, gs = oracle.Model(d).adjoint(8, 2.0 * ca - 3.0 * cb)
    np.testing.assert_allclose(gs, 2.0 * ga - 3.0 * gb, rtol=1e-11, atol=1e-11 * np.abs(gs).max())


def test_adjoint_rejects_unsupported_modes(oracle):
    with pytest.raises(oracle.OracleError):
        oracle.Model(workloads.small_params(n_flavor=3, n_steps=4)).adjoint(2)
    with pytest.raises(oracle.OracleError):
        oracle.Model(_case(n_steps=4)).adjoint(0)


def test_resolved_adjoint_workload_is_resolved(oracle):
    """At the start of the resolved adjoint variant every beam's first-stage rotation
    angle h |B| / cos(theta) is below one radian (vacuum, matter and nu-nu terms of the
    initial state), while at the neutrinosphere it is far above: there the step does not
    resolve the Hamiltonian."""
    d = dict(workloads.adjoint_200k_resolved(), n_energy=20, n_u=50)
    h = (d["r_end_km"] - d["r_start_km"]) / d["n_steps"]
    for r, resolved in ((d["r_start_km"], True), (d["r_nu_km"], False)):
        m = oracle.Model(d)
        j0, j1 = m.moments(r)
        B = m.hamiltonian(r, j0, j1)
        c = np.tile(np.repeat(m.cos_theta(r), d["n_energy"]), 2)
        angle = h * np.linalg.norm(B, axis=1) / c
        assert (angle.max() < 1.0) == resolved, (r, angle.max())
