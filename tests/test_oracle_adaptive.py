"""Pins of the oracle's adaptive step-size control (RKMK4 steps with an embedded error
estimate, the paper integrating with an adaptive radial step, Sec. 3.4).

Each pin checks the oracle against something other than itself: the order of the error
estimator (the exponential midpoint rule's local error grows as h^3, so its square as h^6),
the vacuum closed form of P_ee at r_end, convergence towards a fine fixed-step run as the
tolerance shrinks, and the controller's bookkeeping (rejections retried with half the
step, the run ending exactly at r_end, failures reported).
"""
import numpy as np
import pytest

import workloads
from tests import physref as ref


def _resolved(nf):
    """Every rotation per step small: matter and nu-nu terms weak, energies >= 10 MeV."""
    d = workloads.small_params(n_flavor=nf, n_energy=6, n_u=3, n_steps=100, r_start_km=200.0,
                               r_end_km=300.0)
    d.update(n0_cm3=1e31, e_min_mev=10.0, e_max_mev=50.0)
    return d


@pytest.mark.parametrize("nf", [2, 3])
def test_error_estimate_is_sixth_order(oracle, nf):
    """|Theta - F_2|^2 is the square of the midpoint rule's local error, O(h^3): halving h
    divides it by 64.  Using F_1 instead of F_2 would give 16, a generator sum missing its
    1/6 would give 4."""
    m = oracle.Model(_resolved(nf))
    m.step(5)
    hs = [0.04, 0.02, 0.01, 0.005, 0.0025]
    es = [m.step_error(h) for h in hs]
    ratios = [es[i] / es[i + 1] for i in range(len(es) - 1)]
    for r in ratios:
        assert 62.0 < r < 67.0, ratios
    assert m.step_index() == 5                    # the estimate does not advance the state


def _vacuum(nf):
    return workloads.small_params(n_flavor=nf, n_energy=6, n_u=3, n_steps=40, r_start_km=10.0,
                                  r_end_km=40.0, lum_erg_s=[0.0, 0.0, 0.0], n0_cm3=0.0)


def _vacuum_pee(d, nf):
    E, dE, u, du = ref.bins(d)
    L = ref.path_length(d["r_end_km"], d["r_start_km"], d["r_nu_km"], u)[:, None]
    if nf == 2:
        w = ref.omega_km(d["dm2_ev2"][0], E)[None, :]
        return 1.0 - np.sin(2 * d["theta"][0]) ** 2 * np.sin(w * L) ** 2
    U = ref.pmns(*d["theta"])
    m2 = [0.0, d["dm2_ev2"][0], d["dm2_ev2"][1]]
    want = np.ones((len(u), len(E)))
    for i in range(3):
        for j in range(i + 1, 3):
            ph = (m2[j] - m2[i]) / (4.0 * E * 1e6) / ref.HBARC_EV_KM
            want -= 4 * U[0, i] ** 2 * U[0, j] ** 2 * np.sin(ph[None, :] * L) ** 2
    return want


@pytest.mark.parametrize("nf", [2, 3])
def test_adaptive_vacuum_closed_form(oracle, nf):
    """Vacuum: P_ee at r_end (path length measured to exactly r_end) against the closed
    form; the error falls with the tolerance."""
    d = _vacuum(nf)
    want = _vacuum_pee(d, nf)
    errs = []
    for tol, bound in ((1e-4, 1e-7), (1e-6, 3e-10), (1e-8, 1e-12)):
        m = oracle.Model(d)
        st = m.run_adaptive(tol)
        assert m.step_index() == d["n_steps"]
        err = max(np.abs(m.pee()[s] - want).max() for s in range(2))
        assert err < bound, (tol, err, st)
        errs.append(err)
    assert errs[0] > errs[1] > errs[2]


@pytest.mark.parametrize("nf", [2, 3])
def test_adaptive_converges_to_fine_fixed_steps(oracle, nf):
    """A bulb case with matter and neutrino-neutrino terms (100 -> 102 km, n0 = 1e32):
    the adaptive result approaches a fixed-step run with 16000 steps (itself converged to
    1e-10) as the tolerance shrinks."""
    d = workloads.small_params(n_flavor=nf, n_energy=8, n_u=4, n_steps=20, r_start_km=100.0,
                               r_end_km=102.0, n0_cm3=1e32)
    f = oracle.Model(dict(d, n_steps=16000))
    f.run()
    ref_pee = f.pee()
    errs = []
    for tol in (1e-4, 1e-5, 1e-6):
        m = oracle.Model(d)
        m.run_adaptive(tol)
        errs.append(np.abs(m.pee() - ref_pee).max())
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[2] < 3e-6, errs


@pytest.mark.parametrize("ratio,doubles", [(110.0, False), (150.0, True)])
def test_growth_threshold_is_tol2_over_128(oracle, ratio, doubles):
    """The step doubles after an accepted step only if its estimate E <= tol^2/128.  With
    four steps of h and the first estimate E1 = tol^2/ratio (the estimate changes by a few
    per cent from step to step here): at ratio 110 the step never doubles (four accepted
    steps; a threshold of tol^2/64 would double it, giving h, 2h, h); at ratio 150 it
    doubles after the first step (three accepted steps; tol^2/256 would not)."""
    d = _resolved(2)
    d.update(r_start_km=200.0, r_end_km=200.08, n_steps=4)      # h = 0.02 km
    m = oracle.Model(d)
    e1 = m.step_error(0.02)
    es = []
    for k in range(4):
        es.append(m.step_error(0.02))
        m.step(1)
    assert max(es) / min(es) < 1.05                              # E nearly constant
    assert e1 * 64 * 1.05 < e1 * ratio                          # the doubled step passes
    tol = float(np.sqrt(e1 * ratio))
    st = oracle.Model(d).run_adaptive(tol)
    assert st["rejected"] == 0
    assert st["accepted"] == (3 if doubles else 4), (st, es)


def test_rejected_steps_are_retried_with_half_the_step(oracle):
    """A first step far too long for the tolerance is rejected and retried with h/2 until
    it passes; the tally adds up, and the step never grows above h_max."""
    d = workloads.small_params(n_flavor=2, n_energy=8, n_u=4, n_steps=1, r_start_km=100.0,
                               r_end_km=102.0, n0_cm3=1e32)
    m = oracle.Model(d)
    st = m.run_adaptive(1e-6, h_max=0.05)
    assert st["rejected"] >= 5                        # 2 km -> below 0.05 km takes 6 halvings
    assert st["h_last"] <= 0.05
    # same run with a generous cap on attempts: identical result, and the cap is enforced
    m2 = oracle.Model(d)
    st2 = m2.run_adaptive(1e-6, h_max=0.05, max_attempts=st["accepted"] + st["rejected"])
    assert st2 == st
    np.testing.assert_array_equal(m.pee(), m2.pee())
    m3 = oracle.Model(d)
    with pytest.raises(Exception):
        m3.run_adaptive(1e-6, h_max=0.05, max_attempts=st["accepted"] + st["rejected"] - 1)


def test_adaptive_argument_checks(oracle):
    d = _vacuum(2)
    with pytest.raises(Exception):
        oracle.Model(d).run_adaptive(0.0)
    m = oracle.Model(d)
    m.step(1)
    with pytest.raises(Exception):
        m.run_adaptive(1e-6)                          # not at the start
    with pytest.raises(Exception):
        oracle.Model(d, integrator=1).run_adaptive(1e-6)
