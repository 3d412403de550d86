"""Reverse-mode adjoint on the GPU: against the oracle's adjoint, against central
differences of the GPU forward integration, checkpoint-period invariance, the autograd
wrapper, and a prefix of the 200k-beam adjoint workload.

Tolerance against the oracle: the forward states are the same bits on both sides, and
the reverse passes differ only in the order of the FP64 sums of the moment adjoints (a
grid-wide sum per stage on the GPU, a sequential sum in the oracle) and in the sin/cos of
the rotation Jacobians (the library's own against libm).  Those are rounding-level
differences of a linear recursion, so gradients agree to 1e-9 relative, far inside the
1e-6 that central differences can confirm.
"""
import copy
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

RTOL = 1e-9


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


def _case(**kw):
    args = dict(n_flavor=2, n_energy=13, n_u=4, n_steps=60, r_start_km=60.0, r_end_km=80.0,
                n0_cm3=1e31, lum_erg_s=[3e50, 2e50, 1e50], theta=[0.5, 0.0, 0.0])
    args.update(kw)
    return workloads.small_params(**args)


CASES = {
    "fd104": (_case(), 7),
    "ragged1260": (_case(n_energy=70, n_u=9, n_steps=40, r_end_km=75.0), 16),
    # the 1024-beam shape with its step length, started where the step resolves it
    "resolved1024": (workloads.resolved(dict(workloads.two_flavor_small(), n_steps=90), 700.0), 64),
}


def _cot(nb_beams, seed):
    return np.random.default_rng(seed).uniform(-1.0, 1.0, nb_beams) / nb_beams


def _gpu_adjoint(nb, d, ckpt, c=None, state_bar=True):
    import torch
    m = nb.Model(d, adjoint_ckpt=ckpt)
    ct = None if c is None else torch.as_tensor(c, device="cuda")
    g, sb = m.adjoint(ct, want_state_bar=True)
    return m, g, sb.cpu().numpy()


@pytest.mark.parametrize("name", list(CASES))
def test_adjoint_matches_oracle(nb, oracle, name):
    d, ckpt = CASES[name]
    _say(f"adjoint vs oracle: {name}")
    o = oracle.Model(d)
    c = _cot(o.nb, 11)
    Lo, go, sbo = o.adjoint(ckpt, c, want_state_bar=True)
    m, g, sb = _gpu_adjoint(nb, d, ckpt, c)
    assert m.step_index() == d["n_steps"]
    # same forward bits: the loss and the final state agree exactly
    pee = m.pee().cpu().numpy()
    np.testing.assert_array_equal(pee, o.pee().reshape(-1))
    assert float(c @ pee) == pytest.approx(Lo, rel=1e-13)    # numpy and the oracle sum in different orders
    np.testing.assert_allclose(g, go, rtol=RTOL, atol=0)
    np.testing.assert_allclose(sb, sbo, rtol=RTOL, atol=RTOL * np.abs(sbo).max())


def test_adjoint_default_cotangent_matches_oracle(nb, oracle):
    d, ckpt = CASES["ragged1260"]
    _, go = oracle.Model(d).adjoint(ckpt)
    m = nb.Model(d, adjoint_ckpt=ckpt)
    np.testing.assert_allclose(m.adjoint(), go, rtol=RTOL, atol=0)


def test_adjoint_matches_central_differences(nb):
    """dL/d{L_e, L_ebar, L_x, theta_v, n0} from the GPU adjoint against central
    differences of GPU forward runs, step 1e-6 of each parameter."""
    import torch
    d, ckpt = CASES["fd104"]
    m = nb.Model(d, adjoint_ckpt=ckpt)
    c = _cot(m.nb, 3)
    g = m.adjoint(torch.as_tensor(c, device="cuda"))
    x0 = [*d["lum_erg_s"], d["theta"][0], d["n0_cm3"]]

    def loss(x):
        f = nb.Model(nb._with_params(d, x))
        f.run()
        return float(c @ f.pee().cpu().numpy())

    for i in range(5):
        h = 1e-6 * abs(x0[i])
        xp = list(x0); xp[i] += h
        xm = list(x0); xm[i] -= h
        fd = (loss(xp) - loss(xm)) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-6), (nb.PARAM_NAMES[i], g[i], fd)


def test_adjoint_checkpoint_periods_bitwise(nb):
    """Every checkpoint period recomputes the same forward bits and sums the moment
    adjoints in the same order: identical gradients and state adjoints."""
    d = _case(n_steps=23, r_end_km=70.0)
    fwd = nb.Model(d); fwd.run()
    ref = None
    for k in (1, 5, 23, 64):
        m = nb.Model(d, adjoint_ckpt=64)
        g, sb = m.adjoint(None, ckpt=k, want_state_bar=True)
        np.testing.assert_array_equal(m.get_state().cpu().numpy(), fwd.get_state().cpu().numpy())
        if ref is None:
            ref = (g, sb.cpu().numpy())
        else:
            np.testing.assert_array_equal(g, ref[0], err_msg=f"ckpt {k}")
            np.testing.assert_array_equal(sb.cpu().numpy(), ref[1], err_msg=f"ckpt {k}")


def test_adjoint_from_mid_run_and_repeat(nb, oracle):
    d, ckpt = CASES["ragged1260"]
    o = oracle.Model(d); o.step(13)
    _, go = o.adjoint(ckpt)
    m = nb.Model(d, adjoint_ckpt=ckpt)
    m.step(13)
    g1 = m.adjoint()
    np.testing.assert_allclose(g1, go, rtol=RTOL, atol=0)
    m.reset(); m.step(13)
    np.testing.assert_array_equal(m.adjoint(), g1)      # bit-for-bit repeatable
    g_end = m.adjoint()                                   # already at r_end: nothing to do
    np.testing.assert_array_equal(g_end, np.zeros(5))


def test_autograd_function(nb):
    import torch
    d, ckpt = CASES["fd104"]
    x = torch.tensor([*d["lum_erg_s"], d["theta"][0], d["n0_cm3"]], dtype=torch.float64,
                     requires_grad=True)
    pee = nb.bulb_pee(x, d, ckpt)
    c = torch.as_tensor(_cot(pee.numel(), 5), device=pee.device)
    (c * pee).sum().backward()
    m = nb.Model(d, adjoint_ckpt=ckpt)
    np.testing.assert_array_equal(x.grad.numpy(), m.adjoint(c))


def test_adjoint_rejects_unsupported(nb):
    d3 = workloads.small_params(n_flavor=3, n_steps=4)
    with pytest.raises(nb.NubulbError):
        nb.Model(d3, adjoint_ckpt=2)
    m = nb.Model(_case(n_steps=8))                        # created without adjoint_ckpt
    with pytest.raises(nb.NubulbError):
        m.adjoint()
    m = nb.Model(_case(n_steps=40), adjoint_ckpt=8)       # 5 + 8 slots reserved
    with pytest.raises(nb.NubulbError):
        m.adjoint(ckpt=20)                                 # 2 + 20 slots needed
    assert m.step_index() == 0


def test_adjoint_200k_full_run_against_central_differences(nb):
    """The 200k-beam adjoint workload (200 E x 500 u x 2, 5000 steps, checkpoints every 64
    steps) in its resolved variant (500 -> 790 km), loss = energy-integrated final P_ee of
    both species (summed exactly, math.fsum, then scaled by dE/N_u): the five gradients
    against central differences of full GPU forward runs.

    At x +- 1e-6 |x| every gradient must agree to 1e-6 except where the difference quotient
    itself is limited by the rounding of the forward runs: the loss (about 50) carries a
    rounding of a few 1e-15 whatever the parameter (measured: 4e-15), against a change
    2h dL/dx of 8e-11 for L_x (x dL/dx = -4e-5), a floor of 5e-5 relative.  Where that floor
    exceeds 5e-7 the quotient at h = 1e-6 must stay within twice it, and the gradient must
    agree to 1e-6 with the quotient at x +- 1e-4 |x|, where the floor is a hundred times
    lower and the truncation error (h^2/6 of the third derivative) of a luminosity, on
    which the loss depends smoothly this far out, stays near 1e-9 relative.  (theta_v is not
    such a parameter: the loss oscillates in it, and at 1e-4 the truncation error is 8e-5;
    at 1e-6 its quotient agrees to 2e-9.)
    """
    import math
    d = workloads.adjoint_200k_resolved()
    m = nb.Model(d, adjoint_ckpt=64)
    g = m.adjoint()
    cw = ((d["e_max_mev"] - d["e_min_mev"]) / d["n_energy"]) / d["n_u"]
    x0 = [*d["lum_erg_s"], d["theta"][0], d["n0_cm3"]]
    del m

    def loss(x):
        f = nb.Model(nb._with_params(d, x))
        f.run()
        return cw * math.fsum(f.pee().cpu().numpy().tolist())

    def central(i, rel):
        h = rel * abs(x0[i])
        xp = list(x0); xp[i] += h
        xm = list(x0); xm[i] -= h
        return (loss(xp) - loss(xm)) / (2 * h)

    for i in range(5):
        f6, f4 = central(i, 1e-6), central(i, 1e-4)
        r6, r4 = abs(g[i] - f6) / abs(f6), abs(g[i] - f4) / abs(f4)
        _say(f"200k full run: dL/d{nb.PARAM_NAMES[i]} adjoint {g[i]:.10e} central(1e-6) {f6:.10e} "
             f"rel {r6:.2e}; central(1e-4) {f4:.10e} rel {r4:.2e}")
        floor = 4e-15 / (2e-6 * abs(x0[i] * g[i]))     # loss rounding over 2h dL/dx
        if floor <= 5e-7:
            assert r6 <= 1e-6, (nb.PARAM_NAMES[i], g[i], f6, floor)
        else:
            assert r6 <= 2.0 * floor, (nb.PARAM_NAMES[i], g[i], f6, floor)
            assert r4 <= 1e-6, (nb.PARAM_NAMES[i], g[i], f4)


def test_adjoint_beyond_four_beams_per_thread(nb, oracle):
    """1.1M beams (500 E x 1100 u x 2), more than four per resident thread of the reverse
    kernel: its spill variant keeps the beams' adjoint registers in the workspace between
    phases.  Against the oracle adjoint, 6 steps with checkpoints every 4 (a full and a
    short segment), the 200k workload's step length from 500 km, random cotangent."""
    import torch
    d = workloads.adjoint_200k_resolved()
    h = (d["r_end_km"] - d["r_start_km"]) / d["n_steps"]
    d = dict(d, n_energy=500, n_u=1100, n_steps=6, r_end_km=d["r_start_km"] + 6 * h)
    _say("adjoint 1.1M beams: oracle")
    o = oracle.Model(d)
    c = _cot(o.nb, 17)
    _, go, sbo = o.adjoint(4, c, want_state_bar=True)
    _say("adjoint 1.1M beams: gpu")
    m = nb.Model(d, adjoint_ckpt=4)
    g, sb = m.adjoint(torch.as_tensor(c, device="cuda"), want_state_bar=True)
    _say(f"grad gpu {g} oracle {go}")
    np.testing.assert_allclose(g, go, rtol=RTOL, atol=0)
    sb = sb.cpu().numpy()
    np.testing.assert_allclose(sb, sbo, rtol=RTOL, atol=RTOL * np.abs(sbo).max())
    np.testing.assert_array_equal(m.pee().cpu().numpy(), o.pee().reshape(-1))


def test_adjoint_200k_prefix(nb, oracle):
    """The 200k-beam adjoint workload (200 E x 500 u x 2) in its resolved variant, its
    first 70 steps with checkpoints every 64 steps (a full and a ragged segment)."""
    d = copy.deepcopy(workloads.adjoint_200k_resolved())
    h = (d["r_end_km"] - d["r_start_km"]) / d["n_steps"]
    d["n_steps"] = 70
    d["r_end_km"] = d["r_start_km"] + 70 * h
    _say("adjoint 200k prefix: oracle")
    _, go = oracle.Model(d).adjoint(64)
    _say("adjoint 200k prefix: gpu")
    m = nb.Model(d, adjoint_ckpt=64)
    g = m.adjoint()
    _say(f"grad gpu {g} oracle {go}")
    np.testing.assert_allclose(g, go, rtol=RTOL, atol=0)


@pytest.mark.parametrize("name", ["fd104", "ragged1260", "dense_nunu"])
def test_adjoint_dot_product_with_forward_mode(nb, name):
    """<J v, w> = <v, J^T w>: the GPU adjoint (J^T w: parameter gradient and state_bar)
    against forward-mode directional derivatives J v of the two-flavour Bloch form by
    complex-step differentiation (oracle/bloch2.py), for random v (parameters and start
    state) and random cotangents w."""
    import torch
    sys.path.insert(0, __import__("os").path.dirname(__file__))
    from test_oracle_bloch2 import CASES as BCASES, _dot_test
    d = BCASES["dense_nunu"] if name == "dense_nunu" else CASES[name][0]

    def gpu_adjoint(dd, w):
        m = nb.Model(dd, adjoint_ckpt=16)
        g, sb = m.adjoint(torch.as_tensor(w, device="cuda"), want_state_bar=True)
        return g, sb.cpu().numpy()

    worst = _dot_test(gpu_adjoint, d, seed=23)
    _say(f"dot product {name}: worst relative mismatch {worst:.2e}")
    assert worst <= 1e-9, worst
