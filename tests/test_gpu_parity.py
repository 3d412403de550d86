"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle, element by element.

Both sides implement one arithmetic specification from separate sources, so the bar is
bit-for-bit equality of the final state and P_ee (which the tolerance 1e-10 in P_ee
contains).  Sizes span several waves and ragged row tails; the largest cases use the
benchmark's shapes and launch configuration.
"""
import os
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


@pytest.fixture(scope="module")
def hooks():
    from paper_1912_10596_amd import testhooks
    testhooks.lib()
    return testhooks


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


# ------------------------------------------------------------- primitives
def test_sqrt_and_division_correctly_rounded(hooks):
    rng = np.random.default_rng(1)
    a = np.abs(rng.normal(size=200000)) * 10.0 ** rng.uniform(-300, 300, 200000)
    b = rng.normal(size=200000) * 10.0 ** rng.uniform(-150, 150, 200000)
    sq, dv = hooks.test_sqrt_div(_dev(a), _dev(b))
    np.testing.assert_array_equal(sq.cpu().numpy(), np.sqrt(a))
    np.testing.assert_array_equal(dv.cpu().numpy(), a / b)


def test_sincos_bitwise(hooks, oracle):
    rng = np.random.default_rng(2)
    x = np.concatenate([np.linspace(-10, 10, 100001), rng.uniform(-4e6, 4e6, 100000),
                        rng.normal(size=10000) * 1e-8, [0.0, -0.0]])
    s, c = hooks.test_sincos(_dev(x))
    so, co = oracle.sincos(x)
    np.testing.assert_array_equal(s.cpu().numpy(), so)
    np.testing.assert_array_equal(c.cpu().numpy(), co)


def test_rotation_bitwise(hooks, oracle):
    rng = np.random.default_rng(3)
    n = 3000
    x = rng.normal(size=(n, 3)) * 10.0 ** rng.uniform(-6, 6, (n, 1))
    x[0] = 0.0
    p = rng.normal(size=(n, 3))
    p /= np.linalg.norm(p, axis=1, keepdims=True)
    got = hooks.test_rotate(_dev(x), _dev(p)).cpu().numpy()
    want = np.stack([oracle.rotate(x[i], p[i]) for i in range(n)])
    np.testing.assert_array_equal(got, want)


def test_exp3_bitwise(hooks, oracle):
    rng = np.random.default_rng(4)
    ks, ps = [], []
    for scale in (0.0, 1e-6, 0.2, 3.0, 500.0, 3e6):
        for kind in range(4):
            for _ in range(200):
                k9 = rng.normal(size=9) * scale
                if kind == 1:
                    k9[3:] *= 1e-5                     # nearly diagonal
                elif kind == 2:
                    k9[1] = k9[2]; k9[7:] = 0.0        # mu-tau degenerate block
                elif kind == 3:
                    k9[0] += 1e3 * scale               # matter dominated
                ks.append(k9)
                p = rng.normal(size=6)
                ps.append(p / np.linalg.norm(p))
    # the form's range and its special cases: |K| at and around the 2^-100 floor, huge |K|,
    # psi along the isolated eigenvector (P psi from 1e-2 down to 0), flavour eigenstates of
    # a diagonal K, an exactly degenerate pair of eigenvalues
    for scale in (1e-31, 3e-30, 1e-29, 1e-20, 1e9, 1e14):
        for _ in range(50):
            ks.append(rng.normal(size=9) * scale)
            p = rng.normal(size=6)
            ps.append(p / np.linalg.norm(p))
    for scale in (0.3, 50.0):
        for _ in range(20):
            k9 = rng.normal(size=9) * scale
            H = np.diag(k9[:3]).astype(complex)
            for t, (a, b) in enumerate([(0, 1), (0, 2), (1, 2)]):
                H[a, b] = k9[3 + 2 * t] + 1j * k9[4 + 2 * t]
                H[b, a] = np.conj(H[a, b])
            ev, V = np.linalg.eigh(H - np.trace(H) / 3 * np.eye(3))
            i1 = int(np.argmax(np.abs(ev)))
            pl = V[:, [i for i in range(3) if i != i1]] @ (rng.normal(size=2) + 1j * rng.normal(size=2))
            for dlt in (1e-2, 1e-10, 1e-17, 0.0):
                pv = V[:, i1] + dlt * pl / np.linalg.norm(pl)
                pv /= np.linalg.norm(pv)
                ks.append(k9)
                ps.append(np.stack([pv.real, pv.imag], axis=1).ravel())
    for e in range(3):
        k9 = np.zeros(9); k9[:3] = [3.0, -1.0, 0.5]
        p = np.zeros(6); p[2 * e] = 1.0
        ks.append(k9); ps.append(p)
    k9 = np.zeros(9); k9[:3] = [2.0, -1.0, -1.0]          # eigenvalues (2, -1, -1) exactly
    for _ in range(10):
        p = rng.normal(size=6)
        ks.append(k9); ps.append(p / np.linalg.norm(p))
    ks, ps = np.array(ks), np.array(ps)
    got = hooks.test_exp3(_dev(ks), _dev(ps)).cpu().numpy()
    want = np.stack([oracle.exp3_apply(ks[i], ps[i]) for i in range(len(ks))])
    np.testing.assert_array_equal(got, want)


# ---------------------------------------------------------- stepping parity
CASES = [
    # (n_flavor, N_E, N_u, steps, r_start, r_end, max_blocks)
    (2, 37, 5, 40, 60.0, 62.0, 0),       # ragged rows: 37 < 64 lanes
    (2, 130, 7, 25, 10.0, 12.0, 0),      # 3 chunks per row, literal bulb start
    (2, 200, 9, 12, 10.0, 11.0, 3),      # few blocks: many rows per wave
    (2, 1, 1, 5, 30.0, 31.0, 0),         # single beam per species
    (3, 37, 5, 20, 60.0, 61.0, 0),
    (3, 70, 3, 10, 10.0, 10.5, 0),       # literal bulb start, 2 chunks, ragged tail
    (3, 64, 1, 6, 10.0, 10.3, 1),        # one block
    (3, 129, 4, 4, 40.0, 40.4, 2),
    # one row per wavefront (2 N_u a multiple of 8, as in the benchmark's launch) with short
    # last passes of 1-32 busy lanes
    (3, 80, 4, 12, 10.0, 10.6, 0),       # last pass 16 lanes, one block, literal bulb start
    (3, 96, 8, 8, 40.0, 40.8, 0),        # 32 lanes, two blocks
    (3, 400, 4, 6, 10.0, 10.3, 0),       # the benchmark's row length (16 lanes)
    (3, 65, 12, 6, 60.0, 60.6, 0),       # 1 lane, three blocks
    (2, 2200, 1, 4, 30.0, 30.4, 0),      # rows of two 2048-energy segments
    (3, 2100, 1, 3, 40.0, 40.3, 0),      # two segments; tables (151 KB) read from HBM, not LDS
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}f-{c[1]}x{c[2]}-{c[3]}st-b{c[6]}" for c in CASES])
def test_small_models_bitwise(nb, oracle, case):
    nf, ne, nu, steps, rs, re_, mb = case
    d = workloads.small_params(n_flavor=nf, n_energy=ne, n_u=nu, n_steps=steps,
                               r_start_km=rs, r_end_km=re_, max_blocks=mb)
    _say(f"case {case}")
    g = nb.Model(d)
    g.run()
    o = oracle.Model(d)
    o.run()
    np.testing.assert_array_equal(g.get_state().cpu().numpy(), o.get_state())
    np.testing.assert_array_equal(g.pee().cpu().numpy(), o.pee().reshape(-1))


def test_two_flavor_1024_beams_full_run(nb, oracle):
    """The 32 E x 16 u two-flavour model, 10 -> 200 km in 2000 steps: bitwise."""
    d = workloads.two_flavor_small()
    g = nb.Model(d); g.run()
    o = oracle.Model(d); o.run()
    pg, po = g.pee().cpu().numpy(), o.pee().reshape(-1)
    _say(f"max |dPee| = {np.max(np.abs(pg - po)):.3e}")
    np.testing.assert_array_equal(pg, po)


def test_three_flavor_800k_prefix(nb, oracle):
    """Benchmark shape (400 E x 1000 u x 2, 3 flavours) and launch configuration: the first
    100 steps from the neutrinosphere (10 -> 14.95 km), every beam compared bit for bit."""
    d = workloads.three_flavor_800k()
    g = nb.Model(d); g.step(100)
    _say("800k: 100 GPU steps done; oracle")
    o = oracle.Model(d); o.step(100)
    pg, po = g.pee().cpu().numpy(), o.pee().reshape(-1)
    _say(f"800k prefix: min P_ee {po.min():.4f}, max |dPee| = {np.max(np.abs(pg - po)):.3e}")
    np.testing.assert_array_equal(g.get_state().cpu().numpy(), o.get_state())


def test_three_flavor_6m_prefix(nb, oracle):
    """The 6M-beam workload (1000 E x 3000 u x 2, 3 flavours, FP64) in its own launch
    configuration -- rows of 15 full 64-energy passes and a 40-energy tail, the stepper
    without packed tails -- for its first 10 steps from the neutrinosphere, every beam bit
    for bit."""
    d = workloads.three_flavor_6m()
    g = nb.Model(d); g.step(10)
    _say("6M: 10 GPU steps done; oracle")
    o = oracle.Model(d); o.step(10)
    pg, po = g.pee().cpu().numpy(), o.pee().reshape(-1)
    _say(f"6M prefix: min P_ee {po.min():.4f}, max |dPee| = {np.max(np.abs(pg - po)):.3e}")
    np.testing.assert_array_equal(g.get_state().cpu().numpy(), o.get_state())


def test_step_split_and_state_roundtrip_bitwise(nb):
    d = workloads.small_params(n_flavor=3, n_energy=50, n_u=6, n_steps=30)
    a = nb.Model(d); a.run()
    b = nb.Model(d); b.step(7); b.step(11); b.step(100)
    assert b.step_index() == 30
    np.testing.assert_array_equal(a.get_state().cpu().numpy(), b.get_state().cpu().numpy())
    c = nb.Model(d); c.step(13)
    x = c.get_state()
    e = nb.Model(d); e.set_state(x, 13); e.run()
    np.testing.assert_array_equal(a.get_state().cpu().numpy(), e.get_state().cpu().numpy())


def test_repeat_runs_identical(nb):
    d = workloads.small_params(n_flavor=2, n_energy=300, n_u=40, n_steps=20, r_start_km=10.0,
                               r_end_km=11.0)
    outs = []
    for mb in (0, 0, 5):
        d["max_blocks"] = mb
        m = nb.Model(d); m.run(); outs.append(m.get_state().cpu().numpy())
    np.testing.assert_array_equal(outs[0], outs[1])
    np.testing.assert_array_equal(outs[0], outs[2])


def test_nan_state_reports_numeric_error(nb):
    import torch
    d = workloads.small_params(n_flavor=2, n_energy=20, n_u=3, n_steps=4)
    m = nb.Model(d)
    x = m.get_state()
    x[0, 5] = float("nan")
    m.set_state(x, 0)
    with pytest.raises(nb.NubulbError) as e:
        m.step(1)
    assert e.value.code == nb.NB_ENUMERIC
    m.reset()
    m.run()                       # the model is usable again afterwards
    assert torch.isfinite(m.pee()).all()


@pytest.mark.parametrize("case", ["2f", "3f", "3f_fp32_state", "3f_fp32_arith", "batch", "2f_ext"])
def test_renormalisation_factor_far_from_one_reports_numeric_error(nb, case):
    """A state off unit norm by far more than a unitary step's rounding (here 2e-3 in
    |state|^2) is reported as NB_ENUMERIC by the renormalisation; a state off by 2e-10 (FP64)
    is not, and with renormalisation off nothing is checked."""
    import torch
    kw = {}
    if case.startswith("2f"):
        d = workloads.small_params(n_flavor=2, n_energy=40, n_u=3, n_steps=6)
        if case == "2f_ext":
            d["n_phi"] = 2
    elif case == "batch":
        d = [workloads.small_params(n_flavor=2, n_energy=20 + 7 * i, n_u=2 + i, n_steps=6)
             for i in range(3)]
    else:
        d = workloads.small_params(n_flavor=3, n_energy=40, n_u=3, n_steps=6)
        if case != "3f":
            kw["precision"] = nb.NB_FP32_STATE
            # the FP32-arithmetic kernel from step 0: the 6M workload's step length at 600 km
            if case == "3f_fp32_arith":
                d6 = workloads.three_flavor_6m()
                h6 = (d6["r_end_km"] - d6["r_start_km"]) / d6["n_steps"]
                d.update(r_start_km=600.0, r_end_km=600.0 + 6 * h6)
    m = nb.Model(d, **kw)
    if case == "3f_fp32_arith":
        assert m.mixed_fp32_step() == 0
    x = m.get_state()
    m.set_state(x * 1.001, 0)
    with pytest.raises(nb.NubulbError) as e:
        m.step(1)
    assert e.value.code == nb.NB_ENUMERIC and "renormalisation" in str(e.value)
    m.reset()
    m.run()
    assert torch.isfinite(m.pee()).all()
    if not kw:
        m.set_state(x * (1.0 + 1e-10), 0)    # within the bound: accepted and renormalised
        m.step(2)
    if not isinstance(d, list):
        off = nb.Model(dict(d, renorm=0), **kw)
        off.set_state(x * 1.001, 0)
        off.step(1)
