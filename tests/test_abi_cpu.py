"""C-ABI checks that need no GPU: the library loads, exports every declared symbol,
validates parameters, and its host tables equal the oracle's bit for bit."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def nb():
    import paper_1912_10596_amd as nb
    if not os.path.exists(nb.LIB_PATH):
        pytest.fail("libnubulb.so not built (run __graft_entry__.build())")
    return nb


def _declared(header):
    hdr = open(os.path.join(ROOT, "include", header)).read()
    declared = set(re.findall(r"\b(nb_[a-z0-9_]+)\s*\(", hdr))
    assert declared, "no declarations found"
    return declared


def test_every_declared_symbol_is_exported(nb):
    declared = _declared("nubulb.h")
    L = nb.lib()
    for name in sorted(declared):
        assert hasattr(L, name), f"{name} not exported"
    assert declared == set(nb.EXPORTS)
    # the arithmetic test hooks live in their own library, not in the stepper's ABI
    assert not any(n.startswith("nb_test_") for n in declared)


def test_test_hook_library_exports_its_header():
    from paper_1912_10596_amd import testhooks
    if not os.path.exists(testhooks.LIB_PATH):
        pytest.fail("libnubulb_testhooks.so not built (run __graft_entry__.build())")
    declared = _declared("nubulb_testhooks.h")
    L = testhooks.lib()
    for name in sorted(declared):
        assert hasattr(L, name), f"{name} not exported"
    assert declared == set(testhooks.EXPORTS)
    import paper_1912_10596_amd as nb
    assert not hasattr(nb.lib(), "nb_test_sincos")


XBAR = dict(lum_xbar_erg_s=2.3e51, temp_xbar_mev=5.1)


@pytest.mark.parametrize("case", ["2f_small", "3f_small", "2f_batchlike", "3f_800k_shape",
                                  "2f_extended", "3f_extended", "2f_xbar", "2f_track_all",
                                  "3f_track_all_xbar"])
def test_host_tables_equal_oracle(nb, oracle, case):
    species4 = 0
    if case == "2f_small":
        d = workloads.two_flavor_small()
    elif case == "2f_xbar":
        d = dict(workloads.two_flavor_small(), **XBAR)
    elif case == "2f_track_all":
        d = dict(workloads.two_flavor_small(), track_all=1)
        species4 = 1
    elif case == "3f_track_all_xbar":
        d = workloads.small_params(n_flavor=3, n_energy=37, n_u=5, track_all=1, **XBAR)
        species4 = 1
    elif case == "2f_extended":
        d = dict(workloads.two_flavor_small(), n_phi=5)
    elif case == "3f_extended":
        d = workloads.small_params(n_flavor=3, n_energy=37, n_u=5, n_phi=6)
    elif case == "3f_small":
        d = workloads.small_params(n_flavor=3, n_energy=37, n_u=5)
    elif case == "2f_batchlike":
        d = workloads.batch_256(3)[2]
    else:
        d = workloads.three_flavor_800k()
        d["n_u"] = 7
    g = nb.HostModel(d).tables()
    o = oracle.Model(d, species4=species4).tables()
    for k in ("E", "w", "bv"):
        np.testing.assert_array_equal(g[k], o[k], err_msg=k)
    for k in ("lam0", "kappa0", "h", "p2e1", "p2e0", "e1", "e0"):
        assert g[k] == o[k], k


@pytest.mark.parametrize("bad", [
    dict(n_flavor=4), dict(n_energy=0), dict(n_u=0), dict(n_steps=0), dict(r_start_km=5.0),
    dict(r_end_km=10.0), dict(delta_cp=0.1), dict(ne_power=9), dict(e_min_mev=0.0),
    dict(precision=1), dict(temp_mev=[0.0, 1.0, 1.0]), dict(lum_erg_s=[-1.0, 1.0, 1.0]),
    dict(n_phi=-1), dict(n_phi=5000), dict(track_all=2), dict(temp_xbar_mev=-1.0),
    dict(temp_xbar_mev=3.0, lum_xbar_erg_s=-1.0),
])
def test_invalid_parameters_rejected(nb, bad):
    d = workloads.two_flavor_small()
    d.update(bad)
    with pytest.raises(nb.NubulbError) as e:
        nb.HostModel(d)
    assert e.value.code == nb.NB_EINVAL


def test_extended_model_mode_checks(nb):
    """The extended bulb model is a single-model FP64 fixed-step mode."""
    d = dict(workloads.two_flavor_small(), n_phi=4)
    nb.HostModel(d)
    for kw in (dict(adjoint_ckpt=64), dict(adaptive=True)):
        with pytest.raises(nb.NubulbError) as e:
            nb.HostModel(d, **kw)
        assert e.value.code == nb.NB_EINVAL
    d3 = workloads.small_params(n_flavor=3, n_phi=4)
    with pytest.raises(nb.NubulbError) as e:
        nb.HostModel(d3, precision=nb.NB_FP32_STATE)
    assert e.value.code == nb.NB_EINVAL
    with pytest.raises(nb.NubulbError) as e:
        nb.HostModel([d, d])
    assert e.value.code == nb.NB_EINVAL
    assert nb.HostModel(d).nb == 2 * 32 * 16 * 4


def test_species_mode_checks(nb):
    """Explicit tracking multiplies the beams by the flavour count; the adjoint keeps two
    tracked species and anti-nu_x = nu_x; batches track two species."""
    d = workloads.two_flavor_small()
    assert nb.HostModel(dict(d, track_all=1)).nb == 2 * nb.HostModel(d).nb
    d3 = workloads.small_params(n_flavor=3, track_all=1)
    assert nb.HostModel(d3).nb == 6 * 37 * 5
    for bad in (dict(track_all=1), XBAR):
        with pytest.raises(nb.NubulbError) as e:
            nb.HostModel(dict(d, **bad), adjoint_ckpt=64)
        assert e.value.code == nb.NB_EINVAL
    with pytest.raises(nb.NubulbError) as e:
        nb.HostModel([dict(d, track_all=1)] * 2)
    assert e.value.code == nb.NB_EINVAL


def test_unbound_calls_fail_cleanly(nb):
    m = nb.HostModel(workloads.two_flavor_small())
    L = nb.lib()
    assert L.nb_step(m.h, 1) == nb.NB_EUNBOUND
    assert L.nb_run(m.h) == nb.NB_EUNBOUND
    assert L.nb_reset(m.h) == nb.NB_EUNBOUND
    assert L.nb_read_pee(m.h, C.c_void_p(16)) == nb.NB_EUNBOUND
    assert L.nb_step(None, 1) == nb.NB_EINVAL
    assert m.workspace_bytes() > 3 * 8 * m.nb
    t = nb.Tuning(block_threads=512)
    assert L.nb_cancel(m.h, 1) == nb.NB_EUNBOUND
    assert L.nb_cancel(None, 1) == nb.NB_EINVAL
    assert L.nb_set_tuning(m.h, C.byref(t)) == nb.NB_EUNBOUND
    assert L.nb_get_tuning(m.h, C.byref(t)) == nb.NB_EUNBOUND
    assert L.nb_autotune(m.h, 4, None, None) == nb.NB_EUNBOUND
    assert L.nb_autotune(m.h, 4, b"/nonexistent/cache.json", None) == nb.NB_EUNBOUND


def test_product_path_has_no_oracle_dependency():
    """The product package never imports, loads or links the oracle."""
    pkg = os.path.join(ROOT, "paper_1912_10596_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "libnbo" not in txt and "nbo.h" not in txt, f


def _herm(o):
    """3x3 Hermitian matrix from (d0, d1, d2, Re/Im o01, o02, o12)."""
    H = np.diag(o[:3]).astype(complex)
    for i, (a, b) in enumerate(((0, 1), (0, 2), (1, 2))):
        H[a, b] = o[3 + 2 * i] + 1j * o[4 + 2 * i]
        H[b, a] = np.conj(H[a, b])
    return H


@pytest.mark.parametrize("r_start", [440.0, 460.0])
def test_mixed_precision_switch_is_a_valid_angle_bound(oracle, r_start):
    """The library's a-priori bound behind the mixed-precision FP32 switch, checked against
    the oracle's Hamiltonians: from the switch step on, every beam's stage generator
    (h/cos) H, traceless, has eigenvalues below one radian -- on the oracle's own state at
    that step, at the step's three stage radii."""
    import paper_1912_10596_amd as nb
    d0 = workloads.three_flavor_6m()
    h = (d0["r_end_km"] - d0["r_start_km"]) / d0["n_steps"]
    d = workloads.small_params(n_flavor=3, n_energy=37, n_u=5, n_steps=1200, r_start_km=r_start,
                               r_end_km=r_start + 1200 * h)
    k = nb.HostModel(d, precision=1).mixed_fp32_step()
    assert 0 < k < d["n_steps"]
    o = oracle.Model(d)
    o.step(k)
    worst = 0.0
    for r in (d["r_start_km"] + k * h, d["r_start_km"] + (k + 0.5) * h, d["r_start_km"] + (k + 1) * h):
        j0, j1 = o.moments(r)
        H = o.hamiltonian(r, j0, j1)
        c = np.tile(np.repeat(o.cos_theta(r), d["n_energy"]), 2)
        for b in range(0, o.nb, 7):
            K = _herm(H[b]) * (h / c[b])
            K -= np.trace(K) / 3.0 * np.eye(3)
            worst = max(worst, np.abs(np.linalg.eigvalsh(K)).max())
    assert worst < 1.0, worst


def test_fp32_state_beam_limit(nb):
    """The FP32-arithmetic kernel addresses a state plane with 32-bit byte offsets, so FP32
    state is limited to 2^30 - 64 beams; FP64 state of the same size is accepted."""
    d = workloads.small_params(n_flavor=3, n_energy=1024, n_u=1 << 19)
    with pytest.raises(nb.NubulbError) as e:
        nb.HostModel(d, precision=nb.NB_FP32_STATE)
    assert e.value.code == nb.NB_EINVAL
    assert nb.HostModel(d).nb == 1 << 30
    ok = workloads.small_params(n_flavor=3, n_energy=1023, n_u=1 << 19)
    assert nb.HostModel(ok, precision=nb.NB_FP32_STATE).nb == 1023 * 2 ** 20
