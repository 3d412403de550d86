"""Launch shapes, the autotuner's JSON cache, host cancellation and the graph-launch guard,
and the host state exchange: every launch shape gives the same bits; a cache hit applies
the stored shape without timing and keeps the bits; a cancelled model's launches end
normally with NB_ETIMEOUT."""
import json
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


def _cases():
    d3 = workloads.small_params(n_flavor=3, n_energy=130, n_u=7, n_steps=12)
    d2 = workloads.small_params(n_flavor=2, n_energy=100, n_u=9, n_steps=12)
    dx = dict(workloads.small_params(n_flavor=2, n_energy=70, n_u=5, n_steps=8), n_phi=3)
    batch = []
    for i, d in enumerate(workloads.batch_256(9)):
        d = dict(d)
        d.update(n_energy=20 + d["n_energy"] % 130, n_u=2 + d["n_u"] % 11, n_steps=12,
                 r_start_km=10.0, r_end_km=11.0)
        batch.append(d)
    return {"3f_130x7": (d3, {}), "2f_100x9": (d2, {}), "2f_ext_3phi": (dx, {}),
            "3f_mixed": (dict(d3, r_start_km=460.0, r_end_km=470.0), {"precision": 1}),
            "batch9": (batch, {})}


@pytest.mark.parametrize("case", list(_cases()))
def test_every_launch_shape_gives_the_same_bits(nb, case):
    d, kw = _cases()[case]
    ref = nb.Model(d, **kw)
    ref.run()
    want = ref.get_state().cpu().numpy()
    shapes = [(512, 0, 1.0), (256, 0, 1.0), (256, 3, 1.0), (512, 1, 1.0)]
    if isinstance(d, list):
        shapes += [(256, 0, 0.25), (512, 2, 3.0)]
    for bs, blocks, cost in shapes:
        m = nb.Model(d, **kw)
        m.set_tuning(bs, blocks, cost)
        t = m.get_tuning()
        assert t["block_threads"] == bs
        if blocks:
            assert t["blocks"] <= blocks
        m.step(5)
        m.step(100)
        np.testing.assert_array_equal(m.get_state().cpu().numpy(), want,
                                      err_msg=f"{case} shape {(bs, blocks, cost)}")
        _say(f"{case}: {bs} threads x {t['blocks']} blocks (row cost {cost}) equal")


def test_set_tuning_rejects_bad_shapes(nb):
    m = nb.Model(workloads.small_params(n_flavor=2, n_energy=40, n_u=3, n_steps=4))
    assert m.get_tuning()["block_threads"] == 256        # the two-flavour default
    assert nb.Model(workloads.small_params(n_flavor=3, n_energy=40, n_u=3, n_steps=4)
                    ).get_tuning()["block_threads"] == 512
    for bs, blocks in ((128, 0), (1024, 0), (512, -1), (512, 100000)):
        with pytest.raises(nb.NubulbError) as e:
            m.set_tuning(bs, blocks)
        assert e.value.code == nb.NB_EINVAL
    assert m.get_tuning()["block_threads"] == 256


@pytest.mark.parametrize("case", ["3f_130x7", "batch9"])
def test_autotune_cache_hit_keeps_bits(nb, case, tmp_path):
    d, kw = _cases()[case]
    path = tmp_path / "tune.json"
    ref = nb.Model(d, **kw)
    ref.run()
    want = ref.get_state().cpu().numpy()
    a = nb.Model(d, **kw)
    r1 = a.autotune(3, cache=str(path))
    assert r1["from_cache"] == 0 and r1["candidates"] >= 2 and r1["ms"] > 0
    a.run()
    np.testing.assert_array_equal(a.get_state().cpu().numpy(), want)
    doc = json.loads(path.read_text())
    assert len(doc) == 1
    (key, rec), = doc.items()
    assert "gfx" in key and (f"ne{d['n_energy']}" in key if not isinstance(d, list) else "batch9" in key)
    assert rec["block_threads"] == r1["block_threads"] and rec["blocks"] >= 1
    b = nb.Model(d, **kw)
    r2 = b.autotune(3, cache=str(path))
    assert r2["from_cache"] == 1 and r2["candidates"] == 0
    for k in ("block_threads", "blocks", "row_cost"):
        assert r2[k] == r1[k], k
    assert r2["ms"] == pytest.approx(r1["ms"])
    b.run()
    np.testing.assert_array_equal(b.get_state().cpu().numpy(), want)
    # another shape adds an entry and keeps the first
    other = workloads.small_params(n_flavor=2, n_energy=33, n_u=3, n_steps=6)
    nb.Model(other).autotune(2, cache=str(path))
    doc2 = json.loads(path.read_text())
    assert len(doc2) == 2 and doc2[key] == rec
    _say(f"{case}: cache {r1['block_threads']} x {r1['blocks']} ({r1['ms']:.3f} ms) hit")


def test_autotune_rejects_a_malformed_cache(nb, tmp_path):
    path = tmp_path / "bad.json"
    path.write_text('{"k": {"block_threads": 512, "blocks": }')
    m = nb.Model(workloads.small_params(n_flavor=2, n_energy=40, n_u=3, n_steps=4))
    with pytest.raises(nb.NubulbError) as e:
        m.autotune(2, cache=str(path))
    assert e.value.code == nb.NB_EIO
    assert path.read_text() == '{"k": {"block_threads": 512, "blocks": }'
    # an entry the device cannot hold is a miss, re-tuned and replaced
    d = workloads.small_params(n_flavor=2, n_energy=40, n_u=3, n_steps=4)
    m2 = nb.Model(d)
    r = m2.autotune(2, cache=str(tmp_path / "ok.json"))
    doc = json.loads((tmp_path / "ok.json").read_text())
    (key, rec), = doc.items()
    doc[key] = dict(rec, blocks=10**6, extra={"x": [1, 2]})
    (tmp_path / "ok.json").write_text(json.dumps(doc))
    r2 = nb.Model(d).autotune(2, cache=str(tmp_path / "ok.json"))
    assert r2["from_cache"] == 0 and r2["blocks"] <= r["blocks"] * 2


@pytest.mark.parametrize("case", ["3f_130x7", "2f_100x9", "batch9", "3f_mixed"])
def test_cancel_before_launch_leaves_state_and_recovers(nb, case):
    d, kw = _cases()[case]
    ref = nb.Model(d, **kw)
    ref.step(7)
    m = nb.Model(d, **kw)
    m.step(3)
    before = m.get_state().cpu().numpy()
    m.cancel(True)
    with pytest.raises(nb.NubulbError) as e:
        m.step(4)
    assert e.value.code == nb.NB_ETIMEOUT and "cancel" in str(e.value)
    assert m.step_index() == 3
    np.testing.assert_array_equal(m.get_state().cpu().numpy(), before)
    m.cancel(False)
    m.step(4)
    assert m.step_index() == 7
    np.testing.assert_array_equal(m.get_state().cpu().numpy(), ref.get_state().cpu().numpy())
    _say(f"{case}: cancelled launch returned NB_ETIMEOUT, state kept, resumed")


def test_cancel_graph_replay_and_adjoint(nb):
    import torch
    d = workloads.small_params(n_flavor=2, n_energy=64, n_u=4, n_steps=24)
    eager = nb.Model(d)
    g = nb.Model(d, stream=torch.cuda.Stream())
    with torch.cuda.stream(g.stream):
        g.graph_capture(6)
    g.graph_launch()
    eager.step(6)
    g.cancel(True)
    with pytest.raises(nb.NubulbError) as e:
        g.graph_launch()
    assert e.value.code == nb.NB_ETIMEOUT
    assert g.step_index() == 6
    g.cancel(False)
    g.graph_launch()
    eager.step(6)
    with torch.cuda.stream(g.stream):
        st = g.get_state()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(st.cpu().numpy(), eager.get_state().cpu().numpy())
    a = nb.Model(d, adjoint_ckpt=8)
    a.cancel(True)
    with pytest.raises(nb.NubulbError) as e:
        a.adjoint()
    assert e.value.code == nb.NB_ETIMEOUT
    a.cancel(False)
    a.reset()
    g1 = a.adjoint()
    b = nb.Model(d, adjoint_ckpt=8)
    np.testing.assert_array_equal(g1, b.adjoint())


def test_cancel_adaptive(nb):
    d = workloads.small_params(n_flavor=2, n_energy=40, n_u=3, n_steps=16)
    m = nb.Model(d, adaptive=True)
    m.cancel(True)
    with pytest.raises(nb.NubulbError) as e:
        m.run_adaptive(1e-6)
    assert e.value.code == nb.NB_ETIMEOUT
    m.cancel(False)
    m.reset()
    s1 = m.run_adaptive(1e-6)
    r = nb.Model(d, adaptive=True)
    assert r.run_adaptive(1e-6) == s1
    np.testing.assert_array_equal(m.get_state().cpu().numpy(), r.get_state().cpu().numpy())


@pytest.mark.parametrize("case", ["3f_130x7", "3f_mixed", "batch9"])
def test_host_state_exchange(nb, case):
    d, kw = _cases()[case]
    m = nb.Model(d, **kw)
    m.step(4)
    dev = m.get_state().cpu().numpy()
    host = m.get_state_host()
    np.testing.assert_array_equal(host, dev)
    o = nb.Model(d, **kw)
    o.set_state_host(host, 4)
    assert o.step_index() == 4
    np.testing.assert_array_equal(o.get_state().cpu().numpy(), dev)
    m.step(3)
    o.step(3)
    np.testing.assert_array_equal(o.get_state_host(), m.get_state_host())
