"""Batched models (one persistent launch for many uneven two-flavour models), HIP-graph
replay and the autotuner, checked bit for bit against single-model runs and the oracle."""
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


def small_batch(n=12, steps=20, r_start=10.0, r_end=11.0):
    """Seeded uneven models (the 256-model recipe with bin counts scaled down)."""
    out = []
    for d in workloads.batch_256(n):
        d = dict(d)
        d["n_energy"] = 20 + d["n_energy"] % 130        # 20..149, ragged against 64 lanes
        d["n_u"] = 2 + d["n_u"] % 11
        d.update(n_steps=steps, r_start_km=r_start, r_end_km=r_end)
        out.append(d)
    return out


def _split(pee, offsets):
    return [pee[offsets[i]:offsets[i + 1]] for i in range(len(offsets) - 1)]


def test_batch_equals_single_runs_and_oracle(nb, oracle):
    ds = small_batch()
    b = nb.Model(ds)
    b.run()
    parts = _split(b.pee().cpu().numpy(), b.offsets())
    for i, d in enumerate(ds):
        s = nb.Model(d)
        s.run()
        np.testing.assert_array_equal(parts[i], s.pee().cpu().numpy(), err_msg=f"model {i}")
        if i % 4 == 0:
            o = oracle.Model(d)
            o.run()
            np.testing.assert_array_equal(parts[i], o.pee().reshape(-1), err_msg=f"oracle {i}")


def test_batch_short_rows_equal_single_runs(nb, oracle):
    """Rows shorter than a 64-lane chunk (down to one energy): a chunk holds several rows,
    a lane's next beam (whose state and table values the batch kernel loads one chunk
    ahead) lies one or more rows further on, and rows end in every chunk."""
    ds = []
    for i, d in enumerate(workloads.batch_256(8)):
        d = dict(d)
        d.update(n_energy=(1, 3, 7, 20, 31, 33, 64, 65)[i], n_u=2 + i % 5, n_steps=15,
                 r_start_km=10.0, r_end_km=10.8)
        ds.append(d)
    b = nb.Model(ds)
    b.run()
    parts = _split(b.pee().cpu().numpy(), b.offsets())
    for i, d in enumerate(ds):
        s = nb.Model(d)
        s.run()
        np.testing.assert_array_equal(parts[i], s.pee().cpu().numpy(),
                                      err_msg=f"model {i} (N_E {d['n_energy']})")
        if i in (0, 2, 4):
            o = oracle.Model(d)
            o.run()
            np.testing.assert_array_equal(parts[i], o.pee().reshape(-1), err_msg=f"oracle {i}")
    _say("short-row batch: every model equals its single run")


def test_batch_resolved_and_repeatable(nb):
    ds = small_batch(n=9, steps=30, r_start=60.0, r_end=63.0)
    a = nb.Model(ds); a.run()
    b = nb.Model(ds); b.step(11); b.step(19)
    np.testing.assert_array_equal(a.get_state().cpu().numpy(), b.get_state().cpu().numpy())


def test_graph_replay_equals_eager(nb):
    import torch
    ds = small_batch(n=7, steps=24)
    eager = nb.Model(ds)
    g = nb.Model(ds, stream=torch.cuda.Stream())
    with torch.cuda.stream(g.stream):
        g.graph_capture(6)
    for rep in range(4):
        g.graph_launch()
        eager.step(6)
        assert g.step_index() == eager.step_index() == 6 * (rep + 1)
        # eager work of the program between replays
        with torch.cuda.stream(g.stream):
            pg = g.pee()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(pg.cpu().numpy(), eager.pee().cpu().numpy(),
                                      err_msg=f"replay {rep}")
    g.graph_launch()                     # past r_end: clamped, no further change
    assert g.step_index() == 24


def test_single_model_graph_replay(nb):
    import torch
    d = workloads.small_params(n_flavor=3, n_energy=70, n_u=4, n_steps=12)
    eager = nb.Model(d)
    eager.run()
    g = nb.Model(d, stream=torch.cuda.Stream())
    with torch.cuda.stream(g.stream):
        g.graph_capture(4)
    for _ in range(3):
        g.graph_launch()
    with torch.cuda.stream(g.stream):
        st = g.get_state()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(st.cpu().numpy(), eager.get_state().cpu().numpy())


def test_autotune_keeps_results(nb):
    ds = small_batch(n=10, steps=16)
    ref = nb.Model(ds); ref.run()
    t = nb.Model(ds)
    res = t.autotune(4)
    assert res["ms"] > 0 and res["candidates"] >= 2 and t.step_index() == 0
    assert res["block_threads"] in (256, 512)
    t.run()
    np.testing.assert_array_equal(ref.get_state().cpu().numpy(), t.get_state().cpu().numpy())


def test_batch_256_shape_prefix(nb, oracle):
    """The 256-model workload (64M beams) in one launch: 50 steps from the neutrinosphere;
    every model against its own single-model run and 8 of them against the oracle, bit for
    bit."""
    ds = workloads.batch_256()
    b = nb.Model(ds)
    _say(f"batch: {b.n_models} models, {b.nb} beams")
    b.step(50)
    parts = _split(b.pee().cpu().numpy(), b.offsets())
    for i in range(len(ds)):
        s = nb.Model(ds[i]); s.step(50)
        np.testing.assert_array_equal(parts[i], s.pee().cpu().numpy(), err_msg=f"model {i}")
        del s
    _say("batch: 256 single-model runs equal; oracle")
    for i in (0, 37, 77, 101, 150, 199, 230, 255):
        o = oracle.Model(ds[i]); o.step(50)
        np.testing.assert_array_equal(parts[i], o.pee().reshape(-1), err_msg=f"oracle {i}")
        _say(f"  oracle model {i}: {ds[i]['n_energy']}x{ds[i]['n_u']} equal")
