#!/usr/bin/env python
"""Benchmark of the MI355X bulb-model radial stepper.

One "step" is one radial RKMK4 step of the whole hot path over every beam of the
three-flavour 800k-beam model (400 E x 1000 u x 2 species, 10 -> 1000 km in 20000 steps):
four stage moment reductions (J0, J1), the Hamiltonian assembly, the exact exponentials
and the renormalised state update.  Inputs are synthetic (seeded parameters); the state
is resident in HBM before timing starts.  Prints ONE JSON line on stdout.

Algorithmic cost per beam-step (counted from the kernel's arithmetic, fma = 2 flops,
div/sqrt = 1; terms that are the same for a whole (species, angle) row are counted once
per row and omitted here):
  3 flavours: 4 exponentials exp(-iK) psi (406 flops each: characteristic cubic by three
  Halley steps, eigenvector as an adjugate column, the 2x2 propagator on the eigen-plane,
  two sin/cos), 4 generators alpha V_k + e_k P + Q from the per-row constants (84 in all),
  renormalisation (19), 4 moment contributions with the state check (48 each)
  ->  1919 flops.
  2 flavours: 4 quaternion rotations (85), 8 B-vector builds (7), 2 cross products,
  combinations, renormalisation, 4 moment contributions with the state check (12 each)
  ->  508 flops.
Algorithmic HBM bytes per beam-step: the state is read at stages 2, 3, 4 and the final
pass and written once: 5 x (state reals) x (bytes per real): 3f FP64 psi 240 B, 3f FP32
psi 120 B, 2f Bloch vector 120 B.  The same five passes over a full density matrix (n^2
reals per beam) would move 360 B for 3f FP64; the line reports that accounting beside
the one of the stored state.  A device-to-device copy of 1 GiB, timed the same way, gives
the bandwidth a streaming kernel can reach on the box: the second ceiling.

Clock warm-up: while the device idles (model set-up, host work) its shader clock falls to
about 2.0 GHz, and it climbs back to the loaded 2.3-2.4 GHz only over the first ~20 ms of
stepping; the cycles per step stay the same.  Before each timed measurement the model is
therefore stepped, untimed, for --clock-warmup seconds and then reset to step 0; the W
warm-up steps and the K timed steps follow from step 0 as without it.  The batch,
extended-model and adjoint timings start the same way.  The line records the untimed
steps and launches this took.
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOPS_PER_BEAM_STEP = {2: 508.0, 3: 1919.0}
PEAK_HBM_GBS = 8000.0          # MI355X HBM3E, published
PEAK_FP64_VALU_TFLOPS = 78.6   # MI355X FP64 vector, published (256 CU x 2.4 GHz x 128)
METRIC = "beam-steps/sec + HBM GB/s (3-flavor 800k beams); adjoint/forward time ratio"
KERNEL_SOURCES = ["paper_1912_10596_amd/csrc/nb_kernels.hip",
                  "paper_1912_10596_amd/csrc/nb_device.h",
                  "paper_1912_10596_amd/csrc/nb_device32.h",
                  "paper_1912_10596_amd/csrc/nb_stage.h",
                  "paper_1912_10596_amd/csrc/nb_internal.h"]
CLOCK_WARMUP_S = 0.3           # --clock-warmup


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bytes_per_beam_step(nf: int, fp32: bool) -> float:
    nsc = 3 if nf == 2 else 6
    return 5.0 * nsc * (4.0 if fp32 else 8.0)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def warm_clock(m, seconds: float) -> dict:
    """Untimed stepping of model m for about `seconds` (launches of 1, 2, 4, ... 32
    steps, each one nb_step call and one launch), then nb_reset: the shader clock is at
    its loaded level when the caller's timed launches start from step 0."""
    steps = launches = 0
    n_max = min(int(x["n_steps"]) for x in m.ds)
    t0 = time.perf_counter()
    k = 1
    while time.perf_counter() - t0 < seconds:
        s0 = m.step_index()
        if s0 + k > n_max:
            break
        m.step(k)
        launches += 1
        steps += m.step_index() - s0
        k = min(2 * k, 32)
    m.reset()
    return dict(seconds=round(time.perf_counter() - t0, 3), steps=steps, launches=launches)


def timed_steps(m, K: int, W: int):
    """W untimed steps, then exactly K steps between synchronisations; HIP events on
    the stream the kernels are launched on (torch's current stream, bound at nb_bind)."""
    import torch
    if W:
        m.step(W)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    m.step(K)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, e0.elapsed_time(e1) / 1e3


def traffic_from_profile(name: str, launch_steps: int, nb: int):
    """HBM bytes per launch from committed counter runs, scaled by the copy-kernel
    calibration, or None if missing or taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{name}.json")
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    per_beam_step = t["hbm_bytes_per_beam_step"]
    return per_beam_step * launch_steps * nb


def copy_probe_gbs(reps: int = 5) -> float:
    """Bandwidth of a 1 GiB device-to-device copy (read + write bytes over the median
    HIP-event time of `reps` copies): the streaming ceiling measured on this device."""
    import torch
    n = 1 << 27                          # 2^27 doubles = 1 GiB each way
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3)
    del src, dst
    torch.cuda.empty_cache()
    ts.sort()
    return 2.0 * 8.0 * n / ts[len(ts) // 2] / 1e9


def adjoint_timing(nb, workloads):
    """Forward run and reverse-mode adjoint (which redoes the forward pass with
    checkpoints every 64 steps, then runs backwards) of the 200k-beam two-flavour workload
    in its resolved variant: same shapes, step length and 5000 steps, started at 500 km
    (nearer the neutrinosphere the step does not resolve the Hamiltonian and the gradients
    overflow).  Wall-clock with the stream drained on both sides."""
    import torch
    d = workloads.adjoint_200k_resolved()
    m = nb.Model(d, adjoint_ckpt=64)
    cw = warm_clock(m, CLOCK_WARMUP_S)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.run()
    torch.cuda.synchronize()
    tf = time.perf_counter() - t0
    m.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = m.adjoint()
    torch.cuda.synchronize()
    ta = time.perf_counter() - t0
    x = [*d["lum_erg_s"], d["theta"][0], d["n0_cm3"]]
    return dict(workload=f"2-flavour bulb model, {d['n_energy']} E x {d['n_u']} u x 2 = "
                         f"{m.nb} beams, {d['n_steps']} steps, {d['r_start_km']:g} -> "
                         f"{d['r_end_km']:g} km (resolved variant of 10 -> 300 km)",
                ckpt=64, forward_s=round(tf, 4), adjoint_s=round(ta, 4),
                ratio=round(ta / tf, 3), loss="sum of dE/N_u Pee over all beams",
                grad={k: float(v) for k, v in zip(nb.PARAM_NAMES, g)},
                grad_times_param={k: float(v * xi) for k, v, xi in zip(nb.PARAM_NAMES, g, x)},
                clock_warmup=cw)


def batch_timing(nb, workloads, steps: int):
    """The 256 uneven two-flavour models in one persistent launch: `steps` steps eager
    (HIP events) and the same number as replays of a captured HIP graph."""
    import torch
    ds = workloads.batch_256()
    s = torch.cuda.Stream()
    m = nb.Model(ds, stream=s)
    with torch.cuda.stream(s):
        cw = warm_clock(m, CLOCK_WARMUP_S)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        m.step(steps)
        e1.record(s)
    torch.cuda.synchronize()
    eager = e0.elapsed_time(e1) / 1e3
    with torch.cuda.stream(s):
        m.reset()
        m.graph_capture(steps // 4)
        torch.cuda.synchronize()
        e0.record(s)
        for _ in range(4):
            m.graph_launch()
        e1.record(s)
    torch.cuda.synchronize()
    graph = e0.elapsed_time(e1) / 1e3
    beams = m.nb
    del m
    torch.cuda.empty_cache()
    return dict(workload=f"256 two-flavour models, {beams} beams in one launch, 10 -> 300 km, "
                         f"{steps} of 5000 steps", beam_steps_per_s_eager=beams * steps / eager,
                ms_per_step_eager=round(eager * 1e3 / steps, 4),
                ms_per_step_graph=round(graph * 1e3 / (4 * (steps // 4)), 4), clock_warmup=cw)


def mixed_precision(nb, workloads, literal_steps: int):
    """Mixed precision (FP32 state and, where the step resolves every beam, FP32 stage
    arithmetic; FP64 moments and renormalisation) against FP64 on the 6M-beam 3-flavour
    workload: the full resolved variant (600 -> 1090 km, 10000 steps, FP32 arithmetic from
    the first step) and a prefix of the literal run (10 -> 500 km, unresolved throughout, so
    the mixed mode keeps FP64 arithmetic there).  Times are HIP events around the stepping
    calls; max |dP_ee| is against the FP64 GPU run, which is bitwise the oracle."""
    import numpy as np
    import torch

    def one(d, precision, steps):
        m = nb.Model(d, precision=precision)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        m.step(steps)
        e1.record()
        torch.cuda.synchronize()
        pee = m.pee().cpu().numpy()
        k = m.mixed_fp32_step() if precision else None
        del m
        torch.cuda.empty_cache()
        return e0.elapsed_time(e1) / 1e3, pee, k

    out = {}
    for label, d, steps in (("resolved_full", workloads.three_flavor_6m_resolved(), None),
                            ("literal_prefix", workloads.three_flavor_6m(), literal_steps)):
        steps = d["n_steps"] if steps is None else steps
        t64, p64, _ = one(d, 0, steps)
        t32, p32, k = one(d, 1, steps)
        out[label] = dict(
            workload=f"3-flavour, {d['n_energy']} E x {d['n_u']} u x 2 = "
                     f"{2 * d['n_energy'] * d['n_u']} beams, {d['r_start_km']:g} -> "
                     f"{d['r_end_km']:g} km, {steps} of {d['n_steps']} steps",
            fp32_arithmetic_from_step=k, fp64_s=round(t64, 4), mixed_s=round(t32, 4),
            speed_ratio=round(t64 / t32, 3), max_abs_dpee=float(np.abs(p64 - p32).max()),
            mean_abs_dpee=float(np.abs(p64 - p32).mean()))
    return out


def adaptive_timing(nb, workloads):
    """Adaptive step-size control (nb_run_adaptive).  (a) The 800k-beam 3-flavour shape over
    a resolved span (600 -> 700 km): attempts, time per attempt against the fixed-step
    kernel on the same span, and max |dP_ee| against a fine fixed-step run (8000 steps).
    (b) A prefix of the literal 1024-beam two-flavour run (10 -> 10.1 km), where the
    controller shrinks the step to a few microns of km."""
    import numpy as np
    import torch

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    d = dict(workloads.three_flavor_800k(), r_start_km=600.0, r_end_km=700.0, n_steps=500)
    m = nb.Model(dict(d, n_steps=8000))
    _, t_fix = timed(m.run)
    p_ref = m.pee().cpu().numpy()
    del m
    torch.cuda.empty_cache()
    out = {"fixed_8000_steps": dict(s=round(t_fix, 4), ms_per_step=round(t_fix / 8000 * 1e3, 4))}
    for tol in (1e-6, 1e-7):
        m = nb.Model(d, adaptive=True)
        st, t = timed(lambda: m.run_adaptive(tol))
        out[f"tol_{tol:g}"] = dict(
            st, s=round(t, 4), ms_per_attempt=round(t / st["attempts"] * 1e3, 4),
            max_abs_dpee_vs_fixed_8000=float(np.abs(m.pee().cpu().numpy() - p_ref).max()))
        del m
        torch.cuda.empty_cache()
    out["workload"] = ("3-flavour, 400 E x 1000 u x 2 = 800000 beams, 600 -> 700 km, first step "
                       "0.2 km")
    lit = dict(workloads.two_flavor_small(), r_end_km=10.1, n_steps=20)
    m = nb.Model(lit, adaptive=True)
    st, t = timed(lambda: m.run_adaptive(1e-3, max_attempts=10**7))
    out["literal_1024_prefix"] = dict(
        st, s=round(t, 3), us_per_attempt=round(t / st["attempts"] * 1e6, 2),
        workload="2-flavour, 32 E x 16 u x 2 = 1024 beams, 10 -> 10.1 km, tol 1e-3")
    return out


def extended_timing(nb, workloads):
    """The extended bulb model (azimuthal bins, four moments) in the shape of the paper's
    multi-node benchmark: 10 azimuthal x 100 energy x 10k and 30k polar bins x 2 species
    (20M and 60M two-flavour beams), a prefix of the 10 -> 200 km run timed with HIP
    events after a short warm-up."""
    import torch
    out = {}
    for n_u, K in ((10000, 20), (30000, 10)):
        d = workloads.extended_paper(n_u)
        m = nb.Model(d)
        cw = warm_clock(m, CLOCK_WARMUP_S)
        m.step(2)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        m.step(K)
        e1.record()
        torch.cuda.synchronize()
        s = e0.elapsed_time(e1) / 1e3
        out[f"n_u_{n_u}"] = dict(
            workload=f"2-flavour extended bulb model, 10 phi x 100 E x {n_u} u x 2 = {m.nb} beams",
            steps=K, ms_per_step=round(s / K * 1e3, 4), beam_steps_per_s=m.nb * K / s,
            hbm_gbs_algorithmic=round(m.nb * K * bytes_per_beam_step(2, False) / s / 1e9, 1),
            clock_warmup=cw)
        del m
        torch.cuda.empty_cache()
    return out


def track_all_timing(nb, workloads):
    """Every initially populated flavour tracked explicitly (six species rows for three
    flavours) with anti-nu_x on its own spectrum, on the 800k-beam 3-flavour shape
    (400 E x 1000 u x 6 = 2.4M beams): the same per-beam cost as two tracked species is the
    expectation."""
    import torch
    d = dict(workloads.three_flavor_800k(), track_all=1, lum_xbar_erg_s=1e51, temp_xbar_mev=5.5)
    m = nb.Model(d)
    m.step(5)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    K = 200
    e0.record()
    m.step(K)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3
    out = dict(workload=f"3-flavour, 400 E x 1000 u x 6 species (every flavour tracked) = {m.nb} beams",
               steps=K, ms_per_step=round(s / K * 1e3, 4), beam_steps_per_s=m.nb * K / s)
    del m
    torch.cuda.empty_cache()
    return out


def conditioning(nb, workloads, delta: float = 1e-10):
    """Measured conditioning of the discrete evolution, per configuration: every component
    of the start state perturbed by delta * N(0, 1) (then renormalised), both states
    advanced the same steps, kappa = max_b |dP_ee| / delta.  Two correct FP64
    implementations that differ by rounding (~1e-16 per operation) can then disagree by
    about kappa * 1e-16; a dP_ee of order 0.1 or more means the perturbation has saturated
    (kappa is then a lower bound)."""
    import torch
    cases = [
        ("3f 800k literal (10 km start)", workloads.three_flavor_800k(), (100, 2000), None),
        ("3f 800k resolved (600 km start)", workloads.resolved(workloads.three_flavor_800k(), 600.0),
         (30, 2000), None),
        ("2f 200k literal (10 km start)", workloads.adjoint_200k(), (200, 5000), None),
        ("2f 200k resolved (500 km start)", workloads.adjoint_200k_resolved(), (200, 5000), None),
        ("2f 1024-beam literal (10 km start)", workloads.two_flavor_small(), (100, 2000), None),
        ("3f 6M resolved (600 km start)", workloads.three_flavor_6m_resolved(), (2000,), None),
        ("3f 6M literal (10 km start)", workloads.three_flavor_6m(), (2000,), None),
    ]
    out = []
    for label, d, marks, prec in cases:
        a = nb.Model(d, precision=prec)
        b = nb.Model(d, precision=prec)
        x = b.get_state()
        g = torch.Generator(device=x.device).manual_seed(7)
        x = x + delta * torch.randn(x.shape, generator=g, device=x.device, dtype=x.dtype)
        x = x / torch.sqrt((x * x).sum(dim=0, keepdim=True))
        b.set_state(x, 0)
        done = 0
        for n in marks:
            a.step(n - done)
            b.step(n - done)
            done = n
            dp = float((a.pee() - b.pee()).abs().max().item())
            out.append(dict(config=label, beams=a.nb, steps=n, max_dpee=dp, kappa=dp / delta,
                            saturated=dp >= 0.1))
        del a, b, x
        torch.cuda.empty_cache()
    return dict(delta=delta, probes=out)


def cpu_baseline(d: dict, seconds: float):
    """The oracle as it stands, on this host's cores, over a bounded prefix of the same
    workload (whole steps of every beam until `seconds` of CPU time have passed)."""
    import oracle
    m = oracle.Model(d)
    nb = m.nb
    m.step(1)                          # first touch of the state arrays
    n = 0
    t0 = time.perf_counter()
    while True:
        m.step(1)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds or n >= 200:
            break
    cores = oracle.get_threads()
    out = dict(value=n * nb / el, unit="beam-steps/s", cores=cores,
               kind="oracle", sample=f"{n} radial steps of all {nb} beams (steps 2..{n + 1}) "
               f"of the same workload, {el:.1f} s wall")
    # the same oracle on one thread, continuing from where the timed run stopped
    oracle.set_threads(1)
    try:
        n1 = 0
        t0 = time.perf_counter()
        while True:
            m.step(1)
            n1 += 1
            el1 = time.perf_counter() - t0
            if el1 >= seconds / 3 or n1 >= 50:
                break
    finally:
        oracle.set_threads(cores)
    out["single_thread"] = dict(value=n1 * nb / el1, unit="beam-steps/s", cores=1,
                                sample=f"{n1} radial steps of all {nb} beams (steps {n + 2}.."
                                f"{n + n1 + 1}), {el1:.1f} s wall")
    return out


def main():
    global CLOCK_WARMUP_S
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the adjoint and mixed-precision measurements")
    ap.add_argument("--mixed-literal-steps", type=int, default=2000)
    ap.add_argument("--clock-warmup", type=float, default=CLOCK_WARMUP_S,
                    help="seconds of untimed stepping (then a reset to step 0) before the "
                         "headline, adjoint, batch and extended-model timings; 0 turns it off")
    ap.add_argument("--section", choices=["batch", "extended", "adjoint", "track_all", "conditioning",
                                          "mixed", "adaptive"],
                    help="run only this measurement and print its result (for profiling "
                         "runs; no benchmark line)")
    args = ap.parse_args()
    CLOCK_WARMUP_S = max(0.0, args.clock_warmup)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this stepper runs on one GPU only (no multi-GPU path is built); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1912_10596_amd as nb
    import workloads

    assert torch.cuda.is_available(), "no HIP device"
    torch.cuda.set_device(0)
    if args.section:
        fn = {"batch": lambda: batch_timing(nb, workloads, 40),
              "extended": lambda: extended_timing(nb, workloads),
              "adjoint": lambda: adjoint_timing(nb, workloads),
              "track_all": lambda: track_all_timing(nb, workloads),
              "conditioning": lambda: conditioning(nb, workloads),
              "mixed": lambda: mixed_precision(nb, workloads, args.mixed_literal_steps),
              "adaptive": lambda: adaptive_timing(nb, workloads)}[args.section]
        res = fn()
        gc.collect()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        print(json.dumps({args.section: res}), flush=True)
        return
    d = workloads.three_flavor_800k()
    K, W = args.steps, args.warmup
    if K + W > d["n_steps"]:
        raise SystemExit(f"steps + warmup must be <= {d['n_steps']}")
    m = nb.Model(d)
    log(f"3-flavour model: {m.nb} beams, warmup {W}, timed {K} steps")
    cw = warm_clock(m, CLOCK_WARMUP_S)
    wall, ev = timed_steps(m, K, W)
    beam_steps = float(m.nb) * K
    value = beam_steps / wall
    ms_per_step = wall * 1e3 / K
    # roofline of the dominant kernel (one cooperative launch for the K steps)
    flops = FLOPS_PER_BEAM_STEP[3] * beam_steps
    alg_bytes = bytes_per_beam_step(3, False) * beam_steps
    tflops = flops / ev / 1e12
    gbs = alg_bytes / ev / 1e9
    f_alu, f_hbm = tflops / PEAK_FP64_VALU_TFLOPS, gbs / PEAK_HBM_GBS
    traffic = traffic_from_profile("k_advance_3f_fp64_800k", K, m.nb)
    if f_alu >= f_hbm:
        roof = dict(bound="alu", achieved=round(tflops, 3), peak=PEAK_FP64_VALU_TFLOPS,
                    unit="TFLOP/s", frac=round(f_alu, 4), traffic=traffic,
                    other=dict(bound="hbm", achieved=round(gbs, 1), peak=PEAK_HBM_GBS,
                               unit="GB/s", frac=round(f_hbm, 4)))
    else:
        roof = dict(bound="hbm", achieved=round(gbs, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                    frac=round(f_hbm, 4), traffic=traffic,
                    other=dict(bound="alu", achieved=round(tflops, 3),
                               peak=PEAK_FP64_VALU_TFLOPS, unit="TFLOP/s", frac=round(f_alu, 4)))
    roof["kernel"] = "nb::k_advance<3, double>"
    roof["launch_ms"] = round(ev * 1e3, 3)
    roof["bytes_per_beam_step"] = bytes_per_beam_step(3, False)
    # the same passes over full density matrices (9 reals per beam): 360 B per beam-step
    rho_gbs = 5.0 * 9 * 8.0 * beam_steps / ev / 1e9
    roof["rho_accounting"] = dict(bytes_per_beam_step=360.0, achieved=round(rho_gbs, 1),
                                  frac=round(rho_gbs / PEAK_HBM_GBS, 4))
    if traffic:
        meas = traffic / ev / 1e9
        roof["measured_hbm"] = dict(achieved=round(meas, 1), frac=round(meas / PEAK_HBM_GBS, 4),
                                    bytes_per_beam_step=round(traffic / beam_steps, 1))
    out = {
        "metric": METRIC, "value": value, "unit": "beam-steps/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "3-flavour bulb model, 400 E x 1000 u x 2 species = 800000 "
                               "beams, 10 -> 1000 km, 20000 RKMK4 steps (timed: a prefix)",
                   "n_flavor": 3, "n_energy": 400, "n_u": 1000, "beams": m.nb,
                   "n0_cm3": d["n0_cm3"], "state": "psi, FP64"},
        "hbm_gbs_algorithmic": round(gbs, 1),
        "clock_warmup": dict(cw, note="untimed stepping before the W warm-up steps, then the "
                                      "model reset to step 0"),
        "adjoint_forward_ratio": None,
        "roofline": roof,
    }
    del m
    gc.collect()
    torch.cuda.empty_cache()
    log("copy probe (1 GiB device copy) ...")
    cp = copy_probe_gbs()
    roof["copy_probe"] = dict(achieved_gbs=round(cp, 1), frac_of_peak=round(cp / PEAK_HBM_GBS, 4),
                              kernel_frac_of_copy=round(gbs / cp, 4))
    if not args.no_extras:
        log("adjoint timing (200k beams) ...")
        adj = adjoint_timing(nb, workloads)
        out["adjoint"] = adj
        out["adjoint_forward_ratio"] = adj["ratio"]
        torch.cuda.empty_cache()
        log("batched models (256, 63M beams) ...")
        out["batch"] = batch_timing(nb, workloads, 40)
        log("mixed precision (6M beams) ...")
        out["mixed_precision"] = mixed_precision(nb, workloads, args.mixed_literal_steps)
        torch.cuda.empty_cache()
        log("adaptive step control (800k beams, 1024-beam literal prefix) ...")
        out["adaptive"] = adaptive_timing(nb, workloads)
        torch.cuda.empty_cache()
        log("extended bulb model (20M and 60M beams) ...")
        out["extended"] = extended_timing(nb, workloads)
        log("every flavour tracked (2.4M beams) ...")
        out["track_all"] = track_all_timing(nb, workloads)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(d, args.cpu_seconds)
    # release every model (its pinned host word, graphs, workspace) and torch's cached
    # device memory while the runtime and any attached profiler are still up, rather than
    # from finalisers during interpreter shutdown
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
