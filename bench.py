#!/usr/bin/env python3
"""Throughput of the GE sweep on one MI355X.

Workload (one "step"): the moving-wall rod -- N = 2^27 interior points,
r = 4, 5000 time levels, u0 = 0, left wall g_L(t) = sin(2 pi t), right wall
0, source f(x, t) = exp(-t) x (1 - x) -- in FP64 at the library's default
plan.  Step k advances levels 5000k .. 5000(k+1) of the same run (the walls
and the source follow t), so no copy or reset sits in the timed region.
Inputs (state, workspace, wall values, source profile and time factor) are
resident in HBM before the timed region starts.  The metric is grid-point
updates per second (one update = one interior u_i^{m+1}).

Prints one JSON line.  Beside the headline value it carries
  roofline     : the dominant kernel (the temporally blocked tile sweep with
                 a source) against the published FP64 vector peak, timed
                 with HIP events on its stream, its HBM traffic from the
                 committed counter profile, and the instruction floor of the
                 form as a separate, labelled figure;
  cpu_baseline : the CPU oracle (all host cores, one barrier per level) on a
                 bounded number of levels of the same rod, median of 5 runs,
                 with legs on the other workloads (closed-form rod, 2^24
                 rod, sampled batch rods) and a single-thread leg;
  extra        : sampled parity of the headline against the oracle, the
                 depth-1 streaming sweep of the same rod against HBM, the
                 rod in the compensated pair and in plain FP32 with their
                 distance from the FP64 oracle, the 2^24-point rod, the
                 sub-domain scheme (k = 16), the 4096-rod batch in FP32 and
                 in the compensated pair with per-rod errors, the 2D
                 extension and the surrogate;
  paper_e2_shape : the paper's timing runs (about 2.6e5 nodes, 20 to 1200
                 time rows) on the GPU and on the CPU oracle.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GE grid-point updates/s + % HBM roofline; surrogate vs plain at 1e-4 rel L2"
# headline: the moving-wall rod
N5 = 1 << 27
R5 = 4.0
LEVELS5 = 5000
# the 2^24-point rod with zero walls and sine modes
N2 = 1 << 24
R = 2.0
LEVELS = 10000
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
# published MI355X vector peaks (TFLOP/s; an FMA counts 2 flops)
PEAK_TF = {"fp64": 78.6, "fp32": 157.3, "fp32c": 157.3}
# VALU issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-ops/s; a
# wave64 FP64 instruction takes a SIMD 4 cycles (78.6 TFLOP/s = this rate
# x 2 flops of an FMA); FP32 issues at twice the rate
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9
VALU_LANE_OPS_BY_PREC = {"fp64": VALU_LANE_OPS, "fp32": 2 * VALU_LANE_OPS,
                         "fp32c": 2 * VALU_LANE_OPS}
# Algorithmic flops per update (an FMA = 2): the first and second
# differences (2), u + c1 D_i + c2 D_q (two FMAs, 4); a source adds one FMA
# a(t) B_i, B_i = e1 b_i + e2 b_q being fixed by the profile (2).  The pair
# takes both differences for s and e and sums them (5), the increment (mul +
# fma, 3), and Kahan's add (4).  VALU_PER_UPDATE: the fewest instructions the
# form can be written in, the basis of the labelled instruction floor.
FLOPS_PER_UPDATE = {"fp64": 6, "fp32": 6, "fp32c": 12}
FLOPS_SRC = 2
VALU_PER_UPDATE = {"fp64": 4, "fp32": 5, "fp32c": 11}
VALU_SRC = 1
BYTES_PER_POINT = {"fp64": 8, "fp32": 4, "fp32c": 8}
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "moving_wall_c5_fp64_traffic.md")
BF16_PEAK_TFLOPS = 2500.0      # MI355X dense BF16 matrix peak, published
# surrogate: algorithmic flops per point of one 64-level jump (real channels:
# 2->64, four 64->64, 64->1, five taps, multiply-add = 2)
NN_FLOPS_PER_POINT = 2 * 5 * (2 * 64 + 4 * 64 * 64 + 64 * 1)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1310_3422_amd", "csrc", f)
                  for f in ("ge_sweep_kernels.h", "ge_sweep.hip", "ge_sweep_fp64_narrow.hip",
                            "ge_sweep_fp64_mid.hip", "ge_sweep_fp64_wide.hip",
                            "ge_sweep_fp32.hip", "ge_tile.h", "ge_level.h", "ge_kernels.h")]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(key):
    """HBM bytes per launch of the tile sweep from the committed counter
    profile, if it was taken on the current kernel source; else None."""
    try:
        text = open(PROFILE_TRAFFIC).read()
        block = text.split("```json", 1)[1].split("```", 1)[0]
        rec = json.loads(block)
    except (OSError, IndexError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch", {}).get(key)


def launches_per_call(cfg, n_window_fits, nsteps):
    """Kernel launches ge_step_n issues for one call (see ge_api.hip)."""
    if n_window_fits:
        return (nsteps + 65535) // 65536
    k = (nsteps + cfg["depth"] - 1) // cfg["depth"]
    if k % 2 == 1 and nsteps > k:
        k += 1
    return k


def time_runs(torch, stream, fn, warmup, steps):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        fn()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, ev0.elapsed_time(ev1) / 1e3


def _median_of(fn, runs=5):
    ts = []
    for _ in range(runs):
        t = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t)
    return float(np.median(ts))


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def _levels_for(per_level_s, target_s, cap):
    return int(max(2, min(cap, target_s / max(per_level_s, 1e-9))))


def cpu_baseline(inputs, target_s):
    """The oracle as it stands, timed on the host cores, median of 5 runs.

    value: the headline rod (the same inputs as the GPU's) on all host
    threads (one barrier per level) over its first levels, as many as take
    about target_s per run.  Legs: the closed-form rod (n = 1024, r = 1, 1000
    levels, whole) on all threads and on one; the 2^24-point rod over its
    first levels on all threads; 128 sampled rods of the 4096-rod batch
    (whole, 2000 levels, FP64), one rod per thread on all threads; the
    headline rod on one thread over a few levels (its rate extrapolated)."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    threads = os.cpu_count() or 1
    w = inputs.moving_wall_rod(N5, r=R5, nsteps=LEVELS5)
    u = w.u0.copy()

    def c5(levels, nt):
        return lambda: oracle.step_n(u, R5, levels, gl=w.g_left[:levels + 1],
                                     gr=w.g_right[:levels + 1], src_b=w.src_b,
                                     src_a=w.src_a[:levels], nthreads=nt, inplace=True)
    t = time.perf_counter()
    c5(2, threads)()
    lv = _levels_for((time.perf_counter() - t) / 2, target_s, LEVELS5)
    med = _median_of(c5(lv, threads))
    out = {"value": N5 * lv / med, "unit": "updates/s", "cores": threads, "kind": "oracle",
           "sample": f"moving-wall rod (N=2^27, r=4, g_L=sin 2 pi t, source exp(-t)x(1-x)), "
                     f"first {lv} of {LEVELS5} levels, FP64 C oracle, {threads} threads with a "
                     f"barrier per level, median of 5 runs of {med:.2f} s",
           "host_cpu": _cpu_model(), "legs": {}}
    legs = out["legs"]
    # one thread on the same rod
    t = time.perf_counter()
    c5(1, 1)()
    lv1 = _levels_for(time.perf_counter() - t, 0.5 * target_s, LEVELS5)
    med1 = _median_of(c5(lv1, 1))
    legs["moving_wall_1thread"] = {"value": N5 * lv1 / med1, "unit": "updates/s", "cores": 1,
                                   "sample": f"first {lv1} levels, median of 5 runs "
                                             "(rate extrapolated to the whole run)"}
    del u, w
    # closed-form rod, whole
    u1 = inputs.sine_pulse(1024)
    for tag, nt in (("closed_form_all_threads", threads), ("closed_form_1thread", 1)):
        m = _median_of(lambda: oracle.step_n(u1, 1.0, 1000, nthreads=nt))
        legs[tag] = {"value": 1024 * 1000 / m, "unit": "updates/s", "cores": nt,
                     "sample": "n=1024, r=1, 1000 levels, whole run, median of 5"}
    # the 2^24-point rod, first levels
    u2 = inputs.sine_rod(N2, seed=2)
    t = time.perf_counter()
    oracle.step_n(u2, R, 2, nthreads=threads, inplace=True)
    lv2 = _levels_for((time.perf_counter() - t) / 2, target_s, LEVELS)
    m2 = _median_of(lambda: oracle.step_n(u2, R, lv2, nthreads=threads, inplace=True))
    legs["rod_2p24_all_threads"] = {"value": N2 * lv2 / m2, "unit": "updates/s", "cores": threads,
                                    "sample": f"first {lv2} of {LEVELS} levels, median of 5"}
    del u2
    # sampled rods of the batch, whole runs, one rod per thread
    rb = inputs.rod_batch(seed=3, nrods=4096, align=4)
    pick = np.random.default_rng(0).choice(rb.nrods, 128, replace=False)
    rods = [(rb.rod(i)[:rb.n[i]].copy(), rb.r[i], rb.g_left[i], rb.g_right[i]) for i in pick]

    def batch_run():
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(lambda a: oracle.step_n(a[0], a[1], 2000, gl=a[2], gr=a[3]), rods))
    m3 = _median_of(batch_run)
    pts = int(sum(rb.n[i] for i in pick))
    legs["rod_batch_sampled_all_threads"] = {
        "value": pts * 2000 / m3, "unit": "updates/s", "cores": threads,
        "sample": f"128 rods of the 4096-rod batch ({pts} points), 2000 levels each, FP64, "
                  "one rod per thread, median of 5"}
    return out


# The paper's timing runs, reshaped for one MI355X: about 8208 sub-domain
# couples of 32 nodes per time row (k = 16), 20 to 1200 time rows; the GPU
# against the CPU oracle on one thread and on all host cores.
E2_N = 8208 * 32 - 1
E2_ROWS = (20, 100, 400, 1200)


def paper_e2_table(torch, stream, ge, inputs):
    """GPU seconds per run of `rows` levels (median of 5 calls, HIP events on
    the call's stream) for the sub-domain scheme (k = 16) and the two-point
    groups, FP32 and FP64, beside the CPU oracle's seconds for the same run:
    the sub-domain oracle (serial) and the two-point oracle on one thread and
    on all host cores."""
    import oracle
    threads = os.cpu_count() or 1
    u0 = inputs.sine_rod(E2_N, seed=2)
    out = {"n": E2_N, "k": 16, "r": R, "rows": list(E2_ROWS), "gpu_s": {}, "cpu_s": {}}
    for name, k, prec in (("subdomain_k16_fp32", 16, "fp32"), ("subdomain_k16_fp64", 16, "fp64"),
                          ("groups_fp32", 0, "fp32"), ("groups_fp64", 0, "fp64")):
        plan = ge.Plan(E2_N, R, prec, k=k)
        u = ge.pack_state(u0, prec)
        ws = plan.new_workspace()
        col = []
        with torch.cuda.stream(stream):
            for rows in E2_ROWS:
                plan.step_n(u, 0, rows, workspace=ws, stream=stream)
                torch.cuda.synchronize()
                ts = []
                for _ in range(5):
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    plan.step_n(u, 0, rows, workspace=ws, stream=stream)
                    e1.record(stream)
                    torch.cuda.synchronize()
                    ts.append(e0.elapsed_time(e1) / 1e3)
                col.append(float(np.median(ts)))
        out["gpu_s"][name] = col
        del plan, u, ws
    for name, fn in (("subdomain_k16_1thread", lambda rows: oracle.sdc_step_n(u0, R, 16, rows)),
                     ("groups_1thread", lambda rows: oracle.step_n(u0, R, rows, nthreads=1)),
                     ("groups_all_cores", lambda rows: oracle.step_n(u0, R, rows, nthreads=threads))):
        col = []
        for rows in E2_ROWS:
            t = time.perf_counter()
            fn(rows)
            col.append(time.perf_counter() - t)
        out["cpu_s"][name] = col
    last = -1
    out["speedup_at_1200_rows"] = {
        "subdomain_fp32_over_1thread": round(out["cpu_s"]["subdomain_k16_1thread"][last]
                                             / out["gpu_s"]["subdomain_k16_fp32"][last], 1),
        "groups_fp64_over_1thread": round(out["cpu_s"]["groups_1thread"][last]
                                          / out["gpu_s"]["groups_fp64"][last], 1),
        "groups_fp64_over_all_cores": round(out["cpu_s"]["groups_all_cores"][last]
                                            / out["gpu_s"]["groups_fp64"][last], 1)}
    out["cores"] = threads
    out["note"] = ("CPU: FP64 C oracle, untuned; the sub-domain oracle is serial, so the "
                   "all-core figure is the two-point-group scheme's")
    return out


def grid2d_extra(torch, stream, ge, inputs, nx=4096, ny=4096, levels=200, depth=4):
    """The 2D extension on an nx x ny grid (u0 = sine rod profiles in x times
    a sine in y, seed 2), `depth` levels per launch (the library's choice):
    updates/s and the kernel against HBM bandwidth (one read and one write of
    the grid per launch)."""
    fx = inputs.sine_rod(nx, seed=2)
    y = np.arange(1, ny + 1) / (ny + 1)
    u = torch.from_numpy(np.outer(np.sin(np.pi * y), fx)).cuda()
    ws = torch.empty_like(u)
    with torch.cuda.stream(stream):
        torch.cuda.synchronize()
        _, g = time_runs(torch, stream, lambda: ge.step2d_n(u, nx, ny, 2.0, 2.0, 0, levels,
                                                            workspace=ws, stream=stream,
                                                            depth=depth), 1, 3)
    per_launch = g / (3 * levels / depth)
    gbs = 16 * nx * ny / per_launch / 1e9
    return {"updates_per_s": nx * ny * levels * 3 / g, "nx": nx, "ny": ny, "levels": levels,
            "depth": depth,
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "basis": "16 B per point and launch (FP64 read + write), "
                                  f"{depth} levels per launch"}}


def surrogate_extra(torch, stream, train_steps, nrods=4096, width=4096, ntraj=200_000):
    """The learned 64-level propagator against the plain GE sweep on a batch
    of rods: its training (data from the FP64 batch sweep), its distance from
    64 GE levels, and the time per rod-jump of each way to advance 64 levels
    (identity, one GE level at 64 r, 64 GE levels in FP64 and FP32, the
    network, and re-checked stepping at tol 1e-4 every 8 jumps)."""
    from paper_1310_3422_amd import ge, surrogate, inputs
    t0 = time.perf_counter()
    net = ge.Net(width=width, max_batch=nrods, seed=4)
    tr, log = surrogate.train_recipe(
        net, train_steps, seed=4, ntraj=ntraj, minibatch=64, log_every=max(train_steps // 8, 1),
        progress=lambda m: print(f"[bench] surrogate: {m}", file=sys.stderr, flush=True))
    del tr
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0      # trajectory generation included
    res = surrogate.evaluate(net, seed=41, nrods=512, width=width)
    med = {k: {m: float(np.median(v[m])) for m in v} for k, v in res.items()}
    roll = surrogate.rollout(net, seed=41, nrods=256, width=width, njumps=8)
    # timing at a batch of nrods rods
    r, u0 = inputs.surrogate_rods(42, nrods, n=width)
    rf = torch.from_numpy(r.astype(np.float32)).cuda()
    u32 = torch.from_numpy(u0.astype(np.float32).ravel()).cuda()
    r64 = r.astype(np.float32).astype(np.float64)
    fwd_flops = NN_FLOPS_PER_POINT * width                 # algorithmic, one rod-jump
    train_tf = 3 * fwd_flops * 64 * train_steps / train_s / 1e12
    out = {"train_steps": train_steps, "train_minibatch": 64, "trajectories": ntraj,
           "train_s": round(train_s, 2),
           "train_tflops_algorithmic": round(train_tf, 1),
           "loss_log": log, "median_rel_l2_vs_ge64": med,
           "rollout_median_rel_l2_per_jump": [float(np.median(x)) for x in roll],
           "batch_rods": nrods, "width": width}
    times = {}
    plan64 = surrogate.fp64_batch(r64, width)
    ws64 = plan64.new_workspace()
    u64 = ge.f32_to_f64(u32)
    with torch.cuda.stream(stream):
        torch.cuda.synchronize()
        _, g = time_runs(torch, stream, lambda: plan64.solve(u64, 0, 64, ws64, stream=stream), 1, 5)
    times["ge64_fp64"] = g / 5
    n = np.full(nrods, width, dtype=np.int64)
    offs = np.arange(nrods + 1, dtype=np.int64) * width
    plan32 = ge.Batch(n, offs, r64, np.zeros(nrods), np.zeros(nrods), precision="fp32")
    ws32 = plan32.new_workspace()
    u32b = u32.clone()
    with torch.cuda.stream(stream):
        torch.cuda.synchronize()
        _, g = time_runs(torch, stream, lambda: plan32.solve(u32b, 0, 64, ws32, stream=stream), 1, 5)
    times["ge64_fp32"] = g / 5
    big = surrogate.fp64_batch(64.0 * r64, width)
    wsb = big.new_workspace()
    with torch.cuda.stream(stream):
        torch.cuda.synchronize()
        _, g = time_runs(torch, stream, lambda: big.solve(u64, 0, 1, wsb, stream=stream), 1, 5)
    times["big_step_fp64"] = g / 5
    un = torch.empty_like(u32)
    with torch.cuda.stream(stream):
        torch.cuda.synchronize()
        _, g = time_runs(torch, stream, lambda: net.jump(u32, rf, out=un, stream=stream), 1, 5)
    times["surrogate_jump"] = g / 5
    del un, u32b, u64
    ua = u32.clone()
    acc = torch.zeros(nrods, dtype=torch.int32, device="cuda")
    fb = torch.zeros_like(acc)
    err = torch.zeros(nrods, dtype=torch.float64, device="cuda")
    njumps = 16
    with torch.cuda.stream(stream):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nfb = net.advance(plan64, ws64, ua, rf, njumps, check=8, tol=1e-4, accepted=acc,
                          fallbacks=fb, last_err=err, stream=stream)
        torch.cuda.synchronize()
        adv_s = time.perf_counter() - t0
    times["recheck_advance"] = adv_s / njumps
    out["recheck"] = {"jumps": njumps, "check_every": 8, "tol": 1e-4,
                      "rod_windows": nrods * njumps // 8, "fallback_rod_windows": nfb,
                      "median_last_rel_l2": float(err.median().cpu())}
    out["us_per_rod_jump"] = {k: round(v / nrods * 1e6, 4) for k, v in times.items()}
    ach = fwd_flops * nrods / times["surrogate_jump"] / 1e12
    out["roofline_fused_jump"] = {"bound": "mfma", "achieved": round(ach, 1),
                                  "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                                  "frac": round(ach / BF16_PEAK_TFLOPS, 4),
                                  "flops_per_rod_jump": fwd_flops}
    out["speedup_vs_ge64_fp64"] = {k: round(times["ge64_fp64"] / v, 3) for k, v in times.items()}
    return out


def kernel_name(prec, cfg, src):
    t = "double" if prec == "fp64" else "float"
    form = "comp" if prec == "fp32c" else "plain"
    if cfg["schedule"] == 2:
        return f"tile_persistent_kernel<{t},{cfg['tile']},{form},{'src' if src else 'nosrc'}>"
    return (f"tile_kernel<{t},{cfg['tile']},{cfg['waves']},{form},{'src' if src else 'nosrc'},"
            "interior>")


def roofline_of(prec, cfg, n, levels, steps, gpu_s, src, traffic=None):
    """The sweep kernel of a run of `steps` calls of `levels` levels against
    the published vector peak of its precision: algorithmic flops per launch
    over the average launch duration (HIP events on the launch stream, gaps
    between launches included).  The instruction floor of the form and the
    HBM rate of its algorithmic bytes are reported beside it."""
    nl = launches_per_call(cfg, n <= cfg["waves"] * 64 * cfg["tile"], levels) * steps
    kernel_s = gpu_s / nl
    upd = n * levels * steps / nl
    fpu = FLOPS_PER_UPDATE[prec] + (FLOPS_SRC if src else 0)
    vpu = VALU_PER_UPDATE[prec] + (VALU_SRC if src else 0)
    flops = fpu * upd
    ach = flops / kernel_s / 1e12
    floor = VALU_LANE_OPS_BY_PREC[prec] * fpu / vpu / 1e12
    # per launch: one read and one write of the state, one read of the profile
    hbm = (2 + (1 if src else 0)) * BYTES_PER_POINT[prec] * n
    if src and prec == "fp32c":
        hbm -= 4 * n          # the pair's profile is one float per point
    gbs = hbm / kernel_s / 1e9
    return {
        "bound": "alu", "achieved": round(ach, 2), "peak": PEAK_TF[prec], "unit": "TFLOP/s",
        "frac": round(ach / PEAK_TF[prec], 4), "traffic": traffic,
        "kernel": kernel_name(prec, cfg, src), "depth": cfg["depth"], "launches": nl,
        "avg_launch_us": round(kernel_s * 1e6, 2),
        "avg_launch_basis": "per block of levels: the interior-tile kernel, the wall-tile "
                            "kernel (beside it on a second stream for rods of many tiles, "
                            "else before it) and the gaps (HIP events)",
        "flops_per_update": fpu,
        "algorithmic_flops_per_launch": flops,
        "issue_floor": {"peak": round(floor, 2), "frac": round(ach / floor, 4),
                        "basis": f"VALU issue {VALU_LANE_OPS_BY_PREC[prec]:.3g} lane-ops/s x "
                                 f"{fpu} flops / {vpu} VALU instructions per update (the "
                                 "fewest the form can be written in)"},
        "hbm": {"algorithmic_bytes_per_launch": hbm, "gbs": round(gbs, 1),
                "frac": round(gbs / HBM_PEAK_GBS, 4)},
    }


def moving_wall_inputs(torch, inputs, prec, levels_total):
    """Device inputs of the moving-wall rod for levels 0 .. levels_total."""
    w = inputs.moving_wall_rod(N5, r=R5, nsteps=levels_total)
    dt = torch.float64 if prec == "fp64" else torch.float32
    d = {"gl": torch.from_numpy(w.g_left).cuda(), "gr": torch.from_numpy(w.g_right).cuda(),
         "sa": torch.from_numpy(w.src_a).cuda(),
         "sb": torch.from_numpy(w.src_b).to(device="cuda", dtype=dt)}
    return w, d


def moving_wall_windows(got, w, prec, levels):
    """rel-L2 of the walls' and the middle's 256-point blocks against the
    FP64 oracle on each block's dependence window (FP32 forms: the source
    profile rounded as the GPU holds it; u0 = 0 is exact in every form)."""
    import oracle
    sb = w.src_b if prec == "fp64" else w.src_b.astype(np.float32).astype(np.float64)
    out = {}
    for tag, lo in (("left", 0), ("middle", N5 // 2), ("right", N5 - 256)):
        want = oracle.window_step_n(w.u0, lo, lo + 256, R5, levels, gl=w.g_left[:levels + 1],
                                    gr=w.g_right[:levels + 1], src_b=sb,
                                    src_a=w.src_a[:levels])
        g = got[lo:lo + 256]
        out[tag] = float(np.linalg.norm(g - want) / np.linalg.norm(want))
    return out


def moving_wall_precision_extra(torch, stream, ge, inputs, prec):
    """One 5000-level run of the moving-wall rod in `prec`, timed with HIP
    events, and its distance from the FP64 oracle."""
    w, d = moving_wall_inputs(torch, inputs, prec, LEVELS5)
    plan = ge.Plan(N5, R5, prec, src_b=d["sb"])
    u = plan.new_state()
    ws = plan.new_workspace()
    with torch.cuda.stream(stream):
        torch.cuda.synchronize()
        wall, g = time_runs(torch, stream, lambda: plan.step_n(
            u, 0, LEVELS5, workspace=ws, g_left_t=d["gl"], g_right_t=d["gr"],
            src_a_t=d["sa"], stream=stream), 0, 1)
    plan.check(stream)
    got = ge.unpack_state(u, N5, prec)
    cfg = plan.config()
    return {"updates_per_s": N5 * LEVELS5 / g, "config": cfg,
            "rel_l2_vs_fp64_oracle": moving_wall_windows(got, w, prec, LEVELS5),
            "roofline": roofline_of(prec, cfg, N5, LEVELS5, 1, g, True)}


def batch_extra(torch, stream, ge, inputs, prec, sample_errors=True):
    """The 4096-rod batch (N log-uniform in [256, 65536], r in [0.25, 4],
    walls in [-1, 1], seed 3), 2000 levels, one persistent graph-captured
    launch; rods above the on-chip limit of the form run as long-rod tasks.
    Per-rod rel-L2 against the oracle (started from the same rounded values;
    the compensated pair against the extended-precision oracle) on the
    largest and smallest rods and ten random ones."""
    import oracle
    rb = inputs.rod_batch(seed=3, nrods=4096, align=4)
    bt = ge.Batch.from_inputs(rb, prec)
    u0 = ge.pack_batch_state(rb.u0, rb.offsets, rb.n, prec)
    ub = u0.clone()
    wsb = bt.new_workspace()
    with torch.cuda.stream(stream):
        torch.cuda.synchronize()
        wb, gb = time_runs(torch, stream, lambda: bt.solve(ub, 0, 2000, wsb, stream=stream), 1, 3)
    info = bt.info()
    bups = float(rb.n.sum()) * 2000 * 3 / gb
    fpu = FLOPS_PER_UPDATE[prec]
    out = {"roofline": {"bound": "alu", "achieved": round(bups * fpu / 1e12, 2),
                        "peak": PEAK_TF[prec], "unit": "TFLOP/s",
                        "frac": round(bups * fpu / 1e12 / PEAK_TF[prec], 4)},
           "updates_per_s": bups, "ms_per_run": gb / 3 * 1e3, "tasks": info["ntasks"],
           "workgroups": info["grid"], "rods": rb.nrods, "points": int(rb.n.sum()),
           "levels": 2000,
           "long_rod_tasks": int((rb.n > (65536 if prec == "fp32" else 32768)).sum())}
    if sample_errors:
        with torch.cuda.stream(stream):
            ub.copy_(u0)
            bt.solve(ub, 0, 2000, wsb, stream=stream)
        bt.check(stream)
        got = ub.cpu().numpy()
        start = u0.cpu().numpy()
        rng = np.random.default_rng(0)
        pick = sorted(set([int(np.argmax(rb.n)), int(np.argmin(rb.n))] +
                          rng.choice(rb.nrods, 10, replace=False).tolist()))
        errs = []
        for i in pick:
            v0 = ge.unpack_batch_rod(start, rb.offsets, rb.n, i, prec)
            want = oracle.step_n(v0, rb.r[i], 2000, gl=rb.g_left[i], gr=rb.g_right[i],
                                 extended=(prec == "fp32c"))
            g = ge.unpack_batch_rod(got, rb.offsets, rb.n, i, prec)
            errs.append(float(np.linalg.norm(g - want) / np.linalg.norm(want)))
        j = int(np.argmax(errs))
        out["rel_l2_sampled_rods"] = {"max": max(errs), "median": float(np.median(errs)),
                                      "worst_rod": {"i": pick[j], "n": int(rb.n[pick[j]]),
                                                    "r": float(rb.r[pick[j]])},
                                      "rods": len(pick)}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32c", "fp32"])
    ap.add_argument("--cpu-seconds", type=float, default=3.0,
                    help="about this long per timed CPU run (5 runs per leg)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--no-extra", action="store_true", help="skip the extra measurements")
    ap.add_argument("--surrogate-steps", type=int, default=24000,
                    help="training steps of the surrogate extra (0: skip it)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a 1 GiB fill and a 1 GiB streaming read+write (counter "
                         "calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the sweep of one rod runs on a single "
              "MI355X and no multi-GPU path is built (run with --gpus 1).", file=sys.stderr)
        return 3

    import torch
    from paper_1310_3422_amd import ge, inputs
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        return 2

    prec = args.precision
    if args.calibrate_copy:
        # counter calibration: a fill that writes 1 GiB, then a streaming
        # kernel that reads 1 GiB and writes 1 GiB (b = 2 a)
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.mul(a, 2.0, out=b)
        torch.cuda.synchronize()
        del a, b
    total = LEVELS5 * (args.warmup + args.steps)
    print(f"[bench] moving-wall rod N=2^27, {total} levels of walls and source ...",
          file=sys.stderr, flush=True)
    w, d = moving_wall_inputs(torch, inputs, prec, total)
    stream = torch.cuda.Stream()   # default priority
    plan = ge.Plan(N5, R5, prec, src_b=d["sb"])
    cfg = plan.config()
    u = plan.new_state()
    ws = plan.new_workspace()
    torch.cuda.synchronize()

    # Step k advances levels k*LEVELS5 .. (k+1)*LEVELS5 of the same run, with
    # the wall values and source factors of those levels (views into the
    # resident arrays).
    calls = [0]

    def step_chained():
        m = calls[0] * LEVELS5
        plan.step_n(u, m, LEVELS5, workspace=ws, g_left_t=d["gl"][m:m + LEVELS5 + 1],
                    g_right_t=d["gr"][m:m + LEVELS5 + 1], src_a_t=d["sa"][m:m + LEVELS5],
                    stream=stream)
        calls[0] += 1

    print(f"[bench] {prec} config {cfg}, warmup {args.warmup}, steps {args.steps}",
          file=sys.stderr, flush=True)
    with torch.cuda.stream(stream):
        torch.cuda.synchronize()
        wall, gpu_s = time_runs(torch, stream, step_chained, args.warmup, args.steps)
    plan.check(stream)
    value = N5 * LEVELS5 * args.steps / wall
    tkey = f"{prec}_n{N5}_k{cfg['tile']}_w{cfg['waves']}_d{cfg['depth']}_s{cfg['schedule']}_src"
    roofline = roofline_of(prec, cfg, N5, LEVELS5, args.steps, gpu_s, True,
                           traffic=recorded_traffic(tkey))

    out = {
        "metric": METRIC, "value": value, "unit": "updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp32c": "f32x2-compensated"}[prec],
        "data": "synthetic",
        "config": {"workload": "moving-wall rod: N=2^27 interior points, r=4, 5000 levels per "
                               "step (steps continue one run in time), u0=0, g_L=sin(2 pi t), "
                               "g_R=0, source exp(-t) x(1-x), library default plan",
                   "n": N5, "r": R5, "levels": LEVELS5, "precision": prec, **cfg},
        "roofline": roofline,
    }
    del u, ws, plan, d

    if not args.no_extra:
        import oracle
        extra = {}
        # sampled parity of the headline form: one untimed 5000-level run from
        # u0 = 0, the walls' and the middle's blocks against the oracle
        w1, d1 = moving_wall_inputs(torch, inputs, prec, LEVELS5)
        p1 = ge.Plan(N5, R5, prec, src_b=d1["sb"])
        u1 = p1.new_state()
        ws1 = p1.new_workspace()
        with torch.cuda.stream(stream):
            p1.step_n(u1, 0, LEVELS5, workspace=ws1, g_left_t=d1["gl"], g_right_t=d1["gr"],
                      src_a_t=d1["sa"], stream=stream)
        p1.check(stream)
        extra["parity_rel_l2_vs_oracle"] = moving_wall_windows(ge.unpack_state(u1, N5, prec),
                                                               w1, prec, LEVELS5)
        del u1, ws1, p1
        # depth-1 streaming sweep of the same rod: every level reads and
        # writes the rod and reads the source profile (F_1)
        pd = ge.Plan(N5, R5, prec, src_b=d1["sb"], depth=1)
        ud = pd.new_state()
        wsd = pd.new_workspace()
        lv = 20
        with torch.cuda.stream(stream):
            torch.cuda.synchronize()
            wdd, gdd = time_runs(torch, stream, lambda: pd.step_n(
                ud, 0, lv, workspace=wsd, g_left_t=d1["gl"][:lv + 1], g_right_t=d1["gr"][:lv + 1],
                src_a_t=d1["sa"][:lv], stream=stream), 1, 3)
        bpu = 3 * BYTES_PER_POINT[prec] - (4 if prec == "fp32c" else 0)
        bps = bpu * N5 * lv * 3 / gdd / 1e9
        extra["streaming_depth1"] = {"n": N5, "levels": lv * 3,
                                     "updates_per_s": N5 * lv * 3 / gdd,
                                     "bytes_per_update": bpu, "hbm_gbs_algorithmic": round(bps, 1),
                                     "F1": round(bps / HBM_PEAK_GBS, 4), "config": pd.config()}
        del ud, wsd, pd, d1
        if prec == "fp64":
            print("[bench] moving-wall rod in the FP32 forms ...", file=sys.stderr, flush=True)
            extra["moving_wall_fp32c"] = moving_wall_precision_extra(torch, stream, ge, inputs,
                                                                     "fp32c")
            extra["moving_wall_fp32"] = moving_wall_precision_extra(torch, stream, ge, inputs,
                                                                    "fp32")
        # the 2^24-point rod (r = 2, 10^4 levels, zero walls, sine modes)
        print("[bench] 2^24-point rod ...", file=sys.stderr, flush=True)
        u0 = inputs.sine_rod(N2, seed=2)
        for p2 in ("fp64", "fp32c"):
            pl = ge.Plan(N2, R, p2)
            ui = ge.pack_state(u0, p2)
            uu = ui.clone()
            wsp = pl.new_workspace()
            with torch.cuda.stream(stream):
                torch.cuda.synchronize()
                wr, gr_ = time_runs(torch, stream, lambda: pl.step_n(uu, 0, LEVELS, workspace=wsp,
                                                                    stream=stream), 1, 3)
            # parity: one more run from u0
            with torch.cuda.stream(stream):
                uu.copy_(ui)
                pl.step_n(uu, 0, LEVELS, workspace=wsp, stream=stream)
            pl.check(stream)
            c2 = pl.config()
            lo = N2 // 2 - 32
            got = ge.unpack_state(uu, N2, p2)[lo:lo + 64]
            v0 = ge.unpack_state(ui, N2, p2)
            want = oracle.window_step_n(v0, lo, lo + 64, R, LEVELS, extended=(p2 != "fp64"))
            extra[f"rod_2p24_{p2}"] = {
                "updates_per_s": N2 * LEVELS * 3 / gr_, "config": c2,
                "rel_l2_sampled_vs_oracle": float(np.linalg.norm(got - want) / np.linalg.norm(want)),
                "increment_rel_l2_sampled": float(
                    np.linalg.norm((got - v0[lo:lo + 64]) - (want - v0[lo:lo + 64])) /
                    np.linalg.norm(want - v0[lo:lo + 64])),
                "roofline": roofline_of(p2, c2, N2, LEVELS, 3, gr_, False)}
            del pl, ui, uu, wsp
        # the paper's own configuration: sub-domains of k = 16 nodes (couples
        # of 32), FP64, a rod of 2^24 - 1 points (n + 1 a multiple of 32),
        # same r, u0 and level count as the 2^24-point rod
        ns = N2 - 1
        ps = ge.Plan(ns, R, "fp64", k=16)
        us = ge.pack_state(u0[:ns], "fp64")
        wss = ps.new_workspace()
        with torch.cuda.stream(stream):
            torch.cuda.synchronize()
            wsd, gsd = time_runs(torch, stream,
                                 lambda: ps.step_n(us, 0, LEVELS, workspace=wss, stream=stream), 1, 3)
        sups = ns * LEVELS * 3 / gsd
        # a sweep node costs one multiply and two FMAs (5 flops, 3 VALU
        # instructions); the pairs are a small share at k = 16
        sfloor = VALU_LANE_OPS * 5 / 3 / 1e12
        extra["subdomain_k16_fp64"] = {
            "updates_per_s": sups, "n": ns, "k": 16, "levels": LEVELS, "config": ps.config(),
            "roofline": {"bound": "alu", "achieved": round(sups * 5 / 1e12, 2),
                         "peak": PEAK_TF["fp64"], "unit": "TFLOP/s",
                         "frac": round(sups * 5 / 1e12 / PEAK_TF["fp64"], 4),
                         "issue_floor": {"peak": round(sfloor, 1),
                                         "frac": round(sups * 5 / 1e12 / sfloor, 4),
                                         "basis": "VALU issue 3.93e13 lane-ops/s x 5 flops / 3 "
                                                  "VALU instructions per sweep node"}}}
        del us, wss, ps
        print("[bench] 4096-rod batch ...", file=sys.stderr, flush=True)
        extra["rod_batch_4096_fp32"] = batch_extra(torch, stream, ge, inputs, "fp32")
        extra["rod_batch_4096_fp32c"] = batch_extra(torch, stream, ge, inputs, "fp32c")
        # two-dimensional extension: 4096 x 4096 grid, FP64, rx = ry = 2
        extra["grid2d_4096_fp64"] = grid2d_extra(torch, stream, ge, inputs)
        if args.surrogate_steps > 0:
            print("[bench] surrogate ...", file=sys.stderr, flush=True)
            extra["surrogate"] = surrogate_extra(torch, stream, args.surrogate_steps)
        out["extra"] = extra

    if not args.no_cpu:
        print(f"[bench] CPU baseline (~{args.cpu_seconds:.0f} s per run, 5 runs per leg) ...",
              file=sys.stderr, flush=True)
        cb = cpu_baseline(inputs, args.cpu_seconds)
        out["cpu_baseline"] = cb
        # the paper's own comparison (a laptop GPU against one and eight CPU
        # threads of its host, same sweep), as context for these ratios
        out["gpu_over_cpu"] = {
            "all_threads": round(value / cb["value"], 1),
            "single_thread": round(value / cb["legs"]["moving_wall_1thread"]["value"], 1),
            "paper_context": "GT 335M vs i7-720QM: about 5x over 1 thread, about 2x over "
                             "8 threads (sub-domain scheme, relative figures only)"}
        if not args.no_extra:
            print("[bench] paper-shaped timing table ...", file=sys.stderr, flush=True)
            out["paper_e2_shape"] = paper_e2_table(torch, stream, ge, inputs)

    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
