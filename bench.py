#!/usr/bin/env python3
"""Throughput of the GE sweep on one MI355X.

Workload (one "step"): a single rod of N = 2^24 interior points, r = 2,
10^4 time levels, zero walls, u0 = sum_{k=1..16} (z_k/k^2) sin(k pi x) with
z ~ N(0,1) from seed 2 (synthetic, generated on the host).  Inputs are
resident in HBM before the timed region starts.  The metric is grid-point
updates per second (one update = one interior u_i^{m+1}).

Prints one JSON line.  Beside the headline value it carries
  roofline     : the dominant kernel (the temporally blocked tile sweep)
                 against its bound, timed with HIP events on its stream;
  cpu_baseline : the CPU oracle (all host cores, one barrier per level) on a
                 bounded number of levels of the same rod;
  extra        : the depth-1 streaming sweep against HBM bandwidth, the
                 compensated FP32 form on the same rod, a sampled parity
                 check of the timed result against the oracle, the
                 sub-domain scheme (k = 16), the 4096-rod batch, the 2D
                 extension on a 4096 x 4096 grid and the surrogate;
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
N_DEFAULT = 1 << 24
R = 2.0
LEVELS = 10000
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
# VALU issue rate of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-ops/s
# for FP64 (the published 78.6 TFLOP/s FP64 vector peak counts each op as a
# fused multiply-add, 2 flops); FP32 at the published 157.3 TFLOP/s vector
# rate, twice that (the FP32 sweep, which has no packed instructions, ran
# above the single rate on the box, so the single rate is no bound for it).
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9
VALU_LANE_OPS_BY_PREC = {"fp64": VALU_LANE_OPS, "fp32": 2 * VALU_LANE_OPS,
                         "fp32c": 2 * VALU_LANE_OPS}
# per update: algorithmic flops (fma = 2) and the fewest VALU instructions the
# form can be written in -- FP64: 2 subtractions + 2 fma; FP32: 2 sub + mul +
# fma + add (increment first); pair: 5 for D, mul + fma, 4 for the Kahan add
FLOPS_PER_UPDATE = {"fp64": 6, "fp32": 6, "fp32c": 12}
VALU_PER_UPDATE = {"fp64": 4, "fp32": 5, "fp32c": 11}
BYTES_PER_POINT = {"fp64": 8, "fp32": 4, "fp32c": 8}
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "tile_sweep_traffic.md")
BF16_PEAK_TFLOPS = 2500.0      # MI355X dense BF16 matrix peak, published
# surrogate: algorithmic flops per point of one 64-level jump (real channels:
# 2->64, four 64->64, 64->1, five taps, multiply-add = 2)
NN_FLOPS_PER_POINT = 2 * 5 * (2 * 64 + 4 * 64 * 64 + 64 * 1)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1310_3422_amd", "csrc", f)
                  for f in ("ge_sweep.hip", "ge_level.h", "ge_kernels.h")]


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


def cpu_baseline(u0, target_s):
    """The oracle as it stands, all host cores, on the first levels of the
    same rod; the number of levels is chosen to take about target_s."""
    import oracle
    threads = os.cpu_count() or 1
    n = u0.size
    probe = 16
    t = time.perf_counter()
    oracle.step_n(u0, R, probe, nthreads=threads)
    per_level = max(time.perf_counter() - t, 1e-3) / probe
    levels = int(max(probe, min(LEVELS, target_s / per_level)))
    t = time.perf_counter()
    oracle.step_n(u0, R, levels, nthreads=threads)
    dt = time.perf_counter() - t
    # the single-thread form (the paper's one-core comparison), on a few
    # levels, extrapolated per update
    lv1 = max(2, min(levels, int(0.2 * target_s / (per_level * threads))))
    t = time.perf_counter()
    oracle.step_n(u0, R, lv1, nthreads=1)
    dt1 = time.perf_counter() - t
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": n * levels / dt, "unit": "updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"same rod (N={n}), first {levels} of {LEVELS} levels, FP64 C oracle, "
                      f"{threads} threads with a barrier per level, {dt:.1f} s",
            "single_thread": {"value": n * lv1 / dt1, "unit": "updates/s",
                              "sample": f"first {lv1} levels, 1 thread, {dt1:.1f} s "
                                        "(rate extrapolated to the whole run)"},
            "host_cpu": model}


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


def grid2d_extra(torch, stream, ge, inputs, nx=4096, ny=4096, levels=200, depth=2):
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


def surrogate_extra(torch, stream, train_steps, nrods=4096, width=4096):
    """The learned 64-level propagator against the plain GE sweep on a batch
    of rods: its training (data from the FP64 batch sweep), its distance from
    64 GE levels, and the time per rod-jump of each way to advance 64 levels
    (identity, one GE level at 64 r, 64 GE levels in FP64 and FP32, the
    network, and re-checked stepping at tol 1e-4 every 8 jumps)."""
    from paper_1310_3422_amd import ge, surrogate, inputs
    t0 = time.perf_counter()
    net = ge.Net(width=width, max_batch=nrods, seed=4)
    tr, log = surrogate.train_recipe(net, train_steps, seed=4, ntraj=4096, minibatch=64,
                                     log_every=max(train_steps // 8, 1))
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
    out = {"train_steps": train_steps, "train_minibatch": 64, "trajectories": 4096,
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


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32c", "fp32"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
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

    n = N_DEFAULT
    prec = args.precision
    if args.calibrate_copy:
        # counter calibration: a fill that writes 1 GiB, then a streaming
        # kernel that reads 1 GiB and writes 1 GiB (b = 2 a)
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.mul(a, 2.0, out=b)
        torch.cuda.synchronize()
        del a, b
    print(f"[bench] generating rod N={n} ...", file=sys.stderr, flush=True)
    u0 = inputs.sine_rod(n, seed=2)
    stream = torch.cuda.Stream()   # default priority
    plan = ge.Plan(n, R, prec)
    cfg = plan.config()
    u_init = ge.pack_state(u0, prec)
    u = u_init.clone()
    ws = plan.new_workspace()
    torch.cuda.synchronize()

    # Steps chain the level index: step k advances levels k*LEVELS ..
    # (k+1)*LEVELS of the same rod (restarting from u0 would put a copy in the
    # timed region).
    calls = [0]

    def step_chained():
        plan.step_n(u, calls[0] * LEVELS, LEVELS, workspace=ws, stream=stream)
        calls[0] += 1

    print(f"[bench] {prec} config {cfg}, warmup {args.warmup}, steps {args.steps}",
          file=sys.stderr, flush=True)
    with torch.cuda.stream(stream):
        u.copy_(u_init)
        torch.cuda.synchronize()
        wall, gpu_s = time_runs(torch, stream, step_chained, args.warmup, args.steps)
    updates = n * LEVELS * args.steps
    value = updates / wall
    nl = launches_per_call(cfg, n <= 4 * 64 * cfg["tile"], LEVELS) * args.steps
    kernel_s = gpu_s / nl
    upd_per_launch = n * LEVELS / (nl / args.steps)
    flops = FLOPS_PER_UPDATE[prec] * upd_per_launch
    peak_tf = VALU_LANE_OPS_BY_PREC[prec] * FLOPS_PER_UPDATE[prec] / VALU_PER_UPDATE[prec] / 1e12
    achieved_tf = flops / kernel_s / 1e12
    hbm_bytes = 2 * BYTES_PER_POINT[prec] * n      # one read + one write per launch
    tkey = f"{prec}_n{n}_k{cfg['tile']}_w{cfg['waves']}_d{cfg['depth']}_s{cfg['schedule']}"
    roofline = {
        "bound": "alu", "achieved": round(achieved_tf, 3), "peak": round(peak_tf, 2),
        "unit": "TFLOP/s", "frac": round(achieved_tf / peak_tf, 4),
        "traffic": recorded_traffic(tkey),
        "peak_basis": f"VALU issue {VALU_LANE_OPS_BY_PREC[prec]:.3g} lane-ops/s x {FLOPS_PER_UPDATE[prec]} "
                      f"flops / {VALU_PER_UPDATE[prec]} VALU ops per update",
        "kernel": (f"tile_persistent_kernel<{'double' if prec == 'fp64' else 'float'},{cfg['tile']},"
                   f"{'comp' if prec == 'fp32c' else 'plain'}>" if cfg["schedule"] == 2 else
                   f"tile_kernel<{'double' if prec == 'fp64' else 'float'},{cfg['tile']},"
                   f"{cfg['waves']},{'comp' if prec == 'fp32c' else 'plain'}>"),
        "depth": cfg["depth"], "launches": nl, "avg_launch_us": round(kernel_s * 1e6, 2),
        "algorithmic_flops_per_launch": flops,
        "hbm_gbs_algorithmic": round(hbm_bytes / kernel_s / 1e9, 1),
        "hbm_frac_algorithmic": round(hbm_bytes / kernel_s / 1e9 / HBM_PEAK_GBS, 4),
    }

    out = {
        "metric": METRIC, "value": value, "unit": "updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp32c": "f32x2-compensated"}[prec],
        "data": "synthetic",
        "config": {"workload": "single rod, N=2^24 interior points, r=2.0, 10000 levels, "
                               "zero walls, seeded 16-mode sine u0 (seed 2)",
                   "n": n, "r": R, "levels": LEVELS, "precision": prec, **cfg},
        "roofline": roofline,
    }

    if not args.no_extra:
        import oracle
        extra = {}
        # sampled parity: one untimed step from u0, a 64-point block against
        # the oracle on that block's dependence window
        with torch.cuda.stream(stream):
            u.copy_(u_init)
            plan.step_n(u, 0, LEVELS, workspace=ws, stream=stream)
        torch.cuda.synchronize()
        lo = n // 2 - 32
        got = ge.unpack_state(u, n, prec)[lo:lo + 64]
        v0 = ge.unpack_state(u_init, n, prec)
        want = oracle.window_step_n(v0, lo, lo + 64, R, LEVELS, extended=(prec != "fp64"))
        extra["parity_sample_rel_l2"] = float(np.linalg.norm(got - want) / np.linalg.norm(want))
        extra["parity_sample_increment_rel_l2"] = float(
            np.linalg.norm((got - v0[lo:lo + 64]) - (want - v0[lo:lo + 64])) /
            np.linalg.norm(want - v0[lo:lo + 64]))
        # depth-1 streaming sweep on a rod of 2^27 points (1 GiB in FP64, far
        # beyond the last-level cache): every level reads and writes the rod
        n5 = 1 << 27
        p1 = ge.Plan(n5, 4.0, prec, depth=1)
        u1 = ge.pack_state(inputs.sine_pulse(n5), prec)
        ws1 = p1.new_workspace()
        lv = 20
        with torch.cuda.stream(stream):
            torch.cuda.synchronize()
            w1, g1 = time_runs(torch, stream,
                               lambda: p1.step_n(u1, 0, lv, workspace=ws1, stream=stream), 1, 3)
        bps = 2 * BYTES_PER_POINT[prec] * n5 * lv * 3 / g1 / 1e9
        extra["streaming_depth1"] = {"n": n5, "levels": lv * 3, "updates_per_s": n5 * lv * 3 / w1,
                                     "hbm_gbs_algorithmic": round(bps, 1),
                                     "hbm_frac": round(bps / HBM_PEAK_GBS, 4),
                                     "config": p1.config()}
        del u1, ws1, p1
        if prec == "fp64":
            pc = ge.Plan(n, R, "fp32c")
            uc = ge.pack_state(u0, "fp32c")
            wsc = pc.new_workspace()
            with torch.cuda.stream(stream):
                torch.cuda.synchronize()
                wc, gc = time_runs(torch, stream,
                                   lambda: pc.step_n(uc, 0, LEVELS, workspace=wsc, stream=stream),
                                   0, 1)
            extra["fp32_compensated"] = {"updates_per_s": n * LEVELS / wc,
                                         "config": pc.config()}
        # the paper's own configuration: sub-domains of k = 16 nodes (couples
        # of 32), FP64, a rod of 2^24 - 1 points (n + 1 a multiple of 32),
        # same r, u0 and level count as the headline rod
        ns = N_DEFAULT - 1
        ps = ge.Plan(ns, R, "fp64", k=16)
        us = ge.pack_state(u0[:ns], "fp64")
        wss = ps.new_workspace()
        with torch.cuda.stream(stream):
            torch.cuda.synchronize()
            wsd, gsd = time_runs(torch, stream,
                                 lambda: ps.step_n(us, 0, LEVELS, workspace=wss, stream=stream), 1, 3)
        sups = ns * LEVELS * 3 / gsd
        # a sweep node costs one multiply and two FMAs (5 flops); the pairs
        # are a small share at k = 16
        speak = VALU_LANE_OPS * 5 / 3 / 1e12
        extra["subdomain_k16_fp64"] = {
            "updates_per_s": sups, "n": ns, "k": 16, "levels": LEVELS, "config": ps.config(),
            "roofline": {"bound": "alu", "achieved": round(sups * 5 / 1e12, 2),
                         "peak": round(speak, 1), "unit": "TFLOP/s",
                         "frac": round(sups * 5 / 1e12 / speak, 4),
                         "peak_basis": "VALU issue 3.93e13 lane-ops/s x 5 flops / 3 VALU ops "
                                       "per sweep node"}}
        del us, wss, ps
        # batch of 4096 independent rods (N log-uniform in [256, 65536],
        # r in [0.25, 4], walls in [-1, 1], seed 3), 2000 levels, FP32, one
        # persistent graph-captured launch
        rb = inputs.rod_batch(seed=3, nrods=4096, align=4)
        bt = ge.Batch.from_inputs(rb, "fp32")
        ub = ge.pack_batch_state(rb.u0, rb.offsets, rb.n, "fp32")
        wsb = bt.new_workspace()
        with torch.cuda.stream(stream):
            torch.cuda.synchronize()
            wb, gb = time_runs(torch, stream,
                               lambda: bt.solve(ub, 0, 2000, wsb, stream=stream), 1, 3)
        info = bt.info()
        bups = float(rb.n.sum()) * 2000 * 3 / gb
        bpeak = VALU_LANE_OPS_BY_PREC["fp32"] * FLOPS_PER_UPDATE["fp32"] / VALU_PER_UPDATE["fp32"] / 1e12
        extra["rod_batch_4096_fp32"] = {
            "roofline": {"bound": "alu", "achieved": round(bups * 6 / 1e12, 2), "peak": round(bpeak, 1),
                         "unit": "TFLOP/s", "frac": round(bups * 6 / 1e12 / bpeak, 4)},
            "updates_per_s": bups,
            "ms_per_run": gb / 3 * 1e3, "tasks": info["ntasks"], "workgroups": info["grid"],
            "rods": rb.nrods, "points": int(rb.n.sum()), "levels": 2000}
        del ub, wsb, bt
        # two-dimensional extension: 4096 x 4096 grid, FP64, rx = ry = 2,
        # 200 levels (one launch per level, each reading and writing the grid)
        extra["grid2d_4096_fp64"] = grid2d_extra(torch, stream, ge, inputs)
        if args.surrogate_steps > 0:
            print("[bench] surrogate ...", file=sys.stderr, flush=True)
            extra["surrogate"] = surrogate_extra(torch, stream, args.surrogate_steps)
        out["extra"] = extra

    if not args.no_cpu:
        print(f"[bench] CPU baseline (~{args.cpu_seconds:.0f} s) ...", file=sys.stderr, flush=True)
        cb = cpu_baseline(u0, args.cpu_seconds)
        out["cpu_baseline"] = cb
        # the paper's own comparison (a laptop GPU against one and eight CPU
        # threads of its host, same sweep), as context for these ratios
        out["gpu_over_cpu"] = {
            "all_cores": round(value / cb["value"], 1),
            "single_thread": round(value / cb["single_thread"]["value"], 1),
            "paper_context": "GT 335M vs i7-720QM: about 5x over 1 thread, about 2x over "
                             "8 threads (sub-domain scheme, relative figures only)"}
        if not args.no_extra:
            print("[bench] paper-shaped timing table ...", file=sys.stderr, flush=True)
            out["paper_e2_shape"] = paper_e2_table(torch, stream, ge, inputs)

    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
