"""Temporal-block depth study of the GE sweep on a long rod with a moving wall.

Workload: N = 2^27 interior points, r = 4, 5000 levels, u0 = 0, left wall
g_L(t_m) = sin(2 pi t_m), right wall 0, source f(x, t) = e^{-t} x (1 - x)
(taken at the level midpoint), in FP64 and FP32.  For each depth D (levels
fused per launch) the sweep of all levels is timed with HIP events on its
stream, inputs resident in HBM.  Reported per (precision, D):

  updates/s U; levels per launch; the average launch duration;
  F_D = U * b(D) / B_peak with b(D) = 3 s / D the algorithmic HBM bytes per
  update (s bytes per value; per launch one read of the rod and of the
  source profile b(x_i), one write of the rod);
  the speedup U / (B_peak / 3 s) over the depth-1 streaming roof.

FP64 results must be the same bits at every depth (the depth only moves the
launch boundaries; each value is computed by the same operations), which the
study checks; FP32 reports its relative L2 distance from the FP64 result.

Before every (precision, D) segment a one-element fill runs on the same
stream, so a counter or trace run can split the dispatches into segments
(the fill kernels are the separators, in the order the segments are
printed).

    python -m paper_1310_3422_amd.depth_study [--levels 5000] [--n 134217728]
"""
import argparse
import json
import sys
import time

DEPTHS = (1, 2, 4, 8, 16, 32)
PRECISIONS = ("fp64", "fp32")
HBM_PEAK_GBS = 8000.0
BYTES = {"fp64": 8, "fp32": 4}


def launches(nsteps, depth):
    """Launches a ge_step_n call issues: levels spread evenly over an even
    count (ping-pong ends in u)."""
    k = (nsteps + depth - 1) // depth
    if k % 2 == 1 and nsteps > k:
        k += 1
    return k


def run(n, levels, depths=DEPTHS, precisions=PRECISIONS, r=4.0):
    import torch
    from . import ge, inputs

    w = inputs.moving_wall_rod(n, r=r, nsteps=levels)
    stream = torch.cuda.Stream()     # default priority
    mark = torch.zeros(1, device="cuda")
    rows = []
    ref = None
    seg = 0
    for prec in precisions:
        dt = torch.float64 if prec == "fp64" else torch.float32
        gl = torch.tensor(w.g_left, dtype=torch.float64, device="cuda")
        gr = torch.tensor(w.g_right, dtype=torch.float64, device="cuda")
        sa = torch.tensor(w.src_a, dtype=torch.float64, device="cuda")
        sb = torch.tensor(w.src_b, dtype=dt, device="cuda")
        u = torch.zeros(n, dtype=dt, device="cuda")
        for d in depths:
            plan = ge.Plan(n, r, prec, src_b=sb, depth=d)
            cfg = plan.config()
            ws = plan.new_workspace()
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                mark.fill_(float(seg))
                u.zero_()
                # warm-up: the first two launches' worth of levels
                k = min(levels, 2 * cfg["depth"])
                plan.step_n(u, 0, k, workspace=ws, g_left_t=gl[:k + 1], g_right_t=gr[:k + 1],
                            src_a_t=sa[:k], stream=stream)
                u.zero_()
                ev0 = torch.cuda.Event(enable_timing=True)
                ev1 = torch.cuda.Event(enable_timing=True)
                ev0.record(stream)
                t0 = time.perf_counter()
                plan.step_n(u, 0, levels, workspace=ws, g_left_t=gl, g_right_t=gr,
                            src_a_t=sa, stream=stream)
                ev1.record(stream)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            gpu_s = ev0.elapsed_time(ev1) / 1e3
            nl = launches(levels, cfg["depth"])
            s = BYTES[prec]
            ups = n * levels / gpu_s
            per_launch = 3 * s * n          # read u and b(x_i), write u
            row = {"segment": seg, "precision": prec, "depth": d, "config": cfg,
                   "levels": levels, "launches": nl, "levels_per_launch": levels / nl,
                   "updates_per_s": ups, "updates_per_s_wall": n * levels / wall,
                   "avg_launch_us": round(gpu_s / nl * 1e6, 2),
                   "F_D": round(ups * 3 * s / (levels / nl) / 1e9 / HBM_PEAK_GBS, 4),
                   "speedup_over_streaming_roof": round(ups / (HBM_PEAK_GBS * 1e9 / (3 * s)), 3),
                   "algorithmic_bytes_per_launch": per_launch,
                   "hbm_gbs_algorithmic": round(per_launch * nl / gpu_s / 1e9, 1)}
            if prec == "fp64":
                if ref is None:
                    ref = u.clone()
                else:
                    row["same_bits_as_depth_%d" % depths[0]] = bool(torch.equal(u, ref))
            elif ref is not None:
                diff = torch.linalg.vector_norm(u.double() - ref).item()
                row["rel_l2_vs_fp64"] = diff / torch.linalg.vector_norm(ref).item()
            print(json.dumps(row), flush=True)
            rows.append(row)
            seg += 1
            del plan, ws
        del u, gl, gr, sa, sb
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--n", type=int, default=1 << 27)
    ap.add_argument("--levels", type=int, default=5000)
    ap.add_argument("--depths", default=",".join(map(str, DEPTHS)))
    ap.add_argument("--precisions", default=",".join(PRECISIONS))
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a 1 GiB fill and a 1 GiB streaming read+write (counter "
                         "calibration)")
    args = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        print("depth_study needs a HIP device", file=sys.stderr)
        return 2
    if args.calibrate_copy:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.mul(a, 2.0, out=b)
        torch.cuda.synchronize()
        del a, b
    rows = run(args.n, args.levels, tuple(int(x) for x in args.depths.split(",")),
               tuple(args.precisions.split(",")))
    bad = [r for r in rows if r.get("same_bits_as_depth_%d" % rows[0]["depth"]) is False]
    if bad:
        print(f"depth_study: FP64 results differ between depths: {bad}", file=sys.stderr)
        return 1
    return 0


if __name__ == "__main__":
    sys.exit(main())
