"""Single runs of the library's workloads, for profilers and quick timing.

    python -m paper_1310_3422_amd.runs batch [--precision fp32] [--levels 2000]
        the 4096-rod batch (N log-uniform in [256, 65536], r in [0.25, 4],
        walls in [-1, 1], seed 3), one graph-captured solve (rods above the
        form's on-chip limit run as long-rod tasks)
    python -m paper_1310_3422_amd.runs subdomain [--k 16] [--precision fp64] [--levels 960]
        the sub-domain scheme on a rod of 2^24 - 1 points (16-mode sine u0,
        seed 2, r = 2)

    python -m paper_1310_3422_amd.runs occupancy [--precision fp32] [--levels 1200]
        the paper's node-rate experiments at MI355X scale: at the paper's row
        of 8208 x 32 - 1 points, updates/s against the number of workgroups
        (tile and waves of the two-point-group sweep, depth 8, one workgroup
        per tile); then updates/s against the rod length (32 * 2^j - 1
        points, j = 8..19) for the sub-domain scheme (k = 16) and the
        two-point groups at the library's choices

    python -m paper_1310_3422_amd.runs grid2d [--precision fp64] [--levels 200]
        the two-dimensional extension on a 4096 x 4096 grid (rx = ry = 2)

Each prints JSON lines with the elapsed time of the run (HIP events on its
stream, after one untimed warm-up run).
"""
import argparse
import json
import sys


def _timed(torch, stream, fn):
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3


def batch(precision, levels):
    import torch
    from . import ge, inputs
    rb = inputs.rod_batch(seed=3, nrods=4096, align=4)
    b = ge.Batch.from_inputs(rb, precision)
    u = ge.pack_batch_state(rb.u0, rb.offsets, rb.n, precision)
    ws = b.new_workspace()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        s = _timed(torch, stream, lambda: b.solve(u, 0, levels, ws, stream=stream))
    pts = int(rb.n.sum())
    return {"workload": "rod_batch_4096", "precision": precision, "levels": levels,
            "points": pts, "s": s, "updates_per_s": pts * levels / s, **b.info(),
            "rod_k": None}


def subdomain(k, precision, levels, schedule=0, depth=0):
    import torch
    from . import ge, inputs
    n = (1 << 24) - 1
    plan = ge.Plan(n, 2.0, precision, k=k, schedule=schedule, depth=depth)
    u = ge.pack_state(inputs.sine_rod(n, 2), precision)
    ws = plan.new_workspace()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        s = _timed(torch, stream, lambda: plan.step_n(u, 0, levels, workspace=ws, stream=stream))
    return {"workload": "subdomain", "k": k, "precision": precision, "n": n, "levels": levels,
            "s": s, "updates_per_s": n * levels / s, "config": plan.config()}


def grid2d(precision, levels, nx=4096, ny=4096, depth=0):
    import numpy as np
    import torch
    from . import ge, inputs
    fx = inputs.sine_rod(nx, seed=2)
    y = np.arange(1, ny + 1) / (ny + 1)
    dt = torch.float64 if precision == "fp64" else torch.float32
    u = torch.from_numpy(np.outer(np.sin(np.pi * y), fx)).to(dt).cuda()
    ws = torch.empty_like(u)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        s = _timed(torch, stream, lambda: ge.step2d_n(u, nx, ny, 2.0, 2.0, 0, levels,
                                                      precision=precision, workspace=ws,
                                                      stream=stream, depth=depth))
    return {"workload": "grid2d", "precision": precision, "nx": nx, "ny": ny, "levels": levels,
            "depth": depth, "s": s, "updates_per_s": nx * ny * levels / s}


def occupancy(precision, levels):
    import torch
    from . import ge, inputs
    stream = torch.cuda.Stream()
    n = 8208 * 32 - 1
    u0 = inputs.sine_rod(n, 2)
    for waves in (1, 4):
        for tile in ((2, 4, 8, 16, 32) if precision == "fp64" else (4, 8, 16, 32)):
            plan = ge.Plan(n, 2.0, precision, tile=tile, waves=waves, depth=8, schedule=1)
            cfg = plan.config()
            window = 64 * waves * tile
            wgs = 1 if n <= window else -(-n // (window - 2 * cfg["halo"]))
            u = ge.pack_state(u0, precision)
            ws = plan.new_workspace()
            with torch.cuda.stream(stream):
                s = _timed(torch, stream,
                           lambda: plan.step_n(u, 0, levels, workspace=ws, stream=stream))
            yield {"sweep": "workgroups", "precision": precision, "n": n, "levels": levels,
                   "tile": tile, "waves": waves, "workgroups": wgs, "s": s,
                   "updates_per_s": n * levels / s}
            del plan, u, ws
    for j in range(8, 20):
        n = 32 * (1 << j) - 1
        u0 = inputs.sine_rod(n, 2)
        for k in (16, 0):
            plan = ge.Plan(n, 2.0, precision, k=k)
            u = ge.pack_state(u0, precision)
            ws = plan.new_workspace()
            with torch.cuda.stream(stream):
                s = _timed(torch, stream,
                           lambda: plan.step_n(u, 0, levels, workspace=ws, stream=stream))
            yield {"sweep": "length", "precision": precision, "n": n, "levels": levels,
                   "scheme": "subdomain_k16" if k else "groups", "config": plan.config(),
                   "s": s, "updates_per_s": n * levels / s}
            del plan, u, ws


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    b = sub.add_parser("batch")
    b.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "fp32c"])
    b.add_argument("--levels", type=int, default=2000)
    s = sub.add_parser("subdomain")
    s.add_argument("--k", type=int, default=16)
    s.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    s.add_argument("--levels", type=int, default=960)
    s.add_argument("--schedule", type=int, default=0, choices=[0, 1, 2])
    s.add_argument("--depth", type=int, default=0)
    g2 = sub.add_parser("grid2d")
    g2.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    g2.add_argument("--levels", type=int, default=200)
    g2.add_argument("--depth", type=int, default=0, choices=[0, 1, 2, 4])
    o = sub.add_parser("occupancy")
    o.add_argument("--precision", default="fp32", choices=["fp64", "fp32"])
    o.add_argument("--levels", type=int, default=1200)
    args = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        print("runs needs a HIP device", file=sys.stderr)
        return 2
    if args.cmd == "occupancy":
        for line in occupancy(args.precision, args.levels):
            print(json.dumps(line), flush=True)
        return 0
    if args.cmd == "grid2d":
        out = grid2d(args.precision, args.levels, depth=args.depth)
    elif args.cmd == "batch":
        out = batch(args.precision, args.levels)
    else:
        out = subdomain(args.k, args.precision, args.levels, args.schedule, args.depth)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
