"""Single runs of the library's workloads, for profilers and quick timing.

    python -m paper_1310_3422_amd.runs batch [--precision fp32] [--levels 2000]
        the 4096-rod batch (N log-uniform in [256, 65536], r in [0.25, 4],
        walls in [-1, 1], seed 3), one graph-captured solve
    python -m paper_1310_3422_amd.runs subdomain [--k 16] [--precision fp64] [--levels 960]
        the sub-domain scheme on a rod of 2^24 - 1 points (16-mode sine u0,
        seed 2, r = 2)

Each prints one JSON line with the elapsed time of the run (HIP events on
its stream, after one untimed warm-up run).
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
    rb = inputs.rod_batch(seed=3, nrods=4096, nmax=65536 if precision == "fp32" else 32768,
                          align=4)
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


def subdomain(k, precision, levels):
    import torch
    from . import ge, inputs
    n = (1 << 24) - 1
    plan = ge.Plan(n, 2.0, precision, k=k)
    u = ge.pack_state(inputs.sine_rod(n, 2), precision)
    ws = plan.new_workspace()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        s = _timed(torch, stream, lambda: plan.step_n(u, 0, levels, workspace=ws, stream=stream))
    return {"workload": "subdomain", "k": k, "precision": precision, "n": n, "levels": levels,
            "s": s, "updates_per_s": n * levels / s, "config": plan.config()}


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
    args = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        print("runs needs a HIP device", file=sys.stderr)
        return 2
    if args.cmd == "batch":
        out = batch(args.precision, args.levels)
    else:
        out = subdomain(args.k, args.precision, args.levels)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
