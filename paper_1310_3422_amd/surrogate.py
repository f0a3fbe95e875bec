"""Training and use of the learned 64-level propagator (the surrogate).

The network and its training step run in the library (ge_nn_*); this module
generates the training data with the batch GE sweep, drives the optimiser,
measures the surrogate against the sweep, and runs re-checked stepping
(ge_nn_advance).  Data: rods of ``width`` points with zero walls, 16 sine
modes with coefficients z_k / k^2 (z standard normal) and mesh ratios drawn
uniformly from [0.5, 2]; a trajectory is the FP64 GE sweep from such a rod,
sampled every 64 levels.
"""
import time

import numpy as np

from . import ge, inputs

JUMP = 64


def _torch():
    import torch
    return torch


def fp64_batch(r, width):
    """FP64 batch plan for len(r) rods of ``width`` points, zero walls."""
    nr = len(r)
    n = np.full(nr, width, dtype=np.int64)
    offsets = np.arange(nr + 1, dtype=np.int64) * width
    z = np.zeros(nr)
    return ge.Batch(n, offsets, np.asarray(r, dtype=np.float64), z, z, precision="fp64")


class Trajectories:
    """Seeded GE trajectories of ``nrods`` rods, with the FP32-rounded state
    after every 64 levels: states[j] holds level 64 j (j = 0..njumps) of all
    rods, back to back."""

    def __init__(self, seed, nrods, width=4096, njumps=8, rmin=0.5, rmax=2.0, noise=None,
                 modes=None):
        torch = _torch()
        r, u0 = inputs.surrogate_rods(seed, nrods, n=width, rmin=rmin, rmax=rmax, noise=noise,
                                      modes=modes)
        self.nrods, self.width, self.njumps = nrods, width, njumps
        self.r64 = r
        self.r = torch.from_numpy(r.astype(np.float32)).cuda()
        self.plan = fp64_batch(r, width)
        ws = self.plan.new_workspace()
        state = torch.from_numpy(np.ascontiguousarray(u0).ravel()).cuda()
        self.states = torch.empty((njumps + 1, nrods * width), dtype=torch.float32, device="cuda")
        for j in range(njumps + 1):
            ge.f64_to_f32(state, out=self.states[j])
            if j < njumps:
                self.plan.solve(state, JUMP * j, JUMP, ws)
        self.final64 = state            # FP64 state at level 64 njumps

    def rods(self, j):
        return self.states[j].view(self.nrods, self.width)


class SelfRollout:
    """Pairs (v, 64 GE levels from v) where v is the network's own state after
    ``jumps`` jumps from a random state of each rod of a trajectory chunk:
    training on them teaches the network to correct the errors its chained
    jumps accumulate.  Shaped like a one-jump Trajectories."""

    def __init__(self, net, traj, jumps, rng):
        torch = _torch()
        W, nr = net.width, traj.nrods
        self.nrods, self.njumps, self.width, self.r = nr, 1, W, traj.r
        j0 = torch.from_numpy(rng.integers(0, traj.njumps, nr)).cuda()
        st = traj.states.view(traj.njumps + 1, nr, W)
        u = st[j0, torch.arange(nr, device="cuda")].reshape(-1).contiguous()
        nxt = torch.empty_like(u)
        for _ in range(jumps):
            for i in range(0, nr, net.max_batch):
                b = min(net.max_batch, nr - i)
                sl = slice(i * W, (i + b) * W)
                net.jump(u[sl], traj.r[i:i + b].contiguous(), out=nxt[sl])
            u, nxt = nxt, u
        self.states = torch.empty((2, nr * W), dtype=torch.float32, device="cuda")
        self.states[0].copy_(u)
        g = ge.f32_to_f64(u)
        traj.plan.solve(g, 0, JUMP, traj.plan.new_workspace())
        ge.f64_to_f32(g, out=self.states[1])


class Trainer:
    """Adam on minibatches of (u, u after 64 levels) pairs drawn from
    trajectory chunks; chunk c of a data set with seed s uses seed [s, c].
    Optionally, self-rollout pair sets (SelfRollout) are refreshed during
    training and sampled for a share of the minibatches."""

    def __init__(self, net, seed=4, ntraj=2048, chunk=1024, njumps=8, minibatch=64,
                 noise=None, modes=None, progress=None):
        self.net = net
        self.progress = progress
        self.seed, self.ntraj, self.chunk = seed, ntraj, min(chunk, ntraj)
        self.njumps, self.minibatch = njumps, minibatch
        self.rng = np.random.default_rng([seed, 1 << 20])
        self.chunks = []
        for c in range((ntraj + self.chunk - 1) // self.chunk):
            nr = min(self.chunk, ntraj - c * self.chunk)
            self.chunks.append(Trajectories([seed, c], nr, net.width, njumps, noise=noise,
                                            modes=modes))
            if progress and (c + 1) % 32 == 0:
                progress(f"{(c + 1) * self.chunk} trajectories generated")
        torch = _torch()
        B, W = minibatch, net.width
        self.u = torch.empty(B * W, dtype=torch.float32, device="cuda")
        self.u64 = torch.empty_like(self.u)
        self.r = torch.empty(B, dtype=torch.float32, device="cuda")
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        self.steps = 0
        self.selfsets = []
        self.self_share = 0.0
        self.nself = 0

    def refresh_self(self, max_jumps=7, keep=4):
        """Add a self-rollout pair set (jumps cycling 1..max_jumps) from a
        random chunk, keeping the newest ``keep``."""
        c = self.chunks[int(self.rng.integers(len(self.chunks)))]
        jumps = 1 + self.nself % max_jumps
        self.nself += 1
        self.selfsets.append(SelfRollout(self.net, c, jumps, self.rng))
        del self.selfsets[:-keep]

    def _gather(self):
        torch = _torch()
        if self.selfsets and self.rng.random() < self.self_share:
            c = self.selfsets[int(self.rng.integers(len(self.selfsets)))]
        else:
            c = self.chunks[int(self.rng.integers(len(self.chunks)))]
        rods = torch.from_numpy(self.rng.integers(0, c.nrods, self.minibatch)).cuda()
        js = torch.from_numpy(self.rng.integers(0, c.njumps, self.minibatch)).cuda()
        W = self.net.width
        st = c.states.view(c.njumps + 1, c.nrods, W)
        self.u.view(-1, W).copy_(st[js, rods])
        self.u64.view(-1, W).copy_(st[js + 1, rods])
        self.r.copy_(c.r[rods])

    def train(self, steps, lr=1e-3, lr_final=None, log_every=0, self_start=None, self_every=0,
              self_share=0.5):
        """``steps`` Adam steps with the rate decaying geometrically from lr to
        lr_final; from step ``self_start`` on, a self-rollout set is added
        every ``self_every`` steps and drawn for a ``self_share`` of the
        minibatches.  Returns the losses at the logged steps."""
        lr_final = lr if lr_final is None else lr_final
        out = []
        for i in range(steps):
            if self_every and self_start is not None and i >= self_start and \
                    (i - self_start) % self_every == 0:
                self.refresh_self()
                self.self_share = self_share
            rate = lr * (lr_final / lr) ** (i / max(steps - 1, 1))
            self._gather()
            self.net.train_step(self.u, self.u64, self.r, rate, loss=self.loss)
            self.steps += 1
            if log_every and (i % log_every == 0 or i == steps - 1):
                out.append((self.steps, float(self.loss.cpu()[0])))
                if self.progress:
                    self.progress(f"step {self.steps}: loss {out[-1][1]:.3e}")
        return out


# Training data of the bundled recipe: rods whose spectrum runs from 16 up to
# a log-uniform cutoff in [16, 512] modes, plus white noise of relative size
# log-uniform in [1e-9, 1e-5], so that the network sees, and learns how the
# sweep damps, every wavelength it may meet when jumps are chained.
TRAIN_MODES = (16, 512)
TRAIN_NOISE = (1e-9, 1e-5)


# Trajectories of the bundled recipe: 200k seeded rods of 4096 points, each
# swept 8 x 64 levels in FP64 (29.5 GB of FP32 states on the device).
TRAIN_TRAJECTORIES = 200_000


def train_recipe(net, steps, seed=4, ntraj=TRAIN_TRAJECTORIES, minibatch=64, lr=2e-3,
                 lr_final=5e-5, log_every=0, progress=None):
    """Generate the recipe's trajectories with the batch sweep and train
    ``steps`` Adam steps, the second half with self-rollout sets refreshed
    12 times and drawn for half the minibatches; returns (trainer, loss log)."""
    tr = Trainer(net, seed=seed, ntraj=ntraj, chunk=min(1024, ntraj), njumps=8,
                 minibatch=minibatch, noise=TRAIN_NOISE, modes=TRAIN_MODES, progress=progress)
    log = tr.train(steps, lr=lr, lr_final=lr_final, log_every=log_every,
                   self_start=steps // 2, self_every=max(steps // 24, 1), self_share=0.5)
    return tr, log


def rel_l2_rows(x, y):
    """Per-row ||x - y|| / ||y|| of two (rods, width) arrays, in FP64."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return np.linalg.norm(x - y, axis=1) / np.maximum(np.linalg.norm(y, axis=1), 1e-300)


def evaluate(net, seed=41, nrods=256, width=None, start_jump=1):
    """Distances of one 64-level jump from the FP64 GE sweep, per rod, for the
    identity map, one GE level at mesh ratio 64 r (the big step), and the
    network; each as the state and as the increment.  The jump starts at
    level 64 start_jump of a fresh trajectory."""
    torch = _torch()
    width = width or net.width
    tr = Trajectories(seed, nrods, width, njumps=start_jump + 1)
    u = tr.rods(start_jump).contiguous()
    ref = tr.final64.view(nrods, width).cpu().numpy()
    u_np = u.cpu().numpy().astype(np.float64)
    big = fp64_batch(64.0 * tr.r64, width)
    ub = ge.f32_to_f64(u.view(-1))
    big.solve(ub, JUMP * start_jump, 1, big.new_workspace())
    un = torch.empty_like(u.view(-1))
    for i in range(0, nrods, net.max_batch):
        b = min(net.max_batch, nrods - i)
        net.jump(u[i:i + b].reshape(-1), tr.r[i:i + b].contiguous(),
                 out=un[i * width:(i + b) * width])
    torch.cuda.synchronize()
    maps = {"identity": u_np, "big_step": ub.view(nrods, width).cpu().numpy(),
            "surrogate": un.view(nrods, width).cpu().numpy().astype(np.float64)}
    res = {}
    for k, v in maps.items():
        res[k] = {"rel_l2": rel_l2_rows(v, ref),
                  "inc_rel_l2": rel_l2_rows(v - u_np, ref - u_np)}
    return res


def rollout(net, seed=41, nrods=256, width=None, njumps=8, noise=None, modes=None):
    """Per-rod rel-L2 distance from the FP64 GE sweep after each of njumps
    surrogate jumps applied in a row (no re-check), from level 0."""
    torch = _torch()
    width = width or net.width
    tr = Trajectories(seed, nrods, width, njumps=njumps, noise=noise, modes=modes)
    u = tr.rods(0).contiguous().view(-1).clone()
    nxt = torch.empty_like(u)
    out = []
    for j in range(1, njumps + 1):
        for i in range(0, nrods, net.max_batch):
            b = min(net.max_batch, nrods - i)
            sl = slice(i * width, (i + b) * width)
            net.jump(u[sl], tr.r[i:i + b].contiguous(), out=nxt[sl])
        u, nxt = nxt, u
        ref = tr.rods(j).cpu().numpy()
        out.append(rel_l2_rows(u.view(nrods, width).cpu().numpy(), ref))
    return np.stack(out)        # [njumps, nrods]


def advance_with_recheck(net, u, r, njumps, ge_batch=None, r64=None, check=8, tol=1e-4,
                         step0=0, stream=None):
    """Re-checked stepping of FP32 rods u (device, batch x width) with mesh
    ratios r (device FP32); the FP64 GE plan is built from r64 (host) when not
    given.  Returns (fallback rod-windows, accepted per rod, fallbacks per rod,
    last distance per rod)."""
    torch = _torch()
    b = r.numel()
    if ge_batch is None:
        ge_batch = fp64_batch(r64, net.width)
    ws = ge_batch.new_workspace()
    acc = torch.zeros(b, dtype=torch.int32, device="cuda")
    fb = torch.zeros(b, dtype=torch.int32, device="cuda")
    err = torch.zeros(b, dtype=torch.float64, device="cuda")
    nfb = net.advance(ge_batch, ws, u, r, njumps, step0=step0, check=check, tol=tol,
                      accepted=acc, fallbacks=fb, last_err=err, stream=stream)
    return nfb, acc.cpu().numpy(), fb.cpu().numpy(), err.cpu().numpy()


# algorithmic flops of one 64-level jump per point (real channels 2->64,
# four 64->64, 64->1; five taps; multiply-add counted as 2)
FLOPS_PER_POINT = 2 * 5 * (2 * 64 + 4 * 64 * 64 + 64 * 1)


def time_jump(batch=1024, width=4096, reps=5, seed=42):
    """Time the fused jump (an untrained network: the arithmetic does not
    depend on the weights) on ``batch`` seeded rods; returns a dict."""
    torch = _torch()
    net = ge.Net(width=width, max_batch=batch, seed=4)
    r, u0 = inputs.surrogate_rods(seed, batch, n=width)
    u = torch.from_numpy(u0.astype(np.float32).ravel()).cuda()
    rf = torch.from_numpy(r.astype(np.float32)).cuda()
    out = torch.empty_like(u)
    for _ in range(2):
        net.jump(u, rf, out=out)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        net.jump(u, rf, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"batch": batch, "width": width, "ms_per_jump": ms,
            "tflops_algorithmic": FLOPS_PER_POINT * width * batch / ms / 1e9}


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="surrogate utilities")
    sub = ap.add_subparsers(dest="cmd", required=True)
    tj = sub.add_parser("time-jump", help="time the fused 64-level jump")
    tj.add_argument("--batch", type=int, default=1024)
    tj.add_argument("--width", type=int, default=4096)
    tj.add_argument("--reps", type=int, default=5)
    args = ap.parse_args(argv)
    if args.cmd == "time-jump":
        print(json.dumps(time_jump(args.batch, args.width, args.reps)), flush=True)
    return 0


if __name__ == "__main__":
    import sys
    sys.exit(main())
