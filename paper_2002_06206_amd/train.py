"""Training of the learned pressure preconditioner on the GPU.

(b, p) pairs come from the plain FP64 solver (ibm_step, Jacobi PCG) run on seeded
windows of the ellipsoid field; every Adam step goes through ibm_cnn_train_step, i.e.
the library's own BF16 MFMA forward and backward kernels.  This module only drives
those entry points (argument marshalling and the host loop) and forms the training
pairs from the solver's fields with a few torch vector operations.

    python -m paper_2002_06206_amd.train --out weights.npy [--seeds 1 2 3 4] [--n 64]
"""
from __future__ import annotations

import argparse
import time

import numpy as np
import torch

from . import ibm, inputs

TRAIN_SEEDS = tuple(range(101, 121))   # 20 windows
EVAL_SEEDS = (201, 202)


def generate_pairs(case: inputs.Case, steps: int = 24, every: int = 3, tol: float = 1e-8, first: int = 2,
                   depths=(0,)):
    """Runs the plain FP64 solver for `steps` CFL-0.3 steps and keeps (b, p) of every
    `every`-th step from step `first` on (b = the compatible Poisson right-hand side,
    p = its solution).  With depths, the i-th kept pair is taken at Krylov depth
    k = depths[i % len(depths)]: x_k = k Jacobi-PCG iterates from zero on L x = b and
    the pair (b - L x_k, p - x_k), which satisfies the same equation and carries the
    error a Krylov method still has to remove after k iterations.  Depth -1 takes x
    = 2 p^n - p^{n-1}, the extrapolated initial guess of the step's solve (what is left
    for the solver when the step starts from that guess).  Depth -2 takes one damped
    Jacobi step from zero, x = (6/7) b / diag(L) (what the network sees inside the
    smoothed preconditioner: the residual after its pre-smoothing step).  Returns the
    solver (it owns the stencil the pairs belong to) and the pairs."""
    if any(d < -2 for d in depths):
        raise ValueError("training-pair depths are >= 0, -1 (extrapolated guess) or -2 (damped Jacobi step)")
    s = ibm.Solver(case.n, case.dx, case.origin, case.bc, case.u_in, ibm.FP64)
    blocked, _ = s.tag(case.tri, want_theta=False)
    s.build(blocked, None, case.deadend)
    st = s.new_state(case.u_in)
    pairs = []
    diag = laplacian_diagonal(s) if -2 in depths else None
    umax, dt_prev = max(abs(v) for v in case.u_in), 0.0
    p_older = st["p"].clone()   # p^{n-1}
    for k in range(steps):
        dt = min(case.dt, 0.3 * case.dx / max(umax, 1e-30))
        p_old = st["p"].clone()     # p^n
        rc, stats = s.step(st, ibm.step_params(dt, case.nu, csm=case.csm, step=k, dt_prev=dt_prev, tol=tol))
        if rc < 0 or not np.isfinite(stats["umax"]):
            break
        umax, dt_prev = stats["umax"], dt
        if k >= first and (k - first) % every == 0:
            b = s.rhs()
            if float(torch.linalg.vector_norm(b)) > 0.0:
                p = st["p"].clone()
                depth = depths[len(pairs) % len(depths)]
                if depth > 0:
                    x = torch.zeros_like(b)
                    s.poisson(b, x, tol=1e-300, max_iter=depth, kind=ibm.SOLVER_PCG_JACOBI)
                    b, p = b - s.laplacian(x), p - x
                elif depth == -1:
                    x = 2.0 * p_old - p_older
                    b, p = b - s.laplacian(x), p - x
                elif depth == -2:
                    x = torch.where(diag < 0.0, (6.0 / 7.0) * b / diag, torch.zeros_like(b))
                    b, p = b - s.laplacian(x), p - x
                pairs.append((b, p))
        p_older = p_old
    return s, pairs


def laplacian_diagonal(s: ibm.Solver):
    """Diagonal of the solver's pressure operator L, read off its applications to the
    indicator fields of a colouring in which no cell shares its colour with one of its
    six neighbours, periodic wraps included: per axis the index modulo the smallest
    m >= 2 with n mod m != 1 (neighbours differ by one in one index, or sit at 0 and
    n - 1), the colour the tuple of the three residues."""
    nz, ny, nx = s.shape
    dev = s.dev
    mods = []
    for n in (nx, ny, nz):
        m = 2 if n > 1 else 1   # one cell: no neighbour along the axis
        while n > 1 and n % m == 1:
            m += 1
        mods.append(m)
    ci = torch.arange(nx, device=dev).view(1, 1, -1) % mods[0]
    cj = torch.arange(ny, device=dev).view(1, -1, 1) % mods[1]
    ck = torch.arange(nz, device=dev).view(-1, 1, 1) % mods[2]
    col = ci + mods[0] * (cj + mods[1] * ck)
    diag = torch.zeros((nz, ny, nx), dtype=torch.float64, device=dev)
    for c in range(mods[0] * mods[1] * mods[2]):
        e = (col == c).to(torch.float64)
        diag += s.laplacian(e) * e
    return diag


def build_dataset(seeds, n: int = 64, steps: int = 24, every: int = 3, depths=(0,)):
    data = []
    for seed in seeds:
        s, pairs = generate_pairs(inputs.case_ellipsoid_window(seed, n), steps, every, first=min(2, steps - 1),
                                  depths=depths)
        if pairs:
            data.append((s, pairs))
    return data


def mean_loss(net: ibm.Network, data, omega: float = 0.0) -> float:
    ls = [net.loss(s, b, p, omega=omega) for s, pairs in data for b, p in pairs]
    return float(np.mean(ls)) if ls else float("nan")


def train(net: ibm.Network, data, iters: int = 600, lr: float = 1e-3, seed: int = 0, log_every: int = 0,
          lr_final: float | None = None, omega: float = 0.0):
    """Adam on single pairs drawn uniformly at random; the learning rate decays
    geometrically to lr_final (default lr / 10).  omega > 0 trains the network through
    the smoothed form of the preconditioner.  Returns the per-step losses."""
    rng = np.random.default_rng(seed)
    index = [(i, j) for i, (_, pairs) in enumerate(data) for j in range(len(pairs))]
    lr_final = lr / 10.0 if lr_final is None else lr_final
    losses = []
    for k in range(iters):
        i, j = index[rng.integers(len(index))]
        s, pairs = data[i]
        b, p = pairs[j]
        a = lr * (lr_final / lr) ** (k / max(iters - 1, 1))
        losses.append(net.train_step(s, b, p, a, omega))
        if log_every and (k + 1) % log_every == 0:
            print("train step %d loss %.4f (mean of last %d %.4f)" % (k + 1, losses[-1], log_every,
                                                                     np.mean(losses[-log_every:])), flush=True)
    return losses


def solve_iterations(s: ibm.Solver, b, kind, tol: float = 1e-6, warm=None, **kw):
    """Iterations and wall time of one pressure solve of pair right-hand side b."""
    x = torch.zeros_like(b) if warm is None else warm.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, stats = s.poisson(b, x, tol=tol, max_iter=20000, kind=kind, **kw)
    torch.cuda.synchronize()
    return stats, time.perf_counter() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--seeds", type=int, nargs="*", default=list(TRAIN_SEEDS))
    ap.add_argument("--iters", type=int, default=1500)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--init-seed", type=int, default=0)
    args = ap.parse_args()
    torch.cuda.set_device(0)
    t0 = time.time()
    data = build_dataset(args.seeds, args.n)
    held = build_dataset(EVAL_SEEDS, args.n)
    print("pairs: train %d, held-out %d (%.1fs)" % (sum(len(p) for _, p in data), sum(len(p) for _, p in held),
                                                   time.time() - t0), flush=True)
    net = ibm.Network(args.n ** 3, inputs.cnn_init_weights(args.init_seed))
    print("held-out loss before %.4f" % mean_loss(net, held), flush=True)
    train(net, data, args.iters, args.lr, log_every=100)
    print("held-out loss after %.4f (%.1fs)" % (mean_loss(net, held), time.time() - t0), flush=True)
    np.save(args.out, net.weights)


if __name__ == "__main__":
    main()
