"""Training workflow of the learned preconditioner (orchestration only).

Every numeric step runs in libpsc: pairs come from ``psc_pairs_collect``
(preconditioned CG runs whose residuals r_k and V-cycle corrections B r_k are
cropped on the device), training is ``psc_net_train`` (forward/backward
kernels + Adam), evaluation is ``psc_fcg_solve`` with and without the
network. This module only draws the random inputs (right-hand sides, crop
corners, minibatch order) and moves them across the boundary.
"""
from __future__ import annotations

import time

import numpy as np

from . import problems as P
from . import psc


def collect_pairs(h, n, uniform_seeds, bump_seeds, crops, crop=40, seed=0, maxit=200, expect_iters=30):
    """Crops of (r_k/s_k, B r_k/s_k) from PCG runs on an n^3 grid.

    Returns device tensors (r, z) of shape (count, crop, crop, crop).
    """
    import torch
    runs = [("u", s) for s in uniform_seeds] + [("b", s) for s in bump_seeds]
    cpi = max(1, int(np.ceil(crops / (len(runs) * expect_iters))))
    r = torch.empty((crops, crop, crop, crop), dtype=torch.float32, device="cuda")
    z = torch.empty_like(r)
    count = 0
    rng_seed = seed
    for kind, s in runs:
        if count >= crops:
            break
        b = P.rhs_uniform(n ** 3, s) if kind == "u" else P.rhs_bumps(n, s)
        origins = P.crop_origins(rng_seed, cpi * (maxit + 1), (n, n, n), crop)
        rng_seed += 1
        count = psc.pairs_collect(h, torch.from_numpy(b).cuda(), (n, n, n), crop, cpi, origins, r, z,
                                  count=count, rtol=1e-6, maxit=maxit)
    return r[:count], z[:count]


def train(net, r, z, epochs=2, batch=16, margin=3, lr=1e-3, seed=0, holdout=0.05, log=None, lr_min=None,
          chunks_per_epoch=8):
    """Adam on the stored crops; returns (train losses, validation loss before, after).

    With lr_min set, the learning rate follows a cosine from lr to lr_min over
    the run, changed between chunks of an epoch (each chunk is one
    psc_net_train call).
    """
    count = r.shape[0]
    rng = np.random.default_rng(seed)
    perm = rng.permutation(count)
    nval = max(batch, int(holdout * count))
    val, tr = perm[:nval], perm[nval:]

    def val_loss():
        tot = 0.0
        k = 0
        for i in range(0, len(val) - batch + 1, batch):
            ids = val[i:i + batch]
            loss, _ = net.loss_grad(r[ids].contiguous(), z[ids].contiguous(), margin)
            tot += loss
            k += 1
        return tot / max(k, 1)

    v0 = val_loss()
    losses = []
    t0 = time.time()
    steps_per_epoch = len(tr) // batch
    total = epochs * chunks_per_epoch
    k = 0
    for ep in range(epochs):
        order = tr[rng.permutation(len(tr))][:steps_per_epoch * batch].astype(np.int32)
        bounds = np.linspace(0, steps_per_epoch, chunks_per_epoch + 1).astype(int)
        ep_losses = []
        for c in range(chunks_per_epoch):
            lr_k = lr if lr_min is None else lr_min + 0.5 * (lr - lr_min) * (1 + np.cos(np.pi * k / max(total - 1, 1)))
            k += 1
            s0, s1 = bounds[c], bounds[c + 1]
            if s1 <= s0:
                continue
            ep_losses.append(net.train(r, z, order[s0 * batch:s1 * batch], steps=s1 - s0, batch=batch,
                                       margin=margin, lr=float(lr_k)))
        losses.append(np.concatenate(ep_losses))
        if log:
            log(f"epoch {ep}: mean loss {losses[-1].mean():.4e} ({time.time() - t0:.1f}s)")
    v1 = val_loss()
    return np.concatenate(losses) if losses else np.zeros(0), v0, v1


def evaluate(h, net, n, seeds, kinds=("uniform",), rtol=1e-6, reps=1):
    """Held-out solves: FP64 PCG, learned FCG, and both FCG forms with the FP32 V-cycle; iterations and ms.

    The hierarchy must have been built with build_fp32.
    """
    import torch
    out = []
    x = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
    for kind in kinds:
        for s in seeds:
            if kind == "uniform":
                b = P.rhs_uniform(n ** 3, s)
            else:
                b = P.rhs_from_solution(*P.poisson7(n), P.x_true(n ** 3, s))
            bd = torch.from_numpy(b).cuda()
            row = {"kind": kind, "seed": s}
            for name, fn in [("pcg", lambda: h.pcg(bd, x, rtol=rtol)),
                             ("learned", lambda: h.fcg(bd, x, rtol=rtol, net=net)),
                             ("mixed", lambda: h.fcg(bd, x, rtol=rtol, prec=psc.FP32)),
                             ("learned_mixed", lambda: h.fcg(bd, x, rtol=rtol, net=net, prec=psc.FP32))]:
                x.zero_()
                fn()
                torch.cuda.synchronize()
                t = time.perf_counter()
                for _ in range(reps):
                    x.zero_()
                    res = fn()
                torch.cuda.synchronize()
                row[name] = dict(res, ms=(time.perf_counter() - t) * 1e3 / reps)
            out.append(row)
    return out
