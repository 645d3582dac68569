"""Training data and training loop of the mu / expansion-order predictor.

Everything numeric runs in libdm.so; this module only orders the calls.
Data come from the method itself:

* mu*  -- bisection on the exact moments of a moments-only pass over every
          column (dm_batch_run with DM_BATCH_MOMENTS_ONLY) at order `label_order`;
* N*   -- smallest order whose Chebyshev coefficient tail at mu* is below
          `tol_order` (dm_cheb_order);
* x    -- features from 64 stochastic moments of 16 +-1 probe vectors, the
          Lanczos interval, beta and the filling (dm_batch_stoch_moments,
          dm_mlp_features).

Targets are encoded as dm_mlp_predict decodes them:
    y0 = 10 (mu* - Ebar) / dE,   y1 = log2(N*) / 10 - 1.
"""
from __future__ import annotations

import numpy as np

import paper_2108_13478_amd as dmlib

N_MOM = 64
N_VEC = 16
SIZES = [N_MOM + 4, 128, 128, 128, 2]


def make_dataset(ctx, clusters, betas, probes, label_order, tol_order, max_order, chunk=48, log=None):
    """Features X (n x 68), targets T (n x 2) and per-cluster records.

    clusters[i] is solved at inverse temperature betas[i] with its own
    n_electrons; probes[i] is its K x 16 block of +-1 probe vectors.
    Clusters are processed in batches of equal beta."""
    n = len(clusters)
    X = np.zeros((n, SIZES[0]), dtype=np.float32)
    T = np.zeros((n, 2), dtype=np.float32)
    rec = [None] * n
    betas = np.asarray(betas, dtype=np.float64)
    for beta in np.unique(betas):
        idx = np.nonzero(betas == beta)[0]
        for s in range(0, len(idx), chunk):
            part = idx[s:s + chunk]
            cl = [clusters[i] for i in part]
            ctx.dm_batch_set_focks(cl)
            ne = [c.n_electrons for c in cl]
            mu = ctx.dm_batch_run(label_order, float(beta), ne, tol=1e-6, flags=dmlib.DM_BATCH_MOMENTS_ONLY)
            ms = ctx.dm_batch_stoch_moments(N_MOM, [probes[i] for i in part])
            for j, i in enumerate(part):
                lo, hi = ctx.dm_batch_get_bounds(j)
                order = ctx.dm_cheb_order(lo, hi, mu[j], beta, tol_order, max_order)
                order = min(order, max_order)
                X[i] = ctx.dm_mlp_features(ms[j], lo, hi, beta, cl[j].n_electrons, cl[j].K)
                T[i] = dmlib.dm_mlp_encode_targets(mu[j], lo, hi, order)
                rec[i] = dict(K=cl[j].K, beta=float(beta), mu=float(mu[j]), emin=lo, emax=hi, order=int(order))
            if log:
                log(f"  labels: beta={beta:g} clusters {s}..{s + len(part) - 1} of {len(idx)}")
    return X, T, rec


def train(ctx, X, T, epochs=400, batch=64, lr=2e-3, seed=0, log=None):
    """Adam on the mean squared error, minibatches drawn by a seeded permutation."""
    import torch

    rng = np.random.default_rng(seed)
    n = len(X)
    losses = []
    for ep in range(epochs):
        perm = rng.permutation(n)
        Xd = torch.from_numpy(np.ascontiguousarray(X[perm])).cuda()
        Td = torch.from_numpy(np.ascontiguousarray(T[perm])).cuda()
        tot, cnt = 0.0, 0
        step_lr = lr * (0.1 ** (ep / max(1, epochs)))
        for s in range(0, n - batch + 1, batch):
            tot += ctx.dm_mlp_train_step(Xd[s:s + batch], Td[s:s + batch], step_lr) * batch
            cnt += batch
        losses.append(tot / max(cnt, 1))
        if log and (ep % 50 == 0 or ep == epochs - 1):
            log(f"  epoch {ep}: loss {losses[-1]:.3e}")
    return losses
