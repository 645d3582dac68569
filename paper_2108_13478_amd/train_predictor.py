"""Train the mu / expansion-order predictor on clusters labelled by the
method itself, on the GPU with the library's own kernels, and save it.

    python -m paper_2108_13478_amd.train_predictor --out paper_2108_13478_amd/predictor.npz

Training set: n clusters (spheres of n_atoms uniform in [atoms_lo,
atoms_hi], seeds seed0 + i, the bounded on-site variant F = T + (ES + SE)/2
of synth.make_cluster, filling N_e = 2 round(n_atoms u), u ~ U(0.8, 1.2)),
beta drawn from `betas`.  Labels (learn.make_dataset): mu* by bisection on
the exact moments of an FP32 symmetric-form moments pass over every column
at order `label_order`, N* from the coefficient tail at mu* (tol 1e-3).
Features: 64 stochastic moments of 16 +-1 probe vectors, the Lanczos
interval, beta and the filling.  The last tenth of the set is held out:
its RMS error in mu (hartree) and in log2 N is saved with the weights and
sizes the mu window of the network-assisted pass.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import paper_2108_13478_amd as dmlib  # noqa: E402
from paper_2108_13478_amd import learn  # noqa: E402
from synth import make_batch, rademacher  # noqa: E402


def log(msg):
    print(msg, flush=True)


def build_set(n, atoms_lo, atoms_hi, betas, seed0, rng):
    atoms = rng.integers(atoms_lo, atoms_hi + 1, size=n)
    beta = rng.choice(np.asarray(betas, dtype=np.float64), size=n)
    clusters = make_batch(atoms, range(seed0, seed0 + n), processes=16, onsite="scaled")
    for c, a in zip(clusters, atoms):
        c.n_electrons = float(2 * int(round(a * rng.uniform(0.8, 1.2))))
    probes = [rademacher(c.K, learn.N_VEC, seed=seed0 + 500000 + i) for i, c in enumerate(clusters)]
    return clusters, beta, probes


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--n", type=int, default=640)
    ap.add_argument("--atoms-lo", type=int, default=256)
    ap.add_argument("--atoms-hi", type=int, default=1024)
    ap.add_argument("--betas", default="20,30,40")
    ap.add_argument("--label-order", type=int, default=2048)
    ap.add_argument("--epochs", type=int, default=600)
    ap.add_argument("--seed0", type=int, default=20000)
    a = ap.parse_args(argv)
    rng = np.random.default_rng(11)
    t0 = time.perf_counter()
    clusters, betas, probes = build_set(a.n, a.atoms_lo, a.atoms_hi, [float(b) for b in a.betas.split(",")],
                                        a.seed0, rng)
    Ks = [c.K for c in clusters]
    log(f"training set: {a.n} clusters, K {min(Ks)}..{max(Ks)}, built in {time.perf_counter() - t0:.1f} s")
    ctx = dmlib.Context(precision=dmlib.DM_FP32)
    ctx.dm_set_operator_form(dmlib.DM_FORM_SYMMETRIC)
    t0 = time.perf_counter()
    X, T, rec = learn.make_dataset(ctx, clusters, betas, probes, label_order=a.label_order, tol_order=1e-3,
                                   max_order=a.label_order, log=log)
    t_label = time.perf_counter() - t0
    log(f"labelled by the method in {t_label:.1f} s")
    n_val = max(1, a.n // 10)
    Xt, Tt, Xv, Tv = X[:-n_val], T[:-n_val], X[-n_val:], T[-n_val:]
    ctx.dm_mlp_init(learn.SIZES, seed=1)
    t0 = time.perf_counter()
    losses = learn.train(ctx, Xt, Tt, epochs=a.epochs, batch=64, lr=2e-3, log=log)
    t_train = time.perf_counter() - t0
    Y = ctx.dm_mlp_forward(Xv)
    # decode as dm_mlp_predict does: mu = Ebar + dE y0 / 10, log2 N = 10 (y1 + 1)
    de = np.array([0.5 * (r["emax"] - r["emin"]) for r in rec[-n_val:]])
    mu_err = (Y[:, 0] - Tv[:, 0]) * de / 10.0
    logn_err = 10.0 * (Y[:, 1] - Tv[:, 1])
    sigma_mu = float(np.sqrt(np.mean(mu_err ** 2)))
    sigma_logn = float(np.sqrt(np.mean(logn_err ** 2)))
    log(f"trained in {t_train:.1f} s: loss {losses[0]:.3e} -> {losses[-1]:.3e}; held-out {n_val}: "
        f"RMS mu error {sigma_mu:.4f} hartree (max {np.abs(mu_err).max():.4f}), RMS log2 N error {sigma_logn:.3f}")
    meta = dict(n_train=a.n - n_val, n_val=n_val, K_range=[int(min(Ks)), int(max(Ks))], betas=a.betas,
                label_order=a.label_order, epochs=a.epochs, seed0=a.seed0, sigma_mu=sigma_mu,
                max_mu_err=float(np.abs(mu_err).max()), sigma_log2_order=sigma_logn, loss_first=float(losses[0]),
                loss_last=float(losses[-1]), label_seconds=t_label, train_seconds=t_train)
    np.savez(a.out, params=ctx.dm_mlp_get_params(), sizes=np.asarray(learn.SIZES, dtype=np.int64),
             meta=json.dumps(meta))
    log(f"saved {a.out}: {json.dumps(meta)}")


if __name__ == "__main__":
    main()
