"""The predictor network's HIP kernels against the FP64 reference network, and
the order estimate against the oracle's coefficient tail."""
import os
import sys

import numpy as np
import pytest

import oracle as O
import paper_2108_13478_amd as dmlib
from oracle import mlp_oracle as MO
from paper_2108_13478_amd import learn

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def unflatten(flat, sizes):
    params, off = [], 0
    for i in range(len(sizes) - 1):
        nin, nout = sizes[i], sizes[i + 1]
        W = flat[off:off + nin * nout].reshape(nout, nin).astype(np.float64)
        off += nin * nout
        b = flat[off:off + nout].astype(np.float64)
        off += nout
        params.append((W, b))
    return params


def flatten(params):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params])


def test_forward_and_gradients_match_reference():
    say("case: MLP forward / gradients 68-128-128-128-2")
    sizes = learn.SIZES
    ctx = dmlib.Context()
    ctx.dm_mlp_init(sizes, seed=3)
    rng = np.random.default_rng(0)
    X = rng.normal(size=(37, sizes[0])).astype(np.float32)
    T = rng.normal(size=(37, sizes[-1])).astype(np.float32)
    params = unflatten(ctx.dm_mlp_get_params(), sizes)
    Y = ctx.dm_mlp_forward(X)
    Yref, _ = MO.forward(params, X.astype(np.float64))
    ey = np.abs(Y - Yref).max() / np.abs(Yref).max()
    loss, g = ctx.dm_mlp_gradients(X, T)
    gref = flatten(MO.backward(params, X.astype(np.float64), T.astype(np.float64)))
    lref = MO.loss(params, X.astype(np.float64), T.astype(np.float64))
    eg = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    say(f"  forward rel err {ey:.2e}, loss {loss:.6f} vs {lref:.6f}, gradient rel err {eg:.2e}")
    assert ey < 1e-5 and abs(loss - lref) < 1e-5 * lref and eg < 1e-4


def test_adam_step_matches_reference():
    say("case: one Adam step")
    sizes = [9, 16, 16, 3]
    ctx = dmlib.Context()
    ctx.dm_mlp_init(sizes, seed=5)
    rng = np.random.default_rng(1)
    X = rng.normal(size=(20, 9)).astype(np.float32)
    T = rng.normal(size=(20, 3)).astype(np.float32)
    p0 = unflatten(ctx.dm_mlp_get_params(), sizes)
    state = {}
    ref = p0
    for _ in range(3):
        ctx.dm_mlp_train_step(X, T, 1e-2)
        ref = MO.adam_step(ref, MO.backward(ref, X.astype(np.float64), T.astype(np.float64)), state, lr=1e-2)
    got = ctx.dm_mlp_get_params()
    err = np.abs(got - flatten(ref)).max()
    say(f"  max |w_gpu - w_ref| after 3 steps = {err:.2e}")
    assert err < 1e-5


def test_order_estimate_matches_coefficient_tail():
    say("case: coefficient-tail order")
    ctx = dmlib.Context()
    for emin, emax, mu, beta, tol in ((-6.0, 20.0, 0.4, 30.0, 1e-4), (-20.0, 25.0, 1.0, 60.0, 1e-6),
                                      (0.0, 10.0, 9.0, 5.0, 1e-3)):
        N = ctx.dm_cheb_order(emin, emax, mu, beta, tol, 8192)
        a = O.fermi_coefficients(mu, beta, emin, emax, 2 * 8192)
        tail = np.cumsum(np.abs(a)[::-1])[::-1]  # tail[n] = sum_{l >= n} |a_l|
        ref = int(np.argmax(tail <= tol))
        say(f"  [{emin},{emax}] mu={mu} beta={beta} tol={tol}: N = {N} (oracle {ref}), 2 dE beta = {(emax - emin) * beta:.0f}")
        assert abs(N - ref) <= 1


def test_feature_kernel():
    ctx = dmlib.Context()
    m = np.linspace(300.0, -20.0, 64)
    x = ctx.dm_mlp_features(m, -6.0, 20.0, 40.0, 512.0, 1000)
    ebar, de = 7.0, 13.0
    ref = np.concatenate([m / 1000.0, [ebar / de, np.log10(de), 0.25 * np.log10(40.0 * de), 4 * 512 / (2 * 1000) - 2]])
    assert np.allclose(x, ref, rtol=1e-6, atol=1e-7)


def test_training_on_method_labels():
    """The training pipeline end to end on the GPU: labels from the method
    (moments pass, mu bisection, coefficient-tail order), features from
    stochastic moments, Adam steps; the loss must fall by two orders."""
    from synth import make_batch, rademacher

    rng = np.random.default_rng(7)
    n = 96
    atoms = rng.integers(64, 129, size=n)
    betas = rng.choice([20.0, 40.0], size=n)
    clusters = make_batch(atoms, range(1000, 1000 + n), onsite="scaled")
    for c, a in zip(clusters, atoms):
        c.n_electrons = float(2 * int(round(a * rng.uniform(0.8, 1.2))))
    probes = [rademacher(c.K, learn.N_VEC, seed=5000 + i) for i, c in enumerate(clusters)]
    ctx = dmlib.Context(precision=dmlib.DM_FP32)
    ctx.dm_set_operator_form(dmlib.DM_FORM_SYMMETRIC)
    X, T, rec = learn.make_dataset(ctx, clusters, betas, probes, label_order=2048, tol_order=1e-3, max_order=2048)
    say(f"case: training on {n} method-labelled clusters, K {min(r['K'] for r in rec)}..{max(r['K'] for r in rec)}")
    ctx.dm_mlp_init(learn.SIZES, seed=1)
    losses = learn.train(ctx, X, T, epochs=300, batch=32, lr=2e-3)
    say(f"  training loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    assert np.all(np.isfinite(losses)) and losses[-1] < 0.01 * losses[0]


PREDICTOR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2108_13478_amd",
                         "predictor.npz")


def _nodes(center, half, m):
    return center + half * np.cos(np.pi * (np.arange(m) + 0.5) / m)


def _lagrange(nodes, x):
    w = np.ones(len(nodes))
    for q in range(len(nodes)):
        for r in range(len(nodes)):
            if r != q:
                w[q] *= (x - nodes[r]) / (nodes[q] - nodes[r])
    return w


def _network_path(ctx, c, beta, cols, P, Ps, params, sizes, sigma, xi, tol_order, b_target, m_max, N_plain):
    """The network-assisted density matrix on a loaded context (timed by the
    caller): stochastic moments -> mu^; the window mu^ +- 2.5 sigma with the
    fewest nodes m <= m_max whose interpolation bound over the window is
    <= b_target; one multi-set pass; mu_d from the interpolated electron
    count; the Lagrange combination, or (mu_d outside the window, bound
    missed) mu by bisection and a P pass; no window: the plain two passes."""
    g = 2.0
    lo, hi = ctx.dm_get_bounds()
    ctx.dm_reset_moments()
    ctx.dm_mlp_init(sizes)
    ctx.dm_mlp_set_params(params)
    ms = ctx.dm_stoch_moments(learn.N_MOM, xi)
    mu_hat, N_hat = ctx.dm_mlp_predict(ms, beta, c.n_electrons, max_order=16384)
    half = 2.5 * sigma
    probe = np.linspace(mu_hat - half, mu_hat + half, 9)
    N = max(ctx.dm_cheb_order(lo, hi, x, beta, tol_order, 16384) for x in probe)
    m = None
    for mm in range(3, m_max + 1):
        nodes = _nodes(mu_hat, half, mm)
        if max(ctx.dm_combine_sets(nodes, beta, N, x, [], None) for x in probe) <= b_target:
            m = mm
            break
    out = dict(mu_hat=mu_hat, N_hat=N_hat, m=m, accepted=False, how="plain (no window meets the bound)")
    if m is not None:
        ctx.dm_chebyshev_block_multi(cols, N, list(nodes), [beta] * m, Ps[:m])
        trq = np.array([ctx.dm_trace(x, beta)[0] for x in nodes])
        f = lambda x: g * float(_lagrange(nodes, x) @ trq) - c.n_electrons
        a_, b_ = mu_hat - half, mu_hat + half
        out["how"] = f"window m={m}, mu outside: fallback"
        if f(a_) < 0.0 < f(b_):
            for _ in range(100):
                mid = 0.5 * (a_ + b_)
                if f(mid) < 0.0:
                    a_ = mid
                else:
                    b_ = mid
            mu = 0.5 * (a_ + b_)
            bound = ctx.dm_combine_sets(nodes, beta, N, mu, Ps[:m], P)
            out["accepted"] = bound <= b_target
            out["how"] = f"window m={m}, one pass" if out["accepted"] else f"window m={m}, bound {bound:.1e}: fallback"
        if not out["accepted"]:
            mu = ctx.dm_solve_mu(c.n_electrons, beta, tol=1e-6)
            ctx.dm_chebyshev_block(cols, N, mu, beta, P)
        out["nodes"] = nodes
    else:
        N = N_plain
        ctx.dm_chebyshev_block(cols, N, 0.0, beta, None)
        mu = ctx.dm_solve_mu(c.n_electrons, beta, tol=1e-6)
        ctx.dm_chebyshev_block(cols, N, mu, beta, P)
    out.update(mu=mu, N=N, lo=lo, hi=hi)
    return out


def _delivered_count(sp, out, beta, n_e):
    """Oracle electron count of the P a network path delivered: the sum of
    the blocks' counts with the combination weights, or the count at its mu."""
    g = 2.0
    if out["accepted"]:
        wq = _lagrange(out["nodes"], out["mu"])
        tr = sum(wq[q] * O.trace_poly(sp, out["N"], x, beta, out["lo"], out["hi"])[0]
                 for q, x in enumerate(out["nodes"]))
    else:
        tr = O.trace_poly(sp, out["N"], out["mu"], beta, out["lo"], out["hi"])[0]
    return abs(g * tr - n_e)


def test_network_window_pass_gain():
    """The trained predictor (paper_2108_13478_amd/predictor.npz, made by
    paper_2108_13478_amd/train_predictor.py on 640 method-labelled clusters,
    K 1024..4096) against the same symmetric-form path without it.

    Without the network mu is unknown before a pass: a moments pass over
    every column, mu by bisection on the exact moments (electron count to
    1e-6), then the P pass, both at the largest coefficient-tail order
    (tail <= 1e-3) over mu in the Lanczos interval.  With it (_network_path):
    16-probe stochastic moments give mu^; a window of m <= 12 Chebyshev nodes
    around it, checked before the pass by the interpolation bound <= 1e-5;
    one pass accumulating P at the nodes with the exact moments fused; mu_d
    solving the delivered P's electron count g sum_q w_q(mu_d) Tr[P_q S] =
    N_e (linear in the blocks); P = sum_q w_q(mu_d) P_q (dm_combine_sets), so
    the second pass is saved; a fallback to bisection and a P pass when mu_d
    leaves the window; the plain two passes when no window meets the bound
    (large beta against the window).

    Two comparisons, both at max|P - P_exact| <= 1e-2 (P_exact: the oracle's
    Fermi-Dirac matrix at its exact mu): the network alone, FP64 against
    FP64 (delivered electron counts in the oracle's traces within 1e-6 in
    both); and the network with the FP32 recursion against the plain FP64
    path.  The FP32 operator's rounding moves the oracle's count of the
    delivered P by about 4e-4 electrons at K = 4096 (FP32 moments), so that
    path is held to 2e-3; the 1e-6 count needs FP64 moments."""
    import json
    import time

    import torch

    from synth import make_cluster, rademacher

    W = np.load(PREDICTOR)
    meta = json.loads(str(W["meta"]))
    sigma = meta["sigma_mu"]
    sizes = [int(x) for x in W["sizes"]]
    say(f"case: network window pass; predictor trained on {meta['n_train']} clusters K {meta['K_range']}, "
        f"held-out RMS mu error {sigma:.4f} hartree (max {meta['max_mu_err']:.4f}), "
        f"RMS log2 N error {meta['sigma_log2_order']:.3f}")
    tol_order, b_target, m_max, target = 1e-3, 1e-5, 12, 1e-2
    held = [(1024, 41, 20.0), (768, 42, 20.0), (1024, 43, 30.0), (768, 44, 40.0)]
    tot = {"plain": 0.0, "net64": 0.0, "net32": 0.0}
    saved = 0
    for n_atoms, seed, beta in held:
        c = make_cluster(n_atoms, seed=seed, geometry="sphere", onsite="scaled")
        sp = O.spectrum(c)
        mu_x = O.solve_mu_exact(sp, c.n_electrons, beta)
        P_x = O.density_matrix_exact(sp, np.arange(c.K), mu_x, beta)
        cols = torch.arange(c.K, dtype=torch.int64, device="cuda")
        xi = torch.from_numpy(rademacher(c.K, learn.N_VEC, seed=9000 + seed)).cuda()
        P = torch.empty((c.K, c.K), dtype=torch.float64, device="cuda")
        Ps = [torch.empty((c.K, c.K), dtype=torch.float64, device="cuda") for _ in range(m_max)]
        ctx = dmlib.Context(precision=dmlib.DM_FP64)
        ctx.dm_set_operator_form(dmlib.DM_FORM_SYMMETRIC)
        ctx.set_cluster(c)
        lo, hi = ctx.dm_get_bounds()
        # ---- without the network (FP64)
        N_plain = max(ctx.dm_cheb_order(lo, hi, x, beta, tol_order, 16384) for x in np.linspace(lo, hi, 41))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.dm_chebyshev_block(cols, N_plain, 0.0, beta, None)
        mu_p = ctx.dm_solve_mu(c.n_electrons, beta, tol=1e-6)
        ctx.dm_chebyshev_block(cols, N_plain, mu_p, beta, P)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        err_plain = np.abs(P.cpu().numpy().T - P_x).max()
        ne_plain = abs(2.0 * O.trace_poly(sp, N_plain, mu_p, beta, lo, hi)[0] - c.n_electrons)
        res = {}
        for name, prec in (("net64", dmlib.DM_FP64), ("net32", dmlib.DM_FP32)):
            if prec != dmlib.DM_FP64:
                ctx.close()
                ctx = dmlib.Context(precision=prec)
                ctx.dm_set_operator_form(dmlib.DM_FORM_SYMMETRIC)
                ctx.set_cluster(c)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = _network_path(ctx, c, beta, cols, P, Ps, W["params"], sizes, sigma, xi, tol_order, b_target,
                                m_max, N_plain)
            torch.cuda.synchronize()
            out["t"] = time.perf_counter() - t0
            out["err"] = np.abs(P.cpu().numpy().T - P_x).max()
            out["dNe"] = _delivered_count(sp, out, beta, c.n_electrons)
            res[name] = out
        ctx.close()
        n64, n32 = res["net64"], res["net32"]
        tot["plain"] += t_plain
        tot["net64"] += n64["t"]
        tot["net32"] += n32["t"]
        saved += n64["accepted"]
        say(f"  K={c.K} beta={beta:g}: plain FP64 N={N_plain} {t_plain:.2f} s err {err_plain:.2e} "
            f"|dNe| {ne_plain:.1e} max|P| {np.abs(P_x).max():.1f}; mu^-mu={n64['mu_hat'] - mu_x:+.4f} N^={n64['N_hat']}")
        for name, o in (("network FP64", n64), ("network FP32", n32)):
            say(f"    {name}: N={o['N']} {o['how']} {o['t']:.2f} s err {o['err']:.2e} |dNe| {o['dNe']:.1e} "
                f"({t_plain / o['t']:.2f}x)")
        assert err_plain <= target and n64["err"] <= target and n32["err"] <= target
        assert ne_plain <= 1e-6 and n64["dNe"] <= 1e-6 and n32["dNe"] <= 2e-3
        del Ps, P
        torch.cuda.empty_cache()
    say(f"  total: plain FP64 {tot['plain']:.2f} s, network FP64 {tot['net64']:.2f} s "
        f"({tot['plain'] / tot['net64']:.2f}x), network FP32 {tot['net32']:.2f} s "
        f"({tot['plain'] / tot['net32']:.2f}x); second pass saved {saved}/{len(held)}")
    assert saved >= 1 and tot["plain"] / tot["net64"] > 1.0 and tot["plain"] / tot["net32"] > 1.5
