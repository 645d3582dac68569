"""The predictor network's HIP kernels against the FP64 reference network, and
the order estimate against the oracle's coefficient tail."""
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


def test_trained_network_gain():
    """Train the predictor on method-generated data, then compare on held-out
    clusters the plain FP64 path (no network) with the network + FP32 path.

    Plain (FP64): order from the paper's rule N = 2 dE beta; a moments pass,
    mu by bisection, a P pass.  Network (FP32): 16-probe stochastic moments,
    predicted (mu, N); a P pass at the predicted mu with the exact moments
    fused; accepted if |2 Tr[PS] - N_e| <= 1e-6, otherwise mu by bisection
    from those moments and a second P pass (the bisection stays the judge).
    Accuracy is max|P - P_exact| against the oracle's Fermi-Dirac matrix at
    the oracle's own mu; time is the wall time of each path on the GPU."""
    import time

    import torch

    from synth import make_batch, rademacher

    rng = np.random.default_rng(7)
    n_train = 384
    atoms = rng.integers(64, 257, size=n_train)
    betas = rng.choice([20.0, 40.0, 80.0], size=n_train)
    clusters = make_batch(atoms, range(1000, 1000 + n_train), processes=16, onsite="scaled")
    for c, a in zip(clusters, atoms):
        c.n_electrons = float(2 * int(round(a * rng.uniform(0.8, 1.2))))
    probes = [rademacher(c.K, learn.N_VEC, seed=5000 + i) for i, c in enumerate(clusters)]
    tctx = dmlib.Context(precision=dmlib.DM_FP32)
    # features and the network path use the symmetric form: its stochastic
    # moments probe T_l(H~_N), whose Frobenius norm is at most sqrt(K), so the
    # +-1 estimates are far less noisy than with the non-normal S^-1 F
    tctx.dm_set_operator_form(dmlib.DM_FORM_SYMMETRIC)
    t0 = time.perf_counter()
    X, T, rec = learn.make_dataset(tctx, clusters, betas, probes, label_order=4096, tol_order=1e-3,
                                   max_order=8192)
    say(f"case: training set of {n_train} clusters (K {min(r['K'] for r in rec)}..{max(r['K'] for r in rec)}) "
        f"labelled by the method in {time.perf_counter() - t0:.1f} s")
    tctx.dm_mlp_init(learn.SIZES, seed=1)
    losses = learn.train(tctx, X, T, epochs=400, batch=64, lr=2e-3)
    say(f"  training loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    assert losses[-1] < 0.05 * losses[0]
    params = tctx.dm_mlp_get_params()

    held = [(384, 31, 20.0), (448, 32, 40.0), (320, 33, 80.0), (512, 34, 40.0)]
    t_plain, t_net, acc_net, orders = [], [], 0, []
    for n_atoms, seed, beta in held:
        c = make_batch([n_atoms], [seed], processes=1, onsite="scaled")[0]
        c.n_electrons = float(2 * n_atoms)
        sp = O.spectrum(c)
        mu_x = O.solve_mu_exact(sp, c.n_electrons, beta)
        P_x = O.density_matrix_exact(sp, np.arange(c.K), mu_x, beta)
        cols = torch.arange(c.K, dtype=torch.int64, device="cuda")
        P = torch.empty((c.K, c.K), dtype=torch.float64, device="cuda")
        # ---- plain FP64 path
        p64 = dmlib.Context(precision=dmlib.DM_FP64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p64.set_cluster(c)
        lo, hi = p64.dm_get_bounds()
        N_rule = dmlib.dm_cheb_order_rule(lo, hi, beta, 16, 8192)
        p64.dm_chebyshev_block(cols, N_rule, 0.0, beta, None)
        mu_p = p64.dm_solve_mu(c.n_electrons, beta, tol=1e-6)
        p64.dm_chebyshev_block(cols, N_rule, mu_p, beta, P)
        torch.cuda.synchronize()
        t_plain.append(time.perf_counter() - t0)
        err_plain = np.abs(P.cpu().numpy().T - P_x).max()
        # ---- network + FP32 path
        n32 = dmlib.Context(precision=dmlib.DM_FP32)
        n32.dm_set_operator_form(dmlib.DM_FORM_SYMMETRIC)
        n32.dm_mlp_init(learn.SIZES)
        n32.dm_mlp_set_params(params)
        xi = torch.from_numpy(rademacher(c.K, learn.N_VEC, seed=9000 + seed)).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n32.set_cluster(c)
        ms = n32.dm_stoch_moments(learn.N_MOM, xi)
        mu_hat, N_hat = n32.dm_mlp_predict(ms, beta, c.n_electrons, max_order=8192)
        N_use = int(np.ceil(1.1 * N_hat))
        n32.dm_chebyshev_block(cols, N_use, mu_hat, beta, P)
        tr, _ = n32.dm_trace(mu_hat, beta)
        accepted = abs(2.0 * tr - c.n_electrons) <= 1e-6
        if not accepted:
            mu_n = n32.dm_solve_mu(c.n_electrons, beta, tol=1e-4)
            n32.dm_chebyshev_block(cols, N_use, mu_n, beta, P)
        torch.cuda.synchronize()
        t_net.append(time.perf_counter() - t0)
        err_net = np.abs(P.cpu().numpy().T - P_x).max()
        acc_net += accepted
        orders.append((N_rule, N_hat))
        say(f"  K={c.K} beta={beta:g}: plain N={N_rule} {t_plain[-1] * 1e3:.0f} ms err {err_plain:.2e} | "
            f"net N^={N_hat} mu^-mu={mu_hat - mu_p:+.3f} accepted={accepted} {t_net[-1] * 1e3:.0f} ms "
            f"err {err_net:.2e} (max|P| {np.abs(P_x).max():.1f})")
        assert err_net <= max(2.0 * err_plain, 1e-3 * np.abs(P_x).max())
    speed = sum(t_plain) / sum(t_net)
    say(f"  time per density matrix: plain FP64 {np.mean(t_plain) * 1e3:.0f} ms, network + FP32 "
        f"{np.mean(t_net) * 1e3:.0f} ms ({speed:.2f}x); predictions accepted {acc_net}/{len(held)}; "
        f"order N^/N_rule = {[round(b / a, 2) for a, b in orders]}")
    assert speed > 1.0
