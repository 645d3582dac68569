"""Batch of uneven clusters through one persistent, graph-captured launch
sequence (dm_batch_*), against the oracle and against the single-cluster path.

Per cluster c the batch finds mu_c with g Tr[P_c S_c] = N_e,c (eq. Ne) from
exact moments, then forms every column of P_c = p_N(S_c^-1 F_c) S_c^-1."""
import sys
import time

import numpy as np
import pytest

import oracle as O
import paper_2108_13478_amd as dmlib
from synth import batch_cluster_sizes, make_batch

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_batch(ctx, clusters, N, beta, tol, flags=0):
    P = [np.zeros(c.K * c.K) for c in clusters]
    mu = ctx.dm_batch_run(N, beta, [c.n_electrons for c in clusters], tol=tol, P_out=P, flags=flags)
    return mu, [p.reshape(c.K, c.K).T for p, c in zip(P, clusters)]


@pytest.mark.parametrize("form", [dmlib.DM_FORM_GENERAL, dmlib.DM_FORM_SYMMETRIC])
def test_fp64_batch_matches_oracle(form):
    sizes = batch_cluster_sizes(6, lo=25, hi=150, seed=3)  # K = 100 .. 600
    clusters = make_batch(sizes, range(100, 106), processes=1)
    say(f"case: FP64 batch K = {[c.K for c in clusters]}, operator form {form}")
    ctx = dmlib.Context(precision=dmlib.DM_FP64)
    ctx.dm_set_operator_form(form)
    ctx.dm_batch_set_focks(clusters)
    N, beta = 200, 20.0
    mu, P = run_batch(ctx, clusters, N, beta, tol=1e-9)
    for i, c in enumerate(clusters):
        sp = O.spectrum(c)
        lo, hi = ctx.dm_batch_get_bounds(i)
        assert lo <= sp.e[0] and hi >= sp.e[-1]
        tr = O.trace_poly(sp, N, mu[i], beta, lo, hi)[0]
        ref = O.density_matrix_poly(sp, np.arange(c.K), N, mu[i], beta, lo, hi)
        err = np.abs(P[i] - ref).max()
        say(f"  cluster {i} K={c.K}: mu={mu[i]:.9f} 2Tr-N_e={2 * tr - c.n_electrons:.2e} max|dP|={err:.2e}")
        assert abs(2.0 * tr - c.n_electrons) < 1e-7
        assert err <= 1e-9


@pytest.mark.parametrize("mom_prec", [-1, dmlib.DM_FP64])
def test_graph_replays_match_eager_run(mom_prec):
    import torch

    sizes = batch_cluster_sizes(5, lo=40, hi=200, seed=4)
    clusters = make_batch(sizes, range(200, 205), processes=1)
    say(f"case: graph replay K = {[c.K for c in clusters]}, moments precision {mom_prec}")
    ctx = dmlib.Context(precision=dmlib.DM_FP32)
    ctx.dm_set_moments_precision(mom_prec)
    ctx.dm_batch_set_focks(clusters)
    N, beta = 120, 30.0
    mu_e, P_e = run_batch(ctx, clusters, N, beta, tol=1e-6, flags=dmlib.DM_BATCH_EAGER)
    for rep in range(3):
        # eager work of the program between replays
        x = torch.randn(1 << 20, device="cuda")
        torch.cuda.synchronize()
        assert torch.isfinite(x.sum())
        mu_g, P_g = run_batch(ctx, clusters, N, beta, tol=1e-6)
        assert np.array_equal(mu_g, mu_e)
        for a, b in zip(P_g, P_e):
            assert np.array_equal(a, b)
        say(f"  replay {rep}: identical to the eager run")


def test_batch64_fp32_full_configuration():
    """64 clusters, K uniform in [500, 4000], beta 100, order 400, FP32
    recursion with FP64 P and moments, tile shape from the batch autotuner."""
    import torch

    sizes = batch_cluster_sizes()
    t0 = time.perf_counter()
    clusters = make_batch(sizes, range(64))
    Ks = np.array([c.K for c in clusters])
    say(f"case: batch of 64, K in [{Ks.min()}, {Ks.max()}], sum K = {Ks.sum()}, inputs {time.perf_counter() - t0:.1f} s")
    ctx = dmlib.Context(precision=dmlib.DM_FP32)
    t0 = time.perf_counter()
    ctx.dm_batch_set_focks(clusters)
    say(f"  setup of 64 operators {time.perf_counter() - t0:.1f} s")
    best, table = ctx.dm_batch_autotune(steps=8)
    for row in table:
        say(f"  tune tile {int(row[1])}x{int(row[2])}: {row[3]:.2f} ms for 8 steps")
    say(f"  chosen cfg {best}")
    N, beta = 400, 100.0
    ne = [c.n_electrons for c in clusters]
    P = [torch.empty(c.K * c.K, dtype=torch.float64, device="cuda") for c in clusters]
    mu = ctx.dm_batch_run(N, beta, ne, tol=1e-6, P_out=P)  # captures the graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mu2 = ctx.dm_batch_run(N, beta, ne, tol=1e-6, P_out=P)  # replay
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    say(f"  replay: {dt:.2f} s for {Ks.sum()} columns (two passes) = {Ks.sum() / dt:.0f} columns/s")
    assert np.array_equal(mu, mu2)
    # the single-cluster path at the same mu, on the batch's tile shape (same
    # summation order), gives the same P
    j = int(np.argmax(Ks))
    c = clusters[j]
    one = dmlib.Context(precision=dmlib.DM_FP32)
    one.set_cluster(c)
    one.dm_set_pass_shape(c.K, best)
    assert one.dm_get_bounds() == ctx.dm_batch_get_bounds(j)
    P1 = np.zeros((c.K, c.K))
    one.dm_chebyshev_block(np.arange(c.K, dtype=np.int64), N, mu[j], beta, P1)
    Pb = P[j].cpu().numpy().reshape(c.K, c.K)
    d = np.abs(P1 - Pb).max()
    say(f"  largest cluster K={c.K}: batch vs single-cluster path max|dP| = {d:.3e}")
    assert d <= 1e-12 * np.abs(P1).max()
    # sampled clusters against the oracle: the FP32 recursion error is
    # measured (about 1e-5 of max|P|); mu from FP32 moments misses the
    # electron count by hundredths of an electron (FP32 rounding of H_N)
    sample = sorted({int(np.argmin(Ks)), j, 10, 40})
    spectra = {i: O.spectrum(clusters[i]) for i in sample}
    for i in sample:
        c, sp = clusters[i], spectra[i]
        lo, hi = ctx.dm_batch_get_bounds(i)
        ref = O.density_matrix_poly(sp, np.arange(c.K), N, mu[i], beta, lo, hi)
        Pi = P[i].cpu().numpy().reshape(c.K, c.K).T
        err = np.abs(Pi - ref).max()
        ne_err = 2.0 * O.trace_poly(sp, N, mu[i], beta, lo, hi)[0] - c.n_electrons
        say(f"  cluster {i} K={c.K}: FP32 max|dP| = {err:.2e} (max|P| {np.abs(ref).max():.1f}), "
            f"oracle 2Tr - N_e at mu = {ne_err:.2e}")
        assert err < 3e-5 * np.abs(ref).max()
        assert abs(ne_err) < 0.2
    # the same batch with the moments pass in FP64 (dm_set_moments_precision):
    # each mu now reproduces N_e in the oracle's trace to 1e-6
    m64 = dmlib.Context(precision=dmlib.DM_FP32)
    m64.dm_set_moments_precision(dmlib.DM_FP64)
    t0 = time.perf_counter()
    m64.dm_batch_set_focks(clusters)
    say(f"  FP64-moments batch: setup {time.perf_counter() - t0:.1f} s")
    best64, _ = m64.dm_batch_autotune(steps=8)
    say(f"  FP64-moments batch: chosen cfg {best64}")
    tol = 5e-7
    mu64 = m64.dm_batch_run(N, beta, ne, tol=tol, P_out=P)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mu64b = m64.dm_batch_run(N, beta, ne, tol=tol, P_out=P)
    torch.cuda.synchronize()
    dt64 = time.perf_counter() - t0
    assert np.array_equal(mu64, mu64b)
    say(f"  FP64-moments replay: {dt64:.2f} s ({Ks.sum() / dt64:.0f} columns/s; FP32 moments {dt:.2f} s)")
    for i in sample:
        c, sp = clusters[i], spectra[i]
        lo, hi = m64.dm_batch_get_bounds(i)
        ref = O.density_matrix_poly(sp, np.arange(c.K), N, mu64[i], beta, lo, hi)
        Pi = P[i].cpu().numpy().reshape(c.K, c.K).T
        err = np.abs(Pi - ref).max()
        ne_err = 2.0 * O.trace_poly(sp, N, mu64[i], beta, lo, hi)[0] - c.n_electrons
        say(f"  cluster {i} K={c.K}: mu {mu64[i]:.9f} (FP32 moments {mu[i]:.9f}), FP32 max|dP| = {err:.2e}, "
            f"oracle 2Tr - N_e at mu = {ne_err:.2e}")
        assert abs(ne_err) <= 1e-6
        assert err < 3e-5 * np.abs(ref).max()


def test_batch_refuses_other_precision():
    """The batch keeps only H_N, so after a precision switch its calls refuse
    to run (instead of reading H_N in the wrong format) until switched back."""
    clusters = make_batch(batch_cluster_sizes(2, lo=30, hi=60, seed=6), [300, 301], processes=1)
    ctx = dmlib.Context(precision=dmlib.DM_FP32)
    ctx.dm_batch_set_focks(clusters)
    ne = [c.n_electrons for c in clusters]
    ctx.dm_batch_run(50, 10.0, ne, tol=1e-4, flags=dmlib.DM_BATCH_MOMENTS_ONLY)
    ctx.dm_set_precision(dmlib.DM_FP64)
    with pytest.raises(dmlib.DMError):
        ctx.dm_batch_run(50, 10.0, ne, tol=1e-4, flags=dmlib.DM_BATCH_MOMENTS_ONLY)
    with pytest.raises(dmlib.DMError):
        ctx.dm_batch_autotune(steps=4)
    ctx.dm_set_precision(dmlib.DM_FP32)
    ctx.dm_batch_run(50, 10.0, ne, tol=1e-4, flags=dmlib.DM_BATCH_MOMENTS_ONLY)


def test_gang_barrier_give_up_is_reported(monkeypatch):
    """The step barrier of a gang gives up after a bounded number of polls
    and the run reports DM_E_STATE instead of waiting forever or returning
    silently.  Forced from the host: with DM_BATCH_BARRIER_POLLS = 0 a member
    that arrives before the others gives up at once, the launch drains, and
    the context runs normally again once the limit is back to its default."""
    clusters = make_batch([640, 60], [400, 401], processes=1)  # K = 2560 (shared by a gang), 240
    say(f"case: barrier give-up, K = {[c.K for c in clusters]}")
    ne = [c.n_electrons for c in clusters]
    ref = dmlib.Context(precision=dmlib.DM_FP32)
    ref.dm_batch_set_focks(clusters)
    mu_ref = ref.dm_batch_run(60, 10.0, ne, tol=1e-4, flags=dmlib.DM_BATCH_EAGER | dmlib.DM_BATCH_MOMENTS_ONLY)
    ctx = dmlib.Context(precision=dmlib.DM_FP32)
    ctx.dm_batch_set_focks(clusters)
    monkeypatch.setenv("DM_BATCH_BARRIER_POLLS", "0")
    with pytest.raises(dmlib.DMError) as ei:
        ctx.dm_batch_run(60, 10.0, ne, tol=1e-4, flags=dmlib.DM_BATCH_EAGER | dmlib.DM_BATCH_MOMENTS_ONLY)
    say(f"  with no patience: {ei.value}")
    assert ei.value.status == dmlib.DM_E_STATE and "gang" in str(ei.value)
    monkeypatch.delenv("DM_BATCH_BARRIER_POLLS")
    mu = ctx.dm_batch_run(60, 10.0, ne, tol=1e-4, flags=dmlib.DM_BATCH_EAGER | dmlib.DM_BATCH_MOMENTS_ONLY)
    say(f"  default patience again: mu {mu} (fresh context {mu_ref})")
    assert np.array_equal(mu, mu_ref)
