"""Orthonormal basis (S = I): P = f_FD(F) (eq. RDM with S = I) from F in CSR.

Parity against the oracle's same polynomial on the spectrum of F, the
closed-form density matrix of a tight-binding chain, and the operator at the
share shape of the largest workload (K = 131072, 8192 columns, FP32), which
the overlap setup cannot hold in one GPU: there the checks are FP32 against
FP64 on sampled columns, symmetry of the sampled block and m_0 = #columns,
plus the measured time per recursion step."""
import sys
import time

import numpy as np
import pytest

import oracle as O
import paper_2108_13478_amd as dmlib
from synth import WORKLOADS, make_cluster, rademacher, workload

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-9


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def orth_ctx(c, precision=dmlib.DM_FP64):
    ctx = dmlib.Context(precision=precision)
    ctx.set_orthonormal(c.K, c.F_rowptr, c.F_col, c.F_val)
    return ctx


def test_orthonormal_k256_against_oracle():
    c = make_cluster(64, seed=0, geometry="cube")
    sp = O.Spectrum(c.F_dense(), np.eye(c.K))
    say(f"case: orthonormal K={c.K}, spectrum of F [{sp.e[0]:.3f}, {sp.e[-1]:.3f}]")
    ctx = orth_ctx(c)
    lo, hi = ctx.dm_get_bounds()
    assert lo <= sp.e[0] and hi >= sp.e[-1]
    w = sp.e[-1] - sp.e[0]
    emin, emax = sp.e[0] - 0.01 * w, sp.e[-1] + 0.01 * w
    ctx.dm_set_bounds(emin, emax)
    N, beta = 300, 2.0
    mu = 0.5 * (sp.e[127] + sp.e[128])
    cols = np.arange(c.K, dtype=np.int64)
    P = np.zeros((c.K, c.K))
    ctx.dm_chebyshev_block(cols, N, mu, beta, P)
    ref = O.density_matrix_poly(sp, cols, N, mu, beta, emin, emax)
    err = np.abs(P.T - ref).max()
    m, _ = ctx.dm_moments(N + 1)
    dm = np.abs(m - O.moments_from_eigs(sp.e, N + 1, emin, emax)).max()
    say(f"  FP64 max|dP| = {err:.3e}, max|dm| = {dm:.2e}")
    assert err <= TOL_FP64 and dm < 1e-8 * c.K
    xi = rademacher(c.K, 8, 1)
    ms = ctx.dm_stoch_moments(32, xi)
    assert np.abs(ms - O.stochastic_moments(sp, xi, 32, emin, emax)).max() < 1e-9 * c.K
    with pytest.raises(dmlib.DMError):
        ctx.dm_get_operator(dmlib.DM_OP_SINV)
    ctx.dm_set_precision(dmlib.DM_FP32)
    ctx.dm_set_bounds(emin, emax)
    ctx.dm_chebyshev_block(cols, N, mu, beta, P)
    say(f"  FP32 max|dP| = {np.abs(P.T - ref).max():.3e} (max|P| {np.abs(ref).max():.2f})")
    assert np.abs(P.T - ref).max() < 1e-5


def test_tight_binding_chain_closed_form():
    """F tridiagonal with -t off the diagonal: eigenvalues -2t cos(pi k/(n+1)),
    eigenvectors sqrt(2/(n+1)) sin(pi i k/(n+1)); P = V f(e) V^T exactly."""
    n, t, mu, beta = 500, 1.0, 0.3, 4.0
    rp = np.zeros(n + 1, dtype=np.int64)
    col, val = [], []
    for i in range(n):
        for j in (i - 1, i + 1):
            if 0 <= j < n:
                col.append(j)
                val.append(-t)
        rp[i + 1] = len(col)
    ctx = dmlib.Context()
    ctx.set_orthonormal(n, rp, np.array(col, dtype=np.int32), np.array(val))
    ctx.dm_set_bounds(-2.05 * t, 2.05 * t)
    k = np.arange(1, n + 1)
    e = -2 * t * np.cos(np.pi * k / (n + 1))
    V = np.sqrt(2.0 / (n + 1)) * np.sin(np.pi * np.outer(np.arange(1, n + 1), k) / (n + 1))
    exact = (V * O.fermi(e, mu, beta)) @ V.T
    cols = np.array([0, 1, 100, 250, 499], dtype=np.int64)
    P = np.zeros((len(cols), n))
    ctx.dm_chebyshev_block(cols, 200, mu, beta, P)
    err = np.abs(P.T - exact[:, cols]).max()
    say(f"case: tight-binding chain n={n}: max|P - P_exact| = {err:.2e}")
    assert err < 1e-10


def test_share_shape_k131072_fp32():
    w = WORKLOADS["K131072_sphere32768_share8192_fp32"]
    t0 = time.perf_counter()
    c = workload("K131072_sphere32768_share8192_fp32")
    say(f"case: K={c.K} orthonormal operator from the 32768-atom sphere's F "
        f"(nnz/row {c.nnz_per_row[0]:.0f}), inputs {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    ctx = orth_ctx(c, dmlib.DM_FP64)
    lo, hi = ctx.dm_get_bounds()
    say(f"  setup (FP64 H_N {8 * c.K ** 2 / 1e9:.0f} GB) {time.perf_counter() - t0:.1f} s, bounds [{lo:.1f}, {hi:.1f}]")
    rng = np.random.default_rng(3)
    cols = np.sort(rng.choice(c.K, 64, replace=False)).astype(np.int64)
    N, beta = 100, w["beta"]
    mu = 0.5 * (lo + hi)
    P64 = np.zeros((64, c.K))
    ctx.dm_chebyshev_block(cols, N, mu, beta, P64)
    ctx.dm_set_precision(dmlib.DM_FP32)
    P32 = np.zeros((64, c.K))
    ctx.dm_chebyshev_block(cols, N, mu, beta, P32)
    m, nd = ctx.dm_moments(1)
    blk = P64[:, cols]
    d = np.abs(P32 - P64).max()
    say(f"  64 sampled columns, N={N}: FP32 vs FP64 max|dP| = {d:.2e} (max|P| {np.abs(P64).max():.3f}), "
        f"FP64 block asymmetry {np.abs(blk - blk.T).max():.2e}, m0 = {m[0]:.9f}")
    assert d < 1e-4 * max(1.0, np.abs(P64).max())
    assert np.abs(blk - blk.T).max() < 1e-10 * max(1.0, np.abs(blk).max())
    assert abs(m[0] - 64) < 1e-6
    # one GPU's share: 8192 columns, FP32, timed recursion steps
    import torch

    share = torch.arange(8192, dtype=torch.int64, device="cuda")
    ctx.dm_reset_moments()
    steps = 4
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.dm_chebyshev_block(share, steps, mu, beta, None)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tf = 2.0 * c.K ** 2 * 8192 * steps / dt / 1e12
    say(f"  share of 8192 columns: {steps} steps in {dt:.2f} s = {dt / steps * 1e3:.0f} ms/step "
        f"(start block included), {tf:.1f} TFLOP/s")
    m, nd = ctx.dm_moments(1)
    assert nd == 8192 and abs(m[0] - 8192) < 1e-6
