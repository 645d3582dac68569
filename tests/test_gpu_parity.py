"""HIP path against the FP64 oracle, through the C ABI.

The oracle evaluates the same truncated Chebyshev polynomial P_N =
C diag(p_N(x)) C^T (supplement "Chebyshev expansion", eq. RDM) on the same
spectral interval; the FP64 recursion must match it within max|dP| <= 1e-9.
Intervals are pinned with dm_set_bounds to the oracle's exact extreme
eigenvalues widened by 1% on each side, so parity does not depend on the
Lanczos estimate (which has its own enclosure test)."""
import sys

import numpy as np
import pytest

import oracle as O
import paper_2108_13478_amd as dmlib
from synth import make_cluster, rademacher

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-9


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def widened(sp, frac=0.01):
    w = sp.e[-1] - sp.e[0]
    return sp.e[0] - frac * w, sp.e[-1] + frac * w


def run_cols(ctx, K, cols, order, mu, beta):
    P = np.zeros((len(cols), K), dtype=np.float64)  # row j = column j of P
    ctx.dm_chebyshev_block(np.asarray(cols, dtype=np.int64), order, mu, beta, P)
    return P.T


def midgap_mu(sp, nocc):
    return 0.5 * (sp.e[nocc - 1] + sp.e[nocc])


@pytest.fixture(scope="module")
def c1():
    c = make_cluster(64, seed=0, geometry="cube")
    return c, O.spectrum(c)


def test_setup_operators_match_dense_algebra(c1):
    c, sp = c1
    say("case: setup operators K=256")
    ctx = dmlib.Context()
    ctx.set_cluster(c)
    S, F = c.S_dense(), c.F_dense()
    Sinv_ref = np.linalg.inv(S)
    Sinv = ctx.dm_get_operator(dmlib.DM_OP_SINV)
    H = ctx.dm_get_operator(dmlib.DM_OP_H)
    e1 = np.abs(Sinv - Sinv_ref).max() / np.abs(Sinv_ref).max()
    e2 = np.abs(H - Sinv_ref @ F).max() / np.abs(H).max()
    say(f"  rel err S^-1 {e1:.3e}  H {e2:.3e}")
    assert e1 < 1e-10 and e2 < 1e-10


def test_lanczos_bounds_enclose_spectrum(c1):
    c, sp = c1
    say("case: Lanczos bounds K=256")
    ctx = dmlib.Context()
    ctx.set_cluster(c)
    lo, hi = ctx.dm_get_bounds()
    w = sp.e[-1] - sp.e[0]
    say(f"  gpu [{lo:.6f}, {hi:.6f}]  exact [{sp.e[0]:.6f}, {sp.e[-1]:.6f}]")
    assert lo <= sp.e[0] and hi >= sp.e[-1]
    assert sp.e[0] - lo < 0.05 * w and hi - sp.e[-1] < 0.05 * w


def test_c1_fp64_full_density_matrix(c1):
    """K=256 cube, beta=100, order 400, all 256 columns in one block."""
    c, sp = c1
    say("case: K=256 FP64 N=400 all columns")
    emin, emax = widened(sp)
    mu, beta, N = midgap_mu(sp, 64), 100.0, 400
    ctx = dmlib.Context()
    ctx.set_cluster(c)
    ctx.dm_set_bounds(emin, emax)
    P = run_cols(ctx, c.K, np.arange(c.K), N, mu, beta)
    ref = O.density_matrix_poly(sp, np.arange(c.K), N, mu, beta, emin, emax)
    err = np.abs(P - ref).max()
    say(f"  max|dP| = {err:.3e}  (max|P| = {np.abs(ref).max():.3e})")
    assert err <= TOL_FP64
    # moments m_l = Tr T_l(H_N) once every column has been processed
    m, nd = ctx.dm_moments(N + 1)
    assert nd == c.K
    mref = O.moments_from_eigs(sp.e, N + 1, emin, emax)
    say(f"  max|dm| = {np.abs(m - mref).max():.3e}")
    assert abs(m[0] - c.K) < 1e-9
    assert np.abs(m - mref).max() < 1e-8 * c.K
    tr, eb = ctx.dm_trace(mu, beta)
    tr_ref, eb_ref = O.trace_poly(sp, N, mu, beta, emin, emax, spin=2.0)
    say(f"  Tr[PS] {tr:.12f} vs {tr_ref:.12f}; E_band {eb:.10f} vs {eb_ref:.10f}")
    assert abs(tr - tr_ref) < 1e-8 and abs(eb - eb_ref) < 1e-7
    # chemical potential for N_e = 128 (g = 2) from the same moments
    mu_g = ctx.dm_solve_mu(128.0, beta, tol=1e-9)
    tr_at = O.trace_poly(sp, N, mu_g, beta, emin, emax)[0]
    say(f"  mu {mu_g:.12f}: oracle 2 Tr = {2 * tr_at:.12f}")
    assert abs(2.0 * tr_at - 128.0) < 1e-7


def test_ragged_shapes_and_column_subsets():
    """K = 148 (not a tile multiple), unsorted columns, one column, N = 2."""
    c = make_cluster(37, seed=4, geometry="sphere")
    sp = O.spectrum(c)
    say(f"case: ragged K={c.K}")
    emin, emax = widened(sp)
    ctx = dmlib.Context()
    ctx.set_cluster(c)
    ctx.dm_set_bounds(emin, emax)
    for cols, N in (([5, 0, 147, 77], 50), ([31], 7), (list(range(0, 148, 3)), 2)):
        P = run_cols(ctx, c.K, cols, N, 0.2, 20.0)
        ref = O.density_matrix_poly(sp, cols, N, 0.2, 20.0, emin, emax)
        err = np.abs(P - ref).max()
        say(f"  cols={len(cols)} N={N} max|dP|={err:.3e}")
        assert err <= TOL_FP64


def test_moment_accumulation_over_column_shares(c1):
    """Columns split into 4 disjoint shares, run one after another, give the
    moments of one pass over all columns (the multi-GPU sharding, simulated)."""
    c, sp = c1
    say("case: moment shares K=256")
    emin, emax = widened(sp)
    ctx = dmlib.Context()
    ctx.set_cluster(c)
    ctx.dm_set_bounds(emin, emax)
    N = 120
    perm = np.random.default_rng(0).permutation(c.K)
    for share in np.array_split(perm, 4):
        ctx.dm_chebyshev_block(share.astype(np.int64), N, 0.3, 50.0, None)
    m, nd = ctx.dm_moments(N + 1)
    assert nd == c.K
    mref = O.moments_from_eigs(sp.e, N + 1, emin, emax)
    assert np.abs(m - mref).max() < 1e-8 * c.K


def test_fp32_recursion_error_is_reported(c1):
    c, sp = c1
    say("case: K=256 FP32 recursion")
    emin, emax = widened(sp)
    mu, beta, N = midgap_mu(sp, 64), 100.0, 400
    ctx = dmlib.Context(precision=dmlib.DM_FP32)
    ctx.set_cluster(c)
    ctx.dm_set_bounds(emin, emax)
    P = run_cols(ctx, c.K, np.arange(c.K), N, mu, beta)
    ref = O.density_matrix_poly(sp, np.arange(c.K), N, mu, beta, emin, emax)
    err = np.abs(P - ref).max()
    say(f"  FP32 recursion: max|dP| = {err:.3e} vs FP64 oracle (max|P| = {np.abs(ref).max():.1f})")
    # measured 6.0e-4
    assert err < 1.5e-3


def test_stochastic_moments(c1):
    c, sp = c1
    say("case: stochastic moments K=256")
    emin, emax = widened(sp)
    ctx = dmlib.Context()
    ctx.set_cluster(c)
    ctx.dm_set_bounds(emin, emax)
    xi = rademacher(c.K, 16, seed=7)
    m = ctx.dm_stoch_moments(64, xi)
    ref = O.stochastic_moments(sp, xi, 64, emin, emax)
    say(f"  max|dm~| = {np.abs(m - ref).max():.3e}")
    assert np.abs(m - ref).max() < 1e-9 * c.K


def test_error_paths():
    say("case: error paths")
    ctx = dmlib.Context()
    # a symmetric overlap with positive diagonal but a negative eigenvalue
    rp = np.array([0, 2, 4], dtype=np.int64)
    ci = np.array([0, 1, 0, 1], dtype=np.int32)
    S = np.array([1.0, 2.0, 2.0, 1.0])
    F = np.array([0.5, 0.1, 0.1, 0.3])
    with pytest.raises(dmlib.DMError) as ei:
        ctx.dm_set_fock(2, rp, ci, F, rp, ci, S)
    assert ei.value.status == dmlib.DM_E_NOTSPD
    c = make_cluster(8, seed=1, geometry="cube")
    ctx.set_cluster(c)
    with pytest.raises(dmlib.DMError) as ei:
        ctx.dm_chebyshev_block(np.array([0, 0], dtype=np.int64), 10, 0.0, 1.0, None)
    assert ei.value.status == dmlib.DM_E_ARG
    with pytest.raises(dmlib.DMError) as ei:
        ctx.dm_chebyshev_block(np.array([c.K], dtype=np.int64), 10, 0.0, 1.0, None)
    assert ei.value.status == dmlib.DM_E_ARG
    bad = c.F_val.copy()
    bad[3] = np.nan
    with pytest.raises(dmlib.DMError) as ei:
        ctx.dm_set_fock(c.K, c.F_rowptr, c.F_col, bad, c.S_rowptr, c.S_col, c.S_val)
    assert ei.value.status == dmlib.DM_E_ARG
    # an interval that misses most of the spectrum makes T_l grow without bound
    ctx.set_cluster(c)
    lo, hi = ctx.dm_get_bounds()
    ctx.dm_set_bounds(lo + 0.45 * (hi - lo), hi - 0.45 * (hi - lo))
    with pytest.raises(dmlib.DMError) as ei:
        ctx.dm_chebyshev_block(np.arange(c.K, dtype=np.int64), 400, 0.0, 1.0, None)
    assert ei.value.status == dmlib.DM_E_BOUNDS


def test_refined_precision_against_oracle(c1):
    """DM_FP32_ACC64 at K = 256 (all columns, N = 400): FP32 storage with FP64
    products and sums, between the FP32 and FP64 paths in accuracy."""
    c, sp = c1
    emin, emax = widened(sp)
    mu, beta, N = midgap_mu(sp, 64), 100.0, 400
    ref = O.density_matrix_poly(sp, np.arange(c.K), N, mu, beta, emin, emax)
    errs = {}
    for prec in (dmlib.DM_FP32, dmlib.DM_FP32_ACC64):
        ctx = dmlib.Context(precision=prec)
        ctx.set_cluster(c)
        ctx.dm_set_bounds(emin, emax)
        errs[prec] = np.abs(run_cols(ctx, c.K, np.arange(c.K), N, mu, beta) - ref).max()
        m, _ = ctx.dm_moments(N + 1)
        # m_0 = sum_a s_a^T U_0 with U_0 = S^-1 u_a rounded to FP32
        assert abs(m[0] - c.K) < 1e-6 * c.K
    say(f"case: K=256 refined precision: max|dP| {errs[dmlib.DM_FP32_ACC64]:.3e} "
        f"(plain FP32 {errs[dmlib.DM_FP32]:.3e}, max|P| {np.abs(ref).max():.1f})")
    # measured 2.5e-5 against 6.0e-4
    assert errs[dmlib.DM_FP32_ACC64] < 6e-5 and errs[dmlib.DM_FP32_ACC64] < 0.25 * errs[dmlib.DM_FP32]
    with pytest.raises(dmlib.DMError):
        b = dmlib.Context(precision=dmlib.DM_FP32_ACC64)
        b.dm_batch_set_focks([c])
