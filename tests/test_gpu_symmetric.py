"""The Cholesky-orthogonalised symmetric form of the recursion against the
FP64 oracle.

With S = U^T U and L = U^-T the recursion runs on H~ = L F L^T (the same
spectrum as S^-1 F) from V_0 = L u_a, and each pass ends with P u_a =
L^T sum_l a_l V_l, the same P = f(S^-1 F) S^-1 (eq. RDM).  T_l(H~_N) is
bounded by 1 in norm, so the FP32 recursion error should fall well below the
general form's, where S^-1 F is far from normal."""
import sys

import numpy as np
import pytest
import scipy.linalg

import oracle as O
import paper_2108_13478_amd as dmlib
from synth import make_cluster, rademacher

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-9


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def c1():
    c = make_cluster(64, seed=0, geometry="cube")
    sp = O.spectrum(c)
    w = sp.e[-1] - sp.e[0]
    return c, sp, (sp.e[0] - 0.01 * w, sp.e[-1] + 0.01 * w)


def sym_ctx(c, precision, bounds):
    ctx = dmlib.Context(precision=precision)
    ctx.dm_set_operator_form(dmlib.DM_FORM_SYMMETRIC)
    ctx.set_cluster(c)
    ctx.dm_set_bounds(*bounds)
    return ctx


def test_symmetric_operator_matches_dense_algebra(c1):
    c, sp, bounds = c1
    say(f"case: symmetric operator K={c.K}")
    ctx = sym_ctx(c, dmlib.DM_FP64, bounds)
    Hs = ctx.dm_get_operator(dmlib.DM_OP_HSYM)
    U = scipy.linalg.cholesky(c.S_dense(), lower=False)
    L = np.linalg.inv(U).T
    ref = L @ c.F_dense() @ L.T
    e1 = np.abs(Hs - ref).max() / np.abs(ref).max()
    ev = np.linalg.eigvalsh(0.5 * (Hs + Hs.T))
    say(f"  rel err {e1:.2e}, asymmetry {np.abs(Hs - Hs.T).max():.2e}, eigenvalues vs eigh(F, S) "
        f"{np.abs(ev - sp.e).max():.2e}")
    assert e1 < 1e-10
    assert np.abs(ev - sp.e).max() < 1e-9 * np.abs(sp.e).max()
    gen = dmlib.Context()
    gen.set_cluster(c)
    with pytest.raises(dmlib.DMError):
        gen.dm_get_operator(dmlib.DM_OP_HSYM)


def test_symmetric_fp64_matches_oracle(c1):
    """All columns (one pass) and a ragged subset on a 32-column tile (the
    final product pads the pass to 64 columns); two coefficient sets."""
    c, sp, (emin, emax) = c1
    mu = 0.5 * (sp.e[63] + sp.e[64])
    N = 400
    ctx = sym_ctx(c, dmlib.DM_FP64, (emin, emax))
    cols = np.arange(c.K, dtype=np.int64)
    P = np.zeros((c.K, c.K))
    ctx.dm_chebyshev_block(cols, N, mu, 100.0, P)
    ref = O.density_matrix_poly(sp, cols, N, mu, 100.0, emin, emax)
    err = np.abs(P.T - ref).max()
    m, nd = ctx.dm_moments(N + 1)
    mref = O.moments_from_eigs(sp.e, N + 1, emin, emax)
    say(f"case: symmetric FP64 K={c.K} N={N}: max|dP| = {err:.3e}, max|dm| = {np.abs(m - mref).max():.2e}")
    assert err <= TOL_FP64 and nd == c.K
    assert np.abs(m - mref).max() < 1e-8 * c.K
    tr, _ = ctx.dm_trace(mu, 100.0)
    tr_ref, _ = O.trace_poly(sp, N, mu, 100.0, emin, emax)
    assert abs(tr - tr_ref) < 1e-8 * c.K
    ctx.dm_reset_moments()
    sub = np.random.default_rng(1).permutation(c.K)[:20]
    ctx.dm_set_pass_shape(32, 2)
    Ps = [np.zeros((20, c.K)) for _ in range(2)]
    ctx.dm_chebyshev_block_multi(sub, N, [mu, mu + 0.3], [100.0, 40.0], Ps)
    for q, (m_, b_) in enumerate([(mu, 100.0), (mu + 0.3, 40.0)]):
        r = O.density_matrix_poly(sp, sub, N, m_, b_, emin, emax)
        e = np.abs(Ps[q].T - r).max()
        say(f"  ragged 20 columns, set {q}: max|dP| = {e:.3e}")
        assert e <= TOL_FP64


def test_symmetric_fp32_error_below_general(c1):
    c, sp, (emin, emax) = c1
    mu = 0.5 * (sp.e[63] + sp.e[64])
    N = 400
    cols = np.arange(c.K, dtype=np.int64)
    ref = O.density_matrix_poly(sp, cols, N, mu, 100.0, emin, emax)
    errs = {}
    for name, form in (("general", dmlib.DM_FORM_GENERAL), ("symmetric", dmlib.DM_FORM_SYMMETRIC)):
        ctx = dmlib.Context(precision=dmlib.DM_FP32)
        ctx.dm_set_operator_form(form)
        ctx.set_cluster(c)
        ctx.dm_set_bounds(emin, emax)
        P = np.zeros((c.K, c.K))
        ctx.dm_chebyshev_block(cols, N, mu, 100.0, P)
        errs[name] = np.abs(P.T - ref).max()
    say(f"case: FP32 K={c.K} N={N}: max|dP| general {errs['general']:.2e}, symmetric {errs['symmetric']:.2e} "
        f"(max|P| {np.abs(ref).max():.1f})")
    assert errs["symmetric"] < 0.5 * errs["general"]


def test_symmetric_stochastic_moments(c1):
    c, sp, (emin, emax) = c1
    ctx = sym_ctx(c, dmlib.DM_FP64, (emin, emax))
    xi = rademacher(c.K, 8, 4)
    got = ctx.dm_stoch_moments(48, xi)
    ref = O.stochastic_moments_symmetric(sp, xi, 48, emin, emax)
    say(f"case: symmetric stochastic moments: max|dm~| = {np.abs(got - ref).max():.2e}")
    assert np.abs(got - ref).max() < 1e-9 * max(1.0, np.abs(ref).max())


def test_symmetric_setup_with_a_narrow_last_panel():
    """K = 1280: H~ = X^T F X is formed in column panels of 1024, so the
    last panel is 256 wide; the operator against dense algebra and P
    against the oracle on sampled columns."""
    c = make_cluster(320, seed=8, geometry="sphere", onsite="scaled")
    sp = O.spectrum(c)
    w = sp.e[-1] - sp.e[0]
    emin, emax = sp.e[0] - 0.01 * w, sp.e[-1] + 0.01 * w
    say(f"case: symmetric form K={c.K} (panels 1024 + 256)")
    ctx = sym_ctx(c, dmlib.DM_FP64, (emin, emax))
    Hs = ctx.dm_get_operator(dmlib.DM_OP_HSYM)
    U = scipy.linalg.cholesky(c.S_dense(), lower=False)
    L = np.linalg.inv(U).T
    ref = L @ c.F_dense() @ L.T
    e1 = np.abs(Hs - ref).max() / np.abs(ref).max()
    cols = np.random.default_rng(5).permutation(c.K)[:48].astype(np.int64)
    mu, N, beta = 0.5 * (sp.e[c.K // 4 - 1] + sp.e[c.K // 4]), 300, 20.0
    P = np.zeros((len(cols), c.K))
    ctx.dm_chebyshev_block(cols, N, mu, beta, P)
    err = np.abs(P.T - O.density_matrix_poly(sp, cols, N, mu, beta, emin, emax)).max()
    say(f"  H~ rel err {e1:.2e}; 48 columns N={N}: max|dP| = {err:.3e}")
    assert e1 < 1e-10 and err <= TOL_FP64
    # FP32 storage, Lanczos interval from the stored H~
    f32 = dmlib.Context(precision=dmlib.DM_FP32)
    f32.dm_set_operator_form(dmlib.DM_FORM_SYMMETRIC)
    f32.set_cluster(c)
    a, b = f32.dm_get_bounds()
    say(f"  FP32 Lanczos interval [{a:.4f}, {b:.4f}], exact [{sp.e[0]:.4f}, {sp.e[-1]:.4f}]")
    assert a <= sp.e[0] and b >= sp.e[-1]
