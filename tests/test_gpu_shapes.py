"""Every compiled tile shape of the recursion step, pinned with
dm_set_pass_shape, against the FP64 oracle (same truncated polynomial,
supplement "Chebyshev expansion"), including the split-reduction shapes
that cut the operator product into chunked partial products plus a combine
kernel.  Column sets are unsorted and ragged so the last pass is padded."""
import sys

import numpy as np
import pytest

import oracle as O
import paper_2108_13478_amd as dmlib
from synth import make_cluster

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-9


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def k1024():
    c = make_cluster(256, seed=2, geometry="sphere")
    sp = O.spectrum(c)
    w = sp.e[-1] - sp.e[0]
    return c, sp, (sp.e[0] - 0.01 * w, sp.e[-1] + 0.01 * w)


def pass_width(cols):
    return max(cols, 64)


def run(ctx, c, cols, N, mu, beta):
    P = np.zeros((len(cols), c.K), dtype=np.float64)
    ctx.dm_chebyshev_block(np.asarray(cols, dtype=np.int64), N, mu, beta, P)
    m, nd = ctx.dm_moments(N + 1)
    ctx.dm_reset_moments()
    return P.T, m


def test_every_shape_fp64_against_oracle(k1024):
    c, sp, (emin, emax) = k1024
    N, beta = 300, 30.0
    mu = 0.5 * (sp.e[c.K // 4 - 1] + sp.e[c.K // 4])
    cols = np.random.default_rng(3).permutation(c.K)[:100]
    ref = O.density_matrix_poly(sp, cols, N, mu, beta, emin, emax)
    ctx = dmlib.Context(precision=dmlib.DM_FP64)
    ctx.set_cluster(c)
    ctx.dm_set_bounds(emin, emax)
    shapes = dmlib.tile_shapes()
    m_first = None
    rejected = []
    for cfg, (rows, tcols, split) in enumerate(shapes):
        say(f"case: K={c.K} FP64 shape {cfg} ({rows}x{tcols}, split {split}) width {pass_width(tcols)}")
        try:
            ctx.dm_set_pass_shape(pass_width(tcols), cfg)
        except dmlib.DMError:
            rejected.append(cfg)  # register rings compiled for FP32 only
            continue
        P, m = run(ctx, c, cols, N, mu, beta)
        err = np.abs(P - ref).max()
        if m_first is None:
            m_first = m
        dm = np.abs(m - m_first).max() / np.abs(m_first).max()
        say(f"  max|dP| = {err:.3e} (max|P| {np.abs(ref).max():.1f}), moments vs shape 0: {dm:.2e}")
        assert err <= TOL_FP64
        assert dm < 1e-12
    say(f"  FP32-only shapes: {rejected}")
    assert not set(rejected) & set(range(6)) and all(shapes[c][2] == 1 for c in rejected)


def test_every_shape_fp32_error_matches_unsplit(k1024):
    c, sp, (emin, emax) = k1024
    N, beta = 300, 30.0
    mu = 0.5 * (sp.e[c.K // 4 - 1] + sp.e[c.K // 4])
    cols = np.random.default_rng(4).permutation(c.K)[:96]
    ref = O.density_matrix_poly(sp, cols, N, mu, beta, emin, emax)
    ctx = dmlib.Context(precision=dmlib.DM_FP32)
    ctx.set_cluster(c)
    ctx.dm_set_bounds(emin, emax)
    ctx.dm_set_pass_shape(64, 2)  # 128 x 32, no split
    P0, m0 = run(ctx, c, cols, N, mu, beta)
    e0 = np.abs(P0 - ref).max()
    say(f"case: K={c.K} FP32 shape 2 (128x32, no split): max|dP| vs oracle {e0:.3e}")
    rejected = []
    shapes = dmlib.tile_shapes()
    for cfg, (rows, tcols, split) in enumerate(shapes):
        try:
            ctx.dm_set_pass_shape(pass_width(tcols), cfg)
        except dmlib.DMError:
            rejected.append(cfg)  # register rings compiled for FP64 only
            continue
        P, m = run(ctx, c, cols, N, mu, beta)
        e = np.abs(P - ref).max()
        dm = np.abs(m - m0).max() / np.abs(m0).max()
        say(f"  shape {cfg} ({rows}x{tcols}, split {split}): max|dP| vs oracle {e:.3e}, moments vs shape 2 {dm:.2e}")
        assert e <= max(2.0 * e0, 1e-5 * np.abs(ref).max())
        assert dm < 1e-4
    say(f"  FP64-only shapes: {rejected}")
    assert not set(rejected) & set(range(6)) and all(shapes[c][2] == 1 for c in rejected)


def test_pass_shape_rejects_misfits(k1024):
    c, _, _ = k1024
    ctx = dmlib.Context(precision=dmlib.DM_FP64)
    ctx.set_cluster(c)
    shapes = dmlib.tile_shapes()
    split = [i for i, s in enumerate(shapes) if s[2] > 1][0]
    for width, cfg in ((0, 0), (32, len(shapes)), (1024, split), (64, 6)):
        with pytest.raises(dmlib.DMError):
            ctx.dm_set_pass_shape(width, cfg)


def test_every_shape_refined_precision(k1024):
    """DM_FP32_ACC64 (FP32 storage, FP64 products and sums) on every shape
    built for it: against the oracle, well below the plain FP32 recursion's
    error on the same columns, and the moments nearly those of FP64."""
    c, sp, (emin, emax) = k1024
    N, beta = 300, 30.0
    mu = 0.5 * (sp.e[c.K // 4 - 1] + sp.e[c.K // 4])
    cols = np.random.default_rng(4).permutation(c.K)[:96]
    ref = O.density_matrix_poly(sp, cols, N, mu, beta, emin, emax)
    f32 = dmlib.Context(precision=dmlib.DM_FP32)
    f32.set_cluster(c)
    f32.dm_set_bounds(emin, emax)
    f32.dm_set_pass_shape(64, 2)
    e32 = np.abs(run(f32, c, cols, N, mu, beta)[0] - ref).max()
    ctx = dmlib.Context(precision=dmlib.DM_FP32_ACC64)
    ctx.set_cluster(c)
    ctx.dm_set_bounds(emin, emax)
    built = []
    for cfg, (rows, tcols, split) in enumerate(dmlib.tile_shapes()):
        try:
            ctx.dm_set_pass_shape(pass_width(tcols), cfg)
        except dmlib.DMError:
            continue
        built.append(cfg)
        P, m = run(ctx, c, cols, N, mu, beta)
        e = np.abs(P - ref).max()
        say(f"case: refined shape {cfg} ({rows}x{tcols}): max|dP| {e:.3e} (plain FP32 {e32:.3e}, "
            f"max|P| {np.abs(ref).max():.1f})")
        assert e < 0.25 * e32
        assert np.all(np.isfinite(m))
    assert {0, 2, 3, 12}.issubset(built) and len(built) >= 6
