"""Several (mu, beta) coefficient sets in one recursion pass, and the density
of states from the accumulated moments, against the FP64 oracle.

The supplement's coefficients a_l(T, mu) depend on temperature and chemical
potential while the recursion vectors T_l(H_N) S^-1 u_a do not, so one pass
can accumulate P for several (mu, beta); each block must equal the
single-set pass bit for bit.  The DOS follows the broadened form of the
paper's DOS comparison figure (g sum_n G_sigma(E - e_n)) truncated to the
pass's N terms, and the Jackson-kernel KPM form; both are compared with the
oracle's same-truncation values from the eigenvalues.  (The figure's
sigma = 0.01 hartree would need N ~ 1e5 terms on these spectra, which span
hundreds of hartree; the tests use sigma above the order-N resolution.)"""
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
def c1():
    c = make_cluster(64, seed=0, geometry="cube")
    sp = O.spectrum(c)
    w = sp.e[-1] - sp.e[0]
    return c, sp, (sp.e[0] - 0.01 * w, sp.e[-1] + 0.01 * w)


def test_multi_sets_match_oracle_and_single_passes(c1):
    c, sp, (emin, emax) = c1
    mu0 = 0.5 * (sp.e[63] + sp.e[64])
    sets = [(mu0, 100.0), (mu0 + 0.2, 50.0), (mu0 - 0.3, 200.0)]
    N = 400
    say(f"case: K={c.K} FP64 N={N}, {len(sets)} coefficient sets in one pass")
    ctx = dmlib.Context(precision=dmlib.DM_FP64)
    ctx.set_cluster(c)
    ctx.dm_set_bounds(emin, emax)
    cols = np.arange(c.K, dtype=np.int64)
    Ps = [np.zeros((c.K, c.K)) for _ in sets]
    ctx.dm_chebyshev_block_multi(cols, N, [m for m, _ in sets], [b for _, b in sets], Ps)
    m_multi, _ = ctx.dm_moments(N + 1)
    for q, (mu, beta) in enumerate(sets):
        ref = O.density_matrix_poly(sp, cols, N, mu, beta, emin, emax)
        err = np.abs(Ps[q].T - ref).max()
        ctx.dm_reset_moments()
        P1 = np.zeros((c.K, c.K))
        ctx.dm_chebyshev_block(cols, N, mu, beta, P1)
        m1, _ = ctx.dm_moments(N + 1)
        say(f"  set {q} mu={mu:.4f} beta={beta:g}: max|dP| vs oracle {err:.3e}, "
            f"identical to single pass: {np.array_equal(P1, Ps[q])}")
        assert err <= TOL_FP64
        assert np.array_equal(P1, Ps[q])
        assert np.array_equal(m1, m_multi)
    # NULL entries: moments only for those sets
    ctx.dm_reset_moments()
    ctx.dm_chebyshev_block_multi(cols[:40], N, [mu0, mu0], [100.0, 80.0], [None, None])
    assert ctx.dm_moments(2)[1] == 40


def test_multi_sets_on_split_and_panel_shapes_fp32():
    """FP32, ragged column sets, on a split-reduction and an LDS-panel shape."""
    c = make_cluster(256, seed=2, geometry="sphere")
    sp = O.spectrum(c)
    w = sp.e[-1] - sp.e[0]
    emin, emax = sp.e[0] - 0.01 * w, sp.e[-1] + 0.01 * w
    mu0 = 0.5 * (sp.e[255] + sp.e[256])
    cols = np.random.default_rng(8).permutation(c.K)[:100]
    ctx = dmlib.Context(precision=dmlib.DM_FP32)
    ctx.set_cluster(c)
    ctx.dm_set_bounds(emin, emax)
    shapes = dmlib.tile_shapes()
    split = [i for i, s in enumerate(shapes) if s[2] > 1][0]
    for cfg in (split, 2):
        ctx.dm_set_pass_shape(64, cfg)
        Ps = [np.zeros((len(cols), c.K)) for _ in range(2)]
        ctx.dm_chebyshev_block_multi(cols, 300, [mu0, mu0 + 0.1], [30.0, 60.0], Ps)
        for q, (mu, beta) in enumerate([(mu0, 30.0), (mu0 + 0.1, 60.0)]):
            ctx.dm_reset_moments()
            P1 = np.zeros((len(cols), c.K))
            ctx.dm_chebyshev_block(cols, 300, mu, beta, P1)
            ref = O.density_matrix_poly(sp, cols, 300, mu, beta, emin, emax)
            say(f"case: FP32 shape {cfg} set {q}: identical to single pass {np.array_equal(P1, Ps[q])}, "
                f"max|dP| vs oracle {np.abs(Ps[q].T - ref).max():.2e}")
            assert np.array_equal(P1, Ps[q])
            assert np.abs(Ps[q].T - ref).max() < 1e-5 * np.abs(ref).max()
        ctx.dm_reset_moments()


def test_dos_gaussian_and_kpm_match_oracle(c1):
    c, sp, (emin, emax) = c1
    N = 400
    say(f"case: DOS K={c.K} N={N}")
    ctx = dmlib.Context(precision=dmlib.DM_FP64)
    ctx.set_cluster(c)
    ctx.dm_set_bounds(emin, emax)
    with pytest.raises(dmlib.DMError):
        ctx.dm_dos(dmlib.DM_DOS_KPM, [0.0])  # no moments yet
    ctx.dm_chebyshev_block(np.arange(c.K, dtype=np.int64), N, 0.0, 100.0, None)
    E = np.linspace(emin - 5.0, emax + 5.0, 401)
    ebar, de = O.spectral_scale(emin, emax)
    for sigma in (2.0, 0.05 * de):
        got = ctx.dm_dos(dmlib.DM_DOS_GAUSSIAN, E, sigma)
        ref = O.dos_poly(sp, E, sigma, N, emin, emax)
        exact = O.dos_exact(sp, E, sigma)
        say(f"  Gaussian sigma={sigma:.3f}: max|d| vs same-truncation oracle "
            f"{np.abs(got - ref).max() / ref.max():.2e} (rel), vs broadened DOS "
            f"{np.abs(got - exact).max() / exact.max():.2e} (rel)")
        assert np.abs(got - ref).max() <= 1e-9 * ref.max()
    got = ctx.dm_dos(dmlib.DM_DOS_KPM, E)
    ref = O.kpm_dos(sp, E, N, emin, emax)
    say(f"  KPM: max|d| vs oracle {np.abs(got - ref).max() / ref.max():.2e} (rel)")
    assert np.abs(got - ref).max() <= 1e-9 * ref.max()
    # normalisation on the GPU values: Gauss-Chebyshev quadrature of rho dE
    th = O.chebyshev_nodes(4 * N)
    r = ctx.dm_dos(dmlib.DM_DOS_KPM, ebar + de * np.cos(th))
    integral = np.sum(r * de * np.sin(th)) * np.pi / len(th)
    say(f"  KPM integral {integral:.10f} (2K = {2 * c.K})")
    assert abs(integral - 2 * c.K) < 1e-8 * c.K
    for bad in ((7, 1.0), (dmlib.DM_DOS_GAUSSIAN, 0.0), (dmlib.DM_DOS_GAUSSIAN, -1.0)):
        with pytest.raises(dmlib.DMError):
            ctx.dm_dos(bad[0], E[:3], bad[1])
    with pytest.raises(dmlib.DMError):
        ctx.dm_chebyshev_block_multi(np.arange(4), 50, [], [], None)
    with pytest.raises(dmlib.DMError):
        ctx.dm_chebyshev_block_multi(np.arange(4), 50, [0.0] * 17, [1.0] * 17, None)
