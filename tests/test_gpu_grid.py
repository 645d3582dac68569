"""Electron density on the grid from density-matrix columns (eq.
ElectronDensity) on the GPU, against the grid oracle: all columns, disjoint
column shares accumulated into one grid (the paper's reduce), the columns of
a dm_chebyshev_block pass, and the integral h^3 sum n = 2 Tr[P S]."""
import sys

import numpy as np
import pytest

import oracle as O
import paper_2108_13478_amd as dmlib
from oracle import grid_oracle as GO
from synth import basis_functions, grid_around, make_cluster

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_density_matches_oracle_and_shares_add_up():
    c = make_cluster(64, seed=0, geometry="cube")  # K = 256
    sp = O.spectrum(c)
    mu, beta = 0.5 * (sp.e[63] + sp.e[64]), 20.0
    P = O.density_matrix_exact(sp, np.arange(c.K), mu, beta)
    centres, exps = basis_functions(c)
    origin, h, dims = grid_around(c, 0.4, 5.0)
    eta = 1e-6
    say(f"case: grid density K={c.K}, grid {dims} h={h}, eta={eta}")
    ref = GO.density_on_grid(P, np.arange(c.K), centres, exps, origin, h, dims, eta)
    ctx = dmlib.Context()
    cols = np.arange(c.K, dtype=np.int64)
    n = ctx.dm_density_on_grid(centres, exps, origin, h, dims, eta, cols, np.ascontiguousarray(P.T))
    err = np.abs(n - ref).max() / np.abs(ref).max()
    say(f"  all columns: max|dn| / max|n| = {err:.2e}")
    assert err < 1e-12
    acc = np.zeros_like(n)
    for share in np.array_split(np.random.default_rng(5).permutation(c.K), 3):
        ctx.dm_density_on_grid(centres, exps, origin, h, dims, eta, share.astype(np.int64),
                               np.ascontiguousarray(P[:, share].T), acc)
    say(f"  three shares accumulated: max|dn| / max|n| = {np.abs(acc - ref).max() / np.abs(ref).max():.2e}")
    assert np.abs(acc - ref).max() < 1e-12 * np.abs(ref).max()


def test_density_lists_reused_only_for_the_same_inputs():
    """A context keeps the cell lists of its last call and reuses them while
    the basis, grid, eta and columns are the same: every call here must equal
    the same call on a fresh context, bit for bit, whatever came before."""
    c = make_cluster(64, seed=0, geometry="cube")  # K = 256
    sp = O.spectrum(c)
    P = O.density_matrix_exact(sp, np.arange(c.K), 0.5 * (sp.e[63] + sp.e[64]), 20.0)
    centres, exps = basis_functions(c)
    origin, h, dims = grid_around(c, 0.4, 5.0)
    share = np.random.default_rng(3).permutation(c.K)[:100].astype(np.int64)
    moved = centres.copy()
    moved[17] += 0.25
    calls = [  # (centres, h, eta, columns)
        (centres, h, 1e-6, np.arange(c.K, dtype=np.int64)),
        (centres, h, 1e-6, np.arange(c.K, dtype=np.int64)),
        (centres, 0.5, 1e-6, np.arange(c.K, dtype=np.int64)),
        (centres, h, 1e-4, np.arange(c.K, dtype=np.int64)),
        (centres, h, 1e-6, share),
        (moved, h, 1e-6, share),
        (centres, h, 1e-6, np.arange(c.K, dtype=np.int64)),
    ]
    say(f"case: grid lists reuse K={c.K}, {len(calls)} calls")
    ctx = dmlib.Context()
    for i, (cen, hh, eta, cols) in enumerate(calls):
        Pc = np.ascontiguousarray(P[:, cols].T)
        n = ctx.dm_density_on_grid(cen, exps, origin, hh, dims, eta, cols, Pc)
        fresh = dmlib.Context().dm_density_on_grid(cen, exps, origin, hh, dims, eta, cols, Pc)
        assert np.array_equal(n, fresh), f"call {i}"
    # after a refused call the next good call still equals a fresh one
    with pytest.raises(dmlib.DMError):
        ctx.dm_density_on_grid(centres, -exps, origin, h, dims, 1e-6, calls[0][3], np.ascontiguousarray(P.T))
    n = ctx.dm_density_on_grid(centres, exps, origin, h, dims, 1e-6, calls[0][3], np.ascontiguousarray(P.T))
    assert np.array_equal(n, dmlib.Context().dm_density_on_grid(centres, exps, origin, h, dims, 1e-6, calls[0][3],
                                                                 np.ascontiguousarray(P.T)))


def test_density_from_a_pass_integrates_to_electron_count():
    """Columns of P from dm_chebyshev_block (device buffer) on a fine grid:
    h^3 sum n = 2 Tr[P_N S] with the oracle's same-polynomial trace."""
    import torch

    c = make_cluster(8, seed=5, geometry="cube")  # K = 32
    sp = O.spectrum(c)
    w = sp.e[-1] - sp.e[0]
    emin, emax = sp.e[0] - 0.01 * w, sp.e[-1] + 0.01 * w
    mu, beta, N = 0.5 * (sp.e[7] + sp.e[8]), 10.0, 600
    ctx = dmlib.Context()
    ctx.set_cluster(c)
    ctx.dm_set_bounds(emin, emax)
    cols = torch.arange(c.K, dtype=torch.int64, device="cuda")
    Pd = torch.empty((c.K, c.K), dtype=torch.float64, device="cuda")
    ctx.dm_chebyshev_block(cols, N, mu, beta, Pd)
    centres, exps = basis_functions(c)
    origin, h, dims = grid_around(c, 0.2, 9.0)
    nd = torch.zeros(int(np.prod(dims)), dtype=torch.float64, device="cuda")
    ctx.dm_density_on_grid(centres, exps, origin, h, dims, 1e-30, cols, Pd, nd)
    total = h ** 3 * float(nd.sum())
    tr, _ = O.trace_poly(sp, N, mu, beta, emin, emax)
    say(f"case: grid {dims} h={h}: h^3 sum n = {total:.10f}, 2 Tr[P_N S] = {2 * tr:.10f}")
    assert abs(total - 2 * tr) < 1e-8 * 2 * tr
    with pytest.raises(dmlib.DMError):
        ctx.dm_density_on_grid(centres, exps, origin, -1.0, dims, 1e-6, cols, Pd, nd)
    with pytest.raises(dmlib.DMError):
        ctx.dm_density_on_grid(centres, exps, origin, h, dims, 2.0, cols, Pd, nd)
    bad = centres.copy()
    bad[3, 1] = np.nan
    with pytest.raises(dmlib.DMError) as ei:
        ctx.dm_density_on_grid(bad, exps, origin, h, dims, 1e-6, cols, Pd, nd)
    assert ei.value.status == dmlib.DM_E_ARG


def test_density_k4096_from_full_pass_timed():
    """The benchmark cluster (K = 4096): P from a full FP64 pass at the
    electron-count mu, density of all columns on a 0.2-bohr grid; the
    integral against 2 Tr[P_N S] from the moments, and the kernel time."""
    import time

    import torch

    from synth import WORKLOADS, workload

    w = WORKLOADS["K4096_sphere1024_fp64"]
    c = workload("K4096_sphere1024_fp64")
    ctx = dmlib.Context()
    ctx.set_cluster(c)
    N, beta = 200, 5.0
    cols = torch.arange(c.K, dtype=torch.int64, device="cuda")
    ctx.dm_chebyshev_block(cols, N, 0.0, beta, None)
    mu = ctx.dm_solve_mu(c.n_electrons, beta, tol=1e-6)
    ctx.dm_reset_moments()
    Pd = torch.empty((c.K, c.K), dtype=torch.float64, device="cuda")
    ctx.dm_chebyshev_block(cols, N, mu, beta, Pd)
    tr, _ = ctx.dm_trace(mu, beta)
    centres, exps = basis_functions(c)
    origin, h, dims = grid_around(c, 0.2, 8.0)
    nd = torch.zeros(int(np.prod(dims)), dtype=torch.float64, device="cuda")
    ctx.dm_density_on_grid(centres, exps, origin, h, dims, 1e-6, cols[:8], Pd[:8], nd)  # warm-up
    nd.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.dm_density_on_grid(centres, exps, origin, h, dims, 1e-6, cols, Pd, nd)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    total = h ** 3 * float(nd.sum())
    say(f"case: K={c.K} grid {dims} ({int(np.prod(dims)) / 1e6:.1f} M points), eta 1e-6: {dt * 1e3:.0f} ms "
        f"(call, lists and copies included); h^3 sum n = {total:.6f}, 2 Tr[P_N S] = {2 * tr:.6f}")
    assert abs(total - 2 * tr) < 1e-4 * 2 * tr
    # the same basis, grid and columns again (a new P in an SCF loop): the
    # call reuses the cell lists of the last one
    nd2 = torch.zeros_like(nd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.dm_density_on_grid(centres, exps, origin, h, dims, 1e-6, cols, Pd, nd2)
    torch.cuda.synchronize()
    say(f"  same inputs again (lists reused): {(time.perf_counter() - t0) * 1e3:.1f} ms")
    assert torch.equal(nd, nd2)
    # sampled points against the grid oracle, each computed on its own
    # (a one-point grid at that point) from the same P: 48 anywhere on the
    # grid, 48 in the central third where the most functions overlap
    nh = nd.cpu().numpy()
    Pc = Pd.cpu().numpy().T  # column j is column j of P
    rng = np.random.default_rng(11)
    lo = [d // 3 for d in dims]
    idx = np.concatenate([rng.integers(0, dims, size=(48, 3)),
                          rng.integers(lo, [2 * d // 3 for d in dims], size=(48, 3))])
    worst = 0.0
    for i, j, k in idx:
        pt = np.asarray(origin, dtype=np.float64) + h * np.array([i, j, k], dtype=np.float64)
        ref = GO.density_on_grid(Pc, np.arange(c.K), centres, exps, pt, h, (1, 1, 1), 1e-6)[0]
        worst = max(worst, abs(nh[i + dims[0] * (j + dims[1] * k)] - ref))
    say(f"  96 sampled points vs oracle: max|dn| = {worst:.2e} (max|n| {np.abs(nh).max():.3f})")
    assert worst < 1e-12 * np.abs(nh).max()
