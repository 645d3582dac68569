"""Parity at the benchmark's full size and launch configuration.

K = 4096 (1024 atoms in a sphere), beta = 200, order N = 1000, all 4096
columns in one dm_chebyshev_block call with the default pass width, exactly
as bench.py times it.  The oracle computes every column of P_N from the
generalized eigen-decomposition (supplement "Chebyshev expansion", eq. RDM)."""
import sys

import numpy as np
import pytest

import oracle as O
import paper_2108_13478_amd as dmlib
from synth import WORKLOADS, workload

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def k4096():
    c = workload("K4096_sphere1024_fp64")
    return c, O.spectrum(c)


def test_k4096_fp64_all_columns(k4096):
    c, sp = k4096
    w = WORKLOADS["K4096_sphere1024_fp64"]
    N, beta = w["order"], w["beta"]
    say(f"case: K={c.K} FP64 N={N} beta={beta} all columns")
    ww = sp.e[-1] - sp.e[0]
    emin, emax = sp.e[0] - 0.01 * ww, sp.e[-1] + 0.01 * ww
    mu = O.solve_mu_poly(sp, w["n_electrons"], N, beta, emin, emax, tol=1e-9)
    ctx = dmlib.Context()
    ctx.set_cluster(c)
    lo, hi = ctx.dm_get_bounds()
    say(f"  Lanczos [{lo:.4f}, {hi:.4f}] exact [{sp.e[0]:.4f}, {sp.e[-1]:.4f}]")
    assert lo <= sp.e[0] and hi >= sp.e[-1]
    ctx.dm_set_bounds(emin, emax)
    P = np.zeros((c.K, c.K))
    ctx.dm_chebyshev_block(np.arange(c.K, dtype=np.int64), N, mu, beta, P)
    ref = O.density_matrix_poly(sp, np.arange(c.K), N, mu, beta, emin, emax)
    err = np.abs(P.T - ref).max()
    say(f"  max|dP| = {err:.3e} (max|P| = {np.abs(ref).max():.1f})")
    assert err <= 1e-9
    m, nd = ctx.dm_moments(N + 1)
    mref = O.moments_from_eigs(sp.e, N + 1, emin, emax)
    say(f"  max|dm| = {np.abs(m - mref).max():.3e}")
    assert nd == c.K and np.abs(m - mref).max() < 1e-8 * c.K
    tr, eb = ctx.dm_trace(mu, beta)
    tr_ref, eb_ref = O.trace_poly(sp, N, mu, beta, emin, emax)
    say(f"  2 Tr[PS] = {2 * tr:.9f} (oracle {2 * tr_ref:.9f}), E_band {eb:.6f} (oracle {eb_ref:.6f})")
    assert abs(tr - tr_ref) < 1e-7 and abs(eb - eb_ref) < 1e-5 * max(1.0, abs(eb_ref))
    mu_g = ctx.dm_solve_mu(w["n_electrons"], beta, tol=1e-8)
    assert abs(2.0 * O.trace_poly(sp, N, mu_g, beta, emin, emax)[0] - w["n_electrons"]) < 1e-6
