"""The allocation-free entry point dm_chebyshev_block_noalloc against
dm_chebyshev_block (and the oracle), through the C ABI: two calls in a row,
the second with fewer columns and a lower order, so stale contents of the
shared device array would show."""
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
    c = make_cluster(64, seed=0, geometry="cube")  # K = 256
    return c, O.spectrum(c)


def _ref_pass(ctx, K, cols, order, mu, beta):
    P = np.zeros((len(cols), K))
    ctx.dm_reset_moments()
    ctx.dm_chebyshev_block(cols, order, mu, beta, P)
    m, nd = ctx.dm_moments(order + 1)
    assert nd == len(cols)
    return P, m


@pytest.mark.parametrize("precision", [dmlib.DM_FP64, dmlib.DM_FP32])
def test_noalloc_matches_block_entry_point(c1, precision):
    import torch

    c, sp = c1
    w = sp.e[-1] - sp.e[0]
    emin, emax = sp.e[0] - 0.01 * w, sp.e[-1] + 0.01 * w
    mu, beta = 0.5 * (sp.e[63] + sp.e[64]), 100.0
    ctx = dmlib.Context(precision=precision)
    ctx.set_cluster(c)
    ctx.dm_set_bounds(emin, emax)
    cases = [(np.arange(c.K, dtype=np.int64), 400), (np.arange(3, c.K, 7, dtype=np.int64)[::-1].copy(), 150)]
    for k, (cols, order) in enumerate(cases):
        say(f"case: noalloc call {k}: K={c.K} ncols={len(cols)} order={order} precision={precision}")
        P_ref, m_ref = _ref_pass(ctx, c.K, cols, order, mu, beta)
        # host outputs
        P = np.full((len(cols), c.K), np.nan)
        m = np.full(order + 1, np.nan)
        ctx.dm_chebyshev_block_noalloc(cols, order, mu, beta, P, m)
        dP = np.abs(P - P_ref).max()
        dm = np.abs(m - m_ref).max()
        # device inputs and outputs
        Pd = torch.full((len(cols), c.K), float("nan"), dtype=torch.float64, device="cuda")
        md = torch.full((order + 1,), float("nan"), dtype=torch.float64, device="cuda")
        ctx.dm_chebyshev_block_noalloc(torch.from_numpy(cols).cuda(), order, mu, beta, Pd, md)
        torch.cuda.synchronize()
        dPd = np.abs(Pd.cpu().numpy() - P_ref).max()
        say(f"  max|P - P_block| = {dP:.2e} (device {dPd:.2e}), max|m - m_block| = {dm:.2e}")
        assert dP == 0.0 and dPd == 0.0 and dm == 0.0
        if precision == dmlib.DM_FP64:
            ref = O.density_matrix_poly(sp, cols, order, mu, beta, emin, emax)
            err = np.abs(P.T - ref).max()
            say(f"  against the oracle: max|dP| = {err:.2e}")
            assert err <= TOL_FP64
        # the context's accumulator is untouched by the allocation-free call
        m_acc, nd = ctx.dm_moments(order + 1)
        assert nd == len(cols) and np.array_equal(m_acc, m_ref)


def test_noalloc_refuses_what_does_not_fit(c1):
    c, sp = c1
    ctx = dmlib.Context()
    ctx.set_cluster(c)
    cols = np.arange(c.K, dtype=np.int64)
    with pytest.raises(dmlib.DMError) as e:
        ctx.dm_chebyshev_block_noalloc(cols, 1 << 20, 0.0, 10.0)  # partial sums alone exceed the array
    assert e.value.status == dmlib.DM_E_ARG and "bytes" in str(e.value)
    with pytest.raises(dmlib.DMError) as e:
        ctx.dm_chebyshev_block_noalloc(np.array([0, 5, 5], dtype=np.int64), 20, 0.0, 10.0)
    assert e.value.status == dmlib.DM_E_ARG
    with pytest.raises(dmlib.DMError) as e:
        ctx.dm_chebyshev_block_noalloc(np.array([0, c.K], dtype=np.int64), 20, 0.0, 10.0)
    assert e.value.status == dmlib.DM_E_ARG
    sym = dmlib.Context()
    sym.dm_set_operator_form(dmlib.DM_FORM_SYMMETRIC)
    sym.set_cluster(c)
    with pytest.raises(dmlib.DMError) as e:
        sym.dm_chebyshev_block_noalloc(cols, 20, 0.0, 10.0)
    assert e.value.status == dmlib.DM_E_STATE
    # after the refusals a good call still works
    P = np.zeros((4, c.K))
    ctx.dm_chebyshev_block_noalloc(cols[:4], 30, 0.0, 10.0, P)
    assert np.isfinite(P).all()
