"""dm_combine_sets: blocks of one multi-set pass at nodes mu_q combined at
another mu, against the oracle.

The coefficients a_l(mu) of the Fermi-Dirac expansion (supplement "Chebyshev
expansion") are smooth in mu, while the recursion vectors are not functions
of mu at all; so P at mu is approximated by sum_q w_q P(mu_q), w_q the
Lagrange weights of the nodes.  The combination itself is checked element by
element against the same weighted sum of oracle matrices (exact up to
rounding), the returned bound against the oracle's coefficients, and the
result against the oracle's P(mu) within that bound."""
import sys

import numpy as np
import pytest

import oracle as O
import paper_2108_13478_amd as dmlib
from synth import make_cluster

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def lagrange_weights(nodes, x):
    w = np.ones(len(nodes))
    for q in range(len(nodes)):
        for r in range(len(nodes)):
            if r != q:
                w[q] *= (x - nodes[r]) / (nodes[q] - nodes[r])
    return w


@pytest.fixture(scope="module")
def cl():
    c = make_cluster(150, seed=12, geometry="sphere", onsite="scaled")
    return c, O.spectrum(c)


@pytest.mark.parametrize("form", [dmlib.DM_FORM_GENERAL, dmlib.DM_FORM_SYMMETRIC])
@pytest.mark.parametrize("m", [3, 8])
def test_combined_blocks_match_oracle(cl, form, m):
    c, sp = cl
    N, beta = 600, 40.0
    w = sp.e[-1] - sp.e[0]
    lo, hi = sp.e[0] - 0.01 * w, sp.e[-1] + 0.01 * w
    nocc = int(c.n_electrons) // 2
    mu_c = 0.5 * (sp.e[nocc - 1] + sp.e[nocc])
    half = 0.02
    nodes = mu_c + half * np.cos(np.pi * (np.arange(m) + 0.5) / m)
    mu = mu_c + 0.37 * half
    say(f"case: combine {m} sets K={c.K} form {form} N={N} beta={beta}")
    ctx = dmlib.Context(precision=dmlib.DM_FP64)
    ctx.dm_set_operator_form(form)
    ctx.set_cluster(c)
    ctx.dm_set_bounds(lo, hi)
    cols = np.arange(c.K, dtype=np.int64)
    Ps = [np.zeros((c.K, c.K)) for _ in range(m)]
    ctx.dm_chebyshev_block_multi(cols, N, list(nodes), [beta] * m, Ps)
    out = np.zeros((c.K, c.K))
    bound = ctx.dm_combine_sets(nodes, beta, N, mu, Ps, out)
    wq = lagrange_weights(nodes, mu)
    ref_sum = sum(wq[q] * O.density_matrix_poly(sp, cols, N, nodes[q], beta, lo, hi) for q in range(m))
    P_mu = O.density_matrix_poly(sp, cols, N, mu, beta, lo, hi)
    a_mu = O.fermi_coefficients(mu, beta, lo, hi, N)
    a_int = sum(wq[q] * O.fermi_coefficients(nodes[q], beta, lo, hi, N) for q in range(m))
    bound_ref = np.abs(a_mu - a_int).sum()
    e_sum = np.abs(out.T - ref_sum).max()
    e_mu = np.abs(out.T - P_mu).max()
    # |P_ab - P~_ab| <= sup|p - p~| sqrt((S^-1)_aa (S^-1)_bb), sup|p - p~| <= bound
    sinv_diag = np.einsum("ij,ij->i", sp.C, sp.C)
    say(f"  max|out - sum_q w_q P_q| = {e_sum:.2e}; bound {bound:.3e} (oracle {bound_ref:.3e}); "
        f"max|out - P(mu)| = {e_mu:.2e} <= {bound * sinv_diag.max():.2e}")
    assert e_sum <= 1e-9 * np.abs(ref_sum).max()
    assert abs(bound - bound_ref) <= 1e-9 + 1e-6 * bound_ref
    assert e_mu <= bound * sinv_diag.max() + 1e-9
    if m == 8:
        assert bound < 1e-6  # eight nodes over +-0.02 hartree at beta 40 resolve p_N(.; mu)


def test_host_and_device_buffers_agree(cl):
    import torch

    c, sp = cl
    say(f"case: combine sets, device buffers K={c.K}")
    ctx = dmlib.Context(precision=dmlib.DM_FP64)
    ctx.set_cluster(c)
    nodes = np.array([-0.3, -0.25, -0.2, -0.15])
    cols = torch.arange(c.K, dtype=torch.int64, device="cuda")
    Pd = [torch.empty((c.K, c.K), dtype=torch.float64, device="cuda") for _ in nodes]
    ctx.dm_chebyshev_block_multi(cols, 300, list(nodes), [20.0] * 4, Pd)
    Ph = [p.cpu().numpy() for p in Pd]
    od = torch.empty((c.K, c.K), dtype=torch.float64, device="cuda")
    oh = np.zeros((c.K, c.K))
    b1 = ctx.dm_combine_sets(nodes, 20.0, 300, -0.22, Pd, od)
    b2 = ctx.dm_combine_sets(nodes, 20.0, 300, -0.22, Ph, oh)
    b3 = ctx.dm_combine_sets(nodes, 20.0, 300, -0.22, [Pd[0], Ph[1], Pd[2], Ph[3]], oh)
    b0 = ctx.dm_combine_sets(nodes, 20.0, 300, -0.22, [], None)  # bound only
    assert b0 == b1 == b2 == b3
    assert np.array_equal(od.cpu().numpy(), oh)
    # at a node the combination is that node's block
    ctx.dm_combine_sets(nodes, 20.0, 300, nodes[2], Pd, od)
    assert np.abs(od.cpu().numpy() - Ph[2]).max() <= 1e-12 * np.abs(Ph[2]).max()


def test_bad_arguments_are_refused(cl):
    c, _ = cl
    ctx = dmlib.Context(precision=dmlib.DM_FP64)
    out = np.zeros(4)
    with pytest.raises(dmlib.DMError):
        ctx.dm_combine_sets([0.0, 0.1], 10.0, 50, 0.05, [np.zeros(4), np.zeros(4)], out)  # no operator
    ctx.set_cluster(c)
    with pytest.raises(dmlib.DMError):
        ctx.dm_combine_sets([0.0, 0.0], 10.0, 50, 0.05, [np.zeros(4), np.zeros(4)], out)  # repeated node
    with pytest.raises(dmlib.DMError):
        ctx.dm_combine_sets([0.0, np.nan], 10.0, 50, 0.05, [np.zeros(4), np.zeros(4)], out)
    with pytest.raises(dmlib.DMError):
        ctx.dm_combine_sets([0.0, 0.1], -1.0, 50, 0.05, [np.zeros(4), np.zeros(4)], out)
