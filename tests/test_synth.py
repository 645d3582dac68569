"""Pins for the synthetic inputs: closed-form integrals against the paper's
grid-sum definitions of S (eq. Smat) and T (eq. Tmat), and structure."""
import numpy as np
import pytest

from synth import (EXPONENTS, batch_cluster_sizes, cube_sites, make_cluster, rademacher,
                   s_gaussian_pair_integrals, sphere_sites)


def _g1(x, c, a):
    """1-D factor of a normalised 3-D s-Gaussian: (2a/pi)^(1/4) exp(-a (x-c)^2)."""
    return (2.0 * a / np.pi) ** 0.25 * np.exp(-a * (x - c) ** 2)


def _dg1(x, c, a):
    return -2.0 * a * (x - c) * _g1(x, c, a)


def grid_S_T(ra, a, rb, b, h=0.02, L=10.0):
    """S = h^3 sum_g phi_a phi_b and T = 1/2 h^3 sum_g grad phi_a . grad phi_b.

    An s-Gaussian is a product of 1-D factors, so the 3-D grid sums factor
    into per-axis 1-D sums (the tabulated 1-D factors of the supplement's
    basis-to-grid section).  Gradients are analytic, as in the paper.
    """
    s1, d1 = [], []
    for ax in range(3):
        x = np.arange(-L, L + h / 2, h) + 0.5 * (ra[ax] + rb[ax])
        s1.append(h * np.sum(_g1(x, ra[ax], a) * _g1(x, rb[ax], b)))
        d1.append(h * np.sum(_dg1(x, ra[ax], a) * _dg1(x, rb[ax], b)))
    S = s1[0] * s1[1] * s1[2]
    T = 0.5 * (d1[0] * s1[1] * s1[2] + s1[0] * d1[1] * s1[2] + s1[0] * s1[1] * d1[2])
    return S, T


@pytest.mark.parametrize("a,b,R", [(0.3, 0.3, 0.0), (0.3, 5.0, 1.7), (0.8, 2.0, 2.9),
                                   (5.0, 5.0, 0.4), (0.3, 0.8, 6.0), (2.0, 0.3, 3.3)])
def test_closed_form_matches_grid_sums(a, b, R):
    ra = np.array([0.1, -0.2, 0.05])
    d = np.array([1.0, 2.0, -0.5])
    rb = ra + R * d / np.linalg.norm(d)
    Sg, Tg = grid_S_T(ra, a, rb, b)
    S, T = s_gaussian_pair_integrals(a, b, R * R)
    assert abs(S - Sg) <= 1e-12
    assert abs(T - Tg) <= 1e-11


def test_self_overlap_and_kinetic_special_cases():
    for a in EXPONENTS:
        S, T = s_gaussian_pair_integrals(a, a, 0.0)
        # normalisation, and <g|-lap/2|g> = 3a/2 for a normalised s-Gaussian
        assert abs(S - 1.0) < 1e-15
        assert abs(T - 1.5 * a) < 1e-14


def test_two_atom_cluster_matrices_match_grid():
    c = make_cluster(2, seed=3, geometry="sphere")
    S = c.S_dense()
    T = c.F_dense() - np.diag(c.onsite)
    for i in range(c.K):
        for j in range(c.K):
            ai, aj = EXPONENTS[i % 4], EXPONENTS[j % 4]
            Sg, Tg = grid_S_T(c.positions[i // 4], ai, c.positions[j // 4], aj, h=0.025)
            assert abs(S[i, j] - Sg) < 1e-11
            assert abs(T[i, j] - Tg) < 1e-10


def test_structure_and_drop_rule():
    c = make_cluster(64, seed=0, geometry="cube")
    assert c.K == 256
    S, F = c.S_dense(), c.F_dense()
    assert np.array_equal(S, S.T) and np.array_equal(F, F.T)
    # every stored off-diagonal entry is at or above the drop threshold
    for rowptr, col, val in ((c.S_rowptr, c.S_col, c.S_val), (c.F_rowptr, c.F_col, c.F_val)):
        rows = np.repeat(np.arange(c.K), np.diff(rowptr))
        off = rows != col
        assert np.all(np.abs(val[off]) >= 1e-10)
        # sorted, unique columns per row; diagonal present
        for r in range(c.K):
            cr = col[rowptr[r]:rowptr[r + 1]]
            assert np.all(np.diff(cr) > 0) and r in cr
    # recompute every pair densely: dropped entries are below the threshold
    ex = np.array(EXPONENTS)
    pos = np.repeat(c.positions, 4, axis=0)
    a = np.tile(ex, 64)
    R2 = ((pos[:, None, :] - pos[None, :, :]) ** 2).sum(-1)
    Sd, Td = s_gaussian_pair_integrals(a[:, None], a[None, :], R2)
    assert np.all(np.abs(Sd[S == 0]) < 1e-10)
    assert np.allclose(S[S != 0], Sd[S != 0], rtol=0, atol=0)
    Fd = Td + np.diag(c.onsite)
    assert np.all(np.abs(Fd[F == 0]) < 1e-10)
    assert np.all(np.linalg.eigvalsh(S) > 0)


def test_geometry_and_seeds():
    assert np.array_equal(cube_sites(2)[:3], [[0, 0, 0], [0, 0, 1], [0, 1, 0]])
    s = sphere_sites(27)
    assert np.array_equal(s[0], [0, 0, 0])
    r2 = (s ** 2).sum(1)
    assert np.all(np.diff(r2) >= 0) and r2[-1] == 3  # 1 + 6 + 12 + 8 sites
    assert np.array_equal(s[1:7], [[-1, 0, 0], [0, -1, 0], [0, 0, -1], [0, 0, 1], [0, 1, 0], [1, 0, 0]])
    c1 = make_cluster(64, seed=0, geometry="cube")
    c2 = make_cluster(64, seed=0, geometry="cube")
    assert np.array_equal(c1.F_val, c2.F_val)
    assert np.all(np.abs(c1.positions - 2.0 * cube_sites(4)) <= 0.1)
    assert abs(np.std(c1.onsite) - 0.5) < 0.1
    sizes = batch_cluster_sizes()
    assert len(sizes) == 64 and sizes.min() >= 125 and sizes.max() <= 1000
    xi = rademacher(10, 3, 1)
    assert set(np.unique(xi)) <= {-1.0, 1.0}
