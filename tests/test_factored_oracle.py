"""Pins for the factored-form oracle (FSAI preconditioner, conjugate
gradients, recursion with one solve per step), each against something other
than the oracle's own formulas: scipy's Cholesky factor and direct solves,
textbook properties of conjugate gradients, hand-checked patterns, and the
eigen-decomposition route of the density-matrix oracle."""
import numpy as np
import pytest
import scipy.linalg

import oracle as O
from oracle import factored_oracle as FO
from synth import make_cluster


@pytest.fixture(scope="module")
def small():
    c = make_cluster(8, seed=5, geometry="cube")  # K = 32
    return c, O.spectrum(c)


@pytest.fixture(scope="module")
def c1():
    c = make_cluster(64, seed=0, geometry="cube")  # K = 256
    return c, O.spectrum(c)


def test_fsai_whole_lower_pattern_is_inverse_cholesky(small):
    c, _ = small
    S = c.S_dense()
    K = c.K
    G = FO.fsai_factor(S, [np.arange(i + 1) for i in range(K)])
    L = scipy.linalg.cholesky(S, lower=True)
    Linv = scipy.linalg.solve_triangular(L, np.eye(K), lower=True)
    assert np.abs(G - Linv).max() < 1e-9 * np.abs(Linv).max()
    assert np.abs(G @ S @ G.T - np.eye(K)).max() < 1e-9


def test_fsai_diagonal_pattern_is_jacobi(small):
    c, _ = small
    S = c.S_dense()
    G = FO.fsai_factor(S, [np.array([i]) for i in range(c.K)])
    assert np.allclose(G, np.diag(1.0 / np.sqrt(np.diag(S))), rtol=1e-15, atol=0)


def test_fsai_rows_are_orthogonal_to_S_on_their_pattern(c1):
    c, _ = c1
    S = c.S_dense()
    pats = FO.fsai_pattern(S, 0.05, 6)
    G = FO.fsai_factor(S, pats)
    GS = G @ S
    for i, J in enumerate(pats):
        assert J[-1] == i and np.all(np.diff(J) > 0) and len(J) <= 6
        off = J[:-1]
        assert np.abs(GS[i, off]).max(initial=0.0) < 1e-12 * abs(GS[i, i])
        assert abs(GS[i, i] * G[i, i] - 1.0) < 1e-12
    assert np.allclose(np.diag(G @ S @ G.T), 1.0, atol=1e-12)
    assert np.array_equal(G, np.tril(G))


def test_fsai_pattern_rule_by_hand():
    # unit diagonal except S_33 = 4, so relative sizes are easy to read
    S = np.eye(5)
    S[3, 3] = 4.0
    for i, j, v in [(1, 0, 0.5), (2, 0, 0.01), (2, 1, -0.3), (3, 0, 0.2), (3, 1, -0.8), (3, 2, 0.02),
                    (4, 0, 1e-4), (4, 3, 0.6)]:
        S[i, j] = S[j, i] = v
    pats = FO.fsai_pattern(S, 0.015, 3)
    # row 2: |0.01| < 0.015 dropped; row 3: relative 0.1, 0.4, 0.01 -> keeps 0, 1;
    # row 4: relative 5e-5 (dropped) and 0.3
    assert [list(J) for J in pats] == [[0], [0, 1], [1, 2], [0, 1, 3], [3, 4]]
    # cap 2 keeps only the largest lower entry
    assert [list(J) for J in FO.fsai_pattern(S, 0.015, 2)] == [[0], [0, 1], [1, 2], [1, 3], [3, 4]]


def test_pcg_against_direct_solve(c1):
    c, _ = c1
    S = c.S_dense()
    rng = np.random.default_rng(3)
    B = rng.standard_normal((c.K, 5))
    B[:, 2] = 0.0  # a zero right-hand side converges at once
    G = FO.fsai_factor(S, FO.fsai_pattern(S, 1e-3, 128))
    X, its = FO.pcg(S, B, lambda R: G.T @ (G @ R), 1e-12)
    ref = scipy.linalg.cho_solve(scipy.linalg.cho_factor(S), B)
    cond = np.linalg.cond(S)
    for j in range(5):
        r = np.linalg.norm(S @ X[:, j] - B[:, j])
        assert r <= 1.01e-12 * np.linalg.norm(B[:, j]) + 1e-300
        # forward error bounded by cond(S) times the relative residual
        assert np.linalg.norm(X[:, j] - ref[:, j]) <= 2 * cond * 1e-12 * np.linalg.norm(ref[:, j]) + 1e-300
    assert its[2] == 0 and np.all(X[:, 2] == 0.0)
    assert np.all(its[[0, 1, 3, 4]] > 0)


def test_pcg_finite_termination_and_exact_preconditioner():
    rng = np.random.default_rng(11)
    A = rng.standard_normal((6, 6))
    S = A @ A.T + 0.5 * np.eye(6)
    b = rng.standard_normal((6, 1))
    # unpreconditioned CG ends within n steps in exact arithmetic
    x, its = FO.pcg(S, b, lambda R: R, 1e-10)
    assert its[0] <= 7
    assert np.allclose(x, np.linalg.solve(S, b), rtol=1e-8, atol=1e-12)
    # with S^-1 as preconditioner the first step is the solution
    Sinv = np.linalg.inv(S)
    x, its = FO.pcg(S, b, lambda R: Sinv @ R, 1e-10)
    assert its[0] == 1
    assert np.allclose(x, np.linalg.solve(S, b), rtol=1e-10, atol=1e-13)


def test_factored_recursion_equals_eigen_route(small):
    c, sp = small
    F, S = c.F_dense(), c.S_dense()
    emin, emax = sp.e[0] - 0.01, sp.e[-1] + 0.01
    N, mu, beta = 60, 0.4, 5.0
    a = O.fermi_coefficients(mu, beta, emin, emax, N)
    cols = np.arange(c.K)
    P, m = FO.factored_recursion(F, S, cols, a, emin, emax, FO.exact_solver(S))
    ref = O.density_matrix_poly(sp, cols, N, mu, beta, emin, emax)
    assert np.abs(P - ref).max() < 1e-9 * max(1.0, np.abs(ref).max())
    # over all columns the moments are the traces of T_l(H_N)
    assert np.allclose(m, O.moments_from_eigs(sp.e, N + 1, emin, emax), rtol=0, atol=1e-8 * c.K)


def test_factored_recursion_with_pcg(c1):
    c, sp = c1
    F, S = c.F_dense(), c.S_dense()
    emin, emax = sp.e[0] - 1.0, sp.e[-1] + 1.0
    N, beta = 120, 100.0
    mu = 0.5 * (sp.e[c.K // 2 - 1] + sp.e[c.K // 2])
    a = O.fermi_coefficients(mu, beta, emin, emax, N)
    cols = np.array([0, 5, 77, 128, 255])
    G = FO.fsai_factor(S, FO.fsai_pattern(S, 1e-3, 128))
    solve = lambda B: FO.pcg(S, B, lambda R: G.T @ (G @ R), 1e-11)[0]  # noqa: E731
    P, _ = FO.factored_recursion(F, S, cols, a, emin, emax, solve)
    ref = O.density_matrix_poly(sp, cols, N, mu, beta, emin, emax)
    assert np.abs(P - ref).max() < 1e-8 * max(1.0, np.abs(ref).max())
