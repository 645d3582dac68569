"""Factored application of H = S^-1 F: sparse-approximate-inverse
preconditioner, preconditioned conjugate gradients, and the column recursion
with one solve per step.

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the product path;
shares no code with the HIP library.

What it computes.  The paper never forms S^-1 F: each application of H to a
vector is a product with F followed by a solve with S by preconditioned
conjugate gradients (Methods, column-by-column evaluation of the density
matrix, and its footnote on the overlap solve).  The recursion itself is the
supplement's eq. ChebychevExpansion on the unit vectors, U_0 = S^-1 u_a,
U_1 = H_N U_0, U_{l+1} = 2 H_N U_l - U_{l-1}, rho_a = sum_l a_l U_l, with
H_N = (H - Ebar) / dE.  The moments are m_l = sum_a s_a^T U_l (s_a = column
a of S).

The preconditioner is the factorised sparse approximate inverse of
Kolotilina and Yeremin: G lower triangular on a prescribed pattern, row i
the solution of S[J_i, J_i] g = e_i (e_i: the unit vector of the row's own
index, the last of the ascending J_i), scaled so that (G S G^T)_ii = 1; then
S^-1 ~ G^T G.  The pattern rule (lower entries above a relative drop
tolerance, at most cap - 1 of them by magnitude, plus the diagonal) is this
project's choice, not the paper's: the paper uses an incomplete Cholesky
factor.

Parity pins (tests/test_factored_oracle.py): with the whole lower triangle
as pattern G is the inverse Cholesky factor; with the diagonal only it is the
Jacobi scaling; (G S)_ij = 0 on the pattern off the diagonal; conjugate
gradients against a direct solve, finite termination on small systems and
one iteration with the exact inverse as preconditioner; the factored
recursion against the eigen-decomposition route of dm_oracle.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

__all__ = ["fsai_pattern", "fsai_row", "fsai_factor", "pcg", "factored_recursion", "exact_solver"]


def fsai_pattern(S, drop, cap, rows=None):
    """Row patterns J_i (ascending int arrays ending with i) of the FSAI factor,
    for every row or for the listed rows.

    Lower entries j < i of the dense symmetric S with |S_ij| >= drop
    sqrt(S_ii S_jj); if more than cap - 1 qualify, the cap - 1 largest
    (ties: smaller j first), then i itself.
    """
    S = np.asarray(S, dtype=np.float64)
    K = S.shape[0]
    d = np.diag(S)
    pats = []
    for i in (range(K) if rows is None else rows):
        cand = []
        for j in range(i):
            if S[i, j] == 0.0:
                continue
            rel = abs(S[i, j]) / np.sqrt(abs(d[i] * d[j]))
            if rel >= drop:
                cand.append((rel, j))
        if len(cand) > cap - 1:
            cand.sort(key=lambda t: (-t[0], t[1]))
            cand = cand[:cap - 1]
        J = sorted(j for _, j in cand) + [i]
        pats.append(np.asarray(J, dtype=np.int64))
    return pats


def fsai_row(S, J):
    """Values of one FSAI row on its pattern J: S[J, J] g = e_last, g / sqrt(g_last)."""
    S = np.asarray(S, dtype=np.float64)
    e = np.zeros(len(J))
    e[-1] = 1.0
    g = np.linalg.solve(S[np.ix_(J, J)], e)
    return g / np.sqrt(g[-1])


def fsai_factor(S, pats):
    """Dense K x K lower-triangular G from the patterns of all K rows."""
    S = np.asarray(S, dtype=np.float64)
    K = S.shape[0]
    G = np.zeros((K, K))
    for i, J in enumerate(pats):
        G[i, J] = fsai_row(S, J)
    return G


def pcg(S, B, apply_M, tol, max_iter=10000):
    """Preconditioned conjugate gradients, one independent system per column
    of B, each stopped when ||r|| <= tol ||b||.  Returns (X, iterations per
    column).  apply_M(R) applies the preconditioner to a block."""
    S = np.asarray(S, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    if B.ndim == 1:
        B = B[:, None]
    n = B.shape[1]
    X = np.zeros_like(B)
    R = B.copy()
    bb = (B * B).sum(axis=0)
    active = bb > 0
    its = np.zeros(n, dtype=np.int64)
    Z = apply_M(R)
    Pd = Z.copy()
    rz = (R * Z).sum(axis=0)
    for _ in range(max_iter):
        if not active.any():
            break
        Q = S @ Pd
        pq = (Pd * Q).sum(axis=0)
        alpha = np.where(active, rz / np.where(active, pq, 1.0), 0.0)
        X += alpha * Pd
        R -= alpha * Q
        its += active
        rr = (R * R).sum(axis=0)
        active = active & (rr > tol * tol * bb)
        Z = apply_M(R)
        rz_new = (R * Z).sum(axis=0)
        beta = np.where(active, rz_new / np.where(rz > 0, rz, 1.0), 0.0)
        Pd = Z + beta * Pd
        rz = rz_new
    return X, its


def factored_recursion(F, S, cols, a, emin, emax, solve):
    """Columns `cols` of P = sum_l a_l T_l(H_N) S^-1 and the moments
    m_0..m_len(a) of those columns, with every application of H computed as
    solve(F @ U) (solve: block -> S^-1 block).  Returns (P (K x ncols),
    moments (len(a) + 1,))."""
    F = np.asarray(F, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    cols = np.asarray(cols)
    K = F.shape[0]
    N = len(a)
    ebar, de = 0.5 * (emax + emin), 0.5 * (emax - emin)
    E = np.zeros((K, len(cols)))
    E[cols, np.arange(len(cols))] = 1.0
    Zm = S[:, cols]
    U_prev = solve(E)
    P = a[0] * U_prev
    m = np.zeros(N + 1)
    m[0] = (Zm * U_prev).sum()
    U = (solve(F @ U_prev) - ebar * U_prev) / de
    if N > 1:
        P += a[1] * U
    m[1] = (Zm * U).sum()
    for l in range(1, N):
        U_next = 2.0 * (solve(F @ U) - ebar * U) / de - U_prev
        if l + 1 < N:
            P += a[l + 1] * U_next
        m[l + 1] = (Zm * U_next).sum()
        U_prev, U = U, U_next
    return P, m


def exact_solver(S):
    """solve(B) = S^-1 B by a Cholesky factorisation (for pins)."""
    cf = scipy.linalg.cho_factor(np.asarray(S, dtype=np.float64), lower=True)
    return lambda B: scipy.linalg.cho_solve(cf, B)
