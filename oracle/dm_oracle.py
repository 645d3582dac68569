"""Plain, slow FP64 reference for the finite-temperature density matrix.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the HIP library.

What it computes (Method section and supplementary section "Chebyshev
expansion" of Fabian, Shpiro & Baer):

* P = f_FD(S^-1 F) S^-1 (eq. RDM), with the Fermi-Dirac occupation
  f_FD(e) = 1 / (1 + exp(beta (e - mu))) (text before eq. RDM);
* N_e = g Tr[P S] (eq. Ne; the paper's spin factor is g = 2);
* <O> = g Tr[P O] (eq. <O>); with O = F this is the band energy;
* the Chebyshev form f_FD(H) ~ sum_{l<N} a_l T_l(H_N), H_N = (H - Ebar)/dE,
  dE = (Emax - Emin)/2, Ebar = (Emax + Emin)/2, with a_l from a discrete
  cosine transform of f at Chebyshev nodes (supplementary "Chebyshev
  expansion").

The truncated polynomial p_N(x) = sum_{l<N} a_l T_l(x) applied to H = S^-1 F
gives P_N = p_N(S^-1 F) S^-1.  Writing the generalized eigenproblem
F C = S C diag(e) with C^T S C = I (the paper's own route when it replaces the
expansion by diagonalisation, H2 section of the supplement), S^-1 F =
C diag(e) C^T S, hence P_N = C diag(p_N(x)) C^T with x = (e - Ebar)/dE.  This
is the result the column recursion (supplementary eq. ChebychevExpansion)
reaches up to rounding order, and it is what the HIP path is compared with.
The exact finite-temperature matrix is P = C diag(f(e)) C^T.

Readings where the paper is silent (each is listed in the design notes):
* "order" N counts the terms a_0 .. a_{N-1};
* a_0 = (1/M) sum_k f_k, a_l = (2/M) sum_k f_k cos(l theta_k),
  theta_k = pi (k + 1/2) / M, f_k = f(Ebar + dE cos theta_k), M = 4N by
  default, no damping kernel;
* f_FD is evaluated as (1 - tanh(beta (e - mu) / 2)) / 2, which cannot
  overflow;
* mu is found by bisection on [Emin, Emax].
"""
from __future__ import annotations

import numpy as np
import scipy.fft
import scipy.linalg

__all__ = [
    "stochastic_moments_symmetric",
    "gaussian",
    "dos_exact",
    "gaussian_coefficients",
    "dos_poly",
    "jackson_kernel",
    "kpm_dos",
    "fermi",
    "generalized_eigh",
    "spectral_scale",
    "chebyshev_nodes",
    "chebyshev_coefficients",
    "fermi_coefficients",
    "chebyshev_T",
    "chebyshev_series",
    "moments_from_eigs",
    "density_matrix_poly",
    "density_matrix_exact",
    "trace_poly",
    "trace_exact",
    "bisect_mu",
    "solve_mu_poly",
    "solve_mu_exact",
    "stochastic_moments",
    "Spectrum",
    "spectrum",
]


def fermi(e, mu, beta):
    """Fermi-Dirac occupation 1/(1+exp(beta(e-mu))), overflow-free form."""
    e = np.asarray(e, dtype=np.float64)
    return 0.5 * (1.0 - np.tanh(0.5 * beta * (e - mu)))


def generalized_eigh(F, S):
    """Solve F C = S C diag(e), C^T S C = I, eigenvalues ascending."""
    e, C = scipy.linalg.eigh(F, S)
    return e, C


class Spectrum:
    """Eigen-decomposition of one (F, S) pencil, reused by the other calls."""

    def __init__(self, F, S):
        self.F = np.asarray(F, dtype=np.float64)
        self.S = np.asarray(S, dtype=np.float64)
        self.e, self.C = generalized_eigh(self.F, self.S)

    @property
    def K(self):
        return len(self.e)


def spectrum(cluster):
    """Spectrum of a synth.Cluster (dense FP64 copies of its CSR F and S)."""
    return Spectrum(cluster.F_dense(), cluster.S_dense())


def spectral_scale(emin, emax):
    """(Ebar, dE) of the Chebyshev section: midpoint and half-width."""
    return 0.5 * (emax + emin), 0.5 * (emax - emin)


def chebyshev_nodes(M):
    """theta_k = pi (k + 1/2) / M, k = 0..M-1 (Chebyshev-Gauss nodes cos theta_k)."""
    return np.pi * (np.arange(M) + 0.5) / M


def chebyshev_coefficients(fvals_at_nodes, N):
    """Coefficients a_0..a_{N-1} from f sampled at M Chebyshev-Gauss nodes.

    a_l = (c_l / M) sum_k f_k cos(l theta_k), c_0 = 1, c_l = 2, computed with
    an FFT-based type-II DCT (the paper computes the coefficients with FFT
    methods, supplementary "Chebyshev expansion").
    """
    f = np.asarray(fvals_at_nodes, dtype=np.float64)
    M = len(f)
    if N > M:
        raise ValueError("need at least N nodes")
    y = scipy.fft.dct(f, type=2)  # y_l = 2 sum_k f_k cos(pi l (2k+1) / (2M))
    a = y[:N] / M
    a[0] *= 0.5
    return a


def fermi_coefficients(mu, beta, emin, emax, N, M=None):
    """Chebyshev coefficients of f_FD(.; mu, beta) on [emin, emax]."""
    if M is None:
        M = 4 * N
    ebar, de = spectral_scale(emin, emax)
    th = chebyshev_nodes(M)
    return chebyshev_coefficients(fermi(ebar + de * np.cos(th), mu, beta), N)


def chebyshev_T(n, x):
    """Array T[l, i] = T_l(x_i), l = 0..n-1, by T_{l+1} = 2x T_l - T_{l-1}."""
    x = np.asarray(x, dtype=np.float64)
    T = np.empty((n,) + x.shape)
    T[0] = 1.0
    if n > 1:
        T[1] = x
    for l in range(1, n - 1):
        T[l + 1] = 2.0 * x * T[l] - T[l - 1]
    return T


def chebyshev_series(a, x):
    """p(x) = sum_l a_l T_l(x)."""
    T = chebyshev_T(len(a), x)
    return np.tensordot(np.asarray(a), T, axes=(0, 0))


def moments_from_eigs(e, n, emin, emax):
    """m_l = Tr T_l(H_N) = sum_i T_l(x_i), l = 0..n-1."""
    ebar, de = spectral_scale(emin, emax)
    return chebyshev_T(n, (np.asarray(e) - ebar) / de).sum(axis=1)


def _poly_occupations(sp, N, mu, beta, emin, emax, M=None):
    a = fermi_coefficients(mu, beta, emin, emax, N, M)
    ebar, de = spectral_scale(emin, emax)
    return chebyshev_series(a, (sp.e - ebar) / de)


def density_matrix_poly(sp, cols, N, mu, beta, emin, emax, M=None):
    """Columns `cols` of P_N = C diag(p_N(x)) C^T (K x len(cols), FP64)."""
    p = _poly_occupations(sp, N, mu, beta, emin, emax, M)
    cols = np.asarray(cols)
    return (sp.C * p[None, :]) @ sp.C[cols, :].T


def density_matrix_exact(sp, cols, mu, beta):
    """Columns `cols` of P = C diag(f_FD(e)) C^T (eq. RDM)."""
    f = fermi(sp.e, mu, beta)
    cols = np.asarray(cols)
    return (sp.C * f[None, :]) @ sp.C[cols, :].T


def trace_poly(sp, N, mu, beta, emin, emax, spin=2.0, M=None):
    """(Tr[P_N S], g Tr[P_N F]) = (sum_i p_N(e_i), g sum_i p_N(e_i) e_i).

    Tr[P S] = sum_i p(e_i) because P S = p(S^-1 F) (eq. Ne); Tr[P F] =
    sum_i p(e_i) e_i because P F = p(H) H (eq. <O> with O = F).
    """
    p = _poly_occupations(sp, N, mu, beta, emin, emax, M)
    return float(p.sum()), float(spin * (p * sp.e).sum())


def trace_exact(sp, mu, beta, spin=2.0):
    f = fermi(sp.e, mu, beta)
    return float(f.sum()), float(spin * (f * sp.e).sum())


def bisect_mu(trace_fn, target, lo, hi, tol, max_iter=200):
    """Bisection for trace_fn(mu) = target on [lo, hi] (trace increasing in mu).

    Returns the first midpoint whose trace is within tol of target, or the
    last midpoint when the bracket has shrunk to rounding level.
    """
    mid = 0.5 * (lo + hi)
    for _ in range(max_iter):
        mid = 0.5 * (lo + hi)
        t = trace_fn(mid)
        if abs(t - target) <= tol:
            return mid
        if t < target:
            lo = mid
        else:
            hi = mid
        if hi - lo <= 4.0 * np.finfo(float).eps * max(abs(lo), abs(hi), 1.0):
            break
    return mid


def solve_mu_poly(sp, n_electrons, N, beta, emin, emax, spin=2.0, tol=1e-10, M=None):
    """mu with spin * Tr[P_N S] = n_electrons (truncated polynomial)."""
    return bisect_mu(lambda m: spin * trace_poly(sp, N, m, beta, emin, emax, spin, M)[0],
                     n_electrons, emin, emax, tol)


def solve_mu_exact(sp, n_electrons, beta, spin=2.0, tol=1e-10):
    """mu with spin * sum_i f_FD(e_i) = n_electrons (exact occupations)."""
    return bisect_mu(lambda m: spin * trace_exact(sp, m, beta, spin)[0],
                     n_electrons, sp.e[0] - 1.0, sp.e[-1] + 1.0, tol)


def stochastic_moments(sp, xi, n, emin, emax):
    """(1/Ns) sum_s xi_s^T T_l(H_N) xi_s for l < n, xi given as K x Ns.

    T_l(H_N) = C T_l(x) C^T S, so xi^T T_l(H_N) xi = sum_i (C^T xi)_i
    T_l(x_i) (C^T S xi)_i.
    """
    ebar, de = spectral_scale(emin, emax)
    y = sp.C.T @ xi
    z = sp.C.T @ (sp.S @ xi)
    w = (y * z).sum(axis=1) / xi.shape[1]
    T = chebyshev_T(n, (sp.e - ebar) / de)
    return T @ w


# ---------------------------------------------------------------- density of states
def gaussian(e, sigma):
    """Normalised Gaussian exp(-e^2 / (2 sigma^2)) / (sqrt(2 pi) sigma)."""
    e = np.asarray(e, dtype=np.float64)
    return np.exp(-0.5 * (e / sigma) ** 2) / (np.sqrt(2.0 * np.pi) * sigma)


def dos_exact(sp, energies, sigma, spin=2.0):
    """Broadened density of states g sum_n G_sigma(E - e_n) over the
    eigenvalues (the DOS function of the water-cluster validation figure,
    sigma = 0.01 hartree there, g = 2)."""
    E = np.asarray(energies, dtype=np.float64)
    return spin * gaussian(E[:, None] - sp.e[None, :], sigma).sum(axis=1)


def gaussian_coefficients(E, sigma, emin, emax, N, M=None):
    """Chebyshev coefficients of x -> G_sigma(E - (Ebar + dE x)) on [-1, 1],
    from the same node DCT as the Fermi function (M = 4N nodes)."""
    if M is None:
        M = 4 * N
    ebar, de = spectral_scale(emin, emax)
    th = chebyshev_nodes(M)
    return chebyshev_coefficients(gaussian(E - (ebar + de * np.cos(th)), sigma), N)


def dos_poly(sp, energies, sigma, N, emin, emax, spin=2.0, M=None):
    """The broadened DOS with the Gaussian truncated to N Chebyshev terms:
    g sum_n sum_{l<N} c_l(E) T_l(x_n) = g sum_l c_l(E) m_l, i.e. what the
    moments of an order-N pass give (same reading of order and nodes as for
    the Fermi function)."""
    m = moments_from_eigs(sp.e, N, emin, emax)
    out = []
    for E in np.asarray(energies, dtype=np.float64):
        out.append(spin * gaussian_coefficients(E, sigma, emin, emax, N, M) @ m)
    return np.array(out)


def jackson_kernel(N):
    """Jackson damping factors g_0..g_{N-1} of the kernel polynomial method
    (Weisse, Wellein, Alvermann and Fehske, Rev. Mod. Phys. 78, 275 (2006)):
    g_l = [(N - l + 1) cos(pi l / (N+1)) + sin(pi l / (N+1)) cot(pi / (N+1))] / (N+1)."""
    l = np.arange(N, dtype=np.float64)
    q = np.pi / (N + 1)
    return ((N - l + 1) * np.cos(q * l) + np.sin(q * l) / np.tan(q)) / (N + 1)


def kpm_dos(sp, energies, N, emin, emax, spin=2.0):
    """Kernel-polynomial DOS from N moments with the Jackson kernel:
    rho(E) = g [g_0 m_0 + 2 sum_{l>=1} g_l m_l T_l(x)] / (pi dE sqrt(1 - x^2)),
    x = (E - Ebar) / dE, zero outside (-1, 1).  Integrates to g K."""
    ebar, de = spectral_scale(emin, emax)
    m = moments_from_eigs(sp.e, N, emin, emax)
    gk = jackson_kernel(N)
    x = (np.asarray(energies, dtype=np.float64) - ebar) / de
    inside = np.abs(x) < 1.0
    xi = np.where(inside, x, 0.0)
    T = chebyshev_T(N, xi)
    w = gk * m
    w[1:] *= 2.0
    series = np.tensordot(w, T, axes=(0, 0))
    rho = spin * series / (np.pi * de * np.sqrt(1.0 - xi ** 2))
    return np.where(inside, rho, 0.0)


def stochastic_moments_symmetric(sp, xi, n, emin, emax):
    """(1/Ns) sum_s xi_s^T T_l(H~_N) xi_s for the symmetric operator
    H~ = L F L^T, L = U^-T, S = U^T U (U upper Cholesky factor).

    With F C = S C diag(e), C^T S C = I, the columns of W = U C are
    orthonormal eigenvectors of H~ (H~ W = L F C = L S C diag(e) = W diag(e)),
    so xi^T T_l(H~_N) xi = sum_i (W^T xi)_i^2 T_l(x_i).
    """
    import scipy.linalg

    ebar, de = spectral_scale(emin, emax)
    U = scipy.linalg.cholesky(sp.S, lower=False)
    y = (U @ sp.C).T @ xi
    w = (y * y).sum(axis=1) / xi.shape[1]
    T = chebyshev_T(n, (sp.e - ebar) / de)
    return T @ w
