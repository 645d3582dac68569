"""Pins for the FP64 oracle, each independent of the oracle's own formulas:
closed-form eigenproblems, brute-force recursion, textbook special cases and
invariants of eqs. RDM, Ne and <O> and of the supplement's Chebyshev section."""
import numpy as np
import pytest
import scipy.integrate
import scipy.optimize
import scipy.special

import oracle as O
from synth import make_cluster, rademacher


@pytest.fixture(scope="module")
def c1():
    c = make_cluster(64, seed=0, geometry="cube")
    return c, O.spectrum(c)


@pytest.fixture(scope="module")
def small():
    c = make_cluster(8, seed=5, geometry="cube")  # K = 32
    return c, O.spectrum(c)


# ---------------------------------------------------------------- f_FD, T_l
def test_fermi_function():
    assert O.fermi(0.3, 0.3, 50.0) == 0.5
    d = np.linspace(-3, 3, 13)
    assert np.allclose(O.fermi(0.1 + d, 0.1, 7.0), 1.0 - O.fermi(0.1 - d, 0.1, 7.0), atol=1e-15)
    x = np.linspace(-2, 2, 41)
    assert np.allclose(O.fermi(x, 0.2, 3.0), 1.0 / (1.0 + np.exp(3.0 * (x - 0.2))), atol=1e-15)
    # no overflow where exp(beta (e - mu)) would overflow
    with np.errstate(over="raise"):
        assert O.fermi(1e4, 0.0, 1e3) == 0.0 and O.fermi(-1e4, 0.0, 1e3) == 1.0


def test_chebyshev_T_is_cos_l_theta():
    th = np.linspace(0, np.pi, 17)
    T = O.chebyshev_T(50, np.cos(th))
    l = np.arange(50)[:, None]
    assert np.allclose(T, np.cos(l * th[None, :]), atol=1e-12)


# ---------------------------------------------------------------- a_l
def test_coefficients_of_exp_are_bessel():
    # exp(x) = I_0(1) + 2 sum_l I_l(1) T_l(x) (textbook expansion)
    N, M = 20, 80
    th = O.chebyshev_nodes(M)
    a = O.chebyshev_coefficients(np.exp(np.cos(th)), N)
    ref = 2.0 * scipy.special.iv(np.arange(N), 1.0)
    ref[0] *= 0.5
    assert np.allclose(a, ref, rtol=0, atol=1e-15)


def test_coefficients_of_T_m_are_delta():
    N, M = 12, 48
    th = O.chebyshev_nodes(M)
    for m in (0, 1, 5, 11):
        a = O.chebyshev_coefficients(np.cos(m * th), N)
        e = np.zeros(N)
        e[m] = 1.0
        assert np.allclose(a, e, atol=1e-14)


def test_fermi_coefficients_symmetry_at_midpoint():
    # f - 1/2 is odd about mu = Ebar, so a_0 = 1/2 and a_2k = 0
    a = O.fermi_coefficients(mu=1.5, beta=4.0, emin=-1.0, emax=4.0, N=60)
    assert abs(a[0] - 0.5) < 1e-15
    assert np.all(np.abs(a[2::2]) < 1e-15)
    assert np.all(np.abs(a[1::2][:5]) > 1e-3)


def test_fermi_coefficients_match_projection_integral():
    # a_l = (c_l/pi) int_0^pi f(cos t) cos(l t) dt for a smooth f; the DCT at
    # M nodes differs from it only by aliasing, negligible here.
    mu, beta, emin, emax, N = 0.3, 3.0, -2.0, 2.0, 12
    a = O.fermi_coefficients(mu, beta, emin, emax, N, M=256)
    for l in range(N):
        v, _ = scipy.integrate.quad(
            lambda t: 1.0 / (1.0 + np.exp(beta * (2.0 * np.cos(t) - mu))) * np.cos(l * t), 0, np.pi,
            epsabs=1e-14, limit=200)
        ref = v / np.pi * (1.0 if l == 0 else 2.0)
        assert abs(a[l] - ref) < 1e-12


# ---------------------------------------------------------------- eigen-decomposition
def test_generalized_eigh_residual_and_normalisation(c1):
    c, sp = c1
    F, S = c.F_dense(), c.S_dense()
    C, e = sp.C, sp.e
    assert np.abs(C.T @ S @ C - np.eye(c.K)).max() < 1e-9
    assert np.abs(F @ C - S @ C * e[None, :]).max() < 1e-10 * np.abs(F).max() * 100
    # eigenvalues agree with the Cholesky-orthogonalised symmetric problem
    L = np.linalg.cholesky(S)
    Li = np.linalg.inv(L)
    e2 = np.linalg.eigvalsh(Li @ F @ Li.T)
    assert np.abs(e - e2).max() < 1e-8 * np.abs(e).max()


# ---------------------------------------------------------------- closed forms
def test_dimer_closed_form():
    # two equal functions: S = [[1, s], [s, 1]], F = [[e, t], [t, e]]:
    # eigenvalues (e +- t)/(1 +- s), S-normalised vectors (1, +-1)/sqrt(2(1 +- s))
    s, e, t, mu, beta = 0.4, -0.2, -0.35, -0.3, 9.0
    S = np.array([[1.0, s], [s, 1.0]])
    F = np.array([[e, t], [t, e]])
    sp = O.Spectrum(F, S)
    lp, lm = (e + t) / (1 + s), (e - t) / (1 - s)
    vp = np.array([1.0, 1.0]) / np.sqrt(2 * (1 + s))
    vm = np.array([1.0, -1.0]) / np.sqrt(2 * (1 - s))
    fp, fm = [1.0 / (1.0 + np.exp(beta * (x - mu))) for x in (lp, lm)]
    P_ref = fp * np.outer(vp, vp) + fm * np.outer(vm, vm)
    P = O.density_matrix_exact(sp, [0, 1], mu, beta)
    assert np.allclose(P, P_ref, atol=1e-14)
    assert np.allclose(sorted([lp, lm]), sp.e, atol=1e-14)


def test_chain_with_overlap_closed_form():
    # S = tridiag(s, 1, s), F = tridiag(t, e, t) on n sites share the sine
    # eigenvectors: eps_j = (e + 2t cos th_j)/(1 + 2s cos th_j), th_j = pi j/(n+1)
    n, s, e, t, mu, beta = 24, 0.2, 0.1, -0.5, 0.05, 6.0
    S = np.eye(n) + s * (np.eye(n, k=1) + np.eye(n, k=-1))
    F = e * np.eye(n) + t * (np.eye(n, k=1) + np.eye(n, k=-1))
    j = np.arange(1, n + 1)
    th = np.pi * j / (n + 1)
    eps = (e + 2 * t * np.cos(th)) / (1 + 2 * s * np.cos(th))
    V = np.sqrt(2.0 / (n + 1)) * np.sin(np.outer(np.arange(1, n + 1), th))
    V = V / np.sqrt(1 + 2 * s * np.cos(th))[None, :]
    P_ref = (V * (1.0 / (1.0 + np.exp(beta * (eps - mu))))[None, :]) @ V.T
    sp = O.Spectrum(F, S)
    assert np.allclose(np.sort(eps), sp.e, atol=1e-13)
    assert np.allclose(O.density_matrix_exact(sp, np.arange(n), mu, beta), P_ref, atol=1e-13)


def test_orthogonal_basis_reduces_to_matrix_function():
    # S = I: P = f(F), computed by scipy's matrix-function routine
    rng = np.random.default_rng(1)
    A = rng.normal(size=(12, 12))
    F = 0.5 * (A + A.T)
    sp = O.Spectrum(F, np.eye(12))
    mu, beta = 0.3, 2.0
    P_ref = scipy.linalg.funm(F, lambda x: 1.0 / (1.0 + np.exp(beta * (x - mu))))
    assert np.allclose(O.density_matrix_exact(sp, np.arange(12), mu, beta), np.real(P_ref), atol=1e-10)


# ---------------------------------------------------------------- invariants of eq. RDM / Ne / <O>
def test_trace_symmetry_limits(small):
    c, sp = small
    S, F = c.S_dense(), c.F_dense()
    K = c.K
    mu, beta = 0.5, 3.0
    P = O.density_matrix_exact(sp, np.arange(K), mu, beta)
    assert np.abs(P - P.T).max() < 1e-10
    tr, eb = O.trace_exact(sp, mu, beta, spin=2.0)
    assert abs(np.trace(P @ S) - tr) < 1e-9
    assert abs(2.0 * np.trace(P @ F) - eb) < 1e-8
    Sinv = np.linalg.inv(S)
    # beta -> 0: every state half filled, P -> S^-1 / 2
    assert np.abs(O.density_matrix_exact(sp, np.arange(K), mu, 1e-12) - 0.5 * Sinv).max() < 1e-8
    # mu far above / below the spectrum: P -> S^-1 / P -> 0
    assert np.abs(O.density_matrix_exact(sp, np.arange(K), 1e4, 1.0) - Sinv).max() < 1e-8
    assert np.abs(O.density_matrix_exact(sp, np.arange(K), -1e4, 1.0)).max() < 1e-12


def test_idempotency_at_large_beta(c1):
    # with beta * gap >> 1 the occupations are 0/1 and P S P = P
    c, sp = c1
    S = c.S_dense()
    nocc = 64
    mu = 0.5 * (sp.e[nocc - 1] + sp.e[nocc])
    gap = sp.e[nocc] - sp.e[nocc - 1]
    beta = 400.0 / gap
    P = O.density_matrix_exact(sp, np.arange(c.K), mu, beta)
    assert abs(np.trace(P @ S) - nocc) < 1e-9
    assert np.abs(P @ S @ P - P).max() < 1e-8 * np.abs(P).max()


# ---------------------------------------------------------------- polynomial result
def _recursion_all_columns(F, S, a, emin, emax):
    """The supplement's column recursion on all unit vectors at once, with
    S^-1 and S^-1 F from dense solves (no eigen-decomposition)."""
    ebar, de = 0.5 * (emax + emin), 0.5 * (emax - emin)
    H = np.linalg.solve(S, F)
    HN = (H - ebar * np.eye(len(F))) / de
    U0 = np.linalg.inv(S)
    U1 = HN @ U0
    rho = a[0] * U0 + a[1] * U1
    for l in range(2, len(a)):
        U2 = 2.0 * HN @ U1 - U0
        rho = rho + a[l] * U2
        U0, U1 = U1, U2
    return rho


def test_poly_density_matrix_equals_recursion(small):
    c, sp = small
    F, S = c.F_dense(), c.S_dense()
    emin, emax = sp.e[0] - 0.01, sp.e[-1] + 0.01
    N, mu, beta = 60, 0.4, 5.0
    a = O.fermi_coefficients(mu, beta, emin, emax, N)
    ref = _recursion_all_columns(F, S, a, emin, emax)
    P = O.density_matrix_poly(sp, np.arange(c.K), N, mu, beta, emin, emax)
    assert np.abs(P - ref).max() < 1e-9 * max(1.0, np.abs(ref).max())
    # column subset selection
    cols = [3, 0, 17]
    assert np.array_equal(O.density_matrix_poly(sp, cols, N, mu, beta, emin, emax), P[:, cols])


def test_poly_converges_to_exact(small):
    c, sp = small
    emin, emax = sp.e[0] - 0.01, sp.e[-1] + 0.01
    mu, beta = 0.4, 2.0
    Pe = O.density_matrix_exact(sp, np.arange(c.K), mu, beta)
    errs = [np.abs(O.density_matrix_poly(sp, np.arange(c.K), N, mu, beta, emin, emax) - Pe).max()
            for N in (80, 320, 640)]
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-10


def test_moments_trace_and_band_energy_identities(small):
    c, sp = small
    F, S = c.F_dense(), c.S_dense()
    K = c.K
    emin, emax = sp.e[0] - 0.5, sp.e[-1] + 0.5
    ebar, de = 0.5 * (emax + emin), 0.5 * (emax - emin)
    HN = (np.linalg.solve(S, F) - ebar * np.eye(K)) / de
    N = 40
    m = O.moments_from_eigs(sp.e, N + 1, emin, emax)
    assert abs(m[0] - K) < 1e-12
    assert abs(m[1] - np.trace(HN)) < 1e-9
    assert abs(m[2] - (2.0 * np.trace(HN @ HN) - K)) < 1e-8
    mu, beta = 0.3, 4.0
    a = O.fermi_coefficients(mu, beta, emin, emax, N)
    tr, eb = O.trace_poly(sp, N, mu, beta, emin, emax, spin=2.0)
    P = O.density_matrix_poly(sp, np.arange(K), N, mu, beta, emin, emax)
    assert abs(tr - np.trace(P @ S)) < 1e-9
    assert abs(eb - 2.0 * np.trace(P @ F)) < 1e-8
    # Tr P_N S = sum_l a_l m_l; Tr P_N F = sum_l a_l [Ebar m_l + dE (m_{l+1} + m_|l-1|)/2]
    assert abs(tr - a @ m[:N]) < 1e-10
    e_l = np.array([ebar * m[l] + de * 0.5 * (m[l + 1] + m[abs(l - 1)]) for l in range(N)])
    assert abs(eb - 2.0 * (a @ e_l)) < 1e-9


def test_mu_bisection_against_brentq(c1):
    c, sp = c1
    beta, ne = 100.0, 128.0
    mu = O.solve_mu_exact(sp, ne, beta, tol=1e-11)
    ref = scipy.optimize.brentq(lambda m: 2.0 * O.fermi(sp.e, m, beta).sum() - ne,
                                sp.e[0], sp.e[-1], xtol=1e-14)
    assert abs(2.0 * O.trace_exact(sp, mu, beta)[0] - ne) <= 1e-11
    assert abs(mu - ref) < 1e-9
    emin, emax = sp.e[0] - 3.0, sp.e[-1] + 3.0
    mup = O.solve_mu_poly(sp, ne, 400, beta, emin, emax, tol=1e-9)
    assert abs(2.0 * O.trace_poly(sp, 400, mup, beta, emin, emax)[0] - ne) <= 1e-9


def test_stochastic_moments(small):
    c, sp = small
    F, S = c.F_dense(), c.S_dense()
    K = c.K
    emin, emax = sp.e[0] - 0.5, sp.e[-1] + 0.5
    ebar, de = 0.5 * (emax + emin), 0.5 * (emax - emin)
    HN = (np.linalg.solve(S, F) - ebar * np.eye(K)) / de
    xi = rademacher(K, 5, 2)
    n = 16
    ms = O.stochastic_moments(sp, xi, n, emin, emax)
    # brute force: xi^T T_l(H_N) xi by the matrix recursion
    T0, T1 = np.eye(K), HN.copy()
    ref = [np.einsum("is,ij,js->", xi, T0, xi) / 5, np.einsum("is,ij,js->", xi, T1, xi) / 5]
    for _ in range(2, n):
        T0, T1 = T1, 2.0 * HN @ T1 - T0
        ref.append(np.einsum("is,ij,js->", xi, T1, xi) / 5)
    assert np.allclose(ms, ref, atol=1e-8)
    # with all K unit vectors the estimate is exact: K * m~ = m
    m = O.moments_from_eigs(sp.e, n, emin, emax)
    assert np.allclose(K * O.stochastic_moments(sp, np.eye(K), n, emin, emax), m, atol=1e-9)


# ---------------------------------------------------------------- density of states
def test_broadened_dos_normalisation_and_single_level(small):
    """The broadened DOS integrates to g K; one level gives g times a Gaussian
    centred on it (textbook normal density)."""
    c, sp = small
    sigma = 0.3
    E = np.linspace(sp.e[0] - 12 * sigma, sp.e[-1] + 12 * sigma, 200001)
    rho = O.dos_exact(sp, E, sigma, spin=2.0)
    assert abs(np.trapezoid(rho, E) - 2.0 * c.K) < 1e-6 * c.K
    one = type("Sp", (), {"e": np.array([0.7])})()
    x = np.array([0.7, 0.7 + sigma, 0.7 - 2 * sigma])
    ref = 2.0 * np.exp(-0.5 * ((x - 0.7) / sigma) ** 2) / (np.sqrt(2 * np.pi) * sigma)
    assert np.allclose(O.dos_exact(one, x, sigma), ref, rtol=1e-14)


def test_gaussian_coefficients_against_quadrature():
    """Node-DCT coefficients of the Gaussian agree with direct integrals
    (2/pi) int_0^pi G(E - Ebar - dE cos t) cos(l t) dt (halved for l = 0)."""
    from scipy.integrate import quad

    emin, emax, sigma, N = -3.0, 5.0, 0.4, 60
    ebar, de = 1.0, 4.0
    for E in (-1.2, 0.5, 3.9):
        a = O.gaussian_coefficients(E, sigma, emin, emax, N)
        for l in (0, 1, 7, 30):
            v = quad(lambda t: O.gaussian(E - ebar - de * np.cos(t), sigma) * np.cos(l * t), 0, np.pi,
                     limit=400, epsabs=1e-13)[0] * 2 / np.pi
            if l == 0:
                v *= 0.5
            assert abs(a[l] - v) < 1e-11


def test_truncated_dos_converges_to_broadened(small):
    """With N far above dE / sigma the truncated Gaussian is exact to rounding."""
    c, sp = small
    w = sp.e[-1] - sp.e[0]
    emin, emax = sp.e[0] - 0.01 * w, sp.e[-1] + 0.01 * w
    sigma = 0.05 * (emax - emin) / 2
    E = np.linspace(emin, emax, 37)
    ref = O.dos_exact(sp, E, sigma)
    got = O.dos_poly(sp, E, sigma, 400, emin, emax)
    assert np.abs(got - ref).max() < 1e-9 * ref.max()
    coarse = O.dos_poly(sp, E, sigma, 20, emin, emax)
    assert np.abs(coarse - ref).max() > 1e-3 * ref.max()  # too few terms: visibly different


def test_jackson_kernel_hand_values():
    """Weisse et al. (2006), Jackson kernel for N moments,
    g_n = [(N - n + 1) cos(pi n/(N+1)) + sin(pi n/(N+1)) cot(pi/(N+1))]/(N+1),
    evaluated by hand: N = 3 (angle pi/4) gives 1, sqrt(2)/2, 1/4; N = 4
    (angle pi/5, with cos(pi/5) = (1 + sqrt 5)/4) gives 1, (1 + sqrt 5)/4,
    sqrt(5)/5, (5 - sqrt 5)/20.  An off-by-one in N or N + 1 changes them."""
    r5 = np.sqrt(5.0)
    assert np.allclose(O.jackson_kernel(3), [1.0, np.sqrt(2.0) / 2.0, 0.25], rtol=0, atol=1e-15)
    assert np.allclose(O.jackson_kernel(4), [1.0, (1.0 + r5) / 4.0, r5 / 5.0, (5.0 - r5) / 20.0],
                       rtol=0, atol=1e-15)


def test_jackson_kernel_and_kpm_dos_properties(small):
    """g_0 = 1 and g_l decreasing to ~0; the KPM DOS is non-negative,
    integrates to g K, and counts the levels in windows wide compared with
    its resolution pi dE / N."""
    c, sp = small
    N = 400
    g = O.jackson_kernel(N)
    assert abs(g[0] - 1.0) < 1e-14 and np.all(np.diff(g) < 0) and g[-1] < 1e-3
    w = sp.e[-1] - sp.e[0]
    emin, emax = sp.e[0] - 0.01 * w, sp.e[-1] + 0.01 * w
    ebar, de = O.spectral_scale(emin, emax)
    # Gauss-Chebyshev quadrature of rho dE = (g/pi) series dtheta: exact for the polynomial
    th = O.chebyshev_nodes(4 * N)
    rho = O.kpm_dos(sp, ebar + de * np.cos(th), N, emin, emax)
    integral = np.sum(rho * np.pi * de * np.sin(th)) * (np.pi / len(th)) / np.pi
    assert abs(integral - 2.0 * c.K) < 1e-8 * c.K
    E = np.linspace(emin, emax, 20001)[1:-1]
    r = O.kpm_dos(sp, E, N, emin, emax)
    assert r.min() > -1e-9 * r.max()
    res = np.pi * de / N
    edges = np.linspace(sp.e[0] - 5 * res, sp.e[-1] + 5 * res, 5)
    for a, b in zip(edges[:-1], edges[1:]):
        sel = (E >= a) & (E < b)
        count = 2.0 * np.sum((sp.e >= a) & (sp.e < b))
        assert abs(np.trapezoid(r[sel], E[sel]) - count) < 0.05 * c.K + 2.0


def test_symmetric_form_eigenvalues_and_stochastic_moments(small):
    """H~ = L F L^T (L = U^-T, S = U^T U) has the generalized eigenvalues of
    (F, S); xi^T T_l(H~_N) xi by the matrix recursion on the explicitly formed
    H~ matches the oracle, and all K unit vectors give the exact moments."""
    import scipy.linalg

    c, sp = small
    F, S = c.F_dense(), c.S_dense()
    K = c.K
    U = scipy.linalg.cholesky(S, lower=False)
    L = np.linalg.inv(U).T
    Hs = L @ F @ L.T
    assert np.allclose(np.linalg.eigvalsh(0.5 * (Hs + Hs.T)), sp.e, atol=1e-9 * np.abs(sp.e).max())
    emin, emax = sp.e[0] - 0.5, sp.e[-1] + 0.5
    ebar, de = 0.5 * (emax + emin), 0.5 * (emax - emin)
    HN = (Hs - ebar * np.eye(K)) / de
    xi = rademacher(K, 5, 3)
    n = 16
    ms = O.stochastic_moments_symmetric(sp, xi, n, emin, emax)
    T0, T1 = np.eye(K), HN.copy()
    ref = [np.einsum("is,ij,js->", xi, T0, xi) / 5, np.einsum("is,ij,js->", xi, T1, xi) / 5]
    for _ in range(2, n):
        T0, T1 = T1, 2.0 * HN @ T1 - T0
        ref.append(np.einsum("is,ij,js->", xi, T1, xi) / 5)
    assert np.allclose(ms, ref, atol=1e-8)
    m = O.moments_from_eigs(sp.e, n, emin, emax)
    assert np.allclose(K * O.stochastic_moments_symmetric(sp, np.eye(K), n, emin, emax), m, atol=1e-9)
    # P = L^T f(H~) L is the same density matrix as C f(e) C^T
    w, V = np.linalg.eigh(0.5 * (Hs + Hs.T))
    fw = O.fermi(w, 0.3, 5.0)
    P_sym = L.T @ (V * fw) @ V.T @ L
    assert np.allclose(P_sym, O.density_matrix_exact(sp, np.arange(K), 0.3, 5.0), atol=1e-9)
