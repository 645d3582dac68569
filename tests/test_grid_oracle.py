"""Pins for the grid-density oracle (eq. ElectronDensity), each independent of
its own formula: the electron count from the eigenvalues, the closed-form norm
of one Gaussian, additivity over column shares, and brute-force window checks."""
import numpy as np
import pytest

import oracle as O
from oracle import grid_oracle as GO
from synth import basis_functions, grid_around, make_cluster


@pytest.fixture(scope="module")
def small():
    c = make_cluster(8, seed=5, geometry="cube")  # K = 32
    return c, O.spectrum(c)


def test_density_integrates_to_electron_count(small):
    """h^3 sum_g n(r_g) = 2 Tr[P S] (eqs. density, Smat, Ne): with all columns,
    a fine grid and wide windows it equals 2 sum_i f(e_i) from the spectrum
    (uniform sums of Gaussians converge very fast in h)."""
    c, sp = small
    mu, beta = 0.5 * (sp.e[7] + sp.e[8]), 10.0
    P = O.density_matrix_exact(sp, np.arange(c.K), mu, beta)
    centres, exps = basis_functions(c)
    ne = 2.0 * O.fermi(sp.e, mu, beta).sum()
    errs = []
    for h in (0.4, 0.2):
        origin, h, shape = grid_around(c, h, 9.0)
        n = GO.density_on_grid(P, np.arange(c.K), centres, exps, origin, h, shape, eta=1e-30)
        errs.append(abs(h ** 3 * n.sum() - ne))
    # P has entries far above 1 (S^-1 is ill conditioned), which amplifies the
    # grid error: visible at h = 0.4, below 1e-9 of N_e at h = 0.2
    assert errs[1] < 1e-9 * ne and errs[0] > 100 * errs[1]


def test_single_normalised_function():
    """P = e_0 e_0^T: n = 2 phi_0^2, whose integral is 2 (normalised Gaussian);
    the value at the centre is 2 (2a/pi)^{3/2}."""
    a = 0.8
    centres, exps = np.zeros((1, 3)), np.array([a])
    origin, h, shape = np.array([-6.0, -6.0, -6.0]), 0.2, (61, 61, 61)
    n = GO.density_on_grid(np.ones((1, 1)), [0], centres, exps, origin, h, shape, eta=1e-30)
    assert abs(h ** 3 * n.sum() - 2.0) < 1e-9
    assert abs(n.max() - 2.0 * (2 * a / np.pi) ** 1.5) < 1e-12


def test_column_shares_add_up(small):
    """The density of all columns is the sum of the densities of disjoint
    column shares (the paper's reduce over processors)."""
    c, sp = small
    P = O.density_matrix_exact(sp, np.arange(c.K), 0.3, 5.0)
    centres, exps = basis_functions(c)
    origin, h, shape = grid_around(c, 0.5, 4.0)
    full = GO.density_on_grid(P, np.arange(c.K), centres, exps, origin, h, shape, eta=1e-6)
    parts = np.zeros_like(full)
    for share in np.array_split(np.random.default_rng(2).permutation(c.K), 3):
        parts += GO.density_on_grid(P[:, share], share, centres, exps, origin, h, shape, eta=1e-6)
    assert np.allclose(parts, full, rtol=1e-12, atol=1e-14)


def _charge_fraction(d, l):
    """c(d, l) of eq. WindowLength by adaptive quadrature (no special functions)."""
    from scipy.integrate import quad

    num = quad(lambda x: x ** l * np.exp(-x * x), 0.0, d, epsabs=0.0, epsrel=1e-13)[0]
    den = quad(lambda x: x ** l * np.exp(-x * x), 0.0, np.inf, epsabs=0.0, epsrel=1e-13)[0]
    tail = quad(lambda x: x ** l * np.exp(-x * x), d, np.inf, epsabs=0.0, epsrel=1e-13)[0]
    return num / den, tail / den


@pytest.mark.parametrize("l", [0, 1, 2])
@pytest.mark.parametrize("eta", [1e-3, 1e-6, 1e-10])
def test_window_depth_solves_charge_equation(l, eta):
    """Eq. WindowLength: the window depth d = L sqrt(zeta) keeps the fraction
    1 - eta of the primitive's charge, c(d, l) = 1 - eta, with c integrated
    by quadrature (the tail carries eta to 1e-9 relative)."""
    d = float(GO.window_depth(eta, l))
    inside, tail = _charge_fraction(d, l)
    assert abs(inside - (1.0 - eta)) < 1e-12
    assert abs(tail / eta - 1.0) < 1e-9


def test_window_depth_s_values():
    """For s functions c(d, 0) = erf(d): d = erfinv(1 - eta), 2.3263 at
    eta = 1e-3 and 3.4589 at 1e-6 (tabulated inverse-erf values); the
    Gaussian-factor rule sqrt(ln(1/eta)) (3.7169 at 1e-6) is not it."""
    assert abs(GO.window_depth(1e-3) - 2.326753765513525) < 1e-9
    assert abs(GO.window_depth(1e-6) - 3.458910737279500) < 1e-9
    assert abs(GO.window_depth(1e-6) - np.sqrt(np.log(1e6))) > 0.2
    a = np.array([0.3, 5.0])
    assert np.allclose(GO.window_halfwidth(a, 1e-6), GO.window_depth(1e-6) / np.sqrt(a), rtol=1e-15)


def test_window_growth_matches_paper_silicon_example():
    """The paper's cutoff study: as eta drops from 1e-3 to 1e-6 the silicon
    window grows from about 5 to about 7 angstrom (volume x2.7).  The most
    protruding primitive of a split-valence silicon basis is an sp shell,
    and for l = 1 the rule gives L(1e-6)/L(1e-3) = sqrt(2) = 1.414 (7/5 =
    1.4); the l = 0 rule would give 1.487, which the quoted sizes exclude."""
    r1 = GO.window_depth(1e-6, 1) / GO.window_depth(1e-3, 1)
    r0 = GO.window_depth(1e-6, 0) / GO.window_depth(1e-3, 0)
    assert abs(r1 - 7.0 / 5.0) < 0.02
    assert abs(r1 ** 3 - 2.7) < 0.15
    assert abs(r0 - 7.0 / 5.0) > 0.08


def test_windows_truncate_by_brute_force():
    """Inside the cube of half-width L (the root of the charge equation,
    found here by bracketing the quadrature) the function keeps its value,
    outside it is zero; checked point by point."""
    from scipy.optimize import brentq

    a, eta = 0.3, 1e-3
    d = brentq(lambda x: _charge_fraction(x, 0)[1] - eta, 0.5, 10.0, xtol=1e-14)
    R = d / np.sqrt(a)
    assert abs(R - GO.window_halfwidth([a], eta)[0]) < 1e-10
    centres, exps = np.array([[0.1, -0.2, 0.3]]), np.array([a])
    origin, h, shape = np.array([-8.0, -8.0, -8.0]), 0.5, (33, 33, 33)
    Phi = GO.basis_on_grid(centres, exps, origin, h, shape, eta)[0]
    pts = GO.grid_points(origin, h, shape)
    n_out = 0
    for g in np.random.default_rng(0).choice(len(pts), 400, replace=False):
        dv = pts[g] - centres[0]
        inside = all(abs(x) <= R for x in dv)
        n_out += not inside
        ref = (2 * a / np.pi) ** 0.75 * np.exp(-a * float(dv @ dv)) if inside else 0.0
        assert Phi[g] == pytest.approx(ref, rel=1e-14, abs=0.0)
    assert 0 < n_out < 400
    # flattened order: i fastest
    assert np.allclose(pts[1] - pts[0], [h, 0, 0]) and np.allclose(pts[shape[0]] - pts[0], [0, h, 0])
