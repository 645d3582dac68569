"""Electron density on a real-space grid from density-matrix columns.

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the product path;
shares no code with the HIP library.

What it computes (Method, eq. density and the grid-window section with eq.
ElectronDensity): the density carried by column a of P is
n_a(r_g) = 2 phi_a(r_g) sum_b phi_b(r_g) P_ba, and the density of a set of
columns is the sum over the set (the paper's reduce over processors).  The
basis functions are normalised s-type Gaussians phi(r) = (2a/pi)^{3/4}
exp(-a |r - R|^2).  Each is set to zero outside its window, a cube centred
on the function's centre whose half-width L keeps the fraction 1 - eta of
the "charge" of the most protruding primitive (grid-window section, eq.
WindowLength): c(L sqrt(zeta), l) = 1 - eta with
c(d, l) = int_0^d x^l exp(-x^2) dx / int_0^inf x^l exp(-x^2) dx, the
regularised incomplete gamma function P((l + 1)/2, d^2).  The basis here is
s-type (l = 0), where c(d, 0) = erf(d).  Grid points are
r_g = origin + h (i, j, k), with i fastest in the flattened index
g = i + nx (j + ny k).
"""
from __future__ import annotations

import numpy as np

__all__ = ["window_depth", "window_halfwidth", "grid_points", "basis_on_grid", "density_on_grid"]


def window_depth(eta, l=0):
    """d = L sqrt(zeta) solving c(d, l) = 1 - eta (eq. WindowLength).

    c(d, l) = P((l + 1)/2, d^2), so d^2 is the inverse of the upper
    regularised incomplete gamma function at eta (exact for eta far below
    the rounding of 1 - eta)."""
    from scipy.special import gammainccinv

    return np.sqrt(gammainccinv(0.5 * (l + 1), eta))


def window_halfwidth(exponents, eta, l=0):
    """Half-width L of each function's cube window: window_depth / sqrt(zeta)."""
    return window_depth(eta, l) / np.sqrt(np.asarray(exponents, dtype=np.float64))


def grid_points(origin, h, shape):
    """Coordinates (G x 3) of the grid points in flattened order."""
    nx, ny, nz = shape
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    pts = np.stack([i.ravel(order="F"), j.ravel(order="F"), k.ravel(order="F")], axis=1)
    return np.asarray(origin, dtype=np.float64) + h * pts


def basis_on_grid(centres, exponents, origin, h, shape, eta):
    """Phi (K x G): every basis function at every grid point, zero outside its window."""
    r = grid_points(origin, h, shape)
    c = np.asarray(centres, dtype=np.float64)
    a = np.asarray(exponents, dtype=np.float64)
    R = window_halfwidth(a, eta)
    d = r[None, :, :] - c[:, None, :]
    inside = np.all(np.abs(d) <= R[:, None, None], axis=2)
    norm = (2.0 * a / np.pi) ** 0.75
    return np.where(inside, norm[:, None] * np.exp(-a[:, None] * np.sum(d * d, axis=2)), 0.0)


def density_on_grid(P_cols, cols, centres, exponents, origin, h, shape, eta):
    """sum over a in cols of n_a(r_g) = 2 phi_a(r_g) sum_b phi_b(r_g) P[b, a];
    P_cols is K x len(cols) (column j holds column cols[j] of P)."""
    Phi = basis_on_grid(centres, exponents, origin, h, shape, eta)
    T = Phi.T @ np.asarray(P_cols, dtype=np.float64)   # G x ncols: sum_b phi_b P_b,a
    return 2.0 * np.sum(Phi[np.asarray(cols)].T * T, axis=1)
