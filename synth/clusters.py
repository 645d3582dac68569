"""Model clusters: jittered lattices of atoms, four normalised s-Gaussians each.

The paper computes S (eq. Smat) and T (eq. Tmat) as grid sums over
contracted Gaussians and adds pseudopotential and Kohn-Sham terms to get the
Fock matrix (eq. FockMatrix).  Those grid and potential layers are not part of
the density-matrix path, so the inputs here use a stand-in that has the same
structure (atom-centred, non-orthogonal, sparse S and F):

* basis: per atom the normalised s-Gaussians g(r) = (2a/pi)^(3/4) exp(-a r^2)
  with a in EXPONENTS, ordered atom-major, exponents ascending;
* S_ab = (2 sqrt(ab)/(a+b))^(3/2) exp(-mu R^2), mu = ab/(a+b)  (textbook
  closed form of the overlap of two normalised s-Gaussians);
* T_ab = mu (3 - 2 mu R^2) S_ab  (closed form of <g_a| -1/2 lap |g_b>);
* F = T + diag(eps), eps ~ N(0, 0.5) drawn once per basis function
  (onsite="diagonal", the default); or, with onsite="scaled", F_ab = T_ab +
  (eps_a + eps_b) S_ab / 2, the same energies applied through the overlap,
  which keeps the spectrum of S^-1 F near that of S^-1 T instead of
  creating near-null-space states with energies of +-1000 hartree;
* entries with |S_ij| < drop (resp. |F_ij| < drop) are removed from S
  (resp. F) independently; diagonals are always kept.

Geometry: lattice sites (i, j, k) * SPACING bohr plus a uniform jitter in
(-0.1, 0.1) per coordinate.  A "cube" takes n^3 sites in lexicographic order;
a "sphere" takes the first n_atoms sites of the integer lattice sorted by
(i^2+j^2+k^2, i, j, k).  The random stream is numpy's default_rng(seed):
first the (n_atoms, 3) jitter, then the (K,) on-site energies.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp
from scipy.spatial import cKDTree

EXPONENTS = (0.3, 0.8, 2.0, 5.0)
SPACING = 2.0
JITTER = 0.1
ONSITE_SD = 0.5
DROP = 1e-10
# Beyond this atom-atom distance every S and T element of the basis above is
# below 1e-12 (the slowest pair, a = b = 0.3, falls below 1e-10 at 12.9 bohr).
PAIR_CUTOFF = 14.0


@dataclasses.dataclass
class Cluster:
    """Input of one density-matrix problem: CSR F and S plus metadata.

    CSR arrays use int64 row pointers, int32 sorted column indices and
    float64 values, full symmetric storage.
    """

    K: int
    n_atoms: int
    positions: np.ndarray
    onsite: np.ndarray
    F_rowptr: np.ndarray
    F_col: np.ndarray
    F_val: np.ndarray
    S_rowptr: np.ndarray
    S_col: np.ndarray
    S_val: np.ndarray
    n_electrons: float
    seed: int

    def F_sparse(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.F_val, self.F_col, self.F_rowptr), shape=(self.K, self.K))

    def S_sparse(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.S_val, self.S_col, self.S_rowptr), shape=(self.K, self.K))

    def F_dense(self) -> np.ndarray:
        return self.F_sparse().toarray()

    def S_dense(self) -> np.ndarray:
        return self.S_sparse().toarray()

    @property
    def nnz_per_row(self) -> tuple[float, float]:
        return (len(self.F_val) / self.K, len(self.S_val) / self.K)


def cube_sites(n_side: int) -> np.ndarray:
    """Integer lattice sites of an n_side^3 cube in lexicographic (i, j, k) order."""
    r = np.arange(n_side)
    i, j, k = np.meshgrid(r, r, r, indexing="ij")
    return np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)


def sphere_sites(n_atoms: int) -> np.ndarray:
    """First n_atoms integer sites sorted by (i^2+j^2+k^2, i, j, k)."""
    R = int(math.ceil((3.0 * n_atoms / (4.0 * math.pi)) ** (1.0 / 3.0))) + 2
    r = np.arange(-R, R + 1)
    i, j, k = np.meshgrid(r, r, r, indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    r2 = i * i + j * j + k * k
    order = np.lexsort((k, j, i, r2))
    sites = np.stack([i[order], j[order], k[order]], axis=1)[:n_atoms]
    # the ball that was taken must lie inside the candidate cube
    assert r2[order][n_atoms - 1] < R * R
    return sites


def s_gaussian_pair_integrals(a, b, R2):
    """Overlap and kinetic integrals of two normalised s-Gaussians.

    a, b: exponents; R2: squared centre distance (broadcastable arrays).
    Returns (S, T) with S = (2 sqrt(ab)/(a+b))^(3/2) exp(-mu R2) and
    T = mu (3 - 2 mu R2) S, mu = ab/(a+b).
    """
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    R2 = np.asarray(R2, dtype=np.float64)
    mu = a * b / (a + b)
    S = (2.0 * np.sqrt(a * b) / (a + b)) ** 1.5 * np.exp(-mu * R2)
    T = mu * (3.0 - 2.0 * mu * R2) * S
    return S, T


def _to_csr(rows, cols, vals, K):
    m = sp.csr_matrix((vals, (rows, cols)), shape=(K, K))
    m.sum_duplicates()
    m.sort_indices()
    rowptr = m.indptr.astype(np.int64)
    col = m.indices.astype(np.int32)
    val = m.data.astype(np.float64)
    return rowptr, col, val


def make_cluster(
    n_atoms: int,
    seed: int = 0,
    geometry: str = "sphere",
    onsite_sd: float = ONSITE_SD,
    drop: float = DROP,
    n_electrons: float | None = None,
    onsite: str = "diagonal",
) -> Cluster:
    """Build the CSR Fock and overlap matrices of one model cluster.

    geometry "cube" needs n_atoms to be a perfect cube; "sphere" takes the
    nearest lattice sites to the origin.  n_electrons defaults to two per
    atom.
    """
    if onsite not in ("diagonal", "scaled"):
        raise ValueError(f"unknown onsite mode {onsite!r}")
    onsite_mode = onsite
    if geometry == "cube":
        n_side = int(round(n_atoms ** (1.0 / 3.0)))
        if n_side ** 3 != n_atoms:
            raise ValueError("cube geometry needs a perfect-cube atom count")
        sites = cube_sites(n_side)
    elif geometry == "sphere":
        sites = sphere_sites(n_atoms)
    else:
        raise ValueError(f"unknown geometry {geometry!r}")
    nb = len(EXPONENTS)
    K = nb * n_atoms
    rng = np.random.default_rng(seed)
    jitter = rng.uniform(-JITTER, JITTER, size=(n_atoms, 3))
    onsite = rng.normal(0.0, onsite_sd, size=K)
    pos = sites.astype(np.float64) * SPACING + jitter

    tree = cKDTree(pos)
    pairs = tree.query_pairs(PAIR_CUTOFF, output_type="ndarray")  # i < j
    I = np.concatenate([np.arange(n_atoms), pairs[:, 0]])
    J = np.concatenate([np.arange(n_atoms), pairs[:, 1]])
    ex = np.asarray(EXPONENTS)
    rows_S, cols_S, vals_S = [], [], []
    rows_F, cols_F, vals_F = [], [], []
    chunk = 1 << 20
    for c0 in range(0, len(I), chunk):
        Ic, Jc = I[c0:c0 + chunk], J[c0:c0 + chunk]
        d2 = np.sum((pos[Ic] - pos[Jc]) ** 2, axis=1)
        S, T = s_gaussian_pair_integrals(ex[None, :, None], ex[None, None, :], d2[:, None, None])
        r = (nb * Ic)[:, None, None] + np.arange(nb)[None, :, None]
        c = (nb * Jc)[:, None, None] + np.arange(nb)[None, None, :]
        r = np.broadcast_to(r, S.shape).ravel()
        c = np.broadcast_to(c, S.shape).ravel()
        S = S.ravel()
        T = T.ravel()
        same = np.repeat(Ic == Jc, nb * nb)
        diag = r == c
        if onsite_mode == "diagonal":
            T = T + np.where(diag, onsite[r], 0.0)
        else:
            T = T + 0.5 * (onsite[r] + onsite[c]) * S
        keepS = (np.abs(S) >= drop) | diag
        keepF = (np.abs(T) >= drop) | diag
        # atom pairs are stored once (i <= j); mirror the off-atom blocks
        for keep, rows_o, cols_o, vals_o, v in (
            (keepS, rows_S, cols_S, vals_S, S),
            (keepF, rows_F, cols_F, vals_F, T),
        ):
            rk, ck, vk, sk = r[keep], c[keep], v[keep], same[keep]
            rows_o += [rk, ck[~sk]]
            cols_o += [ck, rk[~sk]]
            vals_o += [vk, vk[~sk]]
    S_rowptr, S_col, S_val = _to_csr(np.concatenate(rows_S), np.concatenate(cols_S),
                                     np.concatenate(vals_S), K)
    F_rowptr, F_col, F_val = _to_csr(np.concatenate(rows_F), np.concatenate(cols_F),
                                     np.concatenate(vals_F), K)
    ne = 2.0 * n_atoms if n_electrons is None else float(n_electrons)
    return Cluster(K=K, n_atoms=n_atoms, positions=pos, onsite=onsite,
                   F_rowptr=F_rowptr, F_col=F_col, F_val=F_val,
                   S_rowptr=S_rowptr, S_col=S_col, S_val=S_val,
                   n_electrons=ne, seed=seed)


def rademacher(K: int, n_vec: int, seed: int) -> np.ndarray:
    """K x n_vec matrix of independent +-1 entries (column-major use)."""
    rng = np.random.default_rng(seed)
    return (2.0 * rng.integers(0, 2, size=(K, n_vec)) - 1.0).astype(np.float64)


def batch_cluster_sizes(n_clusters: int = 64, lo: int = 125, hi: int = 1000, seed: int = 0) -> np.ndarray:
    """Atom counts of a batch of uneven clusters, uniform on [lo, hi]."""
    return np.random.default_rng(seed).integers(lo, hi + 1, size=n_clusters)


def _make_one(args):
    n, seed, onsite = args
    return make_cluster(int(n), seed=int(seed), geometry="sphere", onsite=onsite)


def make_batch(sizes, seeds, processes: int = 8, onsite: str = "diagonal"):
    """Clusters of the given atom counts and seeds (spheres), built on
    `processes` threads of this process.

    Threads, never a process pool: a process forked after the GPU runtime
    has been initialised inherits its state, and such workers have died
    with fatal signals.  The heavy parts (pair search, integrals, CSR
    assembly) run in numpy/scipy code that releases the GIL, so threads are
    as fast here as processes were."""
    import concurrent.futures

    jobs = [(n, s, onsite) for n, s in zip(sizes, seeds)]
    if processes <= 1 or len(jobs) < 2:
        return [_make_one(j) for j in jobs]
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(processes, 16)) as ex:
        return list(ex.map(_make_one, jobs))


# Workloads with the shapes of the paper's scaling systems (silicon
# nanocrystals and water clusters of a few thousand to ~10^5 basis functions).
# beta in 1/hartree; order = number of Chebyshev terms N.
WORKLOADS = {
    "K256_cube64_fp64": dict(n_atoms=64, geometry="cube", beta=100.0, n_electrons=128.0,
                             order=400, seed=0, precision="fp64", block=256),
    "K4096_sphere1024_fp64": dict(n_atoms=1024, geometry="sphere", beta=200.0, n_electrons=2048.0,
                                  order=1000, seed=0, precision="fp64", block=64),
    "K32768_sphere8192_fp32": dict(n_atoms=8192, geometry="sphere", beta=200.0, n_electrons=16384.0,
                                   order=2000, seed=0, precision="fp32", block=0),
    "batch64_K500-4000_fp32": dict(n_clusters=64, lo=125, hi=1000, beta=100.0, order=400,
                                   precision="fp32"),
    "K131072_sphere32768_share8192_fp32": dict(n_atoms=32768, geometry="sphere", beta=200.0,
                                               n_electrons=65536.0, share=8192, seed=0,
                                               precision="fp32"),
}


def basis_functions(cluster: Cluster):
    """(centres K x 3, exponents K) of the basis: EXPONENTS on every atom,
    atom-major, the order of F and S."""
    nb = len(EXPONENTS)
    centres = np.repeat(np.asarray(cluster.positions, dtype=np.float64), nb, axis=0)
    exps = np.tile(np.asarray(EXPONENTS, dtype=np.float64), cluster.n_atoms)
    return centres, exps


def grid_around(cluster: Cluster, h: float, margin: float):
    """A uniform grid of spacing h covering the atoms plus `margin` on every
    side: (origin (3,), h, (nx, ny, nz))."""
    pos = np.asarray(cluster.positions, dtype=np.float64)
    lo = pos.min(axis=0) - margin
    hi = pos.max(axis=0) + margin
    n = np.ceil((hi - lo) / h).astype(int) + 1
    return lo, float(h), tuple(int(x) for x in n)


def workload(name: str) -> Cluster:
    w = WORKLOADS[name]
    return make_cluster(w["n_atoms"], seed=w.get("seed", 0), geometry=w["geometry"],
                        n_electrons=w.get("n_electrons"))
