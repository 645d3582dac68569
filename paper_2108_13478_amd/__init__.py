"""Python binding of libdm.so, the MI355X Chebyshev density-matrix library.

Argument marshalling only: every computation runs in the library's HIP
kernels.  Functions keep the names of the C ABI in include/dm.h; `Context`
wraps a dm_ctx handle.  Arrays may be torch tensors (CPU or on the GPU) or
numpy arrays; device tensors are passed to the library as device pointers.
The library must have been built (python -m paper_2108_13478_amd.build); a
missing library raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdm.so")

DM_OK, DM_E_ARG, DM_E_STATE, DM_E_HIP, DM_E_OOM, DM_E_NOTSPD, DM_E_BOUNDS, DM_E_NOCONV = (
    0, -1, -2, -3, -4, -5, -6, -7)
DM_FP64, DM_FP32, DM_FP32_ACC64 = 0, 1, 2
DM_OP_SINV, DM_OP_H, DM_OP_HSYM = 0, 1, 2
DM_FORM_GENERAL, DM_FORM_SYMMETRIC, DM_FORM_FACTORED = 0, 1, 2
DM_DOS_GAUSSIAN, DM_DOS_KPM = 0, 1
DM_MAX_SETS = 16
STATUS_NAMES = {0: "DM_OK", -1: "DM_E_ARG", -2: "DM_E_STATE", -3: "DM_E_HIP", -4: "DM_E_OOM",
                -5: "DM_E_NOTSPD", -6: "DM_E_BOUNDS", -7: "DM_E_NOCONV"}

EXPORTED = ["dm_default_options", "dm_init", "dm_destroy", "dm_last_error", "dm_set_fock",
            "dm_get_bounds", "dm_set_bounds", "dm_get_operator", "dm_set_precision", "dm_chebyshev_block",
            "dm_trace", "dm_solve_mu", "dm_moments", "dm_reset_moments", "dm_stoch_moments",
            "dm_autotune", "dm_batch_set_focks", "dm_batch_get_bounds", "dm_batch_run",
            "dm_batch_autotune", "dm_batch_stoch_moments", "dm_cheb_order", "dm_mlp_init",
            "dm_mlp_num_params", "dm_mlp_get_params", "dm_mlp_set_params", "dm_mlp_forward",
            "dm_mlp_gradients", "dm_mlp_train_step", "dm_mlp_features", "dm_mlp_predict",
            "dm_set_pass_shape", "dm_num_tile_shapes", "dm_tile_shape", "dm_chebyshev_block_multi",
            "dm_dos", "dm_set_operator_form", "dm_set_fock_orthonormal", "dm_density_on_grid",
            "dm_set_factored_options", "dm_solve_overlap", "dm_get_preconditioner", "dm_cg_stats",
            "dm_cg_timing", "dm_cheb_order_rule", "dm_mlp_encode_targets",
            "dm_set_moments_precision", "dm_combine_sets", "dm_chebyshev_block_noalloc"]


class DMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


DM_BATCH_EAGER = 1
DM_BATCH_MOMENTS_ONLY = 2


class dm_csr_pair(ctypes.Structure):
    _fields_ = [
        ("K", ctypes.c_longlong),
        ("F_rowptr", ctypes.c_void_p),
        ("F_col", ctypes.c_void_p),
        ("F_val", ctypes.c_void_p),
        ("S_rowptr", ctypes.c_void_p),
        ("S_col", ctypes.c_void_p),
        ("S_val", ctypes.c_void_p),
    ]


class dm_options(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("precision", ctypes.c_int),
        ("block_width", ctypes.c_int),
        ("spin", ctypes.c_double),
        ("lanczos_steps", ctypes.c_int),
        ("bound_margin", ctypes.c_double),
        ("seed", ctypes.c_ulonglong),
    ]


_lib = None
_P = ctypes.c_void_p
_D = ctypes.c_double
_I = ctypes.c_int
_LL = ctypes.c_longlong


def load(path: str = LIB_PATH):
    """Load libdm.so (once) and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: build it with python -m paper_2108_13478_amd.build")
    # PyTorch ships its own HIP runtime with the same soname (libamdhip64.so.7)
    # as the one libdm.so links.  Loading torch first makes libdm bind to that
    # runtime, so torch tensors, torch streams and libdm share one runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    sig = {
        "dm_default_options": (None, [_P]),
        "dm_init": (_I, [_P, _P]),
        "dm_destroy": (None, [_P]),
        "dm_last_error": (ctypes.c_char_p, [_P]),
        "dm_set_fock": (_I, [_P, _LL, _P, _P, _P, _P, _P, _P, _I]),
        "dm_get_bounds": (_I, [_P, _P, _P]),
        "dm_set_bounds": (_I, [_P, _D, _D]),
        "dm_set_precision": (_I, [_P, _I]),
        "dm_get_operator": (_I, [_P, _I, _P]),
        "dm_chebyshev_block": (_I, [_P, _P, _LL, _I, _D, _D, _P]),
        "dm_chebyshev_block_multi": (_I, [_P, _P, _LL, _I, _I, _P, _P, _P]),
        "dm_chebyshev_block_noalloc": (_I, [_P, _P, _LL, _I, _D, _D, _P, _P]),
        "dm_dos": (_I, [_P, _I, _I, _P, _D, _P]),
        "dm_set_operator_form": (_I, [_P, _I]),
        "dm_set_factored_options": (_I, [_P, _D, _I, _D, _I]),
        "dm_solve_overlap": (_I, [_P, _P, _LL, _P]),
        "dm_get_preconditioner": (_I, [_P, _P, _P, _P, _P]),
        "dm_cg_stats": (_I, [_P, _P, _P, _P]),
        "dm_cg_timing": (_I, [_P, _I, _P, _P]),
        "dm_set_fock_orthonormal": (_I, [_P, _LL, _P, _P, _P]),
        "dm_density_on_grid": (_I, [_P, _LL, _P, _P, _P, _D, _P, _D, _P, _LL, _P, _P]),
        "dm_trace": (_I, [_P, _D, _D, _P, _P]),
        "dm_solve_mu": (_I, [_P, _D, _D, _D, _P]),
        "dm_moments": (_I, [_P, _P, _I, _P]),
        "dm_reset_moments": (_I, [_P]),
        "dm_stoch_moments": (_I, [_P, _I, _I, _P, _P]),
        "dm_autotune": (_I, [_P, _LL, _I, _P, _P, _P, _P]),
        "dm_set_pass_shape": (_I, [_P, _I, _I]),
        "dm_num_tile_shapes": (_I, []),
        "dm_tile_shape": (_I, [_I, _P, _P, _P]),
        "dm_batch_set_focks": (_I, [_P, _I, _P]),
        "dm_batch_get_bounds": (_I, [_P, _I, _P, _P]),
        "dm_batch_run": (_I, [_P, _I, _D, _P, _D, _P, _P, _I]),
        "dm_batch_autotune": (_I, [_P, _I, _P, _P, _P]),
        "dm_batch_stoch_moments": (_I, [_P, _I, _I, _P, _P]),
        "dm_cheb_order": (_I, [_P, _D, _D, _D, _D, _D, _I, _P]),
        "dm_mlp_init": (_I, [_P, _I, _P, ctypes.c_ulonglong]),
        "dm_mlp_num_params": (_I, [_P, _P]),
        "dm_mlp_get_params": (_I, [_P, _P]),
        "dm_mlp_set_params": (_I, [_P, _P]),
        "dm_mlp_forward": (_I, [_P, _P, _I, _P]),
        "dm_mlp_gradients": (_I, [_P, _P, _P, _I, _P, _P]),
        "dm_mlp_train_step": (_I, [_P, _P, _P, _I, ctypes.c_float, _P]),
        "dm_mlp_features": (_I, [_P, _P, _I, _D, _D, _D, _D, _LL, _P]),
        "dm_mlp_predict": (_I, [_P, _P, _I, _D, _D, _I, _P, _P]),
        "dm_cheb_order_rule": (_I, [_D, _D, _D, _I, _I, _P]),
        "dm_set_moments_precision": (_I, [_P, _I]),
        "dm_combine_sets": (_I, [_P, _I, _P, _D, _I, _D, _LL, _P, _P, _P]),
        "dm_mlp_encode_targets": (_I, [_D, _D, _D, _I, _P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(x, dtype):
    """(pointer, keepalive) for a torch tensor or array-like of the given numpy dtype."""
    if x is None:
        return None, None
    try:
        import torch
        if isinstance(x, torch.Tensor):
            want = {np.float64: torch.float64, np.int64: torch.int64, np.int32: torch.int32}[dtype]
            if x.dtype != want or not x.is_contiguous():
                raise TypeError(f"tensor must be contiguous {want}")
            return ctypes.c_void_p(x.data_ptr()), x
    except ImportError:
        pass
    a = np.ascontiguousarray(x, dtype=dtype)
    return ctypes.c_void_p(a.ctypes.data), a


def tile_shapes():
    """[(rows, cols, split)] of every compiled recursion tile shape, by index."""
    lib = load()
    out = []
    for cfg in range(lib.dm_num_tile_shapes()):
        r, c, sp = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        if lib.dm_tile_shape(cfg, ctypes.byref(r), ctypes.byref(c), ctypes.byref(sp)) != DM_OK:
            raise DMError(DM_E_ARG, f"tile shape {cfg}")
        out.append((r.value, c.value, sp.value))
    return out


def dm_cheb_order_rule(emin, emax, beta, min_order=16, max_order=1 << 16):
    """The paper's expansion length N_C ~ 2 dE beta, clamped (dm_cheb_order_rule)."""
    lib = load()
    o = ctypes.c_int()
    st = lib.dm_cheb_order_rule(float(emin), float(emax), float(beta), int(min_order), int(max_order),
                                ctypes.byref(o))
    if st != DM_OK:
        raise DMError(st, "dm_cheb_order_rule: bad arguments")
    return o.value


def dm_mlp_encode_targets(mu, emin, emax, order):
    """Predictor targets (2 float32) for (mu, order) on [emin, emax]."""
    lib = load()
    y = np.zeros(2, dtype=np.float32)
    st = lib.dm_mlp_encode_targets(float(mu), float(emin), float(emax), int(order),
                                   ctypes.c_void_p(y.ctypes.data))
    if st != DM_OK:
        raise DMError(st, "dm_mlp_encode_targets: bad arguments")
    return y


def _numel(x):
    n = getattr(x, "numel", None)
    return n() if callable(n) else int(np.asarray(x).size)


class Context:
    """One dm_ctx: a loaded (F, S) pair, its operator and moment accumulator."""

    def __init__(self, device=0, stream=None, precision=DM_FP64, block_width=0, spin=2.0,
                 lanczos_steps=100, bound_margin=0.01, seed=12345):
        lib = load()
        opt = dm_options()
        lib.dm_default_options(ctypes.byref(opt))
        opt.device = device
        opt.stream = stream
        opt.precision = precision
        opt.block_width = block_width
        opt.spin = spin
        opt.lanczos_steps = lanczos_steps
        opt.bound_margin = bound_margin
        opt.seed = seed
        h = ctypes.c_void_p()
        st = lib.dm_init(ctypes.byref(h), ctypes.byref(opt))
        if st != DM_OK:
            raise DMError(st, lib.dm_last_error(None).decode())
        self._lib = lib
        self.h = h
        self.K = None
        self.spin = spin

    def _check(self, st):
        if st != DM_OK:
            raise DMError(st, self._lib.dm_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self._lib.dm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- calls
    def dm_set_fock(self, K, F_rowptr, F_col, F_val, S_rowptr, S_col, S_val, atom_block=1):
        keep = [_ptr(F_rowptr, np.int64), _ptr(F_col, np.int32), _ptr(F_val, np.float64),
                _ptr(S_rowptr, np.int64), _ptr(S_col, np.int32), _ptr(S_val, np.float64)]
        self._check(self._lib.dm_set_fock(self.h, int(K), *[k[0] for k in keep], int(atom_block)))
        self.K = int(K)

    def set_cluster(self, cluster, atom_block=4):
        c = cluster
        self.dm_set_fock(c.K, c.F_rowptr, c.F_col, c.F_val, c.S_rowptr, c.S_col, c.S_val, atom_block)

    def dm_get_bounds(self):
        lo, hi = ctypes.c_double(), ctypes.c_double()
        self._check(self._lib.dm_get_bounds(self.h, ctypes.byref(lo), ctypes.byref(hi)))
        return lo.value, hi.value

    def dm_set_bounds(self, emin, emax):
        self._check(self._lib.dm_set_bounds(self.h, float(emin), float(emax)))

    def dm_get_operator(self, which):
        """K x K FP64 numpy copy of S^-1 (DM_OP_SINV) or H = S^-1 F (DM_OP_H)."""
        out = np.zeros((self.K, self.K), dtype=np.float64)  # filled column-major
        self._check(self._lib.dm_get_operator(self.h, int(which), ctypes.c_void_p(out.ctypes.data)))
        return out.T

    def dm_set_precision(self, precision):
        self._check(self._lib.dm_set_precision(self.h, int(precision)))

    def dm_chebyshev_block(self, cols, order, mu, beta, P_out=None):
        """P_out: None (moments only) or a contiguous float64 buffer of
        ncols * K elements (torch tensor on the GPU or host, or numpy) that
        receives P column-major (column j contiguous)."""
        cp, ck = _ptr(cols, np.int64)
        n = int(len(cols))
        pp, pk = _ptr(P_out, np.float64) if P_out is not None else (None, None)
        if P_out is not None and _numel(pk) < n * self.K:
            raise ValueError("P_out too small")
        self._check(self._lib.dm_chebyshev_block(self.h, cp, n, int(order), float(mu), float(beta), pp))
        return P_out

    def dm_chebyshev_block_noalloc(self, cols, order, mu, beta, P_out=None, m_out=None):
        """Allocation-free pass (library-owned scratch); m_out receives the
        order + 1 moments of these columns (not accumulated)."""
        c, kc = _ptr(cols, np.int64)
        p, kp = (None, None) if P_out is None else _ptr(P_out, np.float64)
        m, km = (None, None) if m_out is None else _ptr(m_out, np.float64)
        self._check(self._lib.dm_chebyshev_block_noalloc(self.h, c, _numel(cols), int(order), float(mu),
                                                         float(beta), p, m))
        if P_out is not None and kp is not P_out and not hasattr(P_out, "data_ptr"):
            np.copyto(P_out, kp.reshape(np.shape(P_out)))
        if m_out is not None and km is not m_out and not hasattr(m_out, "data_ptr"):
            np.copyto(m_out, km.reshape(np.shape(m_out)))

    def dm_combine_sets(self, mus, beta, order, mu, P_ins, P_out):
        """P_out = sum_q w_q(mu) P_ins[q] (Lagrange weights of the nodes mus);
        returns the coefficient-space error bound.  P_out None: the bound only."""
        m = np.ascontiguousarray(mus, dtype=np.float64)
        if P_out is not None and len(P_ins) != len(m):
            raise ValueError("one block per node")
        keep = [_ptr(p, np.float64) for p in P_ins] if P_out is not None else []
        arr = (ctypes.c_void_p * max(len(keep), 1))(*[k[0].value for k in keep])
        op, ok = _ptr(P_out, np.float64)
        n = _numel(P_out) if P_out is not None else 0
        bound = ctypes.c_double()
        self._check(self._lib.dm_combine_sets(self.h, len(m), ctypes.c_void_p(m.ctypes.data), float(beta), int(order),
                                              float(mu), n, arr if keep else None, op, ctypes.byref(bound)))
        if P_out is not None and ok is not P_out and not hasattr(P_out, "data_ptr"):
            np.copyto(P_out, ok.reshape(np.shape(P_out)))
        return bound.value

    def dm_chebyshev_block_multi(self, cols, order, mus, betas, P_outs=None):
        """One pass accumulating len(mus) density-matrix blocks; P_outs: None or
        a sequence of buffers (or None entries) laid out as for dm_chebyshev_block."""
        cp, ck = _ptr(cols, np.int64)
        n = int(len(cols))
        ns = len(mus)
        if len(betas) != ns or (P_outs is not None and len(P_outs) != ns):
            raise ValueError("mus, betas and P_outs must have the same length")
        mu_a = np.ascontiguousarray(mus, dtype=np.float64)
        be_a = np.ascontiguousarray(betas, dtype=np.float64)
        keep = []
        ptrs = (ctypes.c_void_p * ns)()
        for q in range(ns):
            P = None if P_outs is None else P_outs[q]
            if P is not None:
                pp, pk = _ptr(P, np.float64)
                if _numel(pk) < n * self.K:
                    raise ValueError("P_out too small")
                keep.append(pk)
                ptrs[q] = pp.value
        self._check(self._lib.dm_chebyshev_block_multi(
            self.h, cp, n, int(order), ns, ctypes.c_void_p(mu_a.ctypes.data), ctypes.c_void_p(be_a.ctypes.data),
            ptrs if P_outs is not None else None))
        return P_outs

    def dm_set_factored_options(self, cg_tol=1e-11, cg_max_iter=2000, fsai_drop=1e-5, fsai_max_per_row=192):
        self._check(self._lib.dm_set_factored_options(self.h, float(cg_tol), int(cg_max_iter), float(fsai_drop),
                                                      int(fsai_max_per_row)))

    def dm_solve_overlap(self, B):
        """X = S^-1 B for B of shape (K, n) (numpy); returns X (K, n)."""
        Bc = np.asfortranarray(np.asarray(B, dtype=np.float64).reshape(self.K, -1))
        X = np.zeros_like(Bc, order="F")
        n = Bc.shape[1]
        self._check(self._lib.dm_solve_overlap(self.h, ctypes.c_void_p(Bc.ctypes.data), n,
                                               ctypes.c_void_p(X.ctypes.data)))
        return X

    def dm_get_preconditioner(self):
        """(rowptr, col, val) of the FSAI factor G in CSR (numpy)."""
        nnz = ctypes.c_longlong()
        self._check(self._lib.dm_get_preconditioner(self.h, ctypes.byref(nnz), None, None, None))
        rp = np.zeros(self.K + 1, dtype=np.int64)
        col = np.zeros(nnz.value, dtype=np.int32)
        val = np.zeros(nnz.value, dtype=np.float64)
        self._check(self._lib.dm_get_preconditioner(self.h, None, ctypes.c_void_p(rp.ctypes.data),
                                                    ctypes.c_void_p(col.ctypes.data),
                                                    ctypes.c_void_p(val.ctypes.data)))
        return rp, col, val

    def dm_cg_stats(self):
        """(solves, iterations, max_iterations) since the last call."""
        ns, it, mx = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_int()
        self._check(self._lib.dm_cg_stats(self.h, ctypes.byref(ns), ctypes.byref(it), ctypes.byref(mx)))
        return ns.value, it.value, mx.value

    def dm_cg_timing(self, enable):
        """(launches, ms) of the timed S products since the last call; then
        switches the timing on or off."""
        n, ms = ctypes.c_longlong(), ctypes.c_double()
        self._check(self._lib.dm_cg_timing(self.h, int(enable), ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    def dm_dos(self, kind, energies, sigma=0.0):
        """Density of states at `energies` from the accumulated moments
        (DM_DOS_GAUSSIAN with width sigma, or DM_DOS_KPM)."""
        E = np.ascontiguousarray(energies, dtype=np.float64)
        out = np.zeros(E.shape[0], dtype=np.float64)
        self._check(self._lib.dm_dos(self.h, int(kind), int(E.shape[0]), ctypes.c_void_p(E.ctypes.data),
                                     float(sigma), ctypes.c_void_p(out.ctypes.data)))
        return out

    def dm_trace(self, mu, beta):
        tr, eb = ctypes.c_double(), ctypes.c_double()
        self._check(self._lib.dm_trace(self.h, float(mu), float(beta), ctypes.byref(tr), ctypes.byref(eb)))
        return tr.value, eb.value

    def dm_solve_mu(self, n_e, beta, tol=1e-8):
        mu = ctypes.c_double()
        self._check(self._lib.dm_solve_mu(self.h, float(n_e), float(beta), float(tol), ctypes.byref(mu)))
        return mu.value

    def dm_moments(self, n):
        m = np.zeros(n, dtype=np.float64)
        nd = ctypes.c_longlong()
        self._check(self._lib.dm_moments(self.h, ctypes.c_void_p(m.ctypes.data), int(n), ctypes.byref(nd)))
        return m, nd.value

    def dm_reset_moments(self):
        self._check(self._lib.dm_reset_moments(self.h))

    def dm_stoch_moments(self, n_mom, xi):
        """xi: K x n_vec probe vectors (numpy or torch); passed column-major."""
        n_vec = int(xi.shape[1])
        xt = xi.t().contiguous() if hasattr(xi, "t") else np.ascontiguousarray(np.asarray(xi).T)
        xp, xk = _ptr(xt, np.float64)
        m = np.zeros(n_mom, dtype=np.float64)
        self._check(self._lib.dm_stoch_moments(self.h, int(n_mom), n_vec, xp, ctypes.c_void_p(m.ctypes.data)))
        return m

    def dm_autotune(self, ncols, steps=5):
        """Returns (best_width, best_cfg, table) with table rows (width, cfg,
        tile_rows, tile_cols, ms_per_step, column_steps_per_s)."""
        cap = 256
        table = np.zeros((cap, 6), dtype=np.float64)
        n = ctypes.c_int(cap)
        bw, bc = ctypes.c_int(), ctypes.c_int()
        self._check(self._lib.dm_autotune(self.h, int(ncols), int(steps), ctypes.c_void_p(table.ctypes.data),
                                          ctypes.byref(n), ctypes.byref(bw), ctypes.byref(bc)))
        return bw.value, bc.value, table[:min(n.value, cap)].copy()

    def set_orthonormal(self, K, rowptr, col, val):
        """Load F of an orthonormal basis (S = I) from CSR arrays (numpy or torch)."""
        ptrs = [_ptr(rowptr, np.int64), _ptr(col, np.int32), _ptr(val, np.float64)]
        self._check(self._lib.dm_set_fock_orthonormal(self.h, int(K), *[p[0] for p in ptrs]))
        self.K = int(K)

    def dm_density_on_grid(self, centres, exponents, origin, h, dims, eta, cols, P_cols, n_out=None):
        """Accumulate the grid density of columns `cols` of P into n_out (a
        float64 array of nx*ny*nz, i fastest; created zero if None).  P_cols:
        K x ncols column-major, i.e. a (ncols, K) C-order array or tensor."""
        cen = np.ascontiguousarray(centres, dtype=np.float64)
        ex = np.ascontiguousarray(exponents, dtype=np.float64)
        org = np.ascontiguousarray(origin, dtype=np.float64)
        dm_ = np.ascontiguousarray(dims, dtype=np.int32)
        K = ex.shape[0]
        if n_out is None:
            n_out = np.zeros(int(np.prod(dm_)), dtype=np.float64)
        elif isinstance(n_out, np.ndarray) and (n_out.dtype != np.float64 or not n_out.flags.c_contiguous):
            raise TypeError("n_out must be a contiguous float64 array (it is accumulated in place)")
        cp, ck = _ptr(cols, np.int64)
        pp, pk = _ptr(P_cols, np.float64)
        npt, nk = _ptr(n_out, np.float64)
        self._check(self._lib.dm_density_on_grid(
            self.h, K, ctypes.c_void_p(cen.ctypes.data), ctypes.c_void_p(ex.ctypes.data),
            ctypes.c_void_p(org.ctypes.data), float(h), ctypes.c_void_p(dm_.ctypes.data), float(eta),
            cp, _numel(ck), pp, npt))
        return n_out

    def dm_set_operator_form(self, form):
        """DM_FORM_GENERAL or DM_FORM_SYMMETRIC, for Fock matrices loaded afterwards."""
        self._check(self._lib.dm_set_operator_form(self.h, int(form)))

    def dm_set_pass_shape(self, width, cfg):
        self._check(self._lib.dm_set_pass_shape(self.h, int(width), int(cfg)))

    # ---------------------------------------------------------------- batch
    def dm_set_moments_precision(self, precision):
        self._check(self._lib.dm_set_moments_precision(self.h, int(precision)))

    def dm_batch_set_focks(self, clusters):
        """clusters: sequence of objects with K and F_/S_ rowptr, col, val."""
        keep = []
        arr = (dm_csr_pair * len(clusters))()
        for i, c in enumerate(clusters):
            ptrs = [_ptr(c.F_rowptr, np.int64), _ptr(c.F_col, np.int32), _ptr(c.F_val, np.float64),
                    _ptr(c.S_rowptr, np.int64), _ptr(c.S_col, np.int32), _ptr(c.S_val, np.float64)]
            keep.append(ptrs)
            arr[i] = dm_csr_pair(int(c.K), *[p[0].value for p in ptrs])
        self._check(self._lib.dm_batch_set_focks(self.h, len(clusters), arr))
        self.batch_K = [int(c.K) for c in clusters]

    def dm_batch_get_bounds(self, i):
        lo, hi = ctypes.c_double(), ctypes.c_double()
        self._check(self._lib.dm_batch_get_bounds(self.h, int(i), ctypes.byref(lo), ctypes.byref(hi)))
        return lo.value, hi.value

    def dm_batch_run(self, order, beta, n_e, tol=1e-6, P_out=None, flags=0):
        """n_e: per-cluster electron counts.  P_out: None or a list of
        contiguous float64 buffers (K_c * K_c each, column-major; torch on the
        GPU or host, or numpy; entries may be None).  Returns mu per cluster."""
        n = len(self.batch_K)
        ne = np.ascontiguousarray(n_e, dtype=np.float64)
        mu = np.zeros(n, dtype=np.float64)
        keep = []
        parr = None
        if P_out is not None:
            parr = (ctypes.c_void_p * n)()
            for i, p in enumerate(P_out):
                if p is None:
                    parr[i] = None
                    continue
                pp, pk = _ptr(p, np.float64)
                if _numel(pk) < self.batch_K[i] ** 2:
                    raise ValueError("P_out buffer too small")
                keep.append(pk)
                parr[i] = pp.value
        self._check(self._lib.dm_batch_run(self.h, int(order), float(beta), ctypes.c_void_p(ne.ctypes.data),
                                           float(tol), ctypes.c_void_p(mu.ctypes.data), parr, int(flags)))
        return mu

    def dm_batch_autotune(self, steps=8):
        table = np.zeros((16, 4), dtype=np.float64)
        n = ctypes.c_int(16)
        best = ctypes.c_int()
        self._check(self._lib.dm_batch_autotune(self.h, int(steps), ctypes.c_void_p(table.ctypes.data),
                                                ctypes.byref(n), ctypes.byref(best)))
        return best.value, table[:n.value].copy()

    def dm_batch_stoch_moments(self, n_mom, xis):
        """xis: list of K_c x n_vec probe blocks (numpy); returns n x n_mom."""
        n = len(xis)
        n_vec = int(xis[0].shape[1])
        keep = [np.ascontiguousarray(np.asarray(x, dtype=np.float64).T) for x in xis]
        arr = (ctypes.c_void_p * n)(*[k.ctypes.data for k in keep])
        m = np.zeros((n, n_mom), dtype=np.float64)
        self._check(self._lib.dm_batch_stoch_moments(self.h, int(n_mom), n_vec, arr,
                                                     ctypes.c_void_p(m.ctypes.data)))
        return m

    def dm_cheb_order(self, emin, emax, mu, beta, tol, max_order):
        o = ctypes.c_int()
        self._check(self._lib.dm_cheb_order(self.h, float(emin), float(emax), float(mu), float(beta),
                                            float(tol), int(max_order), ctypes.byref(o)))
        return o.value

    # ---------------------------------------------------------------- predictor
    def dm_mlp_init(self, sizes, seed=0):
        arr = (ctypes.c_int * len(sizes))(*[int(x) for x in sizes])
        self._check(self._lib.dm_mlp_init(self.h, len(sizes) - 1, arr, int(seed)))
        self.mlp_sizes = list(sizes)

    def dm_mlp_num_params(self):
        n = ctypes.c_longlong()
        self._check(self._lib.dm_mlp_num_params(self.h, ctypes.byref(n)))
        return n.value

    def dm_mlp_get_params(self):
        out = np.zeros(self.dm_mlp_num_params(), dtype=np.float32)
        self._check(self._lib.dm_mlp_get_params(self.h, ctypes.c_void_p(out.ctypes.data)))
        return out

    def dm_mlp_set_params(self, p):
        a = np.ascontiguousarray(p, dtype=np.float32)
        self._check(self._lib.dm_mlp_set_params(self.h, ctypes.c_void_p(a.ctypes.data)))

    def dm_mlp_forward(self, X):
        xp, xk = _ptr(X, np.float32) if not hasattr(X, "data_ptr") else (ctypes.c_void_p(X.data_ptr()), X)
        B = int(X.shape[0])
        Y = np.zeros((B, self.mlp_sizes[-1]), dtype=np.float32)
        self._check(self._lib.dm_mlp_forward(self.h, xp, B, ctypes.c_void_p(Y.ctypes.data)))
        return Y

    def dm_mlp_gradients(self, X, T):
        xa = np.ascontiguousarray(X, dtype=np.float32)
        ta = np.ascontiguousarray(T, dtype=np.float32)
        loss = ctypes.c_float()
        g = np.zeros(self.dm_mlp_num_params(), dtype=np.float32)
        self._check(self._lib.dm_mlp_gradients(self.h, ctypes.c_void_p(xa.ctypes.data), ctypes.c_void_p(ta.ctypes.data),
                                               int(xa.shape[0]), ctypes.byref(loss), ctypes.c_void_p(g.ctypes.data)))
        return loss.value, g

    def dm_mlp_train_step(self, X, T, lr):
        """X, T: contiguous float32 (numpy, or torch tensors on the GPU)."""
        xp, xk = (ctypes.c_void_p(X.data_ptr()), X) if hasattr(X, "data_ptr") else _ptr(X, np.float32)
        tp, tk = (ctypes.c_void_p(T.data_ptr()), T) if hasattr(T, "data_ptr") else _ptr(T, np.float32)
        loss = ctypes.c_float()
        self._check(self._lib.dm_mlp_train_step(self.h, xp, tp, int(X.shape[0]), float(lr), ctypes.byref(loss)))
        return loss.value

    def dm_mlp_features(self, m_stoch, emin, emax, beta, n_e, K):
        m = np.ascontiguousarray(m_stoch, dtype=np.float64)
        x = np.zeros(len(m) + 4, dtype=np.float32)
        self._check(self._lib.dm_mlp_features(self.h, ctypes.c_void_p(m.ctypes.data), len(m), float(emin), float(emax),
                                              float(beta), float(n_e), int(K), ctypes.c_void_p(x.ctypes.data)))
        return x

    def dm_mlp_predict(self, m_stoch, beta, n_e, max_order=8192):
        m = np.ascontiguousarray(m_stoch, dtype=np.float64)
        mu, order = ctypes.c_double(), ctypes.c_int()
        self._check(self._lib.dm_mlp_predict(self.h, ctypes.c_void_p(m.ctypes.data), len(m), float(beta), float(n_e),
                                             int(max_order), ctypes.byref(mu), ctypes.byref(order)))
        return mu.value, order.value
