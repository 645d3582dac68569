/*
 * dm.h - C ABI of the MI355X Chebyshev density-matrix library (libdm.so).
 *
 * The library computes columns of the finite-temperature density matrix
 *     P = f_FD(S^-1 F) S^-1                                  (eq. RDM)
 * of a non-orthogonal atom-centred basis, with f_FD(e) = 1/(1+exp(beta(e-mu)))
 * (Method section, text before eq. RDM), by the Chebyshev column recursion of
 * the supplement's "Chebyshev expansion" section (eq. ChebychevExpansion):
 *     U_0 = S^-1 u_a,  U_1 = H_N U_0,  U_{l+1} = 2 H_N U_l - U_{l-1},
 *     rho_a = sum_{l<N} a_l U_l,   H_N = (S^-1 F - Ebar) / dE,
 * where u_a is the unit column vector of basis function a (eq. col-by-col).
 * Alongside P it accumulates the moments m_l = sum_a s_a^T U_l (s_a = column
 * a of S), from which the electron count N_e = g Tr[PS] (eq. Ne) and the band
 * energy g Tr[PF] (eq. <O> with O = F) follow for any mu.
 *
 * Conventions for every entry point:
 *  - Return value: a dm_status; DM_OK on success.  No C++ exception crosses
 *    the ABI: one raised inside a call (a host allocation failure) returns
 *    DM_E_OOM.  dm_last_error() gives a message for the last failure.
 *  - After DM_E_HIP the context is poisoned: every later call except
 *    dm_last_error and dm_destroy returns DM_E_STATE.
 *  - Pointers marked "host or device" may point to host memory or to device
 *    memory of the context's GPU; the library tells them apart with
 *    hipPointerGetAttributes.  The caller owns all arrays; the library copies
 *    whatever it keeps.
 *  - Dense matrices are column-major with leading dimension equal to their
 *    row count (K), FP64.
 *  - All GPU work is ordered on the context's stream.  Calls that return
 *    host scalars (dm_get_bounds, dm_trace, dm_solve_mu, dm_moments) and
 *    calls whose output is in host memory synchronise that stream before
 *    returning; other calls may return before the GPU work has finished.
 *  - A context is used by one host thread at a time.
 */
#ifndef DM_H
#define DM_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dm_ctx dm_ctx;

typedef enum {
    DM_OK = 0,
    DM_E_ARG = -1,     /* invalid argument (null pointer, size, range, NaN) */
    DM_E_STATE = -2,   /* call out of order, or context poisoned */
    DM_E_HIP = -3,     /* HIP runtime error; context poisoned */
    DM_E_OOM = -4,     /* device or host allocation failed */
    DM_E_NOTSPD = -5,  /* overlap matrix not positive definite (Cholesky) */
    DM_E_BOUNDS = -6,  /* recursion diverged: spectral bounds do not enclose */
    DM_E_NOCONV = -7   /* iteration did not reach its tolerance */
} dm_status;

/* Precision of H_N and the recursion vectors U_l.  DM_FP32_ACC64 is the
 * refined FP32 path: H_N and U_l are stored in FP32 (half the bytes of
 * FP64), every product and sum runs in FP64 (an FP32 x FP32 product is
 * exact in FP64), and U_{l+1} is rounded to FP32 once, when stored.  It
 * removes the FP32 accumulation error of DM_FP32; the rounding of H_N and
 * U_l to FP32 remains.  Not for the batch or the factored form. */
enum { DM_FP64 = 0, DM_FP32 = 1, DM_FP32_ACC64 = 2 };

typedef struct {
    int device;              /* HIP device ordinal */
    void* stream;            /* hipStream_t to order work on; NULL = library-owned stream */
    int precision;           /* DM_FP64, DM_FP32 or DM_FP32_ACC64: storage and arithmetic of H_N and U_l.
                                P and the moments are always accumulated in FP64. */
    int block_width;         /* columns advanced together per pass; 0 = library choice */
    double spin;             /* g in N_e = g Tr[PS] (eq. Ne); the paper uses 2 */
    int lanczos_steps;       /* Lanczos steps for the spectral bounds; 0 = 100 */
    double bound_margin;     /* relative widening of the Lanczos interval; <= 0 = 0.01 */
    unsigned long long seed; /* seed of the Lanczos start vector */
} dm_options;

/* Fill *opt with the defaults (device 0, library stream, FP64, spin 2). */
void dm_default_options(dm_options* opt);

/* Create a context on opt->device (opt may be NULL: defaults).  *out receives
 * the handle; it is NULL on failure.  Errors: DM_E_ARG (out NULL, bad option),
 * DM_E_HIP (no such device). */
dm_status dm_init(dm_ctx** out, const dm_options* opt);

/* Release every device buffer of the context.  NULL is a no-op. */
void dm_destroy(dm_ctx* ctx);

/* Message of the last failure on ctx ("" if none); ctx may be NULL, then the
 * message of the last failed dm_init of this thread. Valid until the next call. */
const char* dm_last_error(const dm_ctx* ctx);

/* Load the Fock matrix F and overlap S of a K-function basis (eq. FockMatrix,
 * eq. Smat) and build the recursion operator (supplement "Chebyshev
 * expansion"): S = U^T U (Cholesky), S^-1, H = S^-1 F, extreme eigenvalues of
 * H by S-inner-product Lanczos widened by bound_margin, and H_N.
 * CSR arrays (host or device): rowptr[K+1] (int64, rowptr[0] = 0), col[nnz]
 * (int32, sorted ascending within a row, in [0, K)), val[nnz] (FP64); full
 * symmetric storage.  atom_block: functions per atom (K must be a multiple),
 * 1 = no blocking.  Resets the accumulated moments.
 * Errors: DM_E_ARG (K <= 0, malformed CSR, non-finite value, asymmetric
 * pattern size), DM_E_NOTSPD (S not positive definite), DM_E_OOM, DM_E_HIP. */
dm_status dm_set_fock(dm_ctx* ctx, long long K,
                      const long long* F_rowptr, const int* F_col, const double* F_val,
                      const long long* S_rowptr, const int* S_col, const double* S_val,
                      int atom_block);

/* An orthonormal basis (S = I, e.g. an orthogonal tight-binding model or a
 * basis the caller has already orthogonalised): P = f_FD(F) (eq. RDM with
 * S = I).  Only F is given (CSR as for dm_set_fock); the library keeps F in
 * CSR (Lanczos products, re-normalisation) and builds the dense H_N directly
 * from it, with no K x K FP64 temporaries, so the operator needs K^2 x 4
 * bytes in FP32 (69 GB at K = 131072) and K^2 x 8 in FP64.  The start
 * vectors are the unit vectors u_a, the moment vectors too.  Every entry
 * point that works on a dm_set_fock operator works on this one, except
 * dm_get_operator (DM_E_STATE) and the operator form (S = I makes both forms
 * the same).  Errors: as dm_set_fock. */
dm_status dm_set_fock_orthonormal(dm_ctx* ctx, long long K, const long long* F_rowptr, const int* F_col,
                                  const double* F_val);

/* Spectral interval [Emin, Emax] used to normalise H (supplement: Emax and
 * Emin are the extreme eigenvalues of H = S^-1 F).  dm_set_bounds replaces
 * the Lanczos interval (e.g. to pin the interval in a comparison) and resets
 * the accumulated moments.  Errors: DM_E_STATE (no Fock matrix),
 * DM_E_ARG (emin >= emax, non-finite). */
dm_status dm_get_bounds(dm_ctx* ctx, double* emin, double* emax);
dm_status dm_set_bounds(dm_ctx* ctx, double emin, double emax);

/* Copy a setup product to out (host or device, K x K FP64 column-major):
 * which = DM_OP_SINV: S^-1 (the start vectors U_0 = S^-1 u_a are its columns);
 * which = DM_OP_H: H = S^-1 F (supplement "Chebyshev expansion");
 * which = DM_OP_HSYM: H~ = L F L^T, L = U^-T, S = U^T U (symmetric form only).
 * Errors: DM_E_STATE (no Fock matrix; DM_OP_HSYM of a general-form operator),
 * DM_E_ARG. */
enum { DM_OP_SINV = 0, DM_OP_H = 1, DM_OP_HSYM = 2 };
dm_status dm_get_operator(dm_ctx* ctx, int which, double* out);

/* Operator form of the recursion for the Fock matrices loaded afterwards by
 * dm_set_fock or dm_batch_set_focks (operators already loaded keep theirs):
 * DM_FORM_GENERAL (default): the recursion runs on H = S^-1 F as in the
 *   supplement's eq. ChebychevExpansion, from U_0 = S^-1 u_a;
 * DM_FORM_SYMMETRIC: with the Cholesky factor S = U^T U and L = U^-T it runs
 *   on the symmetric H~ = L F L^T (same spectrum: H = U^-1 H~ U), from
 *   V_0 = L u_a, and each pass ends with one FP64 product P u_a =
 *   L^T sum_l a_l V_l, which is the same P = f(S^-1 F) S^-1 (eq. RDM) since
 *   f(H) S^-1 = L^T f(H~) L.  T_l(H~_N) has norm <= 1, so FP32 rounding in
 *   the recursion is not amplified as with the non-normal S^-1 F.  The
 *   moments use z_a = U u_a (u_a^T S T_l(H) S^-1 u_a = (U u_a)^T T_l(H~) L u_a),
 *   so traces, mu and the DOS are unchanged; dm_stoch_moments probes H~.
 *   Costs two K x K FP64 arrays (L, U) and H~ (FP64) more, and K^3 more
 *   setup flops.  dm_batch_set_focks builds every cluster in the form set
 *   here too (dm_batch_run then ends its P pass with the L^T Q products).
 * DM_FORM_FACTORED: H = S^-1 F is never formed.  Every application
 *   H_N U = (S^-1 (F U) - Ebar U) / dE is one sparse product with F and a
 *   solve S X = F U by preconditioned conjugate gradients, the paper's own
 *   route (Methods, column-by-column evaluation; the footnote on the overlap
 *   solve), with a factorised sparse approximate inverse G (S^-1 ~ G^T G, G
 *   lower triangular on a pattern taken from S, see
 *   dm_set_factored_options) in place of the paper's incomplete Cholesky
 *   preconditioner.  F, S and G stay sparse: memory is O(nnz + K x block
 *   width) instead of O(K^2).  Runs in FP64 only (dm_chebyshev_block returns
 *   DM_E_STATE under DM_FP32).  P matches the other forms to within the
 *   solve tolerance amplified by the recursion (about 10 x cg_tol x the
 *   largest |P| entry).  The Lanczos interval is computed through the same
 *   solves, to a tolerance of at most 1e-8.  dm_stoch_moments runs the same
 *   factored recursion from the probe vectors.  Not for dm_batch_set_focks,
 *   dm_autotune, dm_set_pass_shape or dm_get_operator (DM_E_STATE).
 * Errors: DM_E_ARG (unknown form). */
enum { DM_FORM_GENERAL = 0, DM_FORM_SYMMETRIC = 1, DM_FORM_FACTORED = 2 };
dm_status dm_set_operator_form(dm_ctx* ctx, int form);

/* Factored form settings.  cg_tol: a column's solve stops when its
 * residual satisfies ||S x - b|| <= cg_tol ||b|| (default 1e-11);
 * cg_max_iter: iteration limit per solve (default 2000; reaching it fails
 * the call with DM_E_NOCONV).  fsai_drop, fsai_max_per_row: pattern of row
 * i of G, the lower entries j < i of S with |S_ij| >= fsai_drop
 * sqrt(S_ii S_jj), at most fsai_max_per_row - 1 of them (the largest), and
 * the diagonal (defaults 1e-5 and 192); row i of G is then the solution of
 * S[J, J] g = e_i scaled so that (G S G^T)_ii = 1 (Kolotilina-Yeremin
 * factorised sparse approximate inverse).  The tolerance and limit apply
 * from the next call; the pattern from the next dm_set_fock.
 * Errors: DM_E_ARG (cg_tol not in (0, 1), cg_max_iter < 1, fsai_drop < 0,
 * fsai_max_per_row not in [1, 192]). */
dm_status dm_set_factored_options(dm_ctx* ctx, double cg_tol, int cg_max_iter, double fsai_drop,
                                  int fsai_max_per_row);

/* X = S^-1 B by the factored form's preconditioned conjugate gradients,
 * B and X K x nrhs column-major FP64 (host or device); each column to the
 * tolerance of dm_set_factored_options.  Errors: DM_E_STATE (no factored
 * operator loaded), DM_E_ARG, DM_E_NOCONV (iteration limit reached). */
dm_status dm_solve_overlap(dm_ctx* ctx, const double* B, long long nrhs, double* X);

/* The FSAI factor G of the loaded factored operator in CSR: *nnz (host,
 * may be NULL) receives its number of entries; rowptr (K + 1 int64),
 * col (nnz int32, ascending per row, the diagonal last) and val (nnz FP64)
 * are filled when not NULL (host or device).
 * Errors: DM_E_STATE (no factored operator loaded). */
dm_status dm_get_preconditioner(dm_ctx* ctx, long long* nnz, long long* rowptr, int* col, double* val);

/* Conjugate-gradient counters of the factored form since the last call (or
 * the last dm_set_fock): solves run, iterations summed over the solves (for
 * the 64-column group that needed most) and the largest iteration count of
 * one solve.  Any output pointer (host) may be NULL.
 * Errors: DM_E_STATE (no factored operator loaded). */
dm_status dm_cg_stats(dm_ctx* ctx, long long* solves, long long* iterations, int* max_iterations);

/* Timing of the factored form's dominant kernel, the product with S inside
 * every conjugate-gradient iteration of a block solve (single-vector solves,
 * as in the Lanczos bounds, are not timed): with enable = 1 each such launch
 * is bracketed by HIP events on the context's stream (a small cost per
 * launch).
 * Each call returns, and clears, the number of timed launches and their
 * summed duration in ms (host pointers, may be NULL) of the iterations that
 * ran since the previous call, then sets the switch to `enable`.
 * Errors: DM_E_STATE (no factored operator loaded). */
dm_status dm_cg_timing(dm_ctx* ctx, int enable, long long* launches, double* ms);

/* Switch the recursion precision (DM_FP64 / DM_FP32 / DM_FP32_ACC64) of a loaded operator;
 * resets the accumulated moments and forgets a tuned or pinned pass shape.
 * A loaded batch keeps only its H_N and so the precision it was loaded in:
 * the batch calls return DM_E_STATE until dm_batch_set_focks is called
 * again (or the precision is switched back). */
dm_status dm_set_precision(dm_ctx* ctx, int precision);

/* Columns `cols` of P_N = sum_{l<order} a_l T_l(H_N) S^-1 (eq. RDM with the
 * Chebyshev expansion of f_FD at (mu, beta); `order` = N counts the terms
 * a_0..a_{N-1}; a_l from a cosine transform of f_FD at 4N Chebyshev nodes).
 * cols[ncols] (int64, host or device): distinct basis indices in [0, K).
 * P_out (host or device, may be NULL): K x ncols column-major FP64; column j
 * is P u_{cols[j]}.  With P_out NULL only the moments are accumulated.
 * The moments m_0..m_order of the columns are added to the context's
 * accumulator (one more recursion step than P needs gives m_order); a call
 * with a different order restarts the accumulation.
 * Errors: DM_E_STATE (no Fock matrix), DM_E_ARG (order < 2, beta <= 0 or
 * non-finite, ncols < 0, bad or repeated column), DM_E_BOUNDS (the recursion
 * overflowed), DM_E_OOM, DM_E_HIP. */
dm_status dm_chebyshev_block(dm_ctx* ctx, const long long* cols, long long ncols, int order,
                             double mu, double beta, double* P_out);

/* Allocation-free variant of dm_chebyshev_block, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  One pass over all ncols columns with the
 * same kernels, tile shape and arithmetic as dm_chebyshev_block on the
 * general-form or orthonormal operator (DM_E_STATE for the symmetric and
 * factored forms).  It calls no hipMalloc or hipFree: every pass buffer
 * (U_l, U_{l-1}, the moment vectors, the P accumulator, the coefficients,
 * the moment partial sums, a copy of cols) lives in one library-owned device
 * array of DM_NOALLOC_SCRATCH_BYTES per GPU, resident from library load to
 * process end.  A call needs about Kp Bp (2 p + 16) + 8 (order + 1)
 * (Kp Bp / 16384 + 2) + 4 K bytes of it (Kp = K rounded up to 256, Bp =
 * ncols rounded up to the tile width, p = 8 in FP64 and 4 in FP32), e.g.
 * K = 4096 with 512 FP64 columns at order 1000; larger calls fail with
 * DM_E_ARG (the message states the size needed).
 * cols (int64, host or device): ncols distinct indices in [0, K), checked on
 * the device.  P_out (host or device, may be NULL): K x ncols column-major
 * FP64.  m_out (host or device, may be NULL): the order + 1 moments of these
 * columns; they are NOT added to the context's accumulator (dm_trace and
 * dm_solve_mu do not see them).  The array is shared by every call on one
 * GPU and keeps the last call's contents; calls that overlap in time on one
 * GPU (other threads, other streams) race and must not be issued.
 * Synchronises the context's stream before returning.
 * Errors: DM_E_STATE (no operator, other form, array unavailable), DM_E_ARG
 * (as dm_chebyshev_block, or the call does not fit the array), DM_E_BOUNDS,
 * DM_E_HIP. */
#define DM_NOALLOC_SCRATCH_BYTES (128ull << 20)
dm_status dm_chebyshev_block_noalloc(dm_ctx* ctx, const long long* cols, long long ncols, int order,
                                     double mu, double beta, double* P_out, double* m_out);

/* Blocks of one multi-set pass combined at another chemical potential: the
 * expansion coefficients a_l(T, mu) are smooth in mu (supplement "Chebyshev
 * expansion") while the recursion vectors do not depend on it, so blocks
 * P_q accumulated by dm_chebyshev_block_multi at nodes mu_q (same order and
 * beta) give P at mu as P_out = sum_q w_q P_q, w_q the Lagrange weights of
 * the nodes at mu.  *bound (host, may be NULL) receives
 * sum_{l<order} |a_l(mu) - sum_q w_q a_l(mu_q)|, the largest error of the
 * combined polynomial against p_N(.; mu, beta) on the loaded operator's
 * interval (in the symmetric form P's error is at most bound x
 * max_a (S^-1)_aa).  Used with a predicted mu: one pass with nodes around
 * the prediction, mu from the pass's exact moments, then this call instead
 * of a second pass.  P_in: host array of n_sets pointers (host or device,
 * n FP64 each); P_out: host or device, n FP64; with n = 0 only *bound is
 * computed and P_in, P_out may be NULL (to choose nodes before a pass).
 * Errors: DM_E_STATE (no operator loaded), DM_E_ARG (n_sets outside
 * [1, DM_MAX_SETS], repeated or non-finite nodes, order < 2, beta <= 0). */
dm_status dm_combine_sets(dm_ctx* ctx, int n_sets, const double* mus, double beta, int order, double mu,
                          long long n, const double* const* P_in, double* P_out, double* bound);

/* From the accumulated moments (exact once every column 0..K-1 has been
 * processed once): tr_PS = Tr[P_N S] = sum_l a_l m_l (eq. Ne without the spin
 * factor) and e_band = g Tr[P_N F] = g sum_l a_l (Ebar m_l + dE (m_{l+1} +
 * m_|l-1|)/2) (eq. <O>), with a_l the coefficients at (mu, beta) and the
 * accumulated order.  Either output pointer (host) may be NULL.
 * Errors: DM_E_STATE (no moments), DM_E_ARG. */
dm_status dm_trace(dm_ctx* ctx, double mu, double beta, double* tr_PS, double* e_band);

/* One recursion pass over `cols` that accumulates n_sets density-matrix
 * blocks, block q with the coefficients a_l(mu[q], beta[q]) (the supplement's
 * a_l(T, mu) depend on temperature and chemical potential; the recursion
 * vectors T_l(H_N) S^-1 u_a do not, so every set shares them).  mu, beta:
 * host arrays of n_sets values (1 <= n_sets <= DM_MAX_SETS); P_out: host
 * array of n_sets pointers (host or device, each K x ncols column-major
 * FP64 as for dm_chebyshev_block, any may be NULL; P_out itself may be
 * NULL).  Block q equals dm_chebyshev_block with (mu[q], beta[q]) bit for
 * bit; the moments are accumulated once.  Each extra set adds one FP64 read
 * and write of the block per step.  Errors as dm_chebyshev_block, and
 * DM_E_ARG for n_sets out of range or NULL mu / beta. */
enum { DM_MAX_SETS = 16 };
dm_status dm_chebyshev_block_multi(dm_ctx* ctx, const long long* cols, long long ncols, int order,
                                   int n_sets, const double* mu, const double* beta,
                                   double* const* P_out);

/* Density of states from the accumulated moments (those of all K columns
 * give the DOS of H), at n energies (host or device in, host or device
 * out, n values each):
 * kind DM_DOS_GAUSSIAN: g sum_n G_sigma(E - e_n), the broadened DOS of the
 *   paper's DOS comparison figure (g the spin option, G_sigma a normalised
 *   Gaussian, sigma > 0), with the Gaussian expanded in the same N terms and
 *   4N-node cosine transform as f_FD: g sum_k w_k G_sigma(E - Ebar - dE
 *   cos theta_k), w_k the trace quadrature weights of the moments.  Accurate
 *   when N >> dE / sigma;
 * kind DM_DOS_KPM: the kernel-polynomial estimate with the Jackson kernel
 *   g_l (Weisse et al., Rev. Mod. Phys. 78, 275 (2006)): g [g_0 m_0 + 2
 *   sum_{0<l<N} g_l m_l T_l(x)] / (pi dE sqrt(1 - x^2)), x = (E - Ebar)/dE,
 *   zero outside the spectral interval (sigma ignored).  Non-negative,
 *   integrates to g K, resolution about pi dE / N.
 * Errors: DM_E_STATE (no moments), DM_E_ARG (n < 0, NULL arrays with n > 0,
 * unknown kind, sigma <= 0 for DM_DOS_GAUSSIAN). */
enum { DM_DOS_GAUSSIAN = 0, DM_DOS_KPM = 1 };
dm_status dm_dos(dm_ctx* ctx, int kind, int n, const double* energies, double sigma, double* dos);

/* Electron density on a uniform grid from columns of P (Method, eq.
 * ElectronDensity): n(r_g) += sum_j 2 phi_a(r_g) sum_b phi_b(r_g) P_cols[b, j],
 * a = cols[j], so calls over disjoint column shares add up to the density of
 * eq. density (the paper's reduce over processors).  The basis is K
 * normalised s-type Gaussians (2a/pi)^{3/4} exp(-a |r - R|^2): centres (host,
 * K x 3 row-major) and exponents (host, K), in the order of F and S; each is
 * zero outside the cube of half-width L = d / sqrt(a) around its centre, the
 * grid window of eq. WindowLength that keeps the fraction 1 - eta of the
 * function's charge, c(d, 0) = erf(d) = 1 - eta (0 < eta < 1; d = 3.459 at
 * eta = 1e-6).  Grid: r_g = origin (host,
 * 3) + h (i, j, k), dims (host, 3) = (nx, ny, nz), flattened index
 * g = i + nx (j + ny k).  cols (int64, host or device, ncols distinct
 * indices); P_cols (host or device, K x ncols column-major FP64, as written
 * by dm_chebyshev_block); n_out (host or device, nx ny nz FP64) is
 * accumulated.  Independent of any loaded Fock matrix.  Needs device
 * memory for two copies of P_cols (the second with its rows in the
 * library's spatial order of the functions), the grid and the per-cell
 * function lists; the context keeps them until dm_destroy, and a call whose
 * centres, exponents, origin, h, dims, eta and columns equal those of its
 * previous call reuses the lists (they do not depend on P) and only stages P
 * and n.  The result does not depend on timing or on earlier calls.
 * Errors: DM_E_ARG (bad sizes, exponents <= 0, non-finite centres, h <= 0,
 * eta outside (0, 1), bad or repeated columns), DM_E_OOM, DM_E_HIP. */
dm_status dm_density_on_grid(dm_ctx* ctx, long long K, const double* centres, const double* exponents,
                             const double* origin, double h, const int* dims, double eta,
                             const long long* cols, long long ncols, const double* P_cols, double* n_out);

/* Bisection on [Emin, Emax] for mu with g Tr[P_N(mu) S] = n_e from the
 * accumulated moments (the paper adjusts mu to reproduce N_e through eq. Ne;
 * the method is not stated).  Stops when |g Tr - n_e| <= tol or the bracket
 * reaches rounding level (then DM_E_NOCONV, *mu still set to the last
 * midpoint).  Errors: DM_E_STATE (no moments), DM_E_ARG. */
dm_status dm_solve_mu(dm_ctx* ctx, double n_e, double beta, double tol, double* mu);

/* Copy up to n accumulated moments to m (host) and the number of columns
 * they cover to *ncols_done (either may be NULL); n may exceed order + 1,
 * the rest is zero-filled. */
dm_status dm_moments(dm_ctx* ctx, double* m, int n, long long* ncols_done);
dm_status dm_reset_moments(dm_ctx* ctx);

/* Pick the pass width and tile shape of the recursion for this operator and
 * precision by timing `steps` recursion steps of every candidate (widths 32,
 * 64, 128, 256 columns, capped at max(ncols, 32), plus ncols rounded up to
 * 128 (at most 16384) when that is wider; every tile shape that fits the
 * width and the operator, split-reduction shapes up to 512 columns).  The
 * fastest in columns x steps per second is kept in the context and used by
 * dm_chebyshev_block while the block_width option is 0.  table (host, may
 * be NULL) receives up to *ntable rows of (width, tile config, tile rows,
 * tile cols, ms per step, column-steps per second); *ntable returns the
 * number of candidates.  dm_set_fock and dm_set_precision forget the
 * choice.  Errors: DM_E_STATE (no Fock matrix), DM_E_ARG (ncols < 1,
 * steps < 1). */
dm_status dm_autotune(dm_ctx* ctx, long long ncols, int steps, double* table, int* ntable,
                      int* best_width, int* best_cfg);

/* Pin the pass width (columns advanced together, >= 1; a pass is padded to
 * the shape's column tile) and tile shape (an index below
 * dm_num_tile_shapes()) instead of timing them; used by dm_chebyshev_block
 * while the block_width option is 0.  dm_set_fock and dm_set_precision
 * forget the choice.  Errors: DM_E_STATE (no Fock matrix), DM_E_ARG
 * (width < 1, unknown shape, or a shape that does not fit the loaded
 * operator's padded dimension, this width or the current precision). */
dm_status dm_set_pass_shape(dm_ctx* ctx, int width, int cfg);

/* Number of compiled recursion tile shapes, and the rows and columns of one
 * workgroup tile and the number of reduction chunks of shape cfg (split > 1:
 * the recursion step runs as chunked partial products plus a combine kernel
 * that applies the epilogue).  Host outputs may be NULL.
 * Errors: DM_E_ARG (cfg out of range). */
int dm_num_tile_shapes(void);
dm_status dm_tile_shape(int cfg, int* rows, int* cols, int* split);

/* ---------------------------------------------------------------- batch
 * Many independent clusters on one GPU.  Not in the paper, which splits the
 * unit vectors u_a of one system over processors (parallelisation
 * section); here each cluster is a separate problem with its own F, S and
 * mu, and uneven clusters share one persistent launch. */
typedef struct {
    long long K;
    const long long* F_rowptr;
    const int* F_col;
    const double* F_val;
    const long long* S_rowptr;
    const int* S_col;
    const double* S_val;
} dm_csr_pair;

/* Load n clusters (CSR as in dm_set_fock, host or device pointers); each gets
 * its own operator setup and Lanczos interval in the context's precision.
 * Replaces any previous batch; independent of the single operator of
 * dm_set_fock.  Errors: as dm_set_fock (the message names the cluster). */
dm_status dm_batch_set_focks(dm_ctx* ctx, int n, const dm_csr_pair* clusters);

/* Lanczos interval [Emin, Emax] of batch cluster i. */
dm_status dm_batch_get_bounds(dm_ctx* ctx, int i, double* emin, double* emax);

/* flags of dm_batch_run: launch without the graph; stop after the moments
 * pass and the mu bisection (no P pass, P_out ignored) */
enum { DM_BATCH_EAGER = 1, DM_BATCH_MOMENTS_ONLY = 2 };

/* Stochastic moments (as dm_stoch_moments) of every batch cluster: xi[c] is
 * cluster c's K_c x n_vec probe block (host or device, column-major);
 * m_out (host) receives n x n_mom values, cluster-major. */
dm_status dm_batch_stoch_moments(dm_ctx* ctx, int n_mom, int n_vec, const double* const* xi,
                                 double* m_out);

/* Precision of the moments pass of dm_batch_run (and so of each cluster's
 * mu) for batches loaded afterwards: -1 (default) = the recursion
 * precision; DM_FP64 under an FP32 recursion keeps an FP64 H_N of every
 * cluster beside the FP32 one (three times the FP32 operator memory), runs
 * the moments pass in FP64 and only the P pass in FP32.  The FP32 rounding
 * of H_N shifts the trace Tr[P_N S] by far more than an electron-count
 * tolerance of 1e-6 (hundredths of an electron at K ~ 4000 with spectra of
 * +-1000 hartree), so a mu that must reproduce N_e to such a tolerance
 * needs FP64 moments.  DM_FP32 under an FP64 recursion is the same as -1.
 * Errors: DM_E_ARG (other value). */
dm_status dm_set_moments_precision(dm_ctx* ctx, int precision);

/* Full density matrices of every cluster: first a moments-only pass over all
 * columns of all clusters (one persistent launch of exactly the resident
 * workgroups, in gangs of four: a gang runs all order steps of one
 * (cluster, column block) item of a large cluster with its members
 * splitting the row tiles and meeting after each step, or four items of
 * small clusters side by side; items dealt to gangs longest first), then
 * per cluster mu_c by bisection with g Tr[P_c S_c] =
 * n_e[c] (tolerance tol) from those moments, the coefficients at mu_c, and a
 * second persistent launch that accumulates P_c.  The whole sequence is
 * captured once in a hipGraph and replayed while (order, beta, n_e, tol,
 * precision, tile shape) stay the same; flags = DM_BATCH_EAGER launches it
 * without the graph.  n_e: host, n values.  mu_out: host, n values or NULL.
 * P_out: NULL or host array of n pointers (each host or device memory, K_c x
 * K_c column-major FP64, or NULL to skip that cluster).
 * Errors: DM_E_STATE (no batch; or a gang member was not resident, so a
 * step barrier gave up after 2^20 polls and the results are void; the
 * environment variable DM_BATCH_BARRIER_POLLS sets another limit, read when
 * the launch sequence is built: at every eager run, at capture for the
 * graph), DM_E_ARG, DM_E_BOUNDS, DM_E_NOCONV (a bisection stopped at
 * rounding level before tol; mu_out still filled). */
dm_status dm_batch_run(dm_ctx* ctx, int order, double beta, const double* n_e, double tol,
                       double* mu_out, double* const* P_out, int flags);

/* Tile shape of the batch kernel: time `steps` recursion steps of the
 * moments pass for each candidate shape on the loaded batch and keep the
 * fastest (shapes with two register buffers or three k-slabs in flight,
 * 128 x 32 .. 128 x 128; cfg is the shape's index as for dm_tile_shape).
 * table (host, may be NULL) receives up to *ntable rows of (cfg, tile rows,
 * tile cols, ms); *ntable returns the number of candidates. */
dm_status dm_batch_autotune(dm_ctx* ctx, int steps, double* table, int* ntable, int* best_cfg);

/* Smallest expansion order N <= max_order whose coefficient tail
 * sum_{l >= N} |a_l| (coefficients of f_FD(.; mu, beta) on [emin, emax],
 * supplement "Chebyshev expansion") is at most tol; bounds the error of
 * the truncated polynomial on the interval.  *order = max_order + 1 when even
 * max_order terms do not reach tol.  No operator needs to be loaded. */
dm_status dm_cheb_order(dm_ctx* ctx, double emin, double emax, double mu, double beta, double tol,
                        int max_order, int* order);

/* The paper's expansion-length rule N_C ~ 2 dE beta, dE = (emax - emin)/2
 * (supplement "Chebyshev expansion"): *order = ceil(2 dE beta) clamped to
 * [min_order, max_order].  Host arithmetic only; no context.
 * Errors: DM_E_ARG (emax <= emin, beta <= 0, non-finite, min_order < 2,
 * max_order < min_order, order NULL). */
dm_status dm_cheb_order_rule(double emin, double emax, double beta, int min_order, int max_order,
                             int* order);

/* ---------------------------------------------------------------- predictor
 * A small multilayer perceptron: n_layers affine maps sizes[j] -> sizes[j+1]
 * with tanh between them and a linear output, FP32 weights, mean-squared
 * error, Adam (b1 0.9, b2 0.999, eps 1e-8).  Weights W_j (sizes[j+1] x
 * sizes[j], row-major) and biases b_j are stored flat as W_0, b_0, W_1, ...
 * Inputs X and targets T are row-major (batch x features), host or device. */
dm_status dm_mlp_init(dm_ctx* ctx, int n_layers, const int* sizes, unsigned long long seed);
dm_status dm_mlp_num_params(dm_ctx* ctx, long long* n);
dm_status dm_mlp_get_params(dm_ctx* ctx, float* out);
dm_status dm_mlp_set_params(dm_ctx* ctx, const float* in);
dm_status dm_mlp_forward(dm_ctx* ctx, const float* X, int batch, float* Y);
/* loss = mean (Y - T)^2 and its gradient with respect to every parameter
 * (layout of the parameters); either output may be NULL */
dm_status dm_mlp_gradients(dm_ctx* ctx, const float* X, const float* T, int batch, float* loss,
                           float* grads);
dm_status dm_mlp_train_step(dm_ctx* ctx, const float* X, const float* T, int batch, float lr,
                            float* loss);
/* Input row for one problem from n_mom stochastic moments m~ (host or device):
 * x = (m~_l / K for l < n_mom, Ebar/dE, log10 dE, log10(beta dE)/4,
 *      4 n_e/(g K) - 2), n_mom + 4 floats (host or device). */
dm_status dm_mlp_features(dm_ctx* ctx, const double* m_stoch, int n_mom, double emin, double emax,
                          double beta, double n_e, long long K, float* x);
/* Training targets of the predictor, the inverse of dm_mlp_predict's
 * decoding: y[0] = 10 (mu - Ebar)/dE, y[1] = log2(order)/10 - 1 on the
 * interval [emin, emax] (host, 2 floats).  No context.
 * Errors: DM_E_ARG (emax <= emin, order < 1, non-finite, y NULL). */
dm_status dm_mlp_encode_targets(double mu, double emin, double emax, int order, float* y);

/* mu and expansion order for the loaded operator from its stochastic
 * moments: features as dm_mlp_features with the operator's interval, one
 * forward pass (network n_mom + 4 -> ... -> 2), decoded as
 * mu = Ebar + dE y_0 / 10 and order = round(2^(10 (y_1 + 1))), clamped to
 * [16, max_order]. */
dm_status dm_mlp_predict(dm_ctx* ctx, const double* m_stoch, int n_mom, double beta, double n_e,
                         int max_order, double* mu, int* order);

/* Stochastic moments (1/n_vec) sum_s xi_s^T T_l(H_N) xi_s, l < n_mom, with
 * caller-supplied probe vectors xi (host or device, K x n_vec column-major
 * FP64, e.g. independent +-1 entries).  m_out: host, n_mom FP64.
 * Does not touch the accumulated moments.  In the factored form every step
 * is one solve with S (DM_E_NOCONV when one reaches the iteration limit). */
dm_status dm_stoch_moments(dm_ctx* ctx, int n_mom, int n_vec, const double* xi, double* m_out);

#ifdef __cplusplus
}
#endif
#endif /* DM_H */
