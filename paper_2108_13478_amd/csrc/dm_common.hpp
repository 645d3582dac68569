// Internal declarations shared by the HIP kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dm {

// Operator and column dimensions are padded to these multiples so that the
// matrix kernels run without edge checks.  Padding rows/columns of the
// operator are zero, padding columns of a block start at zero and stay zero.
constexpr int kRowPad = 256;
constexpr int kColPad = 128;
// Block size of the blocked Cholesky and triangular inverse.
constexpr int kNb = 64;

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// ----------------------------------------------------------------- launches
// All launch wrappers return the hipError_t of the launch.

// C = alpha A B + beta C, every matrix column-major (A: M x Kred, B: Kred x
// N); a_upper: A is upper triangular (a row tile's sum starts at its first
// row).  M, N multiples of 64, Kred of 32.
hipError_t gemm_nn_f64(int M, int N, int Kred, double alpha, const double* A, long lda, const double* B,
                       long ldb, double beta, double* C, long ldc, bool a_upper, hipStream_t s);
// C[m + n*ldc] = alpha * sum_k A[m*lda + k] * B[n*ldb + k] + beta * C[...]
// M, N multiples of 64, Kred multiple of 32, operands FP64.  With
// upper_only, output tiles entirely below the diagonal (m0 >= n0 + tile) are
// skipped (used where only the upper triangle of a symmetric result is read).
// a_upper_row0 >= 0: column m of A is zero below row a_upper_row0 + m (an
// upper triangular matrix whose columns from a_upper_row0 on are C's rows),
// so a row tile's sum stops after its last row; -1: no such structure.
hipError_t gemm_tn_f64(int M, int N, int Kred, double alpha, const double* A, long lda,
                       const double* B, long ldb, double beta, double* C, long ldc,
                       bool upper_only, hipStream_t s, int a_upper_row0 = -1);

// One step of the Chebyshev column recursion with the fused epilogue:
//   Unext = alpha * (HN * Ucur) - (has_prev ? Uprev : 0)      (storage T)
//   P_j  += coef[j * cstride + l] * Unext, j < nsets          (FP64, P_j = P + j * pstride)
//   partial[l * ntiles + tile] = sum over the tile of Z .* Unext (FP64)
// HN: Kp x Kp, row-major (row m contiguous); U*, P, Z: Kp x Bp column-major
// (ld = Kp).  Unext may alias Uprev.  `cfg` selects the tile shape
// (see cheb_tile_configs); Bp must be a multiple of that shape's column tile.
// Split-reduction shapes (cheb_cfg_split(cfg) > 1) first write one partial
// product per reduction chunk into `work` (cheb_work_bytes(Kp, Bp, cfg,
// precision) bytes), then a second kernel sums the chunks in fixed order and
// applies the epilogue; `ntiles` is then the second kernel's workgroup count.
struct ChebStepArgs {
    int Kp, Bp;
    const void* HN;
    const void* Ucur;
    const void* Uprev;
    void* Unext;
    double alpha;
    int has_prev;
    const double* coef;
    int l;
    double* P;
    const double* Z;
    double* partial;
    void* work;
    int nsets;          // coefficient sets / P blocks accumulated in one pass (>= 1)
    int cstride;        // distance between coefficient sets
    long long pstride;  // distance between P blocks
};
int cheb_num_tile_configs();
bool cheb_cfg_supports(int cfg, int precision);
// The shape runs on this operator size and pass width (divisibility of the
// reduction chunks, width limit of the split shapes).
bool cheb_cfg_fits(int cfg, int precision, int Kp, int Bp);
int cheb_cfg_split(int cfg);
size_t cheb_work_bytes(int Kp, int Bp, int cfg, int precision);
int cheb_tile_cols(int cfg);
int cheb_tile_rows(int cfg);
hipError_t cheb_step_f64(const ChebStepArgs& a, int cfg, hipStream_t s);
hipError_t cheb_step_f32(const ChebStepArgs& a, int cfg, hipStream_t s);
// One recursion step in precision 0 (FP64), 1 (FP32) or 2 (FP32 storage,
// FP64 arithmetic).
hipError_t cheb_step(const ChebStepArgs& a, int cfg, int precision, hipStream_t s);
int cheb_num_tiles(int Kp, int Bp, int cfg);

// Persistent batch recursion.  Each workgroup repeatedly takes the next work
// item (cluster, column block) from an atomic counter and runs all `order`
// steps of that block by itself (row tile after row tile, one workgroup
// barrier between steps), so no workgroup ever waits for another.  Items
// are listed longest first.  Per cluster: U_a holds U_0 on entry; U_a, U_b
// alternate (U_{l+1} overwrites U_{l-1}); with_P adds coef[l] U_l to P;
// partial[l * nblocks + block] receives the block's moment sum of step l.
struct BatchCluster {
    int Kp, Bp, nblocks;
    int Kt;  // K rounded up to 128: the rows and reduction length that carry data
             // (rows Kt..Kp-1 of H_N and of every U_l are zero)
    const void* HN;
    void* Ua;
    void* Ub;
    double* P;
    const double* Z;
    const double* coef;
    double* partial;
};
struct BatchItem {
    int cluster, block;
};
// Workgroups of the batch kernel form gangs of kGang.  A gang works through
// its list of rounds; a round is either one item whose row tiles the gang
// shares (split = 1: member m takes row tiles m, m + kGang, ..., and the
// gang meets at a barrier after every step), or up to kGang items of which
// member m takes item m alone.
constexpr int kGang = 4;
struct BatchRound {
    int split;
    int n;  // items in the round (1 when split)
    BatchItem item[kGang];
};
struct BatchArgs {
    const BatchCluster* clusters;
    const BatchRound* rounds;
    const int* gang_start;  // rounds of gang g: [gang_start[g], gang_start[g + 1])
    int* bar;               // one barrier counter per gang, zero at launch
    int* flag;              // |= 8 when a barrier wait ran out of patience
    int order;
    int with_P;
    int gmap;               // 8: gang g's members share XCD g % 8; 1: gangs of consecutive workgroups
    int max_polls;          // a barrier wait gives up after this many polls
};
hipError_t cheb_batch(const BatchArgs& a, int cfg, int precision, int grid, hipStream_t s);
// Workgroups of tile shape cfg that fit on one CU at once.
int cheb_batch_occupancy(int cfg, int precision);
// The i-th tile shape the batch kernel is built for (an index into the
// recursion shapes), or -1 when i is out of range or the shape is not built
// for this precision; i < cheb_batch_num_cfgs().
int cheb_batch_num_cfgs();
int cheb_batch_cfg(int i, int precision);

// Chebyshev coefficients with mu read from device memory (mu_dev[0]).
hipError_t cheb_coefficients_devmu(int N, int M, double ebar, double de, const double* mu_dev,
                                   double beta, double* fk_scratch, double* a, hipStream_t s);

// U0[:, j] = Sinv[:, cols[j]] (rounded to T), Z[:, j] = column cols[j] of S
// (from its CSR rows; S is symmetric) or, with Zdense, Zdense[:, cols[j]],
// P_s[:, j] = coef[s * cstride] * Sinv[:, cols[j]] for s < nsets (P_s = P +
// s * pstride), partial[t] = per-tile sums of Z .* U0 for t < ntiles(start).
// Columns j >= ncols are zero.  Z must be zero on entry.  With cols NULL
// the source columns are Sinv's own columns 0 .. ncols - 1; with Zdense ==
// Z the moment vectors are taken as already in Z.  (The symmetric form
// passes its start block for Sinv and its moment vectors in Z; an
// orthonormal basis passes no Sinv: U0 and P start from the unit vectors.)
hipError_t cheb_start(int K, int Kp, int Bp, int ncols, const long long* cols, const double* Sinv,
                      const long long* S_rowptr, const int* S_col, const double* S_val,
                      int precision, void* U0, double* Z, double* P, const double* coef,
                      int nsets, long long pstride, int cstride, double* partial, int* ntiles_out,
                      hipStream_t s, const double* Zdense = nullptr);
// Orthonormal basis (S = I): HN = (F - ebar I) / de from F's CSR rows,
// padding zero, in FP64 (precision 0) or FP32; Kp * Kp even.
hipError_t csr_normalize(int K, int Kp, const long long* rp, const int* col, const double* val, double ebar,
                         double de, int precision, void* HN, hipStream_t s);
// dst = src^T (Kp x Kp, Kp % 32 == 0); dst = upper triangle of src.
hipError_t transpose_square(int Kp, const double* src, double* dst, hipStream_t s);
hipError_t copy_upper(int Kp, const double* src, double* dst, hipStream_t s);

// Start block from caller vectors: U0 = X (rounded to T), Z = X * zscale.
hipError_t cheb_start_vectors(int K, int Kp, int Bp, int nvec, const double* X, double zscale,
                              int precision, void* U0, double* Z, double* partial, int* ntiles_out,
                              hipStream_t s);

// mom[l] += sum_t partial[l * ntiles + t], l <= lmax, fixed summation order;
// flag[0] |= 1 if any partial sum is not finite.
hipError_t reduce_moments(int lmax, int ntiles, const double* partial, double* mom, int* flag,
                          hipStream_t s);

// a[l] for l < N: Chebyshev coefficients of f_FD(.; mu, beta) on [ebar-de, ebar+de]
// from M Chebyshev-Gauss nodes; a[N] = 0.
hipError_t cheb_coefficients(int N, int M, double ebar, double de, double mu, double beta,
                             double* fk_scratch, double* a, hipStream_t s);

// order[0] = smallest N with sum_{l >= N} |a_l| <= tol over a[0..n), or
// max_order + 1 if that N exceeds max_order
hipError_t coef_tail_order(int n, int max_order, const double* a, double tol, int* order,
                           hipStream_t s);

// Trace quadrature weights from moments m[0..N] (N terms, m[N] used for the
// band energy): w_k, v_k for k < M.
hipError_t trace_weights(int N, int M, double ebar, double de, const double* m, double* w,
                         double* v, hipStream_t s);

// Density of states at n energies E (device): broadened,
// out_i = scale sum_k w_k G_sigma(E_i - ebar - de cos theta_k) over the M
// trace weights w; kernel-polynomial (Jackson kernel) from the moments
// m[0..N), out_i = scale [g_0 m_0 + 2 sum g_l m_l T_l(x_i)] / (pi de sqrt(1-x_i^2)).
hipError_t dos_gauss(int n, const double* E, int M, double ebar, double de, double sigma, double scale,
                     const double* w, double* out, hipStream_t s);
hipError_t dos_kpm(int n, const double* E, int N, double ebar, double de, double scale, const double* m,
                   double* out, hipStream_t s);

// Single-workgroup bisection/evaluation over the weights.  With max_iter = 0
// evaluates at mu_in.  out[0] = mu, out[1] = Tr[PS], out[2] = Tr[PF] (no spin),
// out[3] = converged (1/0), out[4] = iterations.
hipError_t mu_bisect(int M, double ebar, double de, double beta, double target, double tol,
                     double lo, double hi, double mu_in, int max_iter, const double* w,
                     const double* v, double* out, hipStream_t s);

// ----------------------------------------------------------------- MLP (FP32)
hipError_t mlp_linear_fwd(int B, int nin, int nout, const float* X, const float* W, const float* b,
                          bool use_tanh, float* Y, hipStream_t s);
// G = d(mean (Y-T)^2)/dY, *loss = mean (Y-T)^2 (partial: (n+255)/256 floats)
hipError_t mlp_mse_grad(int n, const float* Y, const float* T, float* G, float* partial,
                        float* loss, hipStream_t s);
// weight/bias gradients of one layer; Gin (may be null) = input gradient
// through the tanh that produced H
hipError_t mlp_linear_bwd(int B, int nin, int nout, const float* G, const float* H, const float* W,
                          float* dW, float* db, float* Gin, hipStream_t s);
hipError_t mlp_adam(long n, float* w, const float* g, float* m, float* v, float lr, int t,
                    hipStream_t s);
hipError_t mlp_init_layer(int nin, int nout, unsigned long long seed, float* W, float* b,
                          hipStream_t s);
hipError_t mlp_features(int n_mom, const double* m, double emin, double emax, double beta,
                        double n_e, double spin, double K, float* x, hipStream_t s);

// ----------------------------------------------------------------- grid density
// Uniform grid r = (ox, oy, oz) + h (i, j, k), i < nx ..., cells of 4^3 points
// (ncx = ceil(nx / 4) ...), cell c = cx + ncx (cy + ncy cz).  Per basis
// function (K): centre, exponent, normalisation (2a/pi)^{3/4} and cube
// window half-width R.  Per cell (CSR over cells): beta_idx = functions whose
// window reaches the cell (ascending), alpha_idx / alpha_col = those whose
// column is in P (column position alpha_col).  P: K x ncols column-major with
// leading dimension ldp.  n (nx ny nz, i fastest) is accumulated.
struct GridArgs {
    int nx, ny, nz, ncx, ncy, ncz;
    double ox, oy, oz, h;
    const double *cx, *cy, *cz, *ex, *norm, *R;
    const int *beta_ptr, *beta_idx, *alpha_ptr, *alpha_idx, *alpha_col;
    const double* P;
    long long ldp;
    double* n;
};
hipError_t density_on_grid(const GridArgs& a, hipStream_t s);
// dst[j K + r] = src[j K + perm[r]]: the rows of a K x ncols column-major
// block in the order perm (new -> old)
hipError_t permute_rows(int K, long long ncols, const int* perm, const double* src, double* dst, hipStream_t s);

// ----------------------------------------------------------------- setup
// flag[0] |= 2 for a column outside [0, K), |= 4 for a repeated one; seen
// holds K ints, zero on entry
hipError_t check_columns(const long long* cols, long long ncols, long long K, int* seen, int* flag,
                         hipStream_t s);
// Weights and (device) blocks of a combination of coefficient sets.
constexpr int kMaxCombine = 16;
struct CombineSets {
    const double* p[kMaxCombine];
    double w[kMaxCombine];
};
// out[i] = sum_q w_q p_q[i], i < n
hipError_t combine_sets(long long n, int nsets, const CombineSets& cs, double* out, hipStream_t s);
// out[0] = sum_{l < N} |A_nsets[l] - sum_q w_q A_q[l]| (A: nsets + 1 rows of
// `stride` coefficients)
hipError_t interp_bound(int N, int nsets, const double* A, int stride, const CombineSets& cs, double* out,
                        hipStream_t s);
// flag[0] |= 1 when some |x_i| > lim or x_i is not finite
hipError_t flag_large(const double* x, long long n, double lim, int* flag, hipStream_t s);
// --- symmetric form built in place (symform.hip)
// A[r + c Kp] = 0 below the diagonal of the Kp x Kp column-major A
hipError_t zero_strict_lower(int Kp, double* A, hipStream_t s);
// the nb x nb block at A (ld) := upper triangle of V (nb x nb), zero below
hipError_t set_upper_block(int nb, double* A, long ld, const double* V, hipStream_t s);
// dst[c + r ldd] = src[r + c lds], r < rows, c < cols
hipError_t transpose_rect(long rows, long cols, const double* src, long lds, double* dst, long ldd, hipStream_t s);
// V[:, j] = X[cols[j], :]^T (rows of the Kp x Kp column-major X), j < ncols
hipError_t gather_rows(int Kp, int ncols, const long long* cols, const double* X, double* V, hipStream_t s);
// Y = F X, X and Y row-major K x w panels (w <= 2048), F in CSR; rows of X
// from kmax on are taken as zero
hipError_t csr_spmm_rm(int K, const long long* rp, const int* col, const double* val, int w, const double* X,
                       int kmax, double* Y, hipStream_t s);
// the same with F in groups of four rows: gp (ceil(K/4) + 1 offsets), gc
// (sorted union of a group's columns), gv (four values per listed column)
hipError_t rg4_spmm_rm(int K, const long long* gp, const int* gc, const double* gv, int w, const double* X, int kmax,
                       double* Y, hipStream_t s);
// rows row0 .. Kp - 1 of columns col0 .. col0 + w - 1 of H (Kp x Kp,
// precision 0: FP64, else FP32) := (C - ebar I) inv_de on the K x K block,
// zero padding; C is Kp x w FP64
hipError_t store_panel(int K, int Kp, int w, int col0, int row0, const double* C, double ebar, double inv_de,
                       int precision, void* H, hipStream_t s);
// upper triangle of H (Kp x Kp) := transpose of its lower triangle (the
// 32 x 32 diagonal tiles are kept)
hipError_t mirror_lower(int Kp, int precision, void* H, hipStream_t s);
// H := (H - ebar I) / de in place on the K x K block
hipError_t normalize_inplace(int K, int Kp, int precision, void* H, double ebar, double de, hipStream_t s);
// y = A x, A row-major in FP64 (precision 0) or FP32, x and y FP64
hipError_t gemv_rows_t(int K, int precision, const void* A, long lda, const double* x, double* y, hipStream_t s);
// Z[:, j] = column cols[j] of the symmetric CSR S (Z zero on entry), j < ncols
hipError_t scatter_s_columns(int Kp, int ncols, const long long* cols, const long long* rowptr, const int* col,
                             const double* val, double* Z, hipStream_t s);
hipError_t fill_f64(double* x, double v, long long n, hipStream_t s);
hipError_t fill_i32(int* x, int v, long long n, hipStream_t s);
// D (Kp x Kp col-major, zero on entry) gets the CSR matrix; padded diagonal
// entries (i >= K) get pad_diag.
hipError_t csr_to_dense(int K, int Kp, const long long* rowptr, const int* col, const double* val,
                        double pad_diag, double* D, hipStream_t s);
// Factor the nb x nb diagonal block at A (ld) as U^T U in place (upper), write
// V = U^-1 (nb x nb col-major).  info[0] = first failing global index + 1.
hipError_t potrf_diag(double* A, long ld, double* V, int* info, int kglobal, hipStream_t s);
// dst[r + c*ldd] = src[c + r*lds]^T for an nb x nb block (transpose copy).
hipError_t copy_transpose_block(const double* src, long lds, double* dst, long ldd, hipStream_t s);
// HN (row-major = HT column-major) = (HT - ebar I) / de on the K x K part,
// zero elsewhere; output FP64 or FP32.
hipError_t normalize_operator(int K, int Kp, const double* HT, double ebar, double de,
                              int precision, void* HN, hipStream_t s);
// ----------------------------------------------------------------- Lanczos
hipError_t random_vector(int K, unsigned long long seed, double* v, hipStream_t s);
hipError_t csr_spmv(int K, const long long* rowptr, const int* col, const double* val,
                    const double* x, double* y, hipStream_t s);
// y[m] = sum_k A[m*lda + k] x[k]  (rows of a row-major matrix), m < K
hipError_t gemv_rows(int K, const double* A, long lda, const double* x, double* y, hipStream_t s);
// out[i] = sum_k X[k + i*ldx] y[k] for i < n  (n dot products against columns)
hipError_t dots_cols(int K, int n, const double* X, long ldx, const double* y, double* out,
                     hipStream_t s);
// Lanczos bookkeeping kernels, scalars live in device memory.
hipError_t lanczos_normalize_start(int K, double* v, double* q, const double* vSv, hipStream_t s);
hipError_t lanczos_three_term(int K, double* w, const double* vj, const double* vjm1,
                              const double* alpha_j, const double* beta_jm1, hipStream_t s);
hipError_t lanczos_reorth(int K, int n, double* w, const double* V, long ldv, const double* c,
                          hipStream_t s);
hipError_t lanczos_next(int K, const double* w, const double* sw, const double* wSw,
                        double* beta_out, double* vnext, double* qnext, hipStream_t s);

// ----------------------------------------------------------------- factored form
// H = S^-1 F applied as a sparse product with F and a conjugate-gradient
// solve with S, preconditioned by an FSAI factor G (S^-1 ~ G^T G), all FP64.
struct FactOp;
FactOp* fact_create();
void fact_destroy(FactOp* f);
// Host CSR F and S (K x K, sorted columns).  The FSAI pattern of row i keeps
// the lower entries with |S_ij| >= drop sqrt(S_ii S_jj), at most cap - 1 of
// them (the largest), plus the diagonal; cap <= 192.  *bad_row = row + 1 of
// a row whose S[J, J] is not positive definite (0 = none).
hipError_t fact_setup(FactOp* f, int K, const long long* Frp, const int* Fcol, const double* Fval,
                      const long long* Srp, const int* Scol, const double* Sval, double drop, int cap,
                      int* bad_row, hipStream_t s);
long long fact_precond_nnz(const FactOp* f);
// G in CSR (K + 1 row pointers, columns, values); host or device pointers, any may be null.
hipError_t fact_precond_copy(const FactOp* f, long long* rp, int* col, double* val, hipStream_t s);
// X = S^-1 B for n columns (K x n column-major, host or device), at most
// wmax columns per solve; *converged = 0 if a solve hit max_iter.
hipError_t fact_solve(FactOp* f, int n, const double* B, long long ldb, double* X, long long ldx, double tol,
                      int max_iter, int wmax, int* converged, hipStream_t s);
// y = S^-1 (F x) for one device K-vector.
hipError_t fact_apply(FactOp* f, const double* x, double* y, double tol, int max_iter, int* converged,
                      hipStream_t s);
// One block of the recursion: U_0 = S^-1 e_cols, U_1 = H_N U_0,
// U_{l+1} = 2 H_N U_l - U_{l-1} up to U_order; P_q = sum_l coef[q cstride + l] U_l;
// mom[l] += sum over the block of S[:, col] . U_l.
struct FactBlockArgs {
    int nc;                 // columns of the block
    const long long* cols;  // device, nc column indices
    int order;
    const double* coef;     // device
    int cstride, nsets;
    double ebar, de;
    double tol;
    int max_iter;
    double* mom;            // device, order + 1 entries, accumulated
    int* flag;              // device, flag[0] |= 1 on a non-finite moment
    double* const* P_out;   // nsets destinations (K x nc column-major, host or device) or null
};
hipError_t fact_block(FactOp* f, const FactBlockArgs& a, int* converged, hipStream_t s);
// Stochastic moments sum_s xi_s^T T_l(H_N) xi_s, l < n_mom, added to mom
// (device, n_mom): the recursion from U_0 = xi (K x n_vec column-major,
// host or device) with one solve per step.
hipError_t fact_stoch(FactOp* f, int n_vec, const double* xi, int n_mom, double ebar, double de, double tol,
                      int max_iter, double* mom, int* flag, int* converged, hipStream_t s);
// Solves since the last reset, the largest per-group sum of iterations and
// the largest iteration count of one solve.
hipError_t fact_stats(FactOp* f, long long* solves, long long* iters, int* max_iters, hipStream_t s);
hipError_t fact_reset_stats(FactOp* f, hipStream_t s);
// With timing on, each S product of the iterations is bracketed by HIP
// events on the solve's stream; fact_take_timing returns and clears the
// number of timed launches and their summed duration.
void fact_set_timing(FactOp* f, bool on);
void fact_take_timing(FactOp* f, long long* launches, double* ms);

}  // namespace dm
