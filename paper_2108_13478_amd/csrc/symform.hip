// Kernels of the symmetric operator form built in place: with S = U^T U the
// library keeps only X = U^-1 (upper triangular, FP64) and the normalised
// H~_N = (X^T F X - Ebar) / dE in the recursion precision, so the setup of a
// K-function basis needs K^2 x (8 + p) bytes instead of several FP64 K x K
// arrays.  Every kernel here is a plain memory-bound pass (transposes,
// gathers, a CSR product against a row-major panel, element-wise stores);
// the flops of the setup run in the MFMA GEMMs of gemm.hip.
#include "dm_common.hpp"

namespace dm {
namespace {

inline dim3 grid_1d(long long n, int bs) {
    long long b = (n + bs - 1) / bs;
    if (b > 65535LL * 64) b = 65535LL * 64;
    return dim3((unsigned)(b < 1 ? 1 : b));
}

// A[r + c Kp] = 0 for r > c (Kp x Kp column-major).
__global__ void zero_strict_lower_kernel(int Kp, double* __restrict__ A) {
    const long long n = (long long)Kp * Kp;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const long long r = i % Kp, c = i / Kp;
        if (r > c) A[i] = 0.0;
    }
}

// The nb x nb diagonal block at A (leading dimension ld) := the upper
// triangle of V (nb x nb column-major), zero below the diagonal.
__global__ void set_upper_block_kernel(int nb, double* __restrict__ A, long ld, const double* __restrict__ V) {
    for (int idx = threadIdx.x; idx < nb * nb; idx += blockDim.x) {
        const int r = idx % nb, c = idx / nb;
        A[r + (long)c * ld] = r <= c ? V[r + (long)c * nb] : 0.0;
    }
}

// dst[c + r ldd] = src[r + c lds] for r < rows, c < cols: 32 x 32 tiles
// through LDS, both sides coalesced; block (bx, by) moves rows 32 bx..,
// columns 32 by..
__global__ void __launch_bounds__(256) transpose_rect_kernel(long rows, long cols, const double* __restrict__ src,
                                                             long lds, double* __restrict__ dst, long ldd) {
    __shared__ double tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const long r0 = (long)blockIdx.x * 32, c0 = (long)blockIdx.y * 32;
    for (int j = ty; j < 32; j += 8) {
        const long r = r0 + tx, c = c0 + j;
        tile[j][tx] = (r < rows && c < cols) ? src[r + c * lds] : 0.0;
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
        const long c = c0 + tx, r = r0 + j;
        if (r < rows && c < cols) dst[c + r * ldd] = tile[tx][j];
    }
}

// V[r + j Kp] = X[cols[j] + r Kp] for r < Kp, j < ncols: row cols[j] of the
// column-major X as column j of V (a column of X^T).  32 x 32 tiles through
// LDS: the reads of one tile row take 32 consecutive columns' rows cols[j]
// (one 256-byte run when the columns are consecutive), the writes 32
// consecutive rows of V.
__global__ void __launch_bounds__(256) gather_rows_kernel(int Kp, int ncols, const long long* __restrict__ cols,
                                                          const double* __restrict__ X, double* __restrict__ V) {
    __shared__ double tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const long j0 = (long)blockIdx.x * 32, r0 = (long)blockIdx.y * 32;
    for (int i = ty; i < 32; i += 8) {
        const long j = j0 + tx, r = r0 + i;
        tile[i][tx] = j < ncols ? X[cols[j] + r * Kp] : 0.0;
    }
    __syncthreads();
    for (int i = ty; i < 32; i += 8) {
        const long j = j0 + i, r = r0 + tx;
        if (j < ncols) V[r + j * Kp] = tile[tx][i];
    }
}

// Y = F X for a row-major panel X (K x w, row k at X + k w) and CSR F, in
// column chunks of kSpmmChunk: workgroup b takes row b % K of chunk b / K,
// so the workgroups in flight share one chunk of the panel (K x 128 FP64,
// 134 MB at K = 131072, within the Infinity Cache) while they gather its
// rows; a thread owns one column.  Row entries come in column order;
// entries with column >= kmax are skipped (X is zero there) and end the
// row.
constexpr int kSpmmChunk = 128;
__global__ void __launch_bounds__(kSpmmChunk) csr_spmm_rm_kernel(int K, const long long* __restrict__ rp,
                                                                 const int* __restrict__ col,
                                                                 const double* __restrict__ val, int w,
                                                                 const double* __restrict__ X, int kmax,
                                                                 double* __restrict__ Y) {
    const long long b = blockIdx.x;
    const int row = (int)(b % K);
    const int j = (int)(b / K) * kSpmmChunk + threadIdx.x;
    double acc = 0.0;
    for (long long p = rp[row]; p < rp[row + 1]; ++p) {
        const int k = col[p];
        if (k >= kmax) break;
        if (j < w) acc += val[p] * X[(long)k * w + j];
    }
    if (j < w) Y[(long)row * w + j] = acc;
}

// The same product with F in groups of four rows (one atom of the
// four-function basis): per group the sorted union of its rows' columns,
// each with four values (zero where a row has no entry).  Every gathered
// row of the panel then serves four rows of Y: a quarter of the gather
// traffic of the CSR form.  Workgroup b: group b % ng, chunk b / ng.
__global__ void __launch_bounds__(kSpmmChunk) rg4_spmm_rm_kernel(int K, int ng, const long long* __restrict__ gp,
                                                                 const int* __restrict__ gc,
                                                                 const double* __restrict__ gv, int w,
                                                                 const double* __restrict__ X, int kmax,
                                                                 double* __restrict__ Y) {
    const long long b = blockIdx.x;
    const int g = (int)(b % ng);
    const int j = (int)(b / ng) * kSpmmChunk + threadIdx.x;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (long long p = gp[g]; p < gp[g + 1]; ++p) {
        const int k = gc[p];
        if (k >= kmax) break;
        if (j < w) {
            const double x = X[(long)k * w + j];
            const double* v = gv + 4 * p;
            a0 += v[0] * x;
            a1 += v[1] * x;
            a2 += v[2] * x;
            a3 += v[3] * x;
        }
    }
    if (j >= w) return;
    const int r0 = 4 * g;
    if (r0 < K) Y[(long)r0 * w + j] = a0;
    if (r0 + 1 < K) Y[(long)(r0 + 1) * w + j] = a1;
    if (r0 + 2 < K) Y[(long)(r0 + 2) * w + j] = a2;
    if (r0 + 3 < K) Y[(long)(r0 + 3) * w + j] = a3;
}

// Rows row0 .. Kp - 1 of columns col0 .. col0 + w - 1 of the Kp x Kp
// matrix H (column-major, type T) := (C - ebar I) inv_de (C: Kp x w
// column-major, FP64), zero outside the K x K block.
template <typename T>
__global__ void store_panel_kernel(int K, int Kp, int w, int col0, int row0, const double* __restrict__ C,
                                   double ebar, double inv_de, T* __restrict__ H) {
    const long long n = (long long)Kp * w;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const long long r = i % Kp, j = i / Kp, c = col0 + j;
        if (r < row0) continue;
        double v = 0.0;
        if (r < K && c < K) v = (C[i] - (r == c ? ebar : 0.0)) * inv_de;
        H[r + c * Kp] = static_cast<T>(v);
    }
}

// Upper triangle of the Kp x Kp matrix H := mirror image of its lower one,
// 32 x 32 tiles through LDS: block (bx, by), bx < by, reads tile (by, bx)
// below the diagonal and writes its transpose to tile (bx, by); diagonal
// tiles are left as they are.
template <typename T>
__global__ void __launch_bounds__(256) mirror_lower_kernel(int Kp, T* __restrict__ H) {
    const int bx = blockIdx.x, by = blockIdx.y;
    if (bx >= by) return;
    __shared__ T tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const long r0 = (long)by * 32, c0 = (long)bx * 32;  // source tile rows by, columns bx
    for (int j = ty; j < 32; j += 8) tile[j][tx] = H[(r0 + tx) + (c0 + j) * Kp];
    __syncthreads();
    for (int j = ty; j < 32; j += 8) H[(c0 + tx) + (r0 + j) * Kp] = tile[tx][j];
}

// H := (H - ebar I) inv_de in place on the K x K block, zero padding.
template <typename T>
__global__ void normalize_inplace_kernel(int K, int Kp, T* __restrict__ H, double ebar, double inv_de) {
    const long long n = (long long)Kp * Kp;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const long long r = i % Kp, c = i / Kp;
        double v = 0.0;
        if (r < K && c < K) v = ((double)H[i] - (r == c ? ebar : 0.0)) * inv_de;
        H[i] = static_cast<T>(v);
    }
}

// y = A x with A row-major (row r at A + r lda) in type T, x and y FP64, FP64
// sums: one wave per row.
template <typename T>
__global__ void gemv_rows_t_kernel(int K, const T* __restrict__ A, long lda, const double* __restrict__ x,
                                   double* __restrict__ y) {
    const int row = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (row >= K) return;
    const T* a = A + (long)row * lda;
    double s = 0.0;
    for (int k = lane; k < K; k += 64) s += (double)a[k] * x[k];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) y[row] = s;
}

}  // namespace

hipError_t zero_strict_lower(int Kp, double* A, hipStream_t s) {
    hipLaunchKernelGGL(zero_strict_lower_kernel, grid_1d((long long)Kp * Kp, 256), dim3(256), 0, s, Kp, A);
    return hipGetLastError();
}

hipError_t set_upper_block(int nb, double* A, long ld, const double* V, hipStream_t s) {
    hipLaunchKernelGGL(set_upper_block_kernel, dim3(1), dim3(256), 0, s, nb, A, ld, V);
    return hipGetLastError();
}

hipError_t transpose_rect(long rows, long cols, const double* src, long lds, double* dst, long ldd, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    if ((rows + 31) / 32 > 0x7fffffffL || (cols + 31) / 32 > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(transpose_rect_kernel, dim3((unsigned)((rows + 31) / 32), (unsigned)((cols + 31) / 32)),
                       dim3(256), 0, s, rows, cols, src, lds, dst, ldd);
    return hipGetLastError();
}

hipError_t gather_rows(int Kp, int ncols, const long long* cols, const double* X, double* V, hipStream_t s) {
    if (ncols <= 0) return hipSuccess;
    if (Kp % 32 || Kp / 32 > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gather_rows_kernel, dim3((ncols + 31) / 32, Kp / 32), dim3(256), 0, s, Kp, ncols, cols, X, V);
    return hipGetLastError();
}

hipError_t csr_spmm_rm(int K, const long long* rp, const int* col, const double* val, int w, const double* X,
                       int kmax, double* Y, hipStream_t s) {
    if (w < 1 || K < 1) return hipErrorInvalidValue;
    const long long nb = (long long)K * ((w + kSpmmChunk - 1) / kSpmmChunk);
    if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(csr_spmm_rm_kernel, dim3((unsigned)nb), dim3(kSpmmChunk), 0, s, K, rp, col, val, w, X, kmax,
                       Y);
    return hipGetLastError();
}

hipError_t rg4_spmm_rm(int K, const long long* gp, const int* gc, const double* gv, int w, const double* X, int kmax,
                       double* Y, hipStream_t s) {
    if (w < 1 || K < 1) return hipErrorInvalidValue;
    const int ng = (K + 3) / 4;
    const long long nb = (long long)ng * ((w + kSpmmChunk - 1) / kSpmmChunk);
    if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(rg4_spmm_rm_kernel, dim3((unsigned)nb), dim3(kSpmmChunk), 0, s, K, ng, gp, gc, gv, w, X, kmax,
                       Y);
    return hipGetLastError();
}

hipError_t store_panel(int K, int Kp, int w, int col0, int row0, const double* C, double ebar, double inv_de,
                       int precision, void* H, hipStream_t s) {
    const dim3 g = grid_1d((long long)Kp * w, 256);
    if (precision == 0)
        hipLaunchKernelGGL(store_panel_kernel<double>, g, dim3(256), 0, s, K, Kp, w, col0, row0, C, ebar, inv_de,
                           static_cast<double*>(H));
    else
        hipLaunchKernelGGL(store_panel_kernel<float>, g, dim3(256), 0, s, K, Kp, w, col0, row0, C, ebar, inv_de,
                           static_cast<float*>(H));
    return hipGetLastError();
}

hipError_t mirror_lower(int Kp, int precision, void* H, hipStream_t s) {
    if (Kp % 32 || Kp / 32 > 65535) return hipErrorInvalidValue;
    const dim3 g(Kp / 32, Kp / 32);
    if (precision == 0)
        hipLaunchKernelGGL(mirror_lower_kernel<double>, g, dim3(256), 0, s, Kp, static_cast<double*>(H));
    else
        hipLaunchKernelGGL(mirror_lower_kernel<float>, g, dim3(256), 0, s, Kp, static_cast<float*>(H));
    return hipGetLastError();
}

hipError_t normalize_inplace(int K, int Kp, int precision, void* H, double ebar, double de, hipStream_t s) {
    const dim3 g = grid_1d((long long)Kp * Kp, 256);
    if (precision == 0)
        hipLaunchKernelGGL(normalize_inplace_kernel<double>, g, dim3(256), 0, s, K, Kp, static_cast<double*>(H), ebar,
                           1.0 / de);
    else
        hipLaunchKernelGGL(normalize_inplace_kernel<float>, g, dim3(256), 0, s, K, Kp, static_cast<float*>(H), ebar,
                           1.0 / de);
    return hipGetLastError();
}

hipError_t gemv_rows_t(int K, int precision, const void* A, long lda, const double* x, double* y, hipStream_t s) {
    const dim3 g((K + 3) / 4);
    if (precision == 0)
        hipLaunchKernelGGL(gemv_rows_t_kernel<double>, g, dim3(256), 0, s, K, static_cast<const double*>(A), lda, x, y);
    else
        hipLaunchKernelGGL(gemv_rows_t_kernel<float>, g, dim3(256), 0, s, K, static_cast<const float*>(A), lda, x, y);
    return hipGetLastError();
}

}  // namespace dm
