// Support kernels of the density-matrix path: operator setup (dense
// scatter, blocked Cholesky pieces, normalisation), the start block of the
// column recursion, moment reduction, Chebyshev coefficients, the trace /
// chemical-potential evaluation and the Lanczos spectral bounds.
#include <cmath>

#include "dm_common.hpp"

namespace dm {
namespace {

constexpr double kPi = 3.14159265358979323846;

__device__ inline double fermi_dirac(double e, double mu, double beta) {
    // 1 / (1 + exp(beta (e - mu))) written with tanh, which cannot overflow
    return 0.5 * (1.0 - tanh(0.5 * beta * (e - mu)));
}

template <int NT>
__device__ inline double block_sum(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < NT / 64; ++w) s += red[w];
    return s;  // every thread gets the same value, summed in wave order
}

// ------------------------------------------------------------------ fills
__global__ void fill_f64_kernel(double* x, double v, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        x[i] = v;
}
__global__ void fill_i32_kernel(int* x, int v, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        x[i] = v;
}

// flag[0] |= 2 for a column index outside [0, K), |= 4 for a repeated one
// (seen: K zeroed ints)
__global__ void check_columns_kernel(const long long* __restrict__ cols, long long ncols, long long K,
                                     int* __restrict__ seen, int* flag) {
    for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < ncols;
         j += (long long)gridDim.x * blockDim.x) {
        const long long x = cols[j];
        if (x < 0 || x >= K)
            atomicOr(flag, 2);
        else if (atomicAdd(seen + x, 1) != 0)
            atomicOr(flag, 4);
    }
}

// out[i] = sum_q w_q P_q[i] (the blocks of one multi-set pass combined)
__global__ void combine_sets_kernel(long long n, int nsets, CombineSets cs, double* __restrict__ out) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int q = 0; q < nsets; ++q) acc += cs.w[q] * cs.p[q][i];
        out[i] = acc;
    }
}

// out[0] = sum_{l <= N - 1} |a_l - sum_q w_q A_q[l]|, a = A_nsets (one
// workgroup, fixed order)
__global__ void __launch_bounds__(256) interp_bound_kernel(int N, int nsets, const double* __restrict__ A, int stride,
                                                           CombineSets cs, double* out) {
    double s = 0.0;
    for (int l = threadIdx.x; l < N; l += 256) {
        double v = A[(long)nsets * stride + l];
        for (int q = 0; q < nsets; ++q) v -= cs.w[q] * A[(long)q * stride + l];
        s += fabs(v);
    }
    __shared__ double red[4];
    s = block_sum<256>(s, red);
    if (threadIdx.x == 0) out[0] = s;
}

// flag[0] |= 1 when some |x_i| exceeds lim or is not finite
__global__ void flag_large_kernel(const double* __restrict__ x, long long n, double lim, int* flag) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        if (!(fabs(x[i]) <= lim)) atomicOr(flag, 1);
}

inline dim3 grid_for(long long n, int bs) {
    long long g = (n + bs - 1) / bs;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return dim3((unsigned)g);
}

// ------------------------------------------------------------------ setup
// One wavefront per CSR row r: its entries go to column r of the column-major
// dense matrix (the matrices are symmetric, so row r equals column r).
__global__ void csr_to_dense_kernel(int K, int Kp, const long long* __restrict__ rowptr,
                                    const int* __restrict__ col, const double* __restrict__ val,
                                    double pad_diag, double* __restrict__ D) {
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (wave >= Kp) return;
    double* dcol = D + (long)wave * Kp;
    if (wave >= K) {
        if (lane == 0) dcol[wave] = pad_diag;
        return;
    }
    for (long long p = rowptr[wave] + lane; p < rowptr[wave + 1]; p += 64) dcol[col[p]] = val[p];
}

// In-LDS factorisation of one 64 x 64 diagonal block A = U^T U (upper) and
// its inverse V = U^-1, 256 threads.
__global__ void __launch_bounds__(256) potrf_diag_kernel(double* A, long ld, double* V, int* info,
                                                         int kglobal) {
    constexpr int nb = kNb;
    __shared__ double s[nb][nb + 1];  // s[r][c] = A[r + c*ld]
    __shared__ double vi[nb][nb + 1];
    __shared__ int fail;
    const int t = threadIdx.x;
    for (int idx = t; idx < nb * nb; idx += 256) {
        const int r = idx % nb, c = idx / nb;
        s[r][c] = A[r + (long)c * ld];
    }
    if (t == 0) fail = 0;
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        if (t == 0) {
            const double d = s[j][j];
            if (!(d > 0.0) || !isfinite(d)) {
                fail = 1;
                if (info[0] == 0) info[0] = kglobal + j + 1;
                s[j][j] = 1.0;
            } else {
                s[j][j] = sqrt(d);
            }
        }
        __syncthreads();
        const double piv = s[j][j];
        for (int c = j + 1 + t; c < nb; c += 256) s[j][c] /= piv;
        __syncthreads();
        const int w = nb - 1 - j;
        for (int idx = t; idx < w * w; idx += 256) {
            const int r = j + 1 + idx / w, c = j + 1 + idx % w;
            if (r <= c) s[r][c] -= s[j][r] * s[j][c];
        }
        __syncthreads();
    }
    // V = U^-1 by back substitution, one column per thread
    if (t < nb) {
        const int c = t;
        for (int r = nb - 1; r >= 0; --r) {
            double acc = (r == c) ? 1.0 : 0.0;
            if (r <= c) {
                for (int p = r + 1; p <= c; ++p) acc -= s[r][p] * vi[p][c];
                vi[r][c] = acc / s[r][r];
            } else {
                vi[r][c] = 0.0;
            }
        }
    }
    __syncthreads();
    for (int idx = t; idx < nb * nb; idx += 256) {
        const int r = idx % nb, c = idx / nb;
        A[r + (long)c * ld] = (r <= c) ? s[r][c] : 0.0;
        V[r + (long)c * nb] = vi[r][c];
    }
    (void)fail;
}

__global__ void copy_transpose_block_kernel(const double* src, long lds, double* dst, long ldd) {
    for (int idx = threadIdx.x; idx < kNb * kNb; idx += blockDim.x) {
        const int r = idx % kNb, c = idx / kNb;
        dst[r + (long)c * ldd] = src[c + (long)r * lds];
    }
}


// dst = src^T for Kp x Kp column-major matrices, 32 x 32 tiles through LDS
// (row padding avoids bank conflicts); block (bx, by) moves tile (bx, by).
__global__ void __launch_bounds__(256) transpose_kernel(int Kp, const double* __restrict__ src,
                                                        double* __restrict__ dst) {
    __shared__ double tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const long r0 = (long)blockIdx.x * 32, c0 = (long)blockIdx.y * 32;
    for (int j = ty; j < 32; j += 8) tile[j][tx] = src[(r0 + tx) + (c0 + j) * Kp];
    __syncthreads();
    for (int j = ty; j < 32; j += 8) dst[(c0 + tx) + (r0 + j) * Kp] = tile[tx][j];
}

// dst = upper triangle of src (column-major), zero below the diagonal.
__global__ void copy_upper_kernel(int Kp, const double* __restrict__ src, double* __restrict__ dst) {
    const long long n = (long long)Kp * Kp;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const int r = (int)(i % Kp), c = (int)(i / Kp);
        dst[i] = r <= c ? src[i] : 0.0;
    }
}

// Z[:, j] = D[:, cols[j]] for j < ncols (column-major, ld = Kp).
__global__ void gather_columns_kernel(int Kp, int ncols, const long long* __restrict__ cols,
                                      const double* __restrict__ D, double* __restrict__ Z) {
    const long long n = (long long)Kp * ncols;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const int r = (int)(i % Kp);
        const long long j = i / Kp;
        Z[i] = D[r + cols[j] * (long long)Kp];
    }
}


// HN = (F - ebar I) * inv_de straight from the CSR rows of a symmetric F
// (orthonormal basis, S = I); HN zero on entry, row r at HN + r * Kp.  One
// thread per row; a row without a stored diagonal gets -ebar * inv_de.
template <typename T>
__global__ void csr_normalize_kernel(int K, int Kp, const long long* __restrict__ rp,
                                     const int* __restrict__ col, const double* __restrict__ val,
                                     double ebar, double inv_de, T* __restrict__ HN) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= K) return;
    bool diag = false;
    T* row = HN + (long)r * Kp;
    for (long long p = rp[r]; p < rp[r + 1]; ++p) {
        const int cc = col[p];
        double v = val[p];
        if (cc == r) {
            v -= ebar;
            diag = true;
        }
        row[cc] = static_cast<T>(v * inv_de);
    }
    if (!diag) row[r] = static_cast<T>(-ebar * inv_de);
}

template <typename T>
__global__ void normalize_operator_kernel(int K, int Kp, const double* __restrict__ HT, double ebar,
                                          double inv_de, T* __restrict__ HN) {
    const long long n = (long long)Kp * Kp;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const int r = (int)(i % Kp), c = (int)(i / Kp);
        double v = 0.0;
        if (r < K && c < K) v = (HT[i] - (r == c ? ebar : 0.0)) * inv_de;
        HN[i] = static_cast<T>(v);
    }
}

// ------------------------------------------------------------------ recursion start
// Tile grid of the start kernel: 256 threads, each thread 4 rows of one
// column; 64 x 16 elements per workgroup.
constexpr int kStartRows = 64, kStartCols = 16;

template <typename T>
__global__ void __launch_bounds__(256)
cheb_start_kernel(int K, int Kp, int Bp, int ncols, const long long* __restrict__ cols,
                  const double* __restrict__ Sinv, T* __restrict__ U0, double* __restrict__ P,
                  const double* __restrict__ Z, const double* __restrict__ coef, int nsets,
                  long long pstride, int cstride, double* __restrict__ partial) {
    const int ntr = Kp / kStartRows;
    const int tr = blockIdx.x % ntr, tc = blockIdx.x / ntr;
    const int r0 = tr * kStartRows + 4 * (threadIdx.x & 15);
    const int j = tc * kStartCols + (threadIdx.x >> 4);
    double msum = 0.0;
    const long idx = (long)r0 + (long)j * Kp;
    if (j < ncols) {
        // no cols: column j of Sinv itself
        const double* src = Sinv ? Sinv + (cols ? cols[j] : (long long)j) * Kp + r0 : nullptr;
        for (int i = 0; i < 4; ++i) {
            const double u = src ? src[i] : (r0 + i == cols[j] ? 1.0 : 0.0);  // no Sinv: S = I
            U0[idx + i] = static_cast<T>(u);
            for (int q = 0; q < nsets; ++q) P[q * pstride + idx + i] = coef[q * cstride] * u;
            msum += Z[idx + i] * static_cast<double>(static_cast<T>(u));
        }
    } else {
        for (int i = 0; i < 4; ++i) {
            U0[idx + i] = static_cast<T>(0);
            for (int q = 0; q < nsets; ++q) P[q * pstride + idx + i] = 0.0;
        }
    }
    __shared__ double red[4];
    const double s = block_sum<256>(msum, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <typename T>
__global__ void __launch_bounds__(256)
cheb_start_vectors_kernel(int K, int Kp, int Bp, int nvec, const double* __restrict__ X,
                          double zscale, T* __restrict__ U0, double* __restrict__ Z,
                          double* __restrict__ partial) {
    const int ntr = Kp / kStartRows;
    const int tr = blockIdx.x % ntr, tc = blockIdx.x / ntr;
    const int r0 = tr * kStartRows + 4 * (threadIdx.x & 15);
    const int j = tc * kStartCols + (threadIdx.x >> 4);
    double msum = 0.0;
    const long idx = (long)r0 + (long)j * Kp;
    for (int i = 0; i < 4; ++i) {
        const int r = r0 + i;
        double x = 0.0;
        if (j < nvec && r < K) x = X[r + (long)j * K];
        const T u = static_cast<T>(x);
        U0[idx + i] = u;
        Z[idx + i] = x * zscale;
        msum += x * zscale * static_cast<double>(u);
    }
    __shared__ double red[4];
    const double s = block_sum<256>(msum, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Z[:, j] = S[:, cols[j]]: one wavefront per column, from CSR row cols[j].
__global__ void scatter_s_columns_kernel(int Kp, int ncols, const long long* __restrict__ cols,
                                         const long long* __restrict__ rowptr,
                                         const int* __restrict__ col, const double* __restrict__ val,
                                         double* __restrict__ Z) {
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (wave >= ncols) return;
    const long long r = cols[wave];
    double* z = Z + (long)wave * Kp;
    for (long long p = rowptr[r] + lane; p < rowptr[r + 1]; p += 64) z[col[p]] = val[p];
}

// ------------------------------------------------------------------ moments
__global__ void reduce_moments_kernel(int lmax, int ntiles, const double* __restrict__ partial,
                                      double* __restrict__ mom, int* flag) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l > lmax) return;
    const double* p = partial + (long)l * ntiles;
    double s = 0.0;
    for (int t = 0; t < ntiles; ++t) s += p[t];
    if (!isfinite(s)) atomicOr(flag, 1);
    mom[l] += s;
}

// ------------------------------------------------------------------ coefficients
// f_k = f_FD(ebar + de cos theta_k), theta_k = pi (k + 1/2) / M
__global__ void fermi_at_nodes_kernel(int M, double ebar, double de, double mu, const double* mu_dev,
                                      double beta, double* fk) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    if (mu_dev) mu = mu_dev[0];
    const double th = kPi * (k + 0.5) / M;
    fk[k] = fermi_dirac(ebar + de * cos(th), mu, beta);
}

// cos(l theta_k) with the angle reduced exactly: l (2k+1) pi / (2M) taken
// modulo 2 pi in integer arithmetic before the cosine.
__device__ inline double cos_node(long long l, long long k, long long M) {
    const long long j = (l * (2 * k + 1)) % (4 * M);
    return cos(kPi * (double)j / (double)(2 * M));
}

// a_l = (c_l / M) sum_k f_k cos(l theta_k), c_0 = 1, c_l = 2; one workgroup
// per l, a[N] = 0.
__global__ void __launch_bounds__(256) dct_coefficients_kernel(int N, int M, const double* fk,
                                                               double* a) {
    const int l = blockIdx.x;
    if (l >= N) {
        if (threadIdx.x == 0) a[N] = 0.0;
        return;
    }
    double s = 0.0;
    for (int k = threadIdx.x; k < M; k += 256) s += fk[k] * cos_node(l, k, M);
    __shared__ double red[4];
    s = block_sum<256>(s, red);
    if (threadIdx.x == 0) a[l] = s * (l == 0 ? 1.0 : 2.0) / M;
}

// w_k = (1/M) sum_{l<N} c_l m_l cos(l theta_k);
// v_k likewise with e_l = ebar m_l + de (m_{l+1} + m_{|l-1|}) / 2,
// so that sum_l a_l m_l = sum_k f_k w_k and sum_l a_l e_l = sum_k f_k v_k.
__global__ void __launch_bounds__(256) trace_weights_kernel(int N, int M, double ebar, double de,
                                                            const double* m, double* w, double* v) {
    const int k = blockIdx.x;
    if (k >= M) return;
    double sw = 0.0, sv = 0.0;
    for (int l = threadIdx.x; l < N; l += 256) {
        const double c = (l == 0 ? 1.0 : 2.0) * cos_node(l, k, M);
        const double el = ebar * m[l] + 0.5 * de * (m[l + 1] + m[l == 0 ? 1 : l - 1]);
        sw += c * m[l];
        sv += c * el;
    }
    __shared__ double red[4];
    sw = block_sum<256>(sw, red);
    sv = block_sum<256>(sv, red);
    if (threadIdx.x == 0) {
        w[k] = sw / M;
        v[k] = sv / M;
    }
}


// Broadened density of states from the trace quadrature weights:
// out_i = scale sum_k w_k G_sigma(E_i - ebar - de cos theta_k), G_sigma the
// normalised Gaussian.  One workgroup per energy, fixed summation order.
__global__ void __launch_bounds__(256) dos_gauss_kernel(int n, const double* __restrict__ E, int M,
                                                        double ebar, double de, double sigma,
                                                        double scale, const double* __restrict__ w,
                                                        double* __restrict__ out) {
    const int i = blockIdx.x;
    if (i >= n) return;
    const double e = E[i];
    double s = 0.0;
    for (int k = threadIdx.x; k < M; k += 256) {
        const double d = (e - ebar - de * cos(kPi * (k + 0.5) / M)) / sigma;
        s += w[k] * exp(-0.5 * d * d);
    }
    __shared__ double red[4];
    s = block_sum<256>(s, red);
    if (threadIdx.x == 0) out[i] = scale * s / (sqrt(2.0 * kPi) * sigma);
}

// Kernel-polynomial density of states with the Jackson kernel
// g_l = [(N - l + 1) cos(q l) + sin(q l) cot q] / (N + 1), q = pi / (N + 1):
// out_i = scale [g_0 m_0 + 2 sum_{0<l<N} g_l m_l cos(l acos x)] / (pi de sqrt(1 - x^2)),
// x = (E_i - ebar) / de, zero for |x| >= 1.  One workgroup per energy.
__global__ void __launch_bounds__(256) dos_kpm_kernel(int n, const double* __restrict__ E, int N,
                                                      double ebar, double de, double scale,
                                                      const double* __restrict__ m,
                                                      double* __restrict__ out) {
    const int i = blockIdx.x;
    if (i >= n) return;
    const double x = (E[i] - ebar) / de;
    if (!(fabs(x) < 1.0)) {
        if (threadIdx.x == 0) out[i] = 0.0;
        return;
    }
    const double th = acos(x);
    const double q = kPi / (N + 1);
    const double cotq = cos(q) / sin(q);
    double s = 0.0;
    for (int l = threadIdx.x; l < N; l += 256) {
        const double g = ((N - l + 1) * cos(q * l) + sin(q * l) * cotq) / (N + 1);
        s += (l == 0 ? 1.0 : 2.0) * g * m[l] * cos(l * th);
    }
    __shared__ double red[4];
    s = block_sum<256>(s, red);
    if (threadIdx.x == 0) out[i] = scale * s / (kPi * de * sqrt(1.0 - x * x));
}

__global__ void __launch_bounds__(1024)
mu_bisect_kernel(int M, double ebar, double de, double beta, double target, double tol, double lo,
                 double hi, double mu_in, int max_iter, const double* __restrict__ w,
                 const double* __restrict__ v, double* out) {
    __shared__ double red[16];
    auto trace_at = [&](double mu) {
        double s = 0.0;
        for (int k = threadIdx.x; k < M; k += 1024) {
            const double x = ebar + de * cos(kPi * (k + 0.5) / M);
            s += fermi_dirac(x, mu, beta) * w[k];
        }
        return block_sum<1024>(s, red);
    };
    double mu = mu_in;
    int conv = 0, it = 0;
    if (max_iter > 0) {
        const double eps = 2.220446049250313e-16;
        for (it = 0; it < max_iter; ++it) {
            mu = 0.5 * (lo + hi);
            const double t = trace_at(mu);
            if (fabs(t - target) <= tol) {
                conv = 1;
                break;
            }
            if (t < target)
                lo = mu;
            else
                hi = mu;
            if (hi - lo <= 4.0 * eps * fmax(fmax(fabs(lo), fabs(hi)), 1.0)) break;
        }
    }
    const double tr = trace_at(mu);
    double e = 0.0;
    for (int k = threadIdx.x; k < M; k += 1024) {
        const double x = ebar + de * cos(kPi * (k + 0.5) / M);
        e += fermi_dirac(x, mu, beta) * v[k];
    }
    e = block_sum<1024>(e, red);
    if (threadIdx.x == 0) {
        out[0] = mu;
        out[1] = tr;
        out[2] = e;
        out[3] = conv;
        out[4] = it;
    }
}

// Smallest N <= max_order with sum_{max_order > l >= N} ... : the coefficient
// tail sum_{l >= N} |a_l| over the n available coefficients is <= tol;
// max_order + 1 when the tail at max_order is already above tol.
__global__ void coef_tail_order_kernel(int n, int max_order, const double* a, double tol, int* order) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double tail = 0.0;
    int N = 0;
    for (int l = n - 1; l >= 0; --l) {
        tail += fabs(a[l]);
        if (tail > tol) {
            N = l + 1;
            break;
        }
    }
    order[0] = N > max_order ? max_order + 1 : N;
}

// ------------------------------------------------------------------ Lanczos
__device__ inline unsigned long long splitmix64(unsigned long long x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__global__ void random_vector_kernel(int K, unsigned long long seed, double* v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K) return;
    const unsigned long long h = splitmix64(seed * 0x100000001B3ull + (unsigned long long)i);
    v[i] = (double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ void csr_spmv_kernel(int K, const long long* __restrict__ rowptr,
                                const int* __restrict__ col, const double* __restrict__ val,
                                const double* __restrict__ x, double* __restrict__ y) {
    const int row = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (row >= K) return;
    double s = 0.0;
    for (long long p = rowptr[row] + lane; p < rowptr[row + 1]; p += 64) s += val[p] * x[col[p]];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) y[row] = s;
}

__global__ void gemv_rows_kernel(int K, const double* __restrict__ A, long lda,
                                 const double* __restrict__ x, double* __restrict__ y) {
    const int row = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (row >= K) return;
    const double* a = A + (long)row * lda;
    double s = 0.0;
    for (int k = lane; k < K; k += 64) s += a[k] * x[k];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) y[row] = s;
}

__global__ void __launch_bounds__(256) dots_cols_kernel(int K, const double* __restrict__ X, long ldx,
                                                        const double* __restrict__ y, double* out) {
    const int i = blockIdx.x;
    const double* x = X + (long)i * ldx;
    double s = 0.0;
    for (int k = threadIdx.x; k < K; k += 256) s += x[k] * y[k];
    __shared__ double red[4];
    s = block_sum<256>(s, red);
    if (threadIdx.x == 0) out[i] = s;
}

__global__ void lanczos_normalize_start_kernel(int K, double* v, double* q, const double* vSv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K) return;
    const double r = 1.0 / sqrt(vSv[0]);
    v[i] *= r;
    q[i] *= r;
}

__global__ void lanczos_three_term_kernel(int K, double* w, const double* vj, const double* vjm1,
                                          const double* alpha_j, const double* beta_jm1) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K) return;
    double r = w[i] - alpha_j[0] * vj[i];
    if (vjm1) r -= beta_jm1[0] * vjm1[i];
    w[i] = r;
}

__global__ void lanczos_reorth_kernel(int K, int n, double* w, const double* V, long ldv,
                                      const double* c) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K) return;
    double r = w[i];
    for (int j = 0; j < n; ++j) r -= c[j] * V[i + (long)j * ldv];
    w[i] = r;
}

__global__ void lanczos_next_kernel(int K, const double* w, const double* sw, const double* wSw,
                                    double* beta_out, double* vnext, double* qnext) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const double b2 = wSw[0];
    const double b = b2 > 0.0 ? sqrt(b2) : 0.0;
    if (i == 0) beta_out[0] = b;
    if (i >= K) return;
    const double r = b > 0.0 ? 1.0 / b : 0.0;
    vnext[i] = w[i] * r;
    qnext[i] = sw[i] * r;
}

}  // namespace

// ====================================================================== wrappers
hipError_t fill_f64(double* x, double v, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_f64_kernel, grid_for(n, 256), dim3(256), 0, s, x, v, n);
    return hipGetLastError();
}
hipError_t fill_i32(int* x, int v, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_i32_kernel, grid_for(n, 256), dim3(256), 0, s, x, v, n);
    return hipGetLastError();
}

hipError_t check_columns(const long long* cols, long long ncols, long long K, int* seen, int* flag,
                         hipStream_t s) {
    if (ncols <= 0) return hipSuccess;
    hipLaunchKernelGGL(check_columns_kernel, grid_for(ncols, 256), dim3(256), 0, s, cols, ncols, K, seen, flag);
    return hipGetLastError();
}

hipError_t combine_sets(long long n, int nsets, const CombineSets& cs, double* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (nsets < 1 || nsets > kMaxCombine) return hipErrorInvalidValue;
    hipLaunchKernelGGL(combine_sets_kernel, grid_for(n, 256), dim3(256), 0, s, n, nsets, cs, out);
    return hipGetLastError();
}

hipError_t interp_bound(int N, int nsets, const double* A, int stride, const CombineSets& cs, double* out,
                        hipStream_t s) {
    if (nsets < 1 || nsets > kMaxCombine) return hipErrorInvalidValue;
    hipLaunchKernelGGL(interp_bound_kernel, dim3(1), dim3(256), 0, s, N, nsets, A, stride, cs, out);
    return hipGetLastError();
}

hipError_t flag_large(const double* x, long long n, double lim, int* flag, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(flag_large_kernel, grid_for(n, 256), dim3(256), 0, s, x, n, lim, flag);
    return hipGetLastError();
}

hipError_t csr_to_dense(int K, int Kp, const long long* rowptr, const int* col, const double* val,
                        double pad_diag, double* D, hipStream_t s) {
    hipLaunchKernelGGL(csr_to_dense_kernel, dim3((Kp + 3) / 4), dim3(256), 0, s, K, Kp, rowptr,
                       col, val, pad_diag, D);
    return hipGetLastError();
}

hipError_t potrf_diag(double* A, long ld, double* V, int* info, int kglobal, hipStream_t s) {
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(256), 0, s, A, ld, V, info, kglobal);
    return hipGetLastError();
}

hipError_t copy_transpose_block(const double* src, long lds, double* dst, long ldd, hipStream_t s) {
    hipLaunchKernelGGL(copy_transpose_block_kernel, dim3(1), dim3(256), 0, s, src, lds, dst, ldd);
    return hipGetLastError();
}

hipError_t transpose_square(int Kp, const double* src, double* dst, hipStream_t s) {
    if (Kp % 32) return hipErrorInvalidValue;
    hipLaunchKernelGGL(transpose_kernel, dim3(Kp / 32, Kp / 32), dim3(256), 0, s, Kp, src, dst);
    return hipGetLastError();
}

hipError_t copy_upper(int Kp, const double* src, double* dst, hipStream_t s) {
    hipLaunchKernelGGL(copy_upper_kernel, grid_for((long long)Kp * Kp, 256), dim3(256), 0, s, Kp, src, dst);
    return hipGetLastError();
}

hipError_t csr_normalize(int K, int Kp, const long long* rp, const int* col, const double* val, double ebar,
                         double de, int precision, void* HN, hipStream_t s) {
    const long long n = (long long)Kp * Kp;
    hipError_t e = fill_f64(static_cast<double*>(HN), 0.0, precision == 0 ? n : n / 2, s);
    if (e != hipSuccess) return e;
    if (precision == 0)
        hipLaunchKernelGGL(csr_normalize_kernel<double>, dim3((K + 255) / 256), dim3(256), 0, s, K, Kp, rp, col,
                           val, ebar, 1.0 / de, static_cast<double*>(HN));
    else
        hipLaunchKernelGGL(csr_normalize_kernel<float>, dim3((K + 255) / 256), dim3(256), 0, s, K, Kp, rp, col,
                           val, ebar, 1.0 / de, static_cast<float*>(HN));
    return hipGetLastError();
}

hipError_t normalize_operator(int K, int Kp, const double* HT, double ebar, double de,
                              int precision, void* HN, hipStream_t s) {
    const long long n = (long long)Kp * Kp;
    if (precision == 0)
        hipLaunchKernelGGL(normalize_operator_kernel<double>, grid_for(n, 256), dim3(256), 0, s, K,
                           Kp, HT, ebar, 1.0 / de, static_cast<double*>(HN));
    else
        hipLaunchKernelGGL(normalize_operator_kernel<float>, grid_for(n, 256), dim3(256), 0, s, K,
                           Kp, HT, ebar, 1.0 / de, static_cast<float*>(HN));
    return hipGetLastError();
}

hipError_t scatter_s_columns(int Kp, int ncols, const long long* cols, const long long* rowptr, const int* col,
                             const double* val, double* Z, hipStream_t s) {
    if (ncols <= 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_s_columns_kernel, dim3((ncols + 3) / 4), dim3(256), 0, s, Kp, ncols, cols, rowptr,
                       col, val, Z);
    return hipGetLastError();
}

hipError_t cheb_start(int K, int Kp, int Bp, int ncols, const long long* cols, const double* Sinv,
                      const long long* S_rowptr, const int* S_col, const double* S_val,
                      int precision, void* U0, double* Z, double* P, const double* coef,
                      int nsets, long long pstride, int cstride, double* partial, int* ntiles_out,
                      hipStream_t s, const double* Zdense) {
    if (nsets < 1) return hipErrorInvalidValue;
    if (Kp % kStartRows || Bp % kStartCols) return hipErrorInvalidValue;
    if (!cols && !Sinv) return hipErrorInvalidValue;
    if (Zdense == Z) {
        // the moment vectors are already in Z
    } else if (ncols > 0 && Zdense)
        hipLaunchKernelGGL(gather_columns_kernel, grid_for((long long)Kp * ncols, 256), dim3(256), 0, s, Kp,
                           ncols, cols, Zdense, Z);
    else if (ncols > 0)
        hipLaunchKernelGGL(scatter_s_columns_kernel, dim3((ncols + 3) / 4), dim3(256), 0, s, Kp,
                           ncols, cols, S_rowptr, S_col, S_val, Z);
    const int ntiles = (Kp / kStartRows) * (Bp / kStartCols);
    if (precision == 0)
        hipLaunchKernelGGL(cheb_start_kernel<double>, dim3(ntiles), dim3(256), 0, s, K, Kp, Bp,
                           ncols, cols, Sinv, static_cast<double*>(U0), P, Z, coef, nsets, pstride, cstride,
                           partial);
    else
        hipLaunchKernelGGL(cheb_start_kernel<float>, dim3(ntiles), dim3(256), 0, s, K, Kp, Bp,
                           ncols, cols, Sinv, static_cast<float*>(U0), P, Z, coef, nsets, pstride, cstride,
                           partial);
    *ntiles_out = ntiles;
    return hipGetLastError();
}

hipError_t cheb_start_vectors(int K, int Kp, int Bp, int nvec, const double* X, double zscale,
                              int precision, void* U0, double* Z, double* partial, int* ntiles_out,
                              hipStream_t s) {
    if (Kp % kStartRows || Bp % kStartCols) return hipErrorInvalidValue;
    const int ntiles = (Kp / kStartRows) * (Bp / kStartCols);
    if (precision == 0)
        hipLaunchKernelGGL(cheb_start_vectors_kernel<double>, dim3(ntiles), dim3(256), 0, s, K, Kp,
                           Bp, nvec, X, zscale, static_cast<double*>(U0), Z, partial);
    else
        hipLaunchKernelGGL(cheb_start_vectors_kernel<float>, dim3(ntiles), dim3(256), 0, s, K, Kp,
                           Bp, nvec, X, zscale, static_cast<float*>(U0), Z, partial);
    *ntiles_out = ntiles;
    return hipGetLastError();
}

hipError_t reduce_moments(int lmax, int ntiles, const double* partial, double* mom, int* flag,
                          hipStream_t s) {
    hipLaunchKernelGGL(reduce_moments_kernel, dim3((lmax + 1 + 255) / 256), dim3(256), 0, s, lmax,
                       ntiles, partial, mom, flag);
    return hipGetLastError();
}

hipError_t cheb_coefficients(int N, int M, double ebar, double de, double mu, double beta,
                             double* fk_scratch, double* a, hipStream_t s) {
    hipLaunchKernelGGL(fermi_at_nodes_kernel, dim3((M + 255) / 256), dim3(256), 0, s, M, ebar, de,
                       mu, (const double*)nullptr, beta, fk_scratch);
    hipLaunchKernelGGL(dct_coefficients_kernel, dim3(N + 1), dim3(256), 0, s, N, M, fk_scratch, a);
    return hipGetLastError();
}

hipError_t cheb_coefficients_devmu(int N, int M, double ebar, double de, const double* mu_dev,
                                   double beta, double* fk_scratch, double* a, hipStream_t s) {
    hipLaunchKernelGGL(fermi_at_nodes_kernel, dim3((M + 255) / 256), dim3(256), 0, s, M, ebar, de,
                       0.0, mu_dev, beta, fk_scratch);
    hipLaunchKernelGGL(dct_coefficients_kernel, dim3(N + 1), dim3(256), 0, s, N, M, fk_scratch, a);
    return hipGetLastError();
}

hipError_t dos_gauss(int n, const double* E, int M, double ebar, double de, double sigma, double scale,
                     const double* w, double* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(dos_gauss_kernel, dim3(n), dim3(256), 0, s, n, E, M, ebar, de, sigma, scale, w, out);
    return hipGetLastError();
}

hipError_t dos_kpm(int n, const double* E, int N, double ebar, double de, double scale, const double* m,
                   double* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(dos_kpm_kernel, dim3(n), dim3(256), 0, s, n, E, N, ebar, de, scale, m, out);
    return hipGetLastError();
}

hipError_t trace_weights(int N, int M, double ebar, double de, const double* m, double* w,
                         double* v, hipStream_t s) {
    hipLaunchKernelGGL(trace_weights_kernel, dim3(M), dim3(256), 0, s, N, M, ebar, de, m, w, v);
    return hipGetLastError();
}

hipError_t mu_bisect(int M, double ebar, double de, double beta, double target, double tol,
                     double lo, double hi, double mu_in, int max_iter, const double* w,
                     const double* v, double* out, hipStream_t s) {
    hipLaunchKernelGGL(mu_bisect_kernel, dim3(1), dim3(1024), 0, s, M, ebar, de, beta, target, tol,
                       lo, hi, mu_in, max_iter, w, v, out);
    return hipGetLastError();
}

hipError_t coef_tail_order(int n, int max_order, const double* a, double tol, int* order,
                           hipStream_t s) {
    hipLaunchKernelGGL(coef_tail_order_kernel, dim3(1), dim3(64), 0, s, n, max_order, a, tol, order);
    return hipGetLastError();
}

hipError_t random_vector(int K, unsigned long long seed, double* v, hipStream_t s) {
    hipLaunchKernelGGL(random_vector_kernel, dim3((K + 255) / 256), dim3(256), 0, s, K, seed, v);
    return hipGetLastError();
}

hipError_t csr_spmv(int K, const long long* rowptr, const int* col, const double* val,
                    const double* x, double* y, hipStream_t s) {
    hipLaunchKernelGGL(csr_spmv_kernel, dim3((K + 3) / 4), dim3(256), 0, s, K, rowptr, col, val, x,
                       y);
    return hipGetLastError();
}

hipError_t gemv_rows(int K, const double* A, long lda, const double* x, double* y, hipStream_t s) {
    hipLaunchKernelGGL(gemv_rows_kernel, dim3((K + 3) / 4), dim3(256), 0, s, K, A, lda, x, y);
    return hipGetLastError();
}

hipError_t dots_cols(int K, int n, const double* X, long ldx, const double* y, double* out,
                     hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(dots_cols_kernel, dim3(n), dim3(256), 0, s, K, X, ldx, y, out);
    return hipGetLastError();
}

hipError_t lanczos_normalize_start(int K, double* v, double* q, const double* vSv, hipStream_t s) {
    hipLaunchKernelGGL(lanczos_normalize_start_kernel, dim3((K + 255) / 256), dim3(256), 0, s, K, v,
                       q, vSv);
    return hipGetLastError();
}

hipError_t lanczos_three_term(int K, double* w, const double* vj, const double* vjm1,
                              const double* alpha_j, const double* beta_jm1, hipStream_t s) {
    hipLaunchKernelGGL(lanczos_three_term_kernel, dim3((K + 255) / 256), dim3(256), 0, s, K, w, vj,
                       vjm1, alpha_j, beta_jm1);
    return hipGetLastError();
}

hipError_t lanczos_reorth(int K, int n, double* w, const double* V, long ldv, const double* c,
                          hipStream_t s) {
    hipLaunchKernelGGL(lanczos_reorth_kernel, dim3((K + 255) / 256), dim3(256), 0, s, K, n, w, V,
                       ldv, c);
    return hipGetLastError();
}

hipError_t lanczos_next(int K, const double* w, const double* sw, const double* wSw,
                        double* beta_out, double* vnext, double* qnext, hipStream_t s) {
    hipLaunchKernelGGL(lanczos_next_kernel, dim3((K + 255) / 256), dim3(256), 0, s, K, w, sw, wSw,
                       beta_out, vnext, qnext);
    return hipGetLastError();
}

}  // namespace dm
