// Factored operator form: the recursion applies H = S^-1 F without forming
// it, as one sparse product with F followed by a solve with S, the way the
// paper applies the overlap inverse (Methods, column-by-column evaluation of
// the density matrix, and its footnote on the overlap solve by preconditioned
// conjugate gradients).  The preconditioner here is a factorised sparse
// approximate inverse (FSAI: S^-1 ~ G^T G with G sparse and lower
// triangular) instead of the paper's incomplete Cholesky factor: applying
// it is two sparse products, with none of the dependency chains of
// triangular solves.
//
// Data layout.  A block of W columns (W a multiple of 64) is stored row-
// interleaved, v[i * W + c]: a wavefront takes 64 adjacent columns in its
// lanes, so each gathered matrix row is one 512-byte coalesced load.  Sparse
// matrices are stored in row groups of kRG = 4 rows (one atom of the
// four-function basis): the group keeps the sorted union of its rows'
// columns, and every listed column carries four values, zero where a row has
// no entry.  One gathered row of the block then feeds four output rows.
//
// The conjugate-gradient iteration runs W independent systems in lock step,
// each with its own step lengths.  Per-column dot products are reduced in
// two fixed orders: the producing kernel writes one partial sum per
// workgroup and column, and a small kernel with one workgroup per 64
// columns adds them in index order and takes the scalar step (step length,
// convergence test).  No workgroup waits for another and no fence is
// needed inside a kernel; results are bitwise reproducible.  Converged
// columns keep their solution; a 64-column group whose columns have all
// converged skips every later kernel of the solve.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include <hip/hip_ext.h>

#include "dm_common.hpp"

namespace dm {
namespace {

constexpr int kRG = 4;              // rows per group
constexpr int kWv = 16;             // waves per workgroup of the row kernels
constexpr int kRowsWG = kRG * kWv;  // 64 rows per workgroup
constexpr int kFsaiMax = 192;       // largest pattern of one FSAI row (packed triangle in LDS)
constexpr int kChunk = 8;           // iterations between convergence polls

struct RgView {
    const long long* ptr;  // ngroups + 1
    const int* col;        // sorted union of the group's columns
    const double* val;     // kRG values per listed column
};

// Workgroup -> (row block x < nx, column group y < ng).  Workgroups are
// dealt to the 8 XCDs round robin; with xcd_split each XCD takes the column
// groups y = xcd (mod 8) one after another, row blocks in order, so the
// 64-column slice of the block that its row blocks gather from (K x 512
// bytes) stays in that XCD's L2 while the group is processed.  Without the
// split (fewer than 8 groups) the order is row blocks fastest.  Returns
// false for the padding workgroups of the split grid.
struct Tiles {
    int nx, ng, xcd_split;
};
__device__ inline bool tile_of(const Tiles& t, int& x, int& y) {
    const int b = blockIdx.x;
    if (t.xcd_split) {
        const int s = b >> 3;
        y = (s / t.nx) * 8 + (b & 7);
        x = s % t.nx;
    } else {
        y = b / t.nx;
        x = b % t.nx;
    }
    return y < t.ng;
}

// Sums v over the 16 waves of the workgroup for each lane (column); the
// result is valid in wave 0.  Fixed order.
__device__ inline double wg_column_sum(double v, double (*red)[64]) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    red[w][lane] = v;
    __syncthreads();
    double s = 0.0;
    if (w == 0)
        for (int k = 0; k < kWv; ++k) s += red[k][lane];
    return s;
}

struct CgArgs {
    int W;
    Tiles t;
    const double* B;
    double *X, *R, *Z, *Pd, *Q, *T;
    double *bb, *rz, *alpha, *beta;
    int* done;
    int* active;  // per 64-column group: columns not yet converged
    int* iters;   // per 64-column group: iterations of the current solve
    double* part; // nx x W: per-workgroup column sums of the last producer
    double tol2;
    int first;
};

enum { kPlain = 0, kPq = 1, kRz = 2 };

// Y = A X over the block (kPlain); the conjugate-gradient products fuse their
// vector updates and the per-workgroup parts of their dot products:
//   kPq: Pd = Z + beta Pd, Q = A Z + beta Q (= A Pd), part = Pd . Q;
//   kRz: Z = A T (the preconditioner's second factor), part = R . Z.
// Each lane takes CPL adjacent columns (CPL = 2: one 16-byte load per
// gathered row and lane, half the matrix reads per multiply-add); a
// workgroup covers 64 CPL columns, tiles.ng counts such column groups.
template <int CPL>
__device__ inline void load_cols(const double* p, double (&x)[CPL]) {
    static_assert(CPL == 1 || CPL == 2, "one or two columns per lane");
    if constexpr (CPL == 1) {
        x[0] = *p;
    } else {
        const double2 v = *reinterpret_cast<const double2*>(p);
        x[0] = v.x;
        x[1] = v.y;
    }
}

template <int MODE, int CPL>
__global__ void __launch_bounds__(1024) rg_spmm_kernel(RgView A, const double* __restrict__ Xin,
                                                       double* __restrict__ Yout, CgArgs a, Tiles t) {
    __shared__ double red[kWv][64 * CPL];
    int bx, y;
    if (!tile_of(t, bx, y)) return;
    if (a.active) {
        bool live = false;
#pragma unroll
        for (int q = 0; q < CPL; ++q) live = live || a.active[y * CPL + q] != 0;
        if (!live) return;
    }
    const int W = a.W;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int g = bx * kWv + wv;
    const int c = y * 64 * CPL + lane * CPL;  // first of this lane's columns
    const long long p0 = A.ptr[g], p1 = A.ptr[g + 1];
    double acc[kRG][CPL];
#pragma unroll
    for (int r = 0; r < kRG; ++r)
#pragma unroll
        for (int q = 0; q < CPL; ++q) acc[r][q] = 0.0;
    const double* xc = Xin + c;
    long long p = p0;
    for (; p + 8 <= p1; p += 8) {
        int j[8];
        double x[8][CPL];
#pragma unroll
        for (int u = 0; u < 8; ++u) j[u] = A.col[p + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) load_cols<CPL>(xc + (size_t)j[u] * W, x[u]);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double* v = A.val + (p + u) * kRG;
#pragma unroll
            for (int r = 0; r < kRG; ++r)
#pragma unroll
                for (int q = 0; q < CPL; ++q) acc[r][q] += v[r] * x[u][q];
        }
    }
    for (; p < p1; ++p) {
        double x[CPL];
        load_cols<CPL>(xc + (size_t)A.col[p] * W, x);
        const double* v = A.val + p * kRG;
#pragma unroll
        for (int r = 0; r < kRG; ++r)
#pragma unroll
            for (int q = 0; q < CPL; ++q) acc[r][q] += v[r] * x[q];
    }
    const size_t base = (size_t)g * kRG * W + c;
    if (MODE == kPlain) {
#pragma unroll
        for (int r = 0; r < kRG; ++r)
#pragma unroll
            for (int q = 0; q < CPL; ++q) Yout[base + (size_t)r * W + q] = acc[r][q];
        return;
    }
    double d[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
        d[q] = 0.0;
        if (MODE == kPq) {
            const double b = a.beta[c + q];
#pragma unroll
            for (int r = 0; r < kRG; ++r) {
                const size_t e = base + (size_t)r * W + q;
                // beta = 0 (first iteration, converged column): Pd and Q may
                // hold anything, so they are not read
                const double pd = b != 0.0 ? Xin[e] + b * a.Pd[e] : Xin[e];
                const double qv = b != 0.0 ? acc[r][q] + b * a.Q[e] : acc[r][q];
                a.Pd[e] = pd;
                a.Q[e] = qv;
                d[q] += pd * qv;
            }
        } else {
#pragma unroll
            for (int r = 0; r < kRG; ++r) {
                const size_t e = base + (size_t)r * W + q;
                a.Z[e] = acc[r][q];
                d[q] += a.R[e] * acc[r][q];
            }
        }
    }
    // column sums over the 16 waves (fixed order), wave 0 writes them
#pragma unroll
    for (int q = 0; q < CPL; ++q) red[wv][lane * CPL + q] = d[q];
    __syncthreads();
    if (wv == 0) {
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            double sum = 0.0;
            for (int k = 0; k < kWv; ++k) sum += red[k][lane * CPL + q];
            a.part[(size_t)bx * W + c + q] = sum;
        }
    }
}

// X = 0, R = B, part = B . B.
__global__ void __launch_bounds__(1024) cg_init_kernel(CgArgs a) {
    __shared__ double red[kWv][64];
    int bx, y;
    if (!tile_of(a.t, bx, y)) return;
    const int W = a.W;
    const int g = bx * kWv + (threadIdx.x >> 6);
    const int c = y * 64 + (threadIdx.x & 63);
    double d = 0.0;
#pragma unroll
    for (int r = 0; r < kRG; ++r) {
        const size_t e = ((size_t)g * kRG + r) * W + c;
        const double b = a.B[e];
        a.X[e] = 0.0;
        a.R[e] = b;
        d += b * b;
    }
    const double s = wg_column_sum(d, red);
    if (threadIdx.x < 64) a.part[(size_t)bx * W + c] = s;
}

// X += alpha Pd, R -= alpha Q, part = R . R.
__global__ void __launch_bounds__(1024) cg_update_kernel(CgArgs a) {
    __shared__ double red[kWv][64];
    int bx, y;
    if (!tile_of(a.t, bx, y)) return;
    const int W = a.W;
    if (a.active[y] == 0) return;
    const int g = bx * kWv + (threadIdx.x >> 6);
    const int c = y * 64 + (threadIdx.x & 63);
    const double al = a.alpha[c];
    double d = 0.0;
#pragma unroll
    for (int r = 0; r < kRG; ++r) {
        const size_t e = ((size_t)g * kRG + r) * W + c;
        a.X[e] += al * a.Pd[e];
        const double rv = a.R[e] - al * a.Q[e];
        a.R[e] = rv;
        d += rv * rv;
    }
    const double s = wg_column_sum(d, red);
    if (threadIdx.x < 64) a.part[(size_t)bx * W + c] = s;
}

enum { kSumBB = 0, kSumPQ = 1, kSumRR = 2, kSumRZ = 3 };

// Column totals of the producer's parts (x < nx, fixed order: 16 strided
// slices, then the slices in order) and the scalar step of the iteration,
// one workgroup per 64-column group:
//   kSumBB: bb = B . B, done = (bb == 0 or not finite), beta = alpha = 0,
//           active count;
//   kSumPQ: alpha = rz / (Pd . Q) (0 for converged columns);
//   kSumRR: done once R . R <= tol^2 bb (or R . R is not finite: a diverged
//           recursion stops its solves at once, its moments report it),
//           active count, iteration count;
//   kSumRZ: beta = rz_new / rz (0 on the first iteration), rz = rz_new.
// The scalar step of column c from its total; returns whether the column is
// still iterating (meaningful for kSumBB and kSumRR).
template <int MODE>
__device__ inline bool cg_column_step(const CgArgs& a, int c, double tot) {
    if (MODE == kSumBB) {
        const bool dn = !(tot > 0.0) || !isfinite(tot);
        a.bb[c] = tot;
        a.done[c] = dn ? 1 : 0;
        a.beta[c] = 0.0;
        a.alpha[c] = 0.0;
        return !dn;
    } else if (MODE == kSumPQ) {
        double al = 0.0;
        if (a.done[c] == 0) {
            if (tot > 0.0)
                al = a.rz[c] / tot;
            else
                a.done[c] = 1;  // zero search direction: the residual is already zero
        }
        a.alpha[c] = al;
        return false;
    } else if (MODE == kSumRR) {
        bool dn = a.done[c] != 0;
        if (!dn && (tot <= a.tol2 * a.bb[c] || !isfinite(tot))) {
            dn = true;
            a.done[c] = 1;
        }
        return !dn;
    } else {
        const bool dn = a.done[c] != 0;
        a.beta[c] = (a.first || dn || !(a.rz[c] > 0.0)) ? 0.0 : tot / a.rz[c];
        a.rz[c] = tot;
        return false;
    }
}

template <int MODE>
__global__ void __launch_bounds__(1024) cg_colsum_kernel(CgArgs a) {
    __shared__ double red[kWv][64];
    const int y = blockIdx.x;
    if (MODE != kSumBB && a.active[y] == 0) return;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c = y * 64 + lane;
    double s = 0.0;
    for (int x = w; x < a.t.nx; x += kWv) s += a.part[(size_t)x * a.W + c];
    const double tot = wg_column_sum(s, red);
    if (w != 0) return;
    const bool live = cg_column_step<MODE>(a, c, tot);
    if (MODE == kSumBB || MODE == kSumRR) {
        const unsigned long long lv = __ballot(live);
        if (lane == 0) {
            a.active[y] = __popcll(lv);
            if (MODE == kSumBB)
                a.iters[y] = 0;
            else
                a.iters[y] += 1;
        }
    }
}

// ------------------------------------------------------ single-vector solves
// The Lanczos bounds apply H to one vector at a time, where a block kernel
// would leave 63 of its 64 lanes idle.  One vector (v[i], i < Kr) has its
// own kernels: a wave per row group with the lanes over the group's listed
// columns (one gathered value per entry), the four row sums reduced by
// butterfly shuffles; one partial dot product per workgroup, added in index
// order by a one-workgroup kernel that takes the same scalar step as the
// block's column sums.  Results do not depend on timing.
constexpr int kVecWv = 4;  // waves per workgroup of the vector product

// Sum of v over a 256-thread workgroup, valid in thread 0 (butterfly within
// each wave, then the four waves in order).
__device__ inline double wg256_sum(double v, double* red4) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red4[threadIdx.x >> 6] = v;
    __syncthreads();
    return ((red4[0] + red4[1]) + red4[2]) + red4[3];
}

// y = A x for one vector (kPlain); kPq: Pd = Z + beta Pd, Q = A Z + beta Q,
// part = Pd . Q; kRz: Z = A T, part = R . Z (x and y as for the block).
template <int MODE>
__global__ void __launch_bounds__(256) rg_spmv_kernel(RgView A, const double* __restrict__ x,
                                                      double* __restrict__ y, CgArgs a) {
    __shared__ double red[kVecWv];
    if (a.active && a.active[0] == 0) return;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = blockIdx.x * kVecWv + wv;
    const long long p0 = A.ptr[g], p1 = A.ptr[g + 1];
    double acc[kRG];
#pragma unroll
    for (int r = 0; r < kRG; ++r) acc[r] = 0.0;
    for (long long p = p0 + lane; p < p1; p += 64) {
        const double xv = x[A.col[p]];
        const double2* v = reinterpret_cast<const double2*>(A.val + p * kRG);
#pragma unroll
        for (int h = 0; h < kRG / 2; ++h) {
            const double2 w = v[h];
            acc[2 * h] += w.x * xv;
            acc[2 * h + 1] += w.y * xv;
        }
    }
#pragma unroll
    for (int r = 0; r < kRG; ++r)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc[r] += __shfl_xor(acc[r], off, 64);
    // every lane holds the row sums; lane r < kRG handles row kRG g + r
    double sr = acc[0];
#pragma unroll
    for (int r = 1; r < kRG; ++r) sr = lane == r ? acc[r] : sr;
    const int i = g * kRG + lane;
    double d = 0.0;
    if (lane < kRG) {
        if (MODE == kPlain) {
            y[i] = sr;
        } else if (MODE == kPq) {
            const double b = a.beta[0];
            const double pd = b != 0.0 ? x[i] + b * a.Pd[i] : x[i];
            const double qv = b != 0.0 ? sr + b * a.Q[i] : sr;
            a.Pd[i] = pd;
            a.Q[i] = qv;
            d = pd * qv;
        } else {
            y[i] = sr;
            d = a.R[i] * sr;
        }
    }
    if (MODE == kPlain) return;
    double dg = __shfl(d, 0, 64);
#pragma unroll
    for (int r = 1; r < kRG; ++r) dg += __shfl(d, r, 64);
    if (lane == 0) red[wv] = dg;
    __syncthreads();
    if (threadIdx.x == 0) a.part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// X = 0, R = B, part = B . B over v[0..n).
__global__ void __launch_bounds__(256) vec_init_kernel(int n, CgArgs a) {
    __shared__ double red[4];
    const int i = blockIdx.x * 256 + threadIdx.x;
    double d = 0.0;
    if (i < n) {
        const double b = a.B[i];
        a.X[i] = 0.0;
        a.R[i] = b;
        d = b * b;
    }
    const double s = wg256_sum(d, red);
    if (threadIdx.x == 0) a.part[blockIdx.x] = s;
}

// X += alpha Pd, R -= alpha Q, part = R . R.
__global__ void __launch_bounds__(256) vec_update_kernel(int n, CgArgs a) {
    __shared__ double red[4];
    if (a.active[0] == 0) return;
    const int i = blockIdx.x * 256 + threadIdx.x;
    double d = 0.0;
    if (i < n) {
        const double al = a.alpha[0];
        a.X[i] += al * a.Pd[i];
        const double rv = a.R[i] - al * a.Q[i];
        a.R[i] = rv;
        d = rv * rv;
    }
    const double s = wg256_sum(d, red);
    if (threadIdx.x == 0) a.part[blockIdx.x] = s;
}

// Total of part[0..nparts) in a fixed order and the scalar step.
template <int MODE>
__global__ void __launch_bounds__(256) vec_sum_kernel(int nparts, CgArgs a) {
    __shared__ double red[4];
    if (MODE != kSumBB && a.active[0] == 0) return;
    double s = 0.0;
    for (int k = threadIdx.x; k < nparts; k += 256) s += a.part[k];
    const double tot = wg256_sum(s, red);
    if (threadIdx.x != 0) return;
    const bool live = cg_column_step<MODE>(a, 0, tot);
    if (MODE == kSumBB) {
        a.active[0] = live ? 1 : 0;
        a.iters[0] = 0;
    } else if (MODE == kSumRR) {
        a.active[0] = live ? 1 : 0;
        a.iters[0] += 1;
    }
}

// Per solve: fold the iteration counts into the totals, flag groups that
// did not converge.
__global__ void cg_fold_kernel(int ngroups, const int* active, const int* iters, long long* tot,
                               int* mx, int* notconv) {
    const int y = threadIdx.x;
    if (y >= ngroups) return;
    tot[y] += iters[y];
    mx[y] = max(mx[y], iters[y]);
    if (active[y] != 0) notconv[0] = 1;
}

// One step of the recursion on the block (eq. ChebychevExpansion):
//   Unew = sx X + su Ucur - (has_prev ? Uprev : 0)   -> Uout (may alias Uprev)
//   P_q (+)= coef[q cstride + l] Unew for q < nsets   (assigned when l == 0)
//   mpart[l * ng * nx + y * nx + x] = this workgroup's sum of Zm . Unew
struct StepArgs {
    int W, l, nsets, cstride, has_prev;
    Tiles t;
    const double* X;
    const double* Ucur;
    const double* Uprev;
    double* Uout;
    double sx, su;
    const double* coef;
    double* P;
    long long pstride;
    const double* Zm;
    double* mpart;
};

__global__ void __launch_bounds__(1024) fact_step_kernel(StepArgs a) {
    __shared__ double red[kWv][64];
    int bx, y;
    if (!tile_of(a.t, bx, y)) return;
    const int W = a.W, nx = a.t.nx;
    const int g = bx * kWv + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int c = y * 64 + lane;
    double d = 0.0;
#pragma unroll
    for (int r = 0; r < kRG; ++r) {
        const size_t e = ((size_t)g * kRG + r) * W + c;
        double u = a.sx * a.X[e];
        if (a.su != 0.0) u += a.su * a.Ucur[e];
        if (a.has_prev) u -= a.Uprev[e];
        a.Uout[e] = u;
        for (int q = 0; q < a.nsets; ++q) {
            double* P = a.P + (size_t)q * a.pstride;
            const double cq = a.coef[q * a.cstride + a.l];
            P[e] = a.l == 0 ? cq * u : P[e] + cq * u;
        }
        d += a.Zm[e] * u;
    }
    double s = wg_column_sum(d, red);
    if (threadIdx.x < 64) {
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (threadIdx.x == 0) a.mpart[((size_t)a.l * a.t.ng + y) * nx + bx] = s;
    }
}

// Y = unit vectors e_{cols[c]} (c < nc), zero elsewhere.
__global__ void fact_unit_kernel(int Kr, int W, int nc, const long long* cols, double* Y) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)Kr * W) return;
    const int c = (int)(e % W);
    const long long i = (long long)(e / W);
    Y[e] = (c < nc && cols[c] == i) ? 1.0 : 0.0;
}

// Zm[:, c] = column cols[c] of S (= its row: S is symmetric); Zm zero on entry.
__global__ void fact_zm_kernel(int W, int nc, const long long* cols, const long long* Srp,
                               const int* Scol, const double* Sval, double* Zm) {
    const int c = blockIdx.x;
    if (c >= nc) return;
    const long long row = cols[c];
    for (long long p = Srp[row] + threadIdx.x; p < Srp[row + 1]; p += blockDim.x)
        Zm[(size_t)Scol[p] * W + c] = Sval[p];
}

// Column-major K x n (ld) <-> row-interleaved block (W), 32 x 32 tiles.
__global__ void to_block_kernel(int K, int n, const double* src, long long ld, int W, double* dst) {
    __shared__ double t[32][33];
    const int i0 = blockIdx.x * 32, c0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: ty < 8
    for (int k = ty; k < 32; k += 8) {
        const int i = i0 + tx, c = c0 + k;
        t[k][tx] = (i < K && c < n) ? src[(size_t)c * ld + i] : 0.0;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int i = i0 + k, c = c0 + tx;
        dst[(size_t)i * W + c] = t[tx][k];
    }
}

__global__ void from_block_kernel(int K, int n, const double* src, int W, double* dst, long long ld) {
    __shared__ double t[32][33];
    const int i0 = blockIdx.x * 32, c0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int k = ty; k < 32; k += 8) {
        const int i = i0 + k, c = c0 + tx;
        t[k][tx] = src[(size_t)i * W + c];
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int i = i0 + tx, c = c0 + k;
        if (i < K && c < n) dst[(size_t)c * ld + i] = t[tx][k];
    }
}

// rg_val[e] = src[idx[e]] (0 where idx[e] < 0)
__global__ void gather_vals_kernel(long long n, const int* idx, const double* src, double* dst) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int k = idx[e];
    dst[e] = k >= 0 ? src[k] : 0.0;
}

// One FSAI row per workgroup: with J the row's pattern (sorted, ending with
// the row itself), factor S[J, J] = L L^T in LDS and solve L^T g = e_last;
// g is row i of G on J (G S G^T then has a unit diagonal, and G = L_S^-1
// when J is the whole lower triangle).  The lower triangle is stored packed
// (row r at r (r + 1) / 2), so patterns of up to 192 entries fit.
// info[0] = some failing row + 1.
__device__ inline int tri(int r, int t) { return r * (r + 1) / 2 + t; }

__global__ void __launch_bounds__(256) fsai_kernel(const long long* Srp, const int* Scol,
                                                   const double* Sval, const long long* Grp,
                                                   const int* Gcol, double* Gval, int* info) {
    __shared__ double A[kFsaiMax * (kFsaiMax + 1) / 2];
    __shared__ int J[kFsaiMax];
    __shared__ double acc[kFsaiMax];
    __shared__ int bad;
    const int i = blockIdx.x, tid = threadIdx.x;
    const int w = tid >> 6, lane = tid & 63;
    const long long q0 = Grp[i];
    const int n = (int)(Grp[i + 1] - q0);
    for (int t = tid; t < n; t += 256) J[t] = Gcol[q0 + t];
    for (int e = tid; e < n * (n + 1) / 2; e += 256) A[e] = 0.0;
    if (tid == 0) bad = 0;
    __syncthreads();
    // lower triangle of S[J, J]: row J[r] of S, columns found in J[0..r]
    for (int r = w; r < n; r += 4) {
        const int jr = J[r];
        for (long long p = Srp[jr] + lane; p < Srp[jr + 1]; p += 64) {
            const int k = Scol[p];
            if (k > jr) continue;
            int lo = 0, hi = r;  // search J[0..r]
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (J[mid] < k) lo = mid + 1; else hi = mid;
            }
            if (J[lo] == k) A[tri(r, lo)] = Sval[p];
        }
    }
    __syncthreads();
    // right-looking Cholesky, lower
    for (int k = 0; k < n; ++k) {
        if (tid == 0) {
            const double dkk = A[tri(k, k)];
            if (!(dkk > 0.0)) bad = 1;
            A[tri(k, k)] = dkk > 0.0 ? sqrt(dkk) : 1.0;
        }
        __syncthreads();
        if (bad) break;
        const double piv = A[tri(k, k)];
        for (int r = k + 1 + tid; r < n; r += 256) A[tri(r, k)] /= piv;
        __syncthreads();
        for (int r = k + 1 + w; r < n; r += 4) {
            const double ark = A[tri(r, k)];
            for (int t = k + 1 + lane; t <= r; t += 64) A[tri(r, t)] -= ark * A[tri(t, k)];
        }
        __syncthreads();
    }
    if (bad) {
        for (int t = tid; t < n; t += 256) Gval[q0 + t] = 0.0;
        if (tid == 0) atomicCAS(info, 0, i + 1);
        return;
    }
    // L^T g = e_{n-1} by columns of L, from the last unknown up
    for (int t = tid; t < n; t += 256) acc[t] = t == n - 1 ? 1.0 : 0.0;
    __syncthreads();
    for (int t = n - 1; t >= 0; --t) {
        const double gt = acc[t] / A[tri(t, t)];
        __syncthreads();
        if (tid == 0) acc[t] = gt;
        for (int r = tid; r < t; r += 256) acc[r] -= A[tri(t, r)] * gt;
        __syncthreads();
    }
    for (int t = tid; t < n; t += 256) Gval[q0 + t] = acc[t];
}

// --------------------------------------------------------------- host side
// Device buffer owned by its holder (freed on release or destruction).
template <typename T>
struct Buf {
    T* p = nullptr;
    size_t n = 0;
    Buf() = default;
    Buf(const Buf&) = delete;
    Buf& operator=(const Buf&) = delete;
    ~Buf() { release(); }
    hipError_t ensure(size_t m) {
        if (m <= n && p) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
        hipError_t e = hipMalloc(&p, std::max<size_t>(m, 1) * sizeof(T));
        if (e == hipSuccess) n = m;
        return e;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
};

struct RgMat {
    Buf<long long> ptr;
    Buf<int> col;
    Buf<double> val;
    Buf<int> src;  // G and G^T: value source index into the CSR values of G
    long long nent = 0;
    RgView view() const { return RgView{ptr.p, col.p, val.p}; }
    void release() {
        ptr.release(); col.release(); val.release(); src.release();
        nent = 0;
    }
};

// Row-group layout of a CSR matrix (rows >= K and groups beyond the matrix
// are empty).  vals may be null; then srcidx[e] receives the CSR position
// of each slot (-1 for the zero slots).
void row_groups(int K, int Kr, const std::vector<long long>& rp, const std::vector<int>& ci,
                const double* vals, std::vector<long long>& gptr, std::vector<int>& gcol,
                std::vector<double>& gval, std::vector<int>& srcidx) {
    const int ng = Kr / kRG;
    gptr.assign((size_t)ng + 1, 0);
    gcol.clear();
    gval.clear();
    srcidx.clear();
    std::vector<long long> pos(kRG);
    for (int g = 0; g < ng; ++g) {
        for (int r = 0; r < kRG; ++r) {
            const long long row = (long long)g * kRG + r;
            pos[r] = row < K ? rp[row] : 0;
        }
        while (true) {
            int next = 0x7fffffff;
            for (int r = 0; r < kRG; ++r) {
                const long long row = (long long)g * kRG + r;
                if (row < K && pos[r] < rp[row + 1]) next = std::min(next, ci[pos[r]]);
            }
            if (next == 0x7fffffff) break;
            gcol.push_back(next);
            for (int r = 0; r < kRG; ++r) {
                const long long row = (long long)g * kRG + r;
                long long k = -1;
                if (row < K && pos[r] < rp[row + 1] && ci[pos[r]] == next) k = pos[r]++;
                if (vals)
                    gval.push_back(k >= 0 ? vals[k] : 0.0);
                else
                    srcidx.push_back((int)k);
            }
        }
        gptr[g + 1] = (long long)gcol.size();
    }
}

}  // namespace

struct FactOp {
    int K = 0, Kr = 0;
    RgMat S, F, G, GT;
    Buf<long long> Srp, Grp;
    Buf<int> Scol, Gcol;
    Buf<double> Sval, Gval;
    long long g_nnz = 0;
    // workspace of width W
    int W = 0;
    Buf<double> B, X, R, Z, Pd, Q, T, U0, U1, Zm, P, Pout;
    Buf<double> bb, rz, alpha, beta, part, mpart;
    Buf<int> done, active, iters, mx, notconv;
    Buf<long long> tot;
    int* h_active = nullptr;  // pinned, 2 x ngroups
    int h_cap = 0;
    int nsets_cap = 0, order_cap = 0;
    long long solves = 0;
    // optional timing of the S products of the iterations (dispatch events)
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    hipEvent_t poll[2] = {nullptr, nullptr};  // convergence polling, one per chunk parity
    long long timed_launches = 0;
    double timed_ms = 0.0;
    ~FactOp() {
        for (RgMat* m : {&S, &F, &G, &GT}) m->release();
        Srp.release(); Grp.release(); Scol.release(); Gcol.release(); Sval.release(); Gval.release();
        for (auto* b : {&B, &X, &R, &Z, &Pd, &Q, &T, &U0, &U1, &Zm, &P, &Pout, &bb, &rz, &alpha, &beta, &part,
                        &mpart})
            b->release();
        for (auto* b : {&done, &active, &iters, &mx, &notconv}) b->release();
        tot.release();
        if (h_active) (void)hipHostFree(h_active);
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
        for (hipEvent_t e : poll)
            if (e) (void)hipEventDestroy(e);
    }
};

namespace {

#define FTRY(expr)                              \
    do {                                        \
        hipError_t e_ = (expr);                 \
        if (e_ != hipSuccess) return e_;        \
    } while (0)

hipError_t upload_rg(RgMat& m, const std::vector<long long>& gptr, const std::vector<int>& gcol,
                     const std::vector<double>& gval, const std::vector<int>& src, hipStream_t s) {
    m.nent = (long long)gcol.size();
    FTRY(m.ptr.ensure(gptr.size()));
    FTRY(m.col.ensure(gcol.size()));
    FTRY(m.val.ensure(gcol.size() * kRG));
    FTRY(hipMemcpyAsync(m.ptr.p, gptr.data(), gptr.size() * 8, hipMemcpyHostToDevice, s));
    if (!gcol.empty()) FTRY(hipMemcpyAsync(m.col.p, gcol.data(), gcol.size() * 4, hipMemcpyHostToDevice, s));
    if (!gval.empty()) FTRY(hipMemcpyAsync(m.val.p, gval.data(), gval.size() * 8, hipMemcpyHostToDevice, s));
    if (!src.empty()) {
        FTRY(m.src.ensure(src.size()));
        FTRY(hipMemcpyAsync(m.src.p, src.data(), src.size() * 4, hipMemcpyHostToDevice, s));
    }
    return hipSuccess;
}

hipError_t ensure_width(FactOp* f, int W, int nsets, int order, hipStream_t s) {
    const size_t nb = (size_t)f->Kr * W;
    const int ng = W / 64, nx = f->Kr / kRowsWG;
    if (W > f->W) {
        for (auto* b : {&f->B, &f->X, &f->R, &f->Z, &f->Pd, &f->Q, &f->T, &f->U0, &f->U1, &f->Zm, &f->Pout})
            FTRY(b->ensure(nb));
        FTRY(f->bb.ensure(W));
        FTRY(f->rz.ensure(W));
        FTRY(f->alpha.ensure(W));
        FTRY(f->beta.ensure(W));
        FTRY(f->done.ensure(W));
        FTRY(f->part.ensure((size_t)nx * W));
        FTRY(f->active.ensure(ng));
        FTRY(f->iters.ensure(ng));
        FTRY(f->mx.ensure(ng));
        FTRY(f->tot.ensure(ng));
        FTRY(f->notconv.ensure(1));
        FTRY(hipMemsetAsync(f->mx.p, 0, (size_t)ng * sizeof(int), s));
        FTRY(hipMemsetAsync(f->tot.p, 0, (size_t)ng * sizeof(long long), s));
        FTRY(hipMemsetAsync(f->notconv.p, 0, sizeof(int), s));
        if (f->h_active) (void)hipHostFree(f->h_active);
        f->h_active = nullptr;
        FTRY(hipHostMalloc((void**)&f->h_active, (size_t)2 * ng * sizeof(int), hipHostMallocDefault));
        f->h_cap = ng;
        f->W = W;
        f->nsets_cap = 0;
        f->order_cap = 0;
    }
    if (nsets > f->nsets_cap) {
        FTRY(f->P.ensure((size_t)f->Kr * f->W * nsets));
        f->nsets_cap = nsets;
    }
    if (order > f->order_cap) {
        FTRY(f->mpart.ensure((size_t)(order + 1) * (f->W / 64) * (f->Kr / kRowsWG)));
        f->order_cap = order;
    }
    return hipSuccess;
}

Tiles tiles_for(const FactOp* f, int W) {
    Tiles t;
    t.nx = f->Kr / kRowsWG;
    t.ng = W / 64;
    t.xcd_split = t.ng >= 8 ? 1 : 0;
    return t;
}

// 1-D grid of the row kernels for these tiles
dim3 tile_grid(const Tiles& t) {
    if (t.xcd_split) return dim3((unsigned)(t.nx * 8 * ((t.ng + 7) / 8)));
    return dim3((unsigned)(t.nx * t.ng));
}

// Launch of a row-group product over the block: two columns per lane when
// the width is a multiple of 128, else one.  (Measured at K = 4096 on the
// whole block, per CG iteration: one column per lane 3.5 ms, two 2.2 ms,
// four 2.9 ms - at 90 registers only one 1024-thread workgroup fits a CU.)
template <int MODE>
void launch_spmm(const FactOp* f, const RgMat& A, const double* X, double* Y, const CgArgs& a, hipStream_t s,
                 hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr) {
    Tiles t = a.t;
    const int cpl = a.W % 128 == 0 ? 2 : 1;
    t.ng = a.W / (64 * cpl);
    t.xcd_split = t.ng >= 8 ? 1 : 0;
    const dim3 grid = tile_grid(t), blk(1024);
    auto k2 = rg_spmm_kernel<MODE, 2>;
    auto k1 = rg_spmm_kernel<MODE, 1>;
    auto k = cpl == 2 ? k2 : k1;
    if (t0)
        hipExtLaunchKernelGGL(k, grid, blk, 0, s, t0, t1, 0, A.view(), X, Y, a, t);
    else
        hipLaunchKernelGGL(k, grid, blk, 0, s, A.view(), X, Y, a, t);
}

CgArgs cg_args(FactOp* f, int W, double tol) {
    CgArgs a{};
    a.W = W;
    a.t = tiles_for(f, W);
    a.B = f->B.p;
    a.X = f->X.p;
    a.R = f->R.p;
    a.Z = f->Z.p;
    a.Pd = f->Pd.p;
    a.Q = f->Q.p;
    a.T = f->T.p;
    a.bb = f->bb.p;
    a.rz = f->rz.p;
    a.alpha = f->alpha.p;
    a.beta = f->beta.p;
    a.done = f->done.p;
    a.active = f->active.p;
    a.iters = f->iters.p;
    a.part = f->part.p;
    a.tol2 = tol * tol;
    a.first = 0;
    return a;
}

// Launches of one CG solve: on a block of width W (a multiple of 64), or,
// with W = 1, on one vector v[0..Kr) in the first Kr elements of the
// workspace buffers.
struct CgLaunch {
    FactOp* f;
    bool vec;
    int ng;          // column groups (1 for a vector)
    int nvp, nve;    // vector: partials of the products and of the element kernels
    dim3 grid, gsum; // block: row-kernel grid, column-sum grid
    hipStream_t s;
    template <int MODE>
    void spmm(const RgMat& A, const double* X, double* Y, const CgArgs& a, hipEvent_t t0 = nullptr,
              hipEvent_t t1 = nullptr) const {
        if (!vec) {
            launch_spmm<MODE>(f, A, X, Y, a, s, t0, t1);
            return;
        }
        auto k = rg_spmv_kernel<MODE>;
        if (t0)
            hipExtLaunchKernelGGL(k, dim3(nvp), dim3(256), 0, s, t0, t1, 0, A.view(), X, Y, a);
        else
            hipLaunchKernelGGL(k, dim3(nvp), dim3(256), 0, s, A.view(), X, Y, a);
    }
    template <int MODE>
    void sum(const CgArgs& a) const {
        if (vec)
            hipLaunchKernelGGL(vec_sum_kernel<MODE>, dim3(1), dim3(256), 0, s,
                               (MODE == kSumPQ || MODE == kSumRZ) ? nvp : nve, a);
        else
            hipLaunchKernelGGL(cg_colsum_kernel<MODE>, gsum, dim3(1024), 0, s, a);
    }
    void init(const CgArgs& a) const {
        if (vec)
            hipLaunchKernelGGL(vec_init_kernel, dim3(nve), dim3(256), 0, s, f->Kr, a);
        else
            hipLaunchKernelGGL(cg_init_kernel, grid, dim3(1024), 0, s, a);
    }
    void update(const CgArgs& a) const {
        if (vec)
            hipLaunchKernelGGL(vec_update_kernel, dim3(nve), dim3(256), 0, s, f->Kr, a);
        else
            hipLaunchKernelGGL(cg_update_kernel, grid, dim3(1024), 0, s, a);
    }
};

// X = S^-1 B on the block (width W <= f->W) or on one vector (W = 1), B and
// X in the workspace.  *converged = 0 when some column needed more than
// max_iter iterations.
hipError_t cg_solve(FactOp* f, int W, double tol, int max_iter, int* converged, hipStream_t s) {
    const bool vec = W == 1;
    const int ng = vec ? 1 : W / 64;
    max_iter = std::max(max_iter, 1);
    CgArgs a = cg_args(f, W, tol);
    CgLaunch L{f, vec, ng, f->Kr / (kRG * kVecWv), (f->Kr + 255) / 256, vec ? dim3(1) : tile_grid(a.t), dim3(ng), s};
    L.init(a);
    L.sum<kSumBB>(a);
    FTRY(hipGetLastError());
    // Z = G^T (G R): preconditioned residual, rz = R . Z
    {
        CgArgs p = a;
        p.first = 1;
        L.spmm<kPlain>(f->G, a.R, a.T, p);
        L.spmm<kRz>(f->GT, a.T, a.Z, p);
        L.sum<kSumRZ>(p);
        FTRY(hipGetLastError());
    }
    int it = 0, chunk = 0, nev = 0;  // nev: timing events used by this solve
    bool conv = false;
    auto timed_event = [&](hipEvent_t* out) -> hipError_t {
        if ((size_t)nev == f->ev_pool.size()) {
            hipEvent_t e;
            FTRY(hipEventCreate(&e));
            f->ev_pool.push_back(e);
        }
        *out = f->ev_pool[nev++];
        return hipSuccess;
    };
    for (hipEvent_t& e : f->poll)
        if (!e) FTRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    hipEvent_t* ev = f->poll;
    hipError_t err = hipSuccess;
    auto check = [&](int k) -> int {  // active columns seen after chunk k
        int n = 0;
        for (int y = 0; y < ng; ++y) n += f->h_active[(k & 1) * f->h_cap + y];
        return n;
    };
    while (err == hipSuccess && it < max_iter) {
        const int n_it = std::min(kChunk, max_iter - it);
        for (int k = 0; k < n_it; ++k) {
            hipEvent_t t0 = nullptr, t1 = nullptr;  // start and stop taken by the dispatch itself
            if (f->timing && !vec &&
                ((err = timed_event(&t0)) != hipSuccess || (err = timed_event(&t1)) != hipSuccess))
                break;
            L.spmm<kPq>(f->S, a.Z, a.Q, a, t0, t1);
            L.sum<kSumPQ>(a);
            L.update(a);
            L.sum<kSumRR>(a);
            L.spmm<kPlain>(f->G, a.R, a.T, a);
            L.spmm<kRz>(f->GT, a.T, a.Z, a);
            L.sum<kSumRZ>(a);
        }
        if (err != hipSuccess) break;
        it += n_it;
        if ((err = hipGetLastError()) != hipSuccess) break;
        const int slot = chunk & 1;
        if ((err = hipMemcpyAsync(f->h_active + slot * f->h_cap, f->active.p, (size_t)ng * sizeof(int),
                                  hipMemcpyDeviceToHost, s)) != hipSuccess)
            break;
        if ((err = hipEventRecord(ev[slot], s)) != hipSuccess) break;
        if (chunk > 0) {
            if ((err = hipEventSynchronize(ev[slot ^ 1])) != hipSuccess) break;
            if (check(chunk - 1) == 0) {
                conv = true;
                break;
            }
        }
        ++chunk;
    }
    if (err == hipSuccess && !conv) {
        // the last chunk decides
        const int last = (chunk > 0 && it >= max_iter) ? chunk - 1 : chunk;
        if ((err = hipEventSynchronize(ev[last & 1])) == hipSuccess) conv = check(last) == 0;
    }
    FTRY(err);
    if (f->timing && nev > 0) {
        // launches after convergence return at once: count only the
        // products of iterations that ran for some column group
        std::vector<int> itg(ng);
        FTRY(hipMemcpyAsync(itg.data(), f->iters.p, (size_t)ng * sizeof(int), hipMemcpyDeviceToHost, s));
        FTRY(hipStreamSynchronize(s));
        int ran = 0;
        for (int v : itg) ran = std::max(ran, v);
        for (int k = 0; k < std::min(ran, nev / 2); ++k) {
            float ms = 0.0f;
            FTRY(hipEventElapsedTime(&ms, f->ev_pool[2 * k], f->ev_pool[2 * k + 1]));
            f->timed_ms += ms;
            f->timed_launches += 1;
        }
    }
    hipLaunchKernelGGL(cg_fold_kernel, dim3(1), dim3(std::max(64, (ng + 63) / 64 * 64)), 0, s, ng, f->active.p,
                       f->iters.p, f->tot.p, f->mx.p, f->notconv.p);
    FTRY(hipGetLastError());
    f->solves += 1;
    *converged = conv ? 1 : 0;
    return hipSuccess;
}

}  // namespace

FactOp* fact_create() { return new FactOp(); }
void fact_destroy(FactOp* f) { delete f; }

hipError_t fact_setup(FactOp* f, int K, const long long* Frp, const int* Fcol, const double* Fval,
                      const long long* Srp, const int* Scol, const double* Sval, double drop, int cap,
                      int* bad_row, hipStream_t s) {
    *bad_row = 0;
    if (cap < 1 || cap > kFsaiMax || K <= 0) return hipErrorInvalidValue;
    f->K = K;
    f->Kr = (K + kRowsWG - 1) / kRowsWG * kRowsWG;
    f->W = 0;
    f->solves = 0;
    const long long snnz = Srp[K], fnnz = Frp[K];
    std::vector<long long> srp(Srp, Srp + K + 1), frp(Frp, Frp + K + 1);
    std::vector<int> scol(Scol, Scol + snnz), fcol(Fcol, Fcol + fnnz);
    // FSAI pattern: lower entries with |S_ij| >= drop sqrt(S_ii S_jj), the
    // cap - 1 largest of them, plus the diagonal (last)
    std::vector<double> diag(K, 0.0);
    for (int i = 0; i < K; ++i)
        for (long long p = srp[i]; p < srp[i + 1]; ++p)
            if (scol[p] == i) diag[i] = Sval[p];
    std::vector<long long> grp((size_t)K + 1, 0);
    std::vector<int> gcol;
    std::vector<std::pair<double, int>> cand;
    for (int i = 0; i < K; ++i) {
        cand.clear();
        for (long long p = srp[i]; p < srp[i + 1]; ++p) {
            const int j = scol[p];
            if (j >= i) continue;
            const double rel = std::fabs(Sval[p]) / std::sqrt(std::fabs(diag[i] * diag[j]) + 1e-300);
            if (rel >= drop) cand.push_back({rel, j});
        }
        if ((int)cand.size() > cap - 1) {
            std::stable_sort(cand.begin(), cand.end(),
                             [](const std::pair<double, int>& x, const std::pair<double, int>& y) {
                                 return x.first > y.first;
                             });
            cand.resize(cap - 1);
        }
        std::vector<int> J;
        for (auto& pr : cand) J.push_back(pr.second);
        std::sort(J.begin(), J.end());
        J.push_back(i);
        gcol.insert(gcol.end(), J.begin(), J.end());
        grp[i + 1] = (long long)gcol.size();
    }
    f->g_nnz = (long long)gcol.size();
    if (f->g_nnz >= 0x7fffffffLL || snnz >= 0x7fffffffLL) return hipErrorInvalidValue;
    // plain CSR copies of S (start vectors, moment columns) and of G's pattern
    FTRY(f->Srp.ensure(K + 1));
    FTRY(f->Scol.ensure(std::max<long long>(snnz, 1)));
    FTRY(f->Sval.ensure(std::max<long long>(snnz, 1)));
    FTRY(hipMemcpyAsync(f->Srp.p, srp.data(), srp.size() * 8, hipMemcpyHostToDevice, s));
    FTRY(hipMemcpyAsync(f->Scol.p, scol.data(), (size_t)snnz * 4, hipMemcpyHostToDevice, s));
    FTRY(hipMemcpyAsync(f->Sval.p, Sval, (size_t)snnz * 8, hipMemcpyHostToDevice, s));
    FTRY(f->Grp.ensure(K + 1));
    FTRY(f->Gcol.ensure(gcol.size()));
    FTRY(f->Gval.ensure(gcol.size()));
    FTRY(hipMemcpyAsync(f->Grp.p, grp.data(), grp.size() * 8, hipMemcpyHostToDevice, s));
    FTRY(hipMemcpyAsync(f->Gcol.p, gcol.data(), gcol.size() * 4, hipMemcpyHostToDevice, s));
    Buf<int> info;
    FTRY(info.ensure(1));
    FTRY(hipMemsetAsync(info.p, 0, sizeof(int), s));
    hipLaunchKernelGGL(fsai_kernel, dim3(K), dim3(256), 0, s, f->Srp.p, f->Scol.p, f->Sval.p, f->Grp.p, f->Gcol.p,
                       f->Gval.p, info.p);
    FTRY(hipGetLastError());
    // row groups: S and F from the host values, G and G^T gathered on the device
    std::vector<long long> gp;
    std::vector<int> gc, src;
    std::vector<double> gv;
    row_groups(K, f->Kr, srp, scol, Sval, gp, gc, gv, src);
    FTRY(upload_rg(f->S, gp, gc, gv, src, s));
    row_groups(K, f->Kr, frp, fcol, Fval, gp, gc, gv, src);
    FTRY(upload_rg(f->F, gp, gc, gv, src, s));
    row_groups(K, f->Kr, grp, gcol, nullptr, gp, gc, gv, src);
    FTRY(upload_rg(f->G, gp, gc, gv, src, s));
    {
        const long long n = (long long)src.size();
        if (n > 0)
            hipLaunchKernelGGL(gather_vals_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, f->G.src.p,
                               (const double*)f->Gval.p, f->G.val.p);
        FTRY(hipGetLastError());
    }
    // G^T in CSR; tpos[d] = position in G of the d-th entry of G^T
    std::vector<long long> trp((size_t)K + 1, 0);
    for (int cidx : gcol) trp[cidx + 1] += 1;
    for (int i = 0; i < K; ++i) trp[i + 1] += trp[i];
    std::vector<int> tcol(gcol.size()), tpos(gcol.size());
    {
        std::vector<long long> fillp(trp.begin(), trp.end() - 1);
        for (int i = 0; i < K; ++i)
            for (long long q = grp[i]; q < grp[i + 1]; ++q) {
                const long long d = fillp[gcol[q]]++;
                tcol[d] = i;
                tpos[d] = (int)q;
            }
    }
    row_groups(K, f->Kr, trp, tcol, nullptr, gp, gc, gv, src);
    for (int& k : src) k = k >= 0 ? tpos[k] : -1;
    FTRY(upload_rg(f->GT, gp, gc, gv, src, s));
    {
        const long long n = (long long)src.size();
        if (n > 0)
            hipLaunchKernelGGL(gather_vals_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                               f->GT.src.p, (const double*)f->Gval.p, f->GT.val.p);
        FTRY(hipGetLastError());
    }
    int hinfo = 0;
    FTRY(hipMemcpyAsync(&hinfo, info.p, sizeof(int), hipMemcpyDeviceToHost, s));
    FTRY(hipStreamSynchronize(s));
    info.release();
    *bad_row = hinfo;
    return hipSuccess;
}

long long fact_precond_nnz(const FactOp* f) { return f->g_nnz; }

hipError_t fact_precond_copy(const FactOp* f, long long* rp, int* col, double* val, hipStream_t s) {
    if (rp) FTRY(hipMemcpyAsync(rp, f->Grp.p, ((size_t)f->K + 1) * 8, hipMemcpyDefault, s));
    if (col) FTRY(hipMemcpyAsync(col, f->Gcol.p, (size_t)f->g_nnz * 4, hipMemcpyDefault, s));
    if (val) FTRY(hipMemcpyAsync(val, f->Gval.p, (size_t)f->g_nnz * 8, hipMemcpyDefault, s));
    return hipStreamSynchronize(s);
}


hipError_t fact_solve(FactOp* f, int n, const double* B, long long ldb, double* X, long long ldx, double tol,
                      int max_iter, int wmax, int* converged, hipStream_t s) {
    *converged = 1;
    const int K = f->K;
    for (int off = 0; off < n; off += wmax) {
        const int nc = std::min(wmax, n - off);
        if (nc == 1) {
            // one right-hand side: the single-vector kernels
            FTRY(ensure_width(f, 64, 1, 1, s));
            if (f->Kr > K) FTRY(fill_f64(f->B.p + K, 0.0, f->Kr - K, s));
            FTRY(hipMemcpyAsync(f->B.p, B + (size_t)off * ldb, (size_t)K * 8, hipMemcpyDefault, s));
            int conv = 1;
            FTRY(cg_solve(f, 1, tol, max_iter, &conv, s));
            if (!conv) *converged = 0;
            FTRY(hipMemcpyAsync(X + (size_t)off * ldx, f->X.p, (size_t)K * 8, hipMemcpyDefault, s));
            continue;
        }
        const int W = (nc + 63) / 64 * 64;
        FTRY(ensure_width(f, W, 1, 1, s));
        // stage B through device memory when it lives on the host
        FTRY(f->Pout.ensure((size_t)f->Kr * f->W));
        FTRY(hipMemcpy2DAsync(f->Pout.p, (size_t)K * 8, B + (size_t)off * ldb, (size_t)ldb * 8, (size_t)K * 8, nc,
                              hipMemcpyDefault, s));
        hipLaunchKernelGGL(to_block_kernel, dim3(f->Kr / 32, W / 32), dim3(256), 0, s, K, nc, (const double*)f->Pout.p,
                           (long long)K, W, f->B.p);
        FTRY(hipGetLastError());
        int conv = 1;
        FTRY(cg_solve(f, W, tol, max_iter, &conv, s));
        if (!conv) *converged = 0;
        hipLaunchKernelGGL(from_block_kernel, dim3(f->Kr / 32, W / 32), dim3(256), 0, s, K, nc, (const double*)f->X.p,
                           W, f->Pout.p, (long long)K);
        FTRY(hipGetLastError());
        FTRY(hipMemcpy2DAsync(X + (size_t)off * ldx, (size_t)ldx * 8, f->Pout.p, (size_t)K * 8, (size_t)K * 8, nc,
                              hipMemcpyDefault, s));
    }
    return hipStreamSynchronize(s);
}

hipError_t fact_apply(FactOp* f, const double* x, double* y, double tol, int max_iter, int* converged,
                      hipStream_t s) {
    const int K = f->K, Kr = f->Kr;
    FTRY(ensure_width(f, 64, 1, 1, s));  // the vector lives in the first Kr elements of each buffer
    if (Kr > K) FTRY(fill_f64(f->U0.p + K, 0.0, Kr - K, s));
    FTRY(hipMemcpyAsync(f->U0.p, x, (size_t)K * 8, hipMemcpyDeviceToDevice, s));
    CgArgs a = cg_args(f, 1, tol);
    a.active = nullptr;
    hipLaunchKernelGGL(rg_spmv_kernel<kPlain>, dim3(Kr / (kRG * kVecWv)), dim3(256), 0, s, f->F.view(),
                       (const double*)f->U0.p, f->B.p, a);
    FTRY(hipGetLastError());
    FTRY(cg_solve(f, 1, tol, max_iter, converged, s));
    return hipMemcpyAsync(y, f->X.p, (size_t)K * 8, hipMemcpyDeviceToDevice, s);
}

hipError_t fact_block(FactOp* f, const FactBlockArgs& b, int* converged, hipStream_t s) {
    *converged = 1;
    const int K = f->K, nc = b.nc;
    const int W = (nc + 63) / 64 * 64;
    FTRY(ensure_width(f, W, b.nsets, b.order, s));
    const int ng = W / 64;
    const Tiles tl = tiles_for(f, W);
    const dim3 grid = tile_grid(tl), blk(1024);
    const size_t nb = (size_t)f->Kr * W;
    // start block and moment columns
    hipLaunchKernelGGL(fact_unit_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, f->Kr, W, nc, b.cols,
                       f->B.p);
    FTRY(fill_f64(f->Zm.p, 0.0, (long long)nb, s));
    hipLaunchKernelGGL(fact_zm_kernel, dim3(nc), dim3(256), 0, s, W, nc, b.cols, (const long long*)f->Srp.p,
                       (const int*)f->Scol.p, (const double*)f->Sval.p, f->Zm.p);
    FTRY(hipGetLastError());
    StepArgs st{};
    st.W = W;
    st.t = tl;
    st.nsets = b.nsets;
    st.cstride = b.cstride;
    st.coef = b.coef;
    st.P = f->P.p;
    st.pstride = (long long)nb;
    st.Zm = f->Zm.p;
    st.mpart = f->mpart.p;
    double* Ucur = f->U0.p;
    double* Uoth = f->U1.p;
    CgArgs plain = cg_args(f, W, b.tol);
    plain.active = nullptr;
    for (int l = 0; l <= b.order; ++l) {
        if (l > 0) {
            launch_spmm<kPlain>(f, f->F, Ucur, f->B.p, plain, s);
            FTRY(hipGetLastError());
        }
        int conv = 1;
        FTRY(cg_solve(f, W, b.tol, b.max_iter, &conv, s));
        if (!conv) {
            *converged = 0;
            return hipSuccess;
        }
        st.l = l;
        st.X = f->X.p;
        if (l == 0) {  // U_0 = S^-1 e_cols
            st.sx = 1.0;
            st.su = 0.0;
            st.has_prev = 0;
            st.Ucur = nullptr;
            st.Uprev = nullptr;
            st.Uout = Ucur;
        } else {  // U_{l+1} = alpha (X - ebar U_l) / de - U_{l-1}
            const double al = l == 1 ? 1.0 : 2.0;
            st.sx = al / b.de;
            st.su = -al * b.ebar / b.de;
            st.has_prev = l > 1;
            st.Ucur = Ucur;
            st.Uprev = Uoth;
            st.Uout = Uoth;
        }
        hipLaunchKernelGGL(fact_step_kernel, grid, blk, 0, s, st);
        FTRY(hipGetLastError());
        if (l > 0) std::swap(Ucur, Uoth);
    }
    FTRY(reduce_moments(b.order, ng * tl.nx, f->mpart.p, b.mom, b.flag, s));
    for (int q = 0; q < b.nsets; ++q) {
        if (!b.P_out || !b.P_out[q]) continue;
        hipLaunchKernelGGL(from_block_kernel, dim3(f->Kr / 32, W / 32), dim3(256), 0, s, K, nc,
                           (const double*)(f->P.p + (size_t)q * nb), W, f->Pout.p, (long long)K);
        FTRY(hipGetLastError());
        FTRY(hipMemcpyAsync(b.P_out[q], f->Pout.p, (size_t)K * nc * 8, hipMemcpyDefault, s));
    }
    return hipSuccess;
}

hipError_t fact_stoch(FactOp* f, int n_vec, const double* xi, int n_mom, double ebar, double de, double tol,
                      int max_iter, double* mom, int* flag, int* converged, hipStream_t s) {
    *converged = 1;
    const int K = f->K;
    const int W = (n_vec + 63) / 64 * 64;
    FTRY(ensure_width(f, W, 1, n_mom, s));
    const Tiles tl = tiles_for(f, W);
    const dim3 grid = tile_grid(tl), blk(1024);
    const size_t nb = (size_t)f->Kr * W;
    // the probe vectors become U_0 (through the solution slot X) and the
    // moment vectors Zm
    FTRY(hipMemcpy2DAsync(f->Pout.p, (size_t)K * 8, xi, (size_t)K * 8, (size_t)K * 8, n_vec, hipMemcpyDefault, s));
    hipLaunchKernelGGL(to_block_kernel, dim3(f->Kr / 32, W / 32), dim3(256), 0, s, K, n_vec, (const double*)f->Pout.p,
                       (long long)K, W, f->X.p);
    hipLaunchKernelGGL(to_block_kernel, dim3(f->Kr / 32, W / 32), dim3(256), 0, s, K, n_vec, (const double*)f->Pout.p,
                       (long long)K, W, f->Zm.p);
    FTRY(hipGetLastError());
    StepArgs st{};
    st.W = W;
    st.t = tl;
    st.nsets = 0;  // moments only
    st.P = f->P.p;
    st.pstride = (long long)nb;
    st.Zm = f->Zm.p;
    st.mpart = f->mpart.p;
    double* Ucur = f->U0.p;
    double* Uoth = f->U1.p;
    CgArgs plain = cg_args(f, W, tol);
    plain.active = nullptr;
    for (int l = 0; l < n_mom; ++l) {
        if (l > 0) {
            launch_spmm<kPlain>(f, f->F, Ucur, f->B.p, plain, s);
            FTRY(hipGetLastError());
            int conv = 1;
            FTRY(cg_solve(f, W, tol, max_iter, &conv, s));
            if (!conv) {
                *converged = 0;
                return hipSuccess;
            }
        }
        st.l = l;
        st.X = f->X.p;
        if (l == 0) {
            st.sx = 1.0;
            st.su = 0.0;
            st.has_prev = 0;
            st.Ucur = nullptr;
            st.Uprev = nullptr;
            st.Uout = Ucur;
        } else {
            const double al = l == 1 ? 1.0 : 2.0;
            st.sx = al / de;
            st.su = -al * ebar / de;
            st.has_prev = l > 1;
            st.Ucur = Ucur;
            st.Uprev = Uoth;
            st.Uout = Uoth;
        }
        hipLaunchKernelGGL(fact_step_kernel, grid, blk, 0, s, st);
        FTRY(hipGetLastError());
        if (l > 0) std::swap(Ucur, Uoth);
    }
    return reduce_moments(n_mom - 1, tl.ng * tl.nx, f->mpart.p, mom, flag, s);
}

hipError_t fact_stats(FactOp* f, long long* solves, long long* iters, int* max_iters, hipStream_t s) {
    *solves = f->solves;
    *iters = 0;
    *max_iters = 0;
    const int ng = f->W / 64;
    if (ng == 0) return hipSuccess;
    std::vector<long long> t(ng);
    std::vector<int> m(ng);
    FTRY(hipMemcpyAsync(t.data(), f->tot.p, (size_t)ng * 8, hipMemcpyDeviceToHost, s));
    FTRY(hipMemcpyAsync(m.data(), f->mx.p, (size_t)ng * 4, hipMemcpyDeviceToHost, s));
    FTRY(hipStreamSynchronize(s));
    for (int y = 0; y < ng; ++y) {
        *iters = std::max(*iters, t[y]);
        *max_iters = std::max(*max_iters, m[y]);
    }
    return hipSuccess;
}

void fact_set_timing(FactOp* f, bool on) { f->timing = on; }

void fact_take_timing(FactOp* f, long long* launches, double* ms) {
    *launches = f->timed_launches;
    *ms = f->timed_ms;
    f->timed_launches = 0;
    f->timed_ms = 0.0;
}

hipError_t fact_reset_stats(FactOp* f, hipStream_t s) {
    f->solves = 0;
    const int ng = f->W / 64;
    if (ng == 0) return hipSuccess;
    FTRY(hipMemsetAsync(f->tot.p, 0, (size_t)ng * 8, s));
    FTRY(hipMemsetAsync(f->mx.p, 0, (size_t)ng * 4, s));
    return hipSuccess;
}

}  // namespace dm
