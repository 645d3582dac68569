// Electron density on a uniform grid from density-matrix columns (Method,
// eq. ElectronDensity): n(r_g) += sum_a 2 phi_a(r_g) sum_b phi_b(r_g) P_ba
// over the columns a of a pass.  Each basis function is a normalised s-type
// Gaussian set to zero outside its cube window (grid-window section).
//
// One workgroup per cell of 4 x 4 x 4 grid points.  The host lists, per
// cell, the functions whose window reaches the cell (b-list) and those of
// them whose column is in the pass (a-list, with the column position).  For
// a chunk of 64 a-entries the workgroup forms t(g, a) = sum_b phi_b(g) P_ba,
// a 64 x 64 x n_b product, on the matrix cores (FP64 MFMA 16 x 16 x 4, one
// z-plane of the cell per wave), 32 b at a time: phi of the b chunk at the
// 64 points and the 32 x 64 block of P are staged in LDS.  The global loads
// of the next b chunk (its P block and its functions' parameters) are
// issued into registers before the products of the current chunk, and the
// list entries they are indexed by one chunk earlier still, so their
// latency overlaps the arithmetic.  Then n(g) += 2 sum_a phi_a(g) t(g, a)
// from the result registers, reduced over lanes in a fixed order.  A
// Gaussian and its cube window factor over x, y and z, so phi of one
// function on the cell's 4 x 4 x 4 points takes 12 exponentials instead of
// 64, computed by the function's lanes and shared by wave shuffles.  Cells
// own disjoint points, so no atomics are needed.
#include "dm_common.hpp"

namespace dm {
namespace {

constexpr int kBc = 32;  // b-functions per staged chunk
constexpr int kPs = 66;  // row stride of the staged P block (doubles)
// phi rows: z-plane q of the cell at 17 q, point (x, y) at x + 4 y; the
// padding puts the four planes in different LDS banks for the stores
constexpr int kPlane = 17, kPhs = 67;

// exp(-a d^2) inside the window |d| <= R, else 0
__device__ inline double axis_factor(double a, double R, double d) {
    return fabs(d) <= R ? exp(-a * d * d) : 0.0;
}

// One b chunk between its global loads and its LDS stores: the thread's
// eight P values (b = tid % 32, a-entries tid / 32 + 8 i) and the
// parameters of function tid / 8 of the chunk.
struct BChunk {
    double pv[8];
    double e, R, nrm, cx, cy, cz;
};

// List entries of a b chunk the thread's loads need: the P row of b =
// tid % 32 and the function tid / 8 (-1 beyond the chunk).  They are loaded
// one chunk before the values, so each chunk's value loads wait for one
// memory latency, not two.
struct BIdx {
    int brow, bfn;
};

__device__ inline void load_bidx(const GridArgs& a, int bs, int nb, BIdx& x) {
    const int tid = threadIdx.x;
    const int k = tid & (kBc - 1), bb = tid >> 3;
    x.brow = k < nb ? a.beta_idx[bs + k] : -1;
    x.bfn = bb < nb ? a.beta_idx[bs + bb] : -1;
}

__device__ inline void load_bchunk(const GridArgs& a, int na, const int (&acol)[8], const BIdx& x, BChunk& c) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int aa = (tid >> 5) + 8 * i;
        c.pv[i] = (x.brow >= 0 && aa < na) ? a.P[(long long)acol[i] * a.ldp + x.brow] : 0.0;
    }
    c.e = 0.0, c.R = -1.0, c.nrm = 0.0, c.cx = 0.0, c.cy = 0.0, c.cz = 0.0;
    if (x.bfn >= 0) {
        const int b = x.bfn;
        c.e = a.ex[b];
        c.R = a.R[b];
        c.nrm = a.norm[b];
        c.cx = a.cx[b];
        c.cy = a.cy[b];
        c.cz = a.cz[b];
    }
}

// 40 KB of LDS: three workgroups per CU
__global__ void __launch_bounds__(256, 3) density_kernel(GridArgs a) {
    __shared__ __align__(16) double phb[kBc][kPhs];  // phi_b(point), b of the chunk x 64 points
    __shared__ __align__(16) double pb[kBc][kPs];   // P_ba, b of the chunk x a of the chunk
    __shared__ double fa[64][13];  // per a-entry: 2 norm fx(x), fy(y), fz(z) at coordinates 0..3
    // workgroups go to the 8 XCDs round robin; XCD x takes the groups of 16
    // consecutive cells x, x + 8, ..., a group at a time, so the 16 cells
    // of a group, which read nearly the same block of P, run together on
    // one L2, and every XCD gets cells from all over the grid
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
    const int cell = (((slot >> 4) << 3) + xcd) * 16 + (slot & 15);
    if (cell >= a.ncx * a.ncy * a.ncz) return;
    const int ccx = cell % a.ncx, ccy = (cell / a.ncx) % a.ncy, ccz = cell / (a.ncx * a.ncy);
    const int tid = threadIdx.x;
    const int w = tid >> 6, lane = tid & 63, li = lane & 15, lq = lane >> 4;
    // MFMA rows: lane li feeds point (x, y) = (li / 4, li % 4) of z-plane w,
    // so result element e of lane (li, lq) is point (e, lq, w) and column li
    const int arow = kPlane * w + (li >> 2) + 4 * (li & 3);
    const int a0 = a.alpha_ptr[cell], a1 = a.alpha_ptr[cell + 1];
    const int b0 = a.beta_ptr[cell], b1 = a.beta_ptr[cell + 1];
    double npt[4] = {0.0, 0.0, 0.0, 0.0};
    for (int as = a0; as < a1; as += 64) {
        const int na = min(64, a1 - as);
        int acol[8];  // columns of the thread's P loads
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int aa = (tid >> 5) + 8 * i;
            acol[i] = aa < na ? a.alpha_col[as + aa] : 0;
        }
        __syncthreads();  // the previous chunk's epilogue has read fa
        // axis factors of the chunk's a-entries: entry tid / 4 at coordinate tid % 4
        {
            const int e = tid >> 2, q = tid & 3;
            double fx = 0.0, fy = 0.0, fz = 0.0;
            if (e < na) {
                const int f = a.alpha_idx[as + e];
                const double ex = a.ex[f], R = a.R[f];
                fx = 2.0 * a.norm[f] * axis_factor(ex, R, a.ox + a.h * (4 * ccx + q) - a.cx[f]);
                fy = axis_factor(ex, R, a.oy + a.h * (4 * ccy + q) - a.cy[f]);
                fz = axis_factor(ex, R, a.oz + a.h * (4 * ccz + q) - a.cz[f]);
            }
            fa[e][q] = fx;
            fa[e][4 + q] = fy;
            fa[e][8 + q] = fz;
        }
        double4_t acc[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = double4_t{0.0, 0.0, 0.0, 0.0};
        BChunk cur;
        BIdx nxt;
        load_bidx(a, b0, min(kBc, b1 - b0), nxt);
        load_bchunk(a, na, acol, nxt, cur);
        if (b0 + kBc < b1) load_bidx(a, b0 + kBc, min(kBc, b1 - b0 - kBc), nxt);
        for (int bs = b0; bs < b1; bs += kBc) {
            const int nb = min(kBc, b1 - bs);
            // phi of the b chunk: the eight lanes of function bb = tid / 8
            // compute its x, y and z factors at coordinate q = tid % 4 (the
            // two halves alike), share them, and lane (q, half) writes the 8
            // points of z-plane q with y = 2 half, 2 half + 1
            {
                const int bb = tid >> 3, q = tid & 3, half = (tid >> 2) & 1;
                const double fxq = axis_factor(cur.e, cur.R, a.ox + a.h * (4 * ccx + q) - cur.cx);
                const double fyq = axis_factor(cur.e, cur.R, a.oy + a.h * (4 * ccy + q) - cur.cy);
                const double fzq = axis_factor(cur.e, cur.R, a.oz + a.h * (4 * ccz + q) - cur.cz);
                const int base = (tid & 63) & ~7;
                double fxv[4], fyv[2];
#pragma unroll
                for (int u = 0; u < 4; ++u) fxv[u] = __shfl(fxq, base + u, 64);
#pragma unroll
                for (int v = 0; v < 2; ++v) fyv[v] = __shfl(fyq, base + 2 * half + v, 64);
                const double s = cur.nrm * fzq;
#pragma unroll
                for (int v = 0; v < 2; ++v)
#pragma unroll
                    for (int u = 0; u < 4; ++u) phb[bb][u + 4 * (2 * half + v) + kPlane * q] = s * fyv[v] * fxv[u];
            }
            // P block: lane k = b of the chunk, thread group tid / 32 holds
            // a-entries tid / 32 + 8 i
            {
                const int k = tid & (kBc - 1), g = tid >> 5;
#pragma unroll
                for (int i = 0; i < 8; ++i) pb[k][g + 8 * i] = cur.pv[i];
            }
            __syncthreads();
            if (bs + kBc < b1) {
                load_bchunk(a, na, acol, nxt, cur);
                if (bs + 2 * kBc < b1) load_bidx(a, bs + 2 * kBc, min(kBc, b1 - bs - 2 * kBc), nxt);
            }
            // t(g, a) += sum_b phi_b(g) P_ba: wave w takes the 16 points of
            // z-plane w and the 64 a-entries (four 16 x 16 tiles), 4 b per
            // MFMA; rows beyond nb hold zeros
            const int nk = (nb + 3) >> 2;
            for (int st = 0; st < nk; ++st) {
                const int kb = 4 * st + lq;
                const double av = phb[kb][arow];
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (16 * c < na)  // tiles past the chunk's a-entries stay zero
                        acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, pb[kb][16 * c + li], acc[c], 0, 0, 0);
            }
            __syncthreads();
        }
        // n(g) += 2 phi_a(g) t(g, a): lane (li, lq) of wave w holds points
        // (e, lq, w), e = 0..3, for a-entries 16 c + li (entries beyond na
        // have zero factors)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (16 * c >= na) break;
            const int aa = 16 * c + li;
            const double s = fa[aa][4 + lq] * fa[aa][8 + w];
#pragma unroll
            for (int e = 0; e < 4; ++e) npt[e] += s * fa[aa][e] * acc[c][e];
        }
    }
    // sums over the 16 lanes of a point row (fixed butterfly order)
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) npt[e] += __shfl_xor(npt[e], off, 64);
    if (li == 0) {
        const int gj = 4 * ccy + lq, gk = 4 * ccz + w;
        if (gj < a.ny && gk < a.nz) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int gi = 4 * ccx + e;
                if (gi < a.nx) a.n[gi + (long long)a.nx * (gj + (long long)a.ny * gk)] += npt[e];
            }
        }
    }
}

// dst[j K + r] = src[j K + perm[r]] for r < K, j < ncols
__global__ void permute_rows_kernel(int K, long long ncols, const int* __restrict__ perm,
                                    const double* __restrict__ src, double* __restrict__ dst) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)K * ncols) return;
    const long long j = e / K;
    const int r = (int)(e - j * K);
    dst[e] = src[j * K + perm[r]];
}

}  // namespace

hipError_t permute_rows(int K, long long ncols, const int* perm, const double* src, double* dst, hipStream_t s) {
    const long long n = (long long)K * ncols;
    if (n <= 0) return hipSuccess;
    const long long nb = (n + 255) / 256;
    if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(permute_rows_kernel, dim3((unsigned)nb), dim3(256), 0, s, K, ncols, perm, src, dst);
    return hipGetLastError();
}

hipError_t density_on_grid(const GridArgs& a, hipStream_t s) {
    const long long ncell = (long long)a.ncx * a.ncy * a.ncz;
    if (ncell <= 0) return hipSuccess;
    const long long nwg = (ncell + 127) / 128 * 128;  // whole rounds of 8 groups of 16 cells
    if (nwg > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(density_kernel, dim3((unsigned)nwg), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace dm
