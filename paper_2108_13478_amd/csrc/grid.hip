// Electron density on a uniform grid from density-matrix columns (Method,
// eq. ElectronDensity): n(r_g) += sum_a 2 phi_a(r_g) sum_b phi_b(r_g) P_ba
// over the columns a of a pass.  Each basis function is a normalised s-type
// Gaussian set to zero outside its cube window (grid-window section).
//
// One workgroup per cell of 4 x 4 x 4 grid points.  The host lists, per
// cell, the functions whose window reaches the cell (b-list) and those of
// them whose column is in the pass (a-list, with the column position).  For
// a chunk of 64 a-entries the workgroup forms t(g, a) = sum_b phi_b(g) P_ba,
// a 64 x 64 x n_b product, 32 b at a time: phi of the b chunk at the 64
// points and the 32 x 64 block of P are staged in LDS, and each thread
// accumulates a 4-point x 4-column block in registers.  The global loads of
// the next b chunk (its P block and its functions' parameters) are issued
// into registers before the products of the current chunk, so their latency
// overlaps the arithmetic.  Then n(g) += 2 sum_a phi_a(g) t(g, a), reduced
// over the threads of a point in a fixed order.  A Gaussian and its cube
// window factor over x, y and z, so phi of one function on the cell's
// 4 x 4 x 4 points takes 12 exponentials, each computed by one lane and
// shared by wave shuffles.  Cells own disjoint points, so no atomics are
// needed.
#include "dm_common.hpp"

namespace dm {
namespace {

constexpr int kBc = 32;  // b-functions per staged chunk
constexpr int kPs = 66;  // row stride of the staged blocks (doubles): 16-byte rows, few bank conflicts

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

__device__ inline void load_bchunk(const GridArgs& a, int bs, int nb, int na, const long long (&acol)[8],
                                   BChunk& c) {
    const int tid = threadIdx.x;
    const int k = tid & (kBc - 1);
    const long long brow = k < nb ? a.beta_idx[bs + k] : 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int aa = (tid >> 5) + 8 * i;
        c.pv[i] = (k < nb && aa < na) ? a.P[acol[i] * a.ldp + brow] : 0.0;
    }
    const int bb = tid >> 3;
    c.e = 0.0, c.R = -1.0, c.nrm = 0.0, c.cx = 0.0, c.cy = 0.0, c.cz = 0.0;
    if (bb < nb) {
        const int b = a.beta_idx[bs + bb];
        c.e = a.ex[b];
        c.R = a.R[b];
        c.nrm = a.norm[b];
        c.cx = a.cx[b];
        c.cy = a.cy[b];
        c.cz = a.cz[b];
    }
}

// 33 KB of LDS and at most 168 registers: three workgroups per CU
__global__ void __launch_bounds__(256, 3) density_kernel(GridArgs a) {
    __shared__ __align__(16) double phb[kBc][kPs];  // phi_b(point), b of the chunk x 64 points
    __shared__ __align__(16) double pb[kBc][kPs];   // P_ba, b of the chunk x a of the chunk
    double(*red)[64] = reinterpret_cast<double(*)[64]>(&phb[0][0]);  // after the last chunk: 16 x 64 sums
    const int cell = blockIdx.x;
    const int ccx = cell % a.ncx, ccy = (cell / a.ncx) % a.ncy, ccz = cell / (a.ncx * a.ncy);
    const int tid = threadIdx.x;
    const int tp = tid & 15, ta = tid >> 4;  // points 4 tp .. 4 tp + 3 (x = 0..3), a-entries 4 ta .. 4 ta + 3
    const int py = tp & 3, pz = tp >> 2;     // the thread's four points differ in x only
    const int a0 = a.alpha_ptr[cell], a1 = a.alpha_ptr[cell + 1];
    const int b0 = a.beta_ptr[cell], b1 = a.beta_ptr[cell + 1];
    double npt[4] = {0.0, 0.0, 0.0, 0.0};
    for (int as = a0; as < a1; as += 64) {
        const int na = min(64, a1 - as);
        long long acol[8];  // columns of the thread's P loads
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int aa = (tid >> 5) + 8 * i;
            acol[i] = aa < na ? a.alpha_col[as + aa] : 0;
        }
        double t[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) t[i][j] = 0.0;
        BChunk cur;
        load_bchunk(a, b0, min(kBc, b1 - b0), na, acol, cur);
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
                    for (int u = 0; u < 4; ++u) phb[bb][u + 4 * (2 * half + v) + 16 * q] = s * fyv[v] * fxv[u];
            }
            // P block: lane k = b of the chunk, thread group w = tid / 32
            // holds a-entries w, w + 8, ...
            {
                const int k = tid & (kBc - 1), w = tid >> 5;
#pragma unroll
                for (int i = 0; i < 8; ++i) pb[k][w + 8 * i] = cur.pv[i];
            }
            __syncthreads();
            if (bs + kBc < b1) load_bchunk(a, bs + kBc, min(kBc, b1 - bs - kBc), na, acol, cur);
            for (int k = 0; k < nb; ++k) {
                const double2 f01 = *reinterpret_cast<const double2*>(&phb[k][4 * tp]);
                const double2 f23 = *reinterpret_cast<const double2*>(&phb[k][4 * tp + 2]);
                const double2 p01 = *reinterpret_cast<const double2*>(&pb[k][4 * ta]);
                const double2 p23 = *reinterpret_cast<const double2*>(&pb[k][4 * ta + 2]);
                const double f[4] = {f01.x, f01.y, f23.x, f23.y};
                const double p[4] = {p01.x, p01.y, p23.x, p23.y};
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) t[i][j] += f[i] * p[j];
            }
            __syncthreads();
        }
        // n(g) += 2 phi_a(g) t(g, a) for the thread's four a-entries.  The
        // 16 lanes sharing an a-entry (same ta) compute its 12 axis factors,
        // lane tp: x (tp < 4), y (4..7) or z (8..11) at coordinate tp % 4.
        {
            const int base = (tid & 63) & ~15;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int aa = 4 * ta + j;
                double fac = 0.0, nrm = 0.0;
                if (aa < na) {
                    const int f = a.alpha_idx[as + aa];
                    const double e = a.ex[f], R = a.R[f];
                    nrm = 2.0 * a.norm[f];
                    const int c = tp & 3;
                    if (tp < 4)
                        fac = axis_factor(e, R, a.ox + a.h * (4 * ccx + c) - a.cx[f]);
                    else if (tp < 8)
                        fac = axis_factor(e, R, a.oy + a.h * (4 * ccy + c) - a.cy[f]);
                    else if (tp < 12)
                        fac = axis_factor(e, R, a.oz + a.h * (4 * ccz + c) - a.cz[f]);
                }
                const double fyv = __shfl(fac, base + 4 + py, 64), fzv = __shfl(fac, base + 8 + pz, 64);
                const double s = nrm * fyv * fzv;
#pragma unroll
                for (int i = 0; i < 4; ++i) npt[i] += s * __shfl(fac, base + i, 64) * t[i][j];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) red[ta][4 * tp + i] = npt[i];
    __syncthreads();
    if (tid < 64) {
        const int p = tid;
        const int gi = 4 * ccx + (p & 3), gj = 4 * ccy + ((p >> 2) & 3), gk = 4 * ccz + (p >> 4);
        if (gi < a.nx && gj < a.ny && gk < a.nz) {
            double sum = 0.0;
            for (int q = 0; q < 16; ++q) sum += red[q][p];
            const long long g = gi + (long long)a.nx * (gj + (long long)a.ny * gk);
            a.n[g] += sum;
        }
    }
}

}  // namespace

hipError_t density_on_grid(const GridArgs& a, hipStream_t s) {
    const long long ncell = (long long)a.ncx * a.ncy * a.ncz;
    if (ncell <= 0) return hipSuccess;
    if (ncell > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(density_kernel, dim3((unsigned)ncell), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace dm
