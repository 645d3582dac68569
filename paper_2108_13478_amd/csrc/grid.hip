// Electron density on a uniform grid from density-matrix columns (Method,
// eq. ElectronDensity): n(r_g) += sum_a 2 phi_a(r_g) sum_b phi_b(r_g) P_ba
// over the columns a of a pass.  Each basis function is a normalised s-type
// Gaussian set to zero outside its cube window (grid-window section).
//
// One workgroup per cell of 4 x 4 x 4 grid points.  The host lists, per
// cell, the functions whose window reaches the cell (b-list) and those of
// them whose column is in the pass (a-list, with the column position).  The
// 64 points x 64 b values of phi are staged in LDS chunk by chunk; wave q
// accumulates t_a(g) = sum_b phi_b(g) P_ba for a-list entries q, q+4, ...
// (the P reads are the same address across the wave, i.e. broadcasts), and
// finally n(g) += 2 sum_a phi_a(g) t_a(g), reduced over the 4 waves in a
// fixed order.  Cells own disjoint points, so no atomics are needed.
#include "dm_common.hpp"

namespace dm {
namespace {

__device__ inline double sgauss(const GridArgs& a, int b, double x, double y, double z) {
    const double dx = x - a.cx[b], dy = y - a.cy[b], dz = z - a.cz[b];
    const double R = a.R[b];
    if (!(fabs(dx) <= R && fabs(dy) <= R && fabs(dz) <= R)) return 0.0;
    return a.norm[b] * exp(-a.ex[b] * (dx * dx + dy * dy + dz * dz));
}

__global__ void __launch_bounds__(256) density_kernel(GridArgs a) {
    constexpr int NA = 16;  // a-list entries per wave and chunk (4 waves x 16 = 64)
    __shared__ double phb[64][64];
    __shared__ double red[4][64];
    const int cell = blockIdx.x;
    const int ccx = cell % a.ncx, ccy = (cell / a.ncx) % a.ncy, ccz = cell / (a.ncx * a.ncy);
    const int tid = threadIdx.x;
    const int p = tid & 63, q = tid >> 6;
    const int gi = 4 * ccx + (p & 3), gj = 4 * ccy + ((p >> 2) & 3), gk = 4 * ccz + (p >> 4);
    const bool valid = gi < a.nx && gj < a.ny && gk < a.nz;
    const double x = a.ox + a.h * gi, y = a.oy + a.h * gj, z = a.oz + a.h * gk;
    const int a0 = a.alpha_ptr[cell], a1 = a.alpha_ptr[cell + 1];
    const int b0 = a.beta_ptr[cell], b1 = a.beta_ptr[cell + 1];
    double nacc = 0.0;
    for (int as = a0; as < a1; as += 4 * NA) {
        double t[NA];
#pragma unroll
        for (int m = 0; m < NA; ++m) t[m] = 0.0;
        for (int bs = b0; bs < b1; bs += 64) {
            const int nb = min(64, b1 - bs);
            // phi of this b-chunk at the cell's 64 points
            for (int e = tid; e < 64 * 64; e += 256) {
                const int pt = e & 63, bb = e >> 6;
                double v = 0.0;
                if (bb < nb) {
                    const int px = 4 * ccx + (pt & 3), py = 4 * ccy + ((pt >> 2) & 3), pz = 4 * ccz + (pt >> 4);
                    v = sgauss(a, a.beta_idx[bs + bb], a.ox + a.h * px, a.oy + a.h * py, a.oz + a.h * pz);
                }
                phb[bb][pt] = v;
            }
            __syncthreads();
            for (int bb = 0; bb < nb; ++bb) {
                const double f = phb[bb][p];
                const long long b = a.beta_idx[bs + bb];
#pragma unroll
                for (int m = 0; m < NA; ++m) {
                    const int ai = as + q + 4 * m;
                    if (ai < a1) t[m] += f * a.P[(long long)a.alpha_col[ai] * a.ldp + b];
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int m = 0; m < NA; ++m) {
            const int ai = as + q + 4 * m;
            if (ai < a1) nacc += 2.0 * sgauss(a, a.alpha_idx[ai], x, y, z) * t[m];
        }
    }
    red[q][p] = nacc;
    __syncthreads();
    if (q == 0 && valid) {
        const long long g = gi + (long long)a.nx * (gj + (long long)a.ny * gk);
        a.n[g] += ((red[0][p] + red[1][p]) + red[2][p]) + red[3][p];
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
