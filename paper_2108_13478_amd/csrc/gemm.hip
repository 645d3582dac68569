// MFMA matrix kernels for gfx950: the Chebyshev recursion step (the hot
// loop of the supplement's eq. ChebychevExpansion) and the FP64 products of
// the operator setup.
//
// Both compute C[m, n] = sum_k A[m*lda + k] * B[n*ldb + k]: each operand has
// its reduction index contiguous, so one lane reads four consecutive k with a
// single vector load.  MFMA 16x16x4 takes A[i][k] from lane i + 16k and
// B[k][j] from lane j + 16k; here lane (i, q = lane/16) holds k = 4q .. 4q+3
// and the s-th MFMA of a 16-wide k slab uses k = 4q + s, which visits every k
// exactly once (the products are summed in a different order, nothing else).
// With the row order of Mfma<T>::a_row, result row i of a tile sits in lane
// j + 16 * (i / 4), element i % 4, so each lane owns four consecutive rows of
// one column: the epilogue reads and writes 4-element vectors of column-major
// blocks.
#include <type_traits>

#include "dm_common.hpp"

namespace dm {
namespace {

template <typename T>
struct Mfma;

// a_row(i): which row of the 16-row A slab lane i feeds.  The f32 result
// puts row 4g + r of the tile in lane j + 16g, element r; the f64 result puts
// row g + 4r there instead.  Feeding slot i from row 4(i % 4) + i / 4 turns
// the f64 layout into the f32 one, so both epilogues see four consecutive
// rows per lane.
template <>
struct Mfma<double> {
    typedef double4_t acc_t;
    typedef double4_t vec_t;
    __device__ static inline acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static inline int a_row(int i) { return 4 * (i & 3) + (i >> 2); }
};

template <>
struct Mfma<float> {
    typedef float4_t acc_t;
    typedef float4_t vec_t;
    __device__ static inline acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static inline int a_row(int i) { return i; }
};

// Storage and arithmetic type of a recursion precision.  W32 is the
// refined mode: H_N and U_l are stored in FP32 (half the bytes of FP64),
// every product and sum runs in FP64 on the f64 MFMA (an FP32 x FP32
// product is exact in FP64), and U_{l+1} is rounded to FP32 once, when it
// is stored.
struct W32 {};
template <typename T>
struct Prec {
    typedef T store;
    typedef T calc;
};
template <>
struct Prec<W32> {
    typedef float store;
    typedef double calc;
};

// Tile placement.  Workgroups are dispatched round-robin over the 8 XCDs
// (workgroup b lands on XCD b % 8); remapping b so that each XCD gets a
// contiguous range of logical tiles, and ordering logical tiles in groups of
// GM tile-rows, keeps the operator rows and column blocks that concurrently
// running workgroups share inside one XCD's L2.
struct TilePos {
    int tile_m, tile_n, logical;
};

template <int GM>
__device__ inline TilePos tile_position(int ntm, int ntn) {
    const int nwg = gridDim.x;
    const int bid = blockIdx.x;
    int logical = bid;
    if ((nwg & 7) == 0) logical = (bid & 7) * (nwg >> 3) + (bid >> 3);
    const int group_size = GM * ntn;
    const int group = logical / group_size;
    const int first_m = group * GM;
    const int gm = min(ntm - first_m, GM);
    const int in_group = logical - group * group_size;
    TilePos p;
    p.tile_m = first_m + in_group % gm;
    p.tile_n = in_group / gm;
    p.logical = logical;
    return p;
}

// The main loop: acc[tm][tn] += A-rows x B-columns over the whole reduction.
// Each lane loads KV consecutive k per operand row/column and slab (one
// vector load of KV elements); a slab is 4 KV wide and takes KV MFMA k-steps.
// Two register buffers keep the next slab's loads in flight while the MFMAs
// of the current slab run; a larger KV puts more bytes in flight per wave,
// which is what the memory-bound narrow-block shapes need.
template <typename T, int KV>
struct VecOf;
template <> struct VecOf<double, 4> { typedef double4_t type; };
template <> struct VecOf<float, 4> { typedef float4_t type; };
template <> struct VecOf<double, 8> { typedef double type __attribute__((ext_vector_type(8))); };
template <> struct VecOf<float, 8> { typedef float type __attribute__((ext_vector_type(8))); };
template <> struct VecOf<float, 16> { typedef float type __attribute__((ext_vector_type(16))); };

// ACM: A is stored column-major (A[m + k lda], the plain product A B): a
// lane then reads its KV values of k one by one, lda apart, and the 16 lanes
// of a row group read 16 consecutive rows of one column together.
template <typename T, int TM, int TN, int KV, int DEPTH = 2, bool NT = false, bool ACM = false>
__device__ inline void gemm_mainloop(int Kred, const typename Prec<T>::store* __restrict__ A, long lda,
                                     const typename Prec<T>::store* __restrict__ B, long ldb, int row0, int col0,
                                     typename Mfma<typename Prec<T>::calc>::acc_t (&acc)[TM][TN]) {
    typedef typename Prec<T>::store S;
    typedef typename Prec<T>::calc C;
    typedef typename VecOf<S, KV>::type vec_t;
    constexpr int SLAB = 4 * KV;
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lq = lane >> 4;
    const S* pa[TM];
    const S* pb[TN];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        if constexpr (ACM)
            pa[i] = A + (long)(row0 + 16 * i + Mfma<C>::a_row(li)) + (long)(KV * lq) * lda;
        else
            pa[i] = A + (long)(row0 + 16 * i + Mfma<C>::a_row(li)) * lda + KV * lq;
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) pb[j] = B + (long)(col0 + 16 * j + li) * ldb + KV * lq;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = typename Mfma<C>::acc_t{0, 0, 0, 0};

    vec_t a0[TM], b0[TN], a1[TM], b1[TN];
    // NT: the A operand is read once per launch, so its loads carry the
    // non-temporal hint and leave the cache to the reused B panel.
    auto load = [&](vec_t(&a)[TM], vec_t(&b)[TN], int k) {
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            if constexpr (ACM) {
#pragma unroll
                for (int s = 0; s < KV; ++s) a[i][s] = pa[i][(long)(k + s) * lda];
            } else if constexpr (NT) {
                a[i] = __builtin_nontemporal_load(reinterpret_cast<const vec_t*>(pa[i] + k));
            } else {
                a[i] = *reinterpret_cast<const vec_t*>(pa[i] + k);
            }
        }
#pragma unroll
        for (int j = 0; j < TN; ++j) b[j] = *reinterpret_cast<const vec_t*>(pb[j] + k);
    };
    auto compute = [&](const vec_t(&a)[TM], const vec_t(&b)[TN]) {
#pragma unroll
        for (int s = 0; s < KV; ++s)
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = Mfma<C>::mma(static_cast<C>(a[i][s]), static_cast<C>(b[j][s]), acc[i][j]);
    };
    if constexpr (DEPTH == 2) {
        // Kred is a multiple of 2 SLAB (checked by the launchers).  The steady
        // state has no branch between a load and the MFMAs that follow it, so
        // the compiler can wait for exactly the older buffer's loads instead
        // of for every load in flight.
        load(a0, b0, 0);
        int k = 0;
        for (; k < Kred - 2 * SLAB; k += 2 * SLAB) {
            load(a1, b1, k + SLAB);
            compute(a0, b0);
            __builtin_amdgcn_sched_barrier(0);
            load(a0, b0, k + 2 * SLAB);
            compute(a1, b1);
            __builtin_amdgcn_sched_barrier(0);
        }
        load(a1, b1, k + SLAB);
        compute(a0, b0);
        compute(a1, b1);
    } else {
        // Ring of DEPTH buffers: DEPTH - 1 slabs stay in flight while one is
        // consumed (Kred is a multiple of DEPTH SLAB).  One slab of MFMA work
        // is far shorter than an HBM or Infinity Cache round trip.
        static_assert((DEPTH & (DEPTH - 1)) == 0, "ring depth is a power of two");
        (void)a0; (void)b0; (void)a1; (void)b1;
        vec_t ra[DEPTH][TM], rb[DEPTH][TN];
#pragma unroll
        for (int d = 0; d < DEPTH - 1; ++d) load(ra[d], rb[d], d * SLAB);
        int k = 0;
        for (; k < Kred - DEPTH * SLAB; k += DEPTH * SLAB) {
#pragma unroll
            for (int d = 0; d < DEPTH; ++d) {
                const int n = (d + DEPTH - 1) & (DEPTH - 1);
                load(ra[n], rb[n], k + (d + DEPTH - 1) * SLAB);
                compute(ra[d], rb[d]);
                // Keep the stages in program order: left alone, the scheduler
                // sinks every load of the next ring turn to the end of the loop
                // body, and each turn then waits for all of them at its start.
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        load(ra[DEPTH - 1], rb[DEPTH - 1], k + (DEPTH - 1) * SLAB);
#pragma unroll
        for (int d = 0; d < DEPTH; ++d) compute(ra[d], rb[d]);
    }
}

// The main loop with the B panel shared through LDS.  All WM waves of the
// workgroup cover the same 16 TN columns, so instead of every wave reading
// the panel from the cache hierarchy (which halves the operator stream when
// the panel is as wide as the wave's row block), the workgroup fetches each
// slab of it once: 16-byte pieces, one (or R) per thread, staged through
// registers in the same ring as the operator, written to one of two LDS
// buffers and read back as MFMA fragments after a barrier.  Piece p of a
// slab holds lane p % 64 of chunk p / 64 = (column group, 16-byte part), so a
// wave reads its fragment of column group j, part h at ((j H + h) 64 + lane)
// * 16 bytes with no bank conflicts.  The barrier waits only for LDS
// traffic; the operator loads of later slabs stay in flight across it.
template <typename T, int TM, int TN, int WM, int KV, int DEPTH>
__device__ inline void gemm_mainloop_ldsb(int Kred, const typename Prec<T>::store* __restrict__ A, long lda,
                                          const typename Prec<T>::store* __restrict__ B, long ldb, int row0,
                                          int col0, typename Mfma<typename Prec<T>::calc>::acc_t (&acc)[TM][TN]) {
    typedef typename Prec<T>::store S;
    typedef typename Prec<T>::calc C;
    typedef typename VecOf<S, KV>::type vec_t;
    typedef float piece_t __attribute__((ext_vector_type(4)));
    constexpr int SLAB = 4 * KV;
    constexpr int H = KV * (int)sizeof(S) / 16;          // 16-byte parts per lane and column group
    constexpr int NPIECE = TN * H * 64;                   // pieces per slab
    constexpr int NT = 64 * WM;
    constexpr int R = NPIECE / NT;                        // pieces per thread and slab
    constexpr int EPP = 16 / (int)sizeof(S);              // elements per piece
    static_assert(NPIECE % NT == 0 && R >= 1, "every thread loads whole pieces");
    static_assert(DEPTH >= 2 && (DEPTH & (DEPTH - 1)) == 0, "ring depth is a power of two");
    __shared__ piece_t lds[2][NPIECE];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int li = lane & 15, lq = lane >> 4;
    const S* pa[TM];
#pragma unroll
    for (int i = 0; i < TM; ++i) pa[i] = A + (long)(row0 + 16 * i + Mfma<C>::a_row(li)) * lda + KV * lq;
    const S* pp[R];
#pragma unroll
    for (int e = 0; e < R; ++e) {
        const int c = (tid + e * NT) >> 6;  // chunk: column group c / H, part c % H
        pp[e] = B + (long)(col0 + 16 * (c / H) + li) * ldb + KV * lq + EPP * (c % H);
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = typename Mfma<C>::acc_t{0, 0, 0, 0};

    vec_t ra[DEPTH][TM];
    piece_t rs[DEPTH][R];
    auto load = [&](vec_t(&a)[TM], piece_t(&st)[R], int k) {
#pragma unroll
        for (int i = 0; i < TM; ++i) a[i] = *reinterpret_cast<const vec_t*>(pa[i] + k);
#pragma unroll
        for (int e = 0; e < R; ++e) st[e] = *reinterpret_cast<const piece_t*>(pp[e] + k);
    };
    auto compute = [&](const vec_t(&a)[TM], const piece_t(&st)[R], int buf) {
#pragma unroll
        for (int e = 0; e < R; ++e) lds[buf][tid + e * NT] = st[e];
        __syncthreads();
        vec_t b[TN];
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            S* bj = reinterpret_cast<S*>(&b[j]);
#pragma unroll
            for (int h = 0; h < H; ++h) {
                const piece_t v = lds[buf][(j * H + h) * 64 + lane];
                __builtin_memcpy(bj + h * EPP, &v, 16);
            }
        }
#pragma unroll
        for (int s = 0; s < KV; ++s)
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = Mfma<C>::mma(static_cast<C>(a[i][s]), static_cast<C>(b[j][s]), acc[i][j]);
    };
    // Slab n uses LDS buffer n & 1 (DEPTH is even, so that is d & 1 below).
    // A buffer is rewritten two slabs later, after every wave has passed the
    // barrier of the slab in between, i.e. after it finished reading.
#pragma unroll
    for (int d = 0; d < DEPTH - 1; ++d) load(ra[d], rs[d], d * SLAB);
    int k = 0;
    for (; k < Kred - DEPTH * SLAB; k += DEPTH * SLAB) {
#pragma unroll
        for (int d = 0; d < DEPTH; ++d) {
            const int n = (d + DEPTH - 1) & (DEPTH - 1);
            load(ra[n], rs[n], k + (d + DEPTH - 1) * SLAB);
            compute(ra[d], rs[d], d & 1);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    load(ra[DEPTH - 1], rs[DEPTH - 1], k + (DEPTH - 1) * SLAB);
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) compute(ra[d], rs[d], d & 1);
}

// ------------------------------------------------------------ plain product
template <int TM, int TN, int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN)
gemm_tn_store_kernel(int M, int N, int Kred, double alpha, const double* __restrict__ A, long lda,
                     const double* __restrict__ B, long ldb, double beta, double* __restrict__ C,
                     long ldc, int upper_only, int k_row0) {
    constexpr int BM = 16 * TM * WM, BN = 16 * TN * WN;
    TilePos tp = tile_position<8>(M / BM, N / BN);
    // with a reduction limit the tiles of the last rows carry the longest
    // sums: they go first, so the launch does not end on them
    if (k_row0 >= 0) tp.tile_m = M / BM - 1 - tp.tile_m;
    if (upper_only && tp.tile_m * BM >= (tp.tile_n + 1) * BN) return;
    const int wave = threadIdx.x >> 6;
    const int row0 = tp.tile_m * BM + (wave % WM) * TM * 16;
    const int col0 = tp.tile_n * BN + (wave / WM) * TN * 16;
    // k_row0 >= 0: column m of A is zero below row k_row0 + m (A upper
    // triangular, C's first row being row k_row0 of it), so the tile's rows
    // need k < k_row0 + its last row + 1 only (rounded up to the slab pair)
    const int kend = k_row0 >= 0 ? min(Kred, (k_row0 + tp.tile_m * BM + BM + 31) / 32 * 32) : Kred;
    double4_t acc[TM][TN];
    if (kend % 64 == 0)  // three slabs in flight (same k order as two buffers)
        gemm_mainloop<double, TM, TN, 4, 4>(kend, A, lda, B, ldb, row0, col0, acc);
    else
        gemm_mainloop<double, TM, TN, 4>(kend, A, lda, B, ldb, row0, col0, acc);
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lq = lane >> 4;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const long idx = (long)(row0 + 16 * i + 4 * lq) + (long)(col0 + 16 * j + li) * ldc;
            double4_t* c = reinterpret_cast<double4_t*>(C + idx);
            double4_t r = alpha * acc[i][j];
            if (beta != 0.0) r += beta * (*c);
            *c = r;
        }
}

// C = alpha A B + beta C with A column-major (M x Kred, lda), B column-major
// (Kred x N, ldb) and C column-major; k_from_row: A is upper triangular, so
// a row tile starting at row r0 only needs k >= r0 (rounded down to the
// slab pair).
template <int TM, int TN, int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN)
gemm_nn_store_kernel(int M, int N, int Kred, double alpha, const double* __restrict__ A, long lda,
                     const double* __restrict__ B, long ldb, double beta, double* __restrict__ C,
                     long ldc, int k_from_row) {
    constexpr int BM = 16 * TM * WM, BN = 16 * TN * WN;
    const TilePos tp = tile_position<8>(M / BM, N / BN);
    const int wave = threadIdx.x >> 6;
    const int row0 = tp.tile_m * BM + (wave % WM) * TM * 16;
    const int col0 = tp.tile_n * BN + (wave / WM) * TN * 16;
    const int k0 = k_from_row ? min(Kred, (tp.tile_m * BM) / 32 * 32) : 0;
    double4_t acc[TM][TN];
    if (k0 < Kred && (Kred - k0) % 64 == 0) {
        gemm_mainloop<double, TM, TN, 4, 4, false, true>(Kred - k0, A + (long)k0 * lda, lda, B + k0, ldb, row0,
                                                         col0, acc);
    } else if (k0 < Kred) {
        gemm_mainloop<double, TM, TN, 4, 2, false, true>(Kred - k0, A + (long)k0 * lda, lda, B + k0, ldb, row0,
                                                         col0, acc);
    } else {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = double4_t{0, 0, 0, 0};
    }
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lq = lane >> 4;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const long idx = (long)(row0 + 16 * i + 4 * lq) + (long)(col0 + 16 * j + li) * ldc;
            double4_t* c = reinterpret_cast<double4_t*>(C + idx);
            double4_t r = alpha * acc[i][j];
            if (beta != 0.0) r += beta * (*c);
            *c = r;
        }
}

// ------------------------------------------------------------ recursion step
template <typename T, int TM, int TN, int WM, int WN, int KV, int DEPTH, bool LDSB = false>
__global__ void __launch_bounds__(64 * WM * WN)
cheb_step_kernel(ChebStepArgs a) {
    typedef typename Prec<T>::store S;
    typedef typename Prec<T>::calc C;
    typedef typename Mfma<S>::vec_t svec_t;  // four stored values
    typedef typename Mfma<C>::vec_t cvec_t;  // four values in the arithmetic type
    constexpr int BM = 16 * TM * WM, BN = 16 * TN * WN;
    const int ntm = a.Kp / BM, ntn = a.Bp / BN;
    const TilePos tp = tile_position<8>(ntm, ntn);
    const int wave = threadIdx.x >> 6;
    const int row0 = tp.tile_m * BM + (wave % WM) * TM * 16;
    const int col0 = tp.tile_n * BN + (wave / WM) * TN * 16;
    typename Mfma<C>::acc_t acc[TM][TN];
    if constexpr (LDSB) {
        static_assert(WN == 1, "the shared panel needs every wave on the same columns");
        gemm_mainloop_ldsb<T, TM, TN, WM, KV, DEPTH>(a.Kp, static_cast<const S*>(a.HN), a.Kp,
                                                     static_cast<const S*>(a.Ucur), a.Kp, row0, col0, acc);
    } else {
        gemm_mainloop<T, TM, TN, KV, DEPTH>(a.Kp, static_cast<const S*>(a.HN), a.Kp,
                                            static_cast<const S*>(a.Ucur), a.Kp, row0, col0, acc);
    }

    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lq = lane >> 4;
    const C alpha = static_cast<C>(a.alpha);
    const double c0 = a.coef[a.l];
    // Uprev and Unext are one buffer (U_{l+1} overwrites U_{l-1} element by
    // element, each element read before it is written), so they carry no
    // __restrict__; the program order below already issues every load of a
    // group before the stores that could alias it.
    const S* Uprev = static_cast<const S*>(a.Uprev);
    S* Unext = static_cast<S*>(a.Unext);
    const double* __restrict__ Zp = a.Z;
    double* __restrict__ Pp = a.P;
    // Epilogue in groups of EG tiles: every load of a group is issued before
    // the group's arithmetic, so a lane waits for memory once per group and
    // coefficient set instead of once per tile.  Per element the arithmetic
    // and the order of the moment sum are those of one tile at a time.  The
    // group is as large as the registers left by the main loop allow (two
    // waves per SIMD, or the refined type's FP64 copies: smaller groups).
    // Register-tile shapes (PIPE) also issue the next group's loads before
    // this group's arithmetic, in straight-line versions for the two uniform
    // conditions (a previous vector; a P block to accumulate); the
    // shared-panel shapes have no registers for a second group.
    constexpr int NTILE = TM * TN;
    constexpr int EGMAX = WM * WN > 4 ? 1 : (std::is_same<T, W32>::value ? 2 : 4);
    constexpr int EG = NTILE % EGMAX == 0 ? EGMAX : 1;
    constexpr int NG = NTILE / EG;
    constexpr bool PIPE = !LDSB;
    double msum = 0.0;
    if constexpr (PIPE) {
        auto at = [&](int g, int t) {
            const int i = (g * EG + t) / TN, j = (g * EG + t) % TN;
            return (long)(row0 + 16 * i + 4 * lq) + (long)(col0 + 16 * j + li) * a.Kp;
        };
        auto pipelined = [&](auto has_prev_c, auto with_p_c) {
            constexpr bool HP = decltype(has_prev_c)::value, WP = decltype(with_p_c)::value;
            svec_t up[2][EG];
            double4_t z[2][EG], pv[2][EG];
            auto load = [&](int g, int buf) {
#pragma unroll
                for (int t = 0; t < EG; ++t) {
                    if constexpr (HP) up[buf][t] = *reinterpret_cast<const svec_t*>(Uprev + at(g, t));
                    z[buf][t] = *reinterpret_cast<const double4_t*>(Zp + at(g, t));
                    if constexpr (WP) pv[buf][t] = *reinterpret_cast<const double4_t*>(Pp + at(g, t));
                }
            };
            load(0, 0);
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                const int buf = g & 1;
                if (g + 1 < NG) load(g + 1, buf ^ 1);
                double4_t od[EG];
#pragma unroll
                for (int t = 0; t < EG; ++t) {
                    const int i = (g * EG + t) / TN, j = (g * EG + t) % TN;
                    cvec_t out = alpha * acc[i][j];
                    if constexpr (HP) out -= __builtin_convertvector(up[buf][t], cvec_t);
                    const svec_t st = __builtin_convertvector(out, svec_t);
                    *reinterpret_cast<svec_t*>(Unext + at(g, t)) = st;
                    od[t] = double4_t{(double)st[0], (double)st[1], (double)st[2], (double)st[3]};
                    msum += z[buf][t][0] * od[t][0] + z[buf][t][1] * od[t][1] + z[buf][t][2] * od[t][2] +
                            z[buf][t][3] * od[t][3];
                    if constexpr (WP) *reinterpret_cast<double4_t*>(Pp + at(g, t)) = pv[buf][t] + c0 * od[t];
                }
                for (int q = 1; q < a.nsets; ++q) {
                    const double c = a.coef[q * a.cstride + a.l];
                    if (c == 0.0) continue;
                    double* __restrict__ Pq = Pp + q * a.pstride;
                    double4_t pq[EG];
#pragma unroll
                    for (int t = 0; t < EG; ++t) pq[t] = *reinterpret_cast<const double4_t*>(Pq + at(g, t));
#pragma unroll
                    for (int t = 0; t < EG; ++t) *reinterpret_cast<double4_t*>(Pq + at(g, t)) = pq[t] + c * od[t];
                }
            }
        };
        typedef std::integral_constant<bool, true> yes;
        typedef std::integral_constant<bool, false> no;
        if (a.has_prev) {
            if (c0 != 0.0) pipelined(yes{}, yes{});
            else pipelined(yes{}, no{});
        } else {
            if (c0 != 0.0) pipelined(no{}, yes{});
            else pipelined(no{}, no{});
        }
    } else {
#pragma unroll
        for (int g0 = 0; g0 < NTILE; g0 += EG) {
            long idx[EG];
            svec_t up[EG];
            double4_t z[EG], pv[EG], od[EG];
#pragma unroll
            for (int t = 0; t < EG; ++t) {
                const int i = (g0 + t) / TN, j = (g0 + t) % TN;
                idx[t] = (long)(row0 + 16 * i + 4 * lq) + (long)(col0 + 16 * j + li) * a.Kp;
                if (a.has_prev) up[t] = *reinterpret_cast<const svec_t*>(Uprev + idx[t]);
                z[t] = *reinterpret_cast<const double4_t*>(Zp + idx[t]);
                if (c0 != 0.0) pv[t] = *reinterpret_cast<const double4_t*>(Pp + idx[t]);
            }
#pragma unroll
            for (int t = 0; t < EG; ++t) {
                const int i = (g0 + t) / TN, j = (g0 + t) % TN;
                cvec_t out = alpha * acc[i][j];
                if (a.has_prev) out -= __builtin_convertvector(up[t], cvec_t);
                const svec_t st = __builtin_convertvector(out, svec_t);
                *reinterpret_cast<svec_t*>(Unext + idx[t]) = st;
                od[t] = double4_t{(double)st[0], (double)st[1], (double)st[2], (double)st[3]};
                msum += z[t][0] * od[t][0] + z[t][1] * od[t][1] + z[t][2] * od[t][2] + z[t][3] * od[t][3];
                if (c0 != 0.0) *reinterpret_cast<double4_t*>(Pp + idx[t]) = pv[t] + c0 * od[t];
            }
            for (int q = 1; q < a.nsets; ++q) {
                const double c = a.coef[q * a.cstride + a.l];
                if (c == 0.0) continue;
                double* __restrict__ Pq = Pp + q * a.pstride;
#pragma unroll
                for (int t = 0; t < EG; ++t) pv[t] = *reinterpret_cast<const double4_t*>(Pq + idx[t]);
#pragma unroll
                for (int t = 0; t < EG; ++t) *reinterpret_cast<double4_t*>(Pq + idx[t]) = pv[t] + c * od[t];
            }
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) msum += __shfl_xor(msum, off, 64);
    __shared__ double red[WM * WN];
    if (lane == 0) red[wave] = msum;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < WM * WN; ++w) s += red[w];
        a.partial[(long)a.l * (ntm * ntn) + tp.logical] = s;
    }
}

// ------------------------------------------------------------ split reduction
// Narrow column blocks leave too few tiles to keep enough operator bytes in
// flight.  The reduction is cut into NSPLIT chunks: workgroup b takes chunk
// b % NSPLIT, and since workgroups are dispatched round-robin over the 8
// XCDs, with NSPLIT = 8 each XCD streams its own slice of every operator row
// and keeps only its slice of the column block (BN x Kp/8) hot in its L2.
// Each workgroup stores its partial product; cheb_combine_kernel sums the
// chunks in chunk order and applies the recursion epilogue.
template <typename T, int TM, int TN, int WM, int WN, int KV, int DEPTH, int NSPLIT, bool NT>
__global__ void __launch_bounds__(64 * WM * WN)
cheb_partial_kernel(ChebStepArgs a) {
    typedef typename Mfma<T>::vec_t vec_t;
    constexpr int BM = 16 * TM * WM, BN = 16 * TN * WN;
    const int ntm = a.Kp / BM;
    const int chunk = blockIdx.x % NSPLIT;
    const int t = blockIdx.x / NSPLIT;
    const int kc = a.Kp / NSPLIT;
    const int wave = threadIdx.x >> 6;
    const int row0 = (t % ntm) * BM + (wave % WM) * TM * 16;
    const int col0 = (t / ntm) * BN + (wave / WM) * TN * 16;
    typename Mfma<T>::acc_t acc[TM][TN];
    const long k0 = (long)chunk * kc;
    gemm_mainloop<T, TM, TN, KV, DEPTH, NT>(kc, static_cast<const T*>(a.HN) + k0, a.Kp,
                                            static_cast<const T*>(a.Ucur) + k0, a.Kp, row0, col0, acc);
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lq = lane >> 4;
    T* W = static_cast<T*>(a.work) + (long)chunk * a.Kp * a.Bp;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const long idx = (long)(row0 + 16 * i + 4 * lq) + (long)(col0 + 16 * j + li) * a.Kp;
            *reinterpret_cast<vec_t*>(W + idx) = acc[i][j];
        }
}

// One thread per four consecutive rows of one column (column-major index
// 4q); 256 threads per workgroup, Kp * Bp / 1024 workgroups.
template <typename T, int NSPLIT>
__global__ void __launch_bounds__(256) cheb_combine_kernel(ChebStepArgs a) {
    typedef typename Mfma<T>::vec_t vec_t;
    const long idx = 4 * ((long)blockIdx.x * 256 + threadIdx.x);
    const long plane = (long)a.Kp * a.Bp;
    const T* W = static_cast<const T*>(a.work);
    vec_t sum = *reinterpret_cast<const vec_t*>(W + idx);
#pragma unroll
    for (int c = 1; c < NSPLIT; ++c) sum += *reinterpret_cast<const vec_t*>(W + c * plane + idx);
    vec_t out = static_cast<T>(a.alpha) * sum;
    if (a.has_prev) out -= *reinterpret_cast<const vec_t*>(static_cast<const T*>(a.Uprev) + idx);
    *reinterpret_cast<vec_t*>(static_cast<T*>(a.Unext) + idx) = out;
    const double4_t z = *reinterpret_cast<const double4_t*>(a.Z + idx);
    double4_t od = {(double)out[0], (double)out[1], (double)out[2], (double)out[3]};
    double msum = z[0] * od[0] + z[1] * od[1] + z[2] * od[2] + z[3] * od[3];
    for (int q = 0; q < a.nsets; ++q) {
        const double c = a.coef[q * a.cstride + a.l];
        if (c != 0.0) {
            double4_t* p = reinterpret_cast<double4_t*>(a.P + q * a.pstride + idx);
            *p = *p + c * od;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) msum += __shfl_xor(msum, off, 64);
    __shared__ double red[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = msum;
    __syncthreads();
    if (threadIdx.x == 0)
        a.partial[(long)a.l * gridDim.x + blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// ------------------------------------------------------------ persistent batch
// Waits until the gang's barrier counter reaches `target` (every member has
// arrived); the release / acquire pair at agent scope orders this
// workgroup's U stores before the other members' loads of them.  Members
// arrive within about one row tile of each other, so a wait of max_polls
// polls (2^20 by default) means a member is not running: the waiter sets
// flag bit 8 and goes on, and once that bit is set no barrier waits any
// more, so the launch drains (the results are then void and the host
// reports it).
__device__ inline void gang_barrier(int* bar, int target, int* flag, int max_polls) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(bar, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        int polls = 0;
        while (__hip_atomic_load(bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 8) break;
            __builtin_amdgcn_s_sleep(1);
            if (++polls > max_polls) {
                atomicOr(flag, 8);
                break;
            }
        }
    }
    __syncthreads();
}

// With gmap = 8 workgroup b belongs to gang (b / 8 / kGang) * 8 + b % 8 as
// member (b / 8) % kGang: workgroups are dealt to the 8 XCDs round robin, so
// a gang's members share one XCD and its L2, where the U panel that all of
// them read for a shared item stays while they walk their row tiles.  The
// grid is exactly the resident workgroups, so every member of a gang runs
// at once.
template <typename T, int TM, int TN, int WM, int WN, int KV, int DEPTH>
__global__ void __launch_bounds__(64 * WM * WN)
cheb_batch_kernel(BatchArgs a) {
    typedef typename Mfma<T>::vec_t vec_t;
    constexpr int BM = 16 * TM * WM, BN = 16 * TN * WN;
    static_assert(128 % (4 * KV * DEPTH) == 0 && 128 % BM == 0, "the live extent Kt is a multiple of 128");
    __shared__ double red[WM * WN];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lq = lane >> 4;
    const int slot = blockIdx.x / a.gmap;
    const int gang = (slot / kGang) * a.gmap + blockIdx.x % a.gmap, member = slot % kGang;
    int nbar = 0;  // barriers this gang has passed
    for (int r = a.gang_start[gang]; r < a.gang_start[gang + 1]; ++r) {
        const BatchRound rd = a.rounds[r];
        if (!rd.split && member >= rd.n) continue;
        const BatchItem item = rd.item[rd.split ? 0 : member];
        const int row_first = rd.split ? member : 0, row_step = rd.split ? kGang : 1;
        const BatchCluster cl = a.clusters[item.cluster];
        const int Kp = cl.Kp;
        const T* HN = static_cast<const T*>(cl.HN);
        T* ua = static_cast<T*>(cl.Ua);
        T* ub = static_cast<T*>(cl.Ub);
        const int col0 = item.block * BN + (wave / WM) * TN * 16;
        for (int l = 1; l <= a.order; ++l) {
            // odd l: U_{l-1} in ua, U_l -> ub; even l: U_{l-1} in ub, U_l -> ua (over U_{l-2})
            const T* ucur = (l & 1) ? ua : ub;
            T* unext = (l & 1) ? ub : ua;
            const double c = a.with_P ? cl.coef[l] : 0.0;
            const T alpha = static_cast<T>(l == 1 ? 1.0 : 2.0);
            double msum = 0.0;
            // rows and reduction only up to Kt: beyond it H_N and U_l are zero
            // (the rows Kt..Kp-1 of U_{l+1} are neither written nor read)
            for (int r0 = row_first * BM; r0 < cl.Kt; r0 += row_step * BM) {
                const int row0 = r0 + (wave % WM) * TM * 16;
                typename Mfma<T>::acc_t acc[TM][TN];
                gemm_mainloop<T, TM, TN, KV, DEPTH>(cl.Kt, HN, Kp, ucur, Kp, row0, col0, acc);
                // the step kernel's epilogue, loads of EG tiles issued together
                // (pairs in FP32; one at a time where the persistent loop's
                // registers are short: FP64, two waves per SIMD); pipelined
                // shapes (four waves) also issue the next group's loads
                // before this group's arithmetic, in straight-line versions
                // for the uniform conditions
                constexpr int NTILE = TM * TN;
                constexpr bool SHORT = WM * WN > 4 || sizeof(T) == 8;
                constexpr int EGMAX = SHORT ? 1 : 2;
                constexpr int EG = NTILE % EGMAX == 0 ? EGMAX : 1;
                constexpr int NG = NTILE / EG;
                // a second group of loads spills registers in the FP32 4 x
                // 4-tile, 4-k, four-slab shape
                constexpr bool PIPE = WM * WN <= 4 && !(sizeof(T) == 4 && TM * TN == 16 && KV == 4 && DEPTH == 4);
                if constexpr (PIPE) {
                    auto at = [&](int g, int t) {
                        const int i = (g * EG + t) / TN, j = (g * EG + t) % TN;
                        return (long)(row0 + 16 * i + 4 * lq) + (long)(col0 + 16 * j + li) * Kp;
                    };
                    auto pipelined = [&](auto has_prev_c, auto with_p_c) {
                        constexpr bool HP = decltype(has_prev_c)::value, WP = decltype(with_p_c)::value;
                        vec_t up[2][EG];
                        double4_t z[2][EG], pv[2][EG];
                        auto load = [&](int g, int buf) {
#pragma unroll
                            for (int t = 0; t < EG; ++t) {
                                if constexpr (HP) up[buf][t] = *reinterpret_cast<const vec_t*>(unext + at(g, t));
                                z[buf][t] = *reinterpret_cast<const double4_t*>(cl.Z + at(g, t));
                                if constexpr (WP) pv[buf][t] = *reinterpret_cast<const double4_t*>(cl.P + at(g, t));
                            }
                        };
                        load(0, 0);
#pragma unroll
                        for (int g = 0; g < NG; ++g) {
                            const int buf = g & 1;
                            if (g + 1 < NG) load(g + 1, buf ^ 1);
#pragma unroll
                            for (int t = 0; t < EG; ++t) {
                                const int i = (g * EG + t) / TN, j = (g * EG + t) % TN;
                                vec_t out = alpha * acc[i][j];
                                if constexpr (HP) out -= up[buf][t];
                                *reinterpret_cast<vec_t*>(unext + at(g, t)) = out;
                                double4_t od = {(double)out[0], (double)out[1], (double)out[2], (double)out[3]};
                                msum += z[buf][t][0] * od[0] + z[buf][t][1] * od[1] + z[buf][t][2] * od[2] +
                                        z[buf][t][3] * od[3];
                                if constexpr (WP)
                                    *reinterpret_cast<double4_t*>(cl.P + at(g, t)) = pv[buf][t] + c * od;
                            }
                        }
                    };
                    typedef std::integral_constant<bool, true> yes;
                    typedef std::integral_constant<bool, false> no;
                    if (l > 1) {
                        if (c != 0.0) pipelined(yes{}, yes{});
                        else pipelined(yes{}, no{});
                    } else {
                        if (c != 0.0) pipelined(no{}, yes{});
                        else pipelined(no{}, no{});
                    }
                } else {
#pragma unroll
                    for (int g0 = 0; g0 < NTILE; g0 += EG) {
                        long idx[EG];
                        vec_t up[EG];
                        double4_t z[EG], pv[EG];
#pragma unroll
                        for (int t = 0; t < EG; ++t) {
                            const int i = (g0 + t) / TN, j = (g0 + t) % TN;
                            idx[t] = (long)(row0 + 16 * i + 4 * lq) + (long)(col0 + 16 * j + li) * Kp;
                            if (l > 1) up[t] = *reinterpret_cast<const vec_t*>(unext + idx[t]);
                            z[t] = *reinterpret_cast<const double4_t*>(cl.Z + idx[t]);
                            if (c != 0.0) pv[t] = *reinterpret_cast<const double4_t*>(cl.P + idx[t]);
                        }
#pragma unroll
                        for (int t = 0; t < EG; ++t) {
                            const int i = (g0 + t) / TN, j = (g0 + t) % TN;
                            vec_t out = alpha * acc[i][j];
                            if (l > 1) out -= up[t];
                            *reinterpret_cast<vec_t*>(unext + idx[t]) = out;
                            double4_t od = {(double)out[0], (double)out[1], (double)out[2], (double)out[3]};
                            msum += z[t][0] * od[0] + z[t][1] * od[1] + z[t][2] * od[2] + z[t][3] * od[3];
                            if (c != 0.0) *reinterpret_cast<double4_t*>(cl.P + idx[t]) = pv[t] + c * od;
                        }
                    }
                }
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) msum += __shfl_xor(msum, off, 64);
            if (lane == 0) red[wave] = msum;
            __syncthreads();
            if (threadIdx.x < kGang) {
                // one partial per (step, block, member); a member working
                // alone writes its sum into slot 0 and zeros elsewhere
                double s = 0.0;
                if (threadIdx.x == (rd.split ? member : 0)) {
#pragma unroll
                    for (int w = 0; w < WM * WN; ++w) s += red[w];
                }
                if (rd.split ? threadIdx.x == member : true)
                    cl.partial[((long)l * cl.nblocks + item.block) * kGang + threadIdx.x] = s;
            }
            // the barrier (or, alone, the workgroup barrier) also orders this
            // step's U writes before the next step's reads
            if (rd.split)
                gang_barrier(a.bar + gang, kGang * ++nbar, a.flag, a.max_polls);
            else
                __syncthreads();
        }
    }
}

struct CfgShape {
    int tm, tn, wm, wn, kv, depth;
    int split = 1;    // reduction chunks (one per XCD)
    bool nt = false;  // non-temporal operator loads
    int precs = 3;     // built for FP64 (bit 0) and/or FP32 (bit 1)
    bool ldsb = false; // B panel shared through LDS
};
// Split shapes serve narrow passes only (the partial products take
// split x Kp x Bp elements).
constexpr int kSplitMaxCols = 512;
// Tile shapes of the recursion step (rows x columns per workgroup, k per
// lane and slab).  The first four suit the compute-bound wide blocks; the
// last three keep more operator bytes in flight for narrow, memory-bound
// blocks.  KV = 16 is FP32 only.
constexpr CfgShape kChebCfgs[] = {
    {4, 4, 2, 2, 4, 2},   // 128 x 128
    {4, 2, 2, 2, 4, 2},   // 128 x 64
    {2, 2, 4, 1, 4, 2},   // 128 x 32
    {2, 2, 2, 2, 4, 2},   // 64 x 64
    {1, 2, 4, 1, 8, 2},   // 64 x 32, 8 k per lane
    {1, 4, 4, 1, 8, 2},   // 64 x 64, 8 k per lane
    {1, 2, 4, 1, 16, 2, 1, false, 2},  // 64 x 32, 16 k per lane (FP32)
    {2, 2, 4, 1, 4, 4},   // 128 x 32, three slabs in flight
    {4, 2, 2, 2, 4, 4},   // 128 x 64, three slabs in flight
    {1, 2, 4, 1, 4, 4},   // 64 x 32, three slabs in flight
    {4, 2, 2, 4, 4, 2},   // 128 x 128, 8 waves: two waves per SIMD
    {2, 4, 4, 2, 4, 2},   // 128 x 128, 8 waves, 32 x 64 per wave
    {4, 4, 2, 2, 4, 4},   // 128 x 128, three slabs in flight
    {1, 2, 4, 1, 4, 4, 8, false},  // 64 x 32, 8 reduction chunks
    {2, 2, 4, 1, 4, 4, 8, false},  // 128 x 32, 8 reduction chunks
    {1, 2, 4, 1, 8, 2, 8, false},  // 64 x 32, 8 chunks, 8 k per lane
    {1, 2, 4, 1, 4, 4, 8, true},   // 64 x 32, 8 chunks, non-temporal operator
    {1, 4, 4, 1, 4, 4, 8, false},  // 64 x 64, 8 chunks
    {2, 4, 4, 1, 4, 4, 8, true},   // 128 x 64, 8 chunks, non-temporal operator
    {1, 2, 4, 1, 4, 4, 16, false}, // 64 x 32, 16 chunks (two per XCD)
    {2, 2, 4, 1, 4, 8},   // 128 x 32, seven slabs in flight
    {1, 2, 4, 1, 4, 8},   // 64 x 32, seven slabs in flight
    {2, 2, 4, 1, 8, 4, 1, false, 2},   // 128 x 32, 8 k per lane, three slabs in flight (FP32)
    {2, 2, 4, 1, 4, 16, 1, false, 2},  // 128 x 32, fifteen slabs in flight (FP32)
    {4, 2, 2, 2, 4, 8, 1, false, 2},   // 128 x 64, seven slabs in flight (FP32)
    {2, 2, 4, 1, 8, 8, 1, false, 2},   // 128 x 32, 8 k per lane, seven slabs in flight (FP32)
    {1, 2, 8, 1, 8, 4, 1, false, 2},   // 128 x 32, 8 waves, 8 k per lane (FP32)
    {4, 4, 2, 2, 8, 4, 1, false, 2},   // 128 x 128, 8 k per lane, three slabs in flight (FP32)
    {4, 2, 2, 2, 8, 4, 1, false, 2},   // 128 x 64, 8 k per lane, three slabs in flight (FP32)
    {2, 2, 4, 1, 8, 8, 1, false, 2, true},   // 128 x 32, panel in LDS, seven slabs (FP32)
    {2, 2, 4, 1, 8, 4, 1, false, 2, true},   // 128 x 32, panel in LDS, three slabs (FP32)
    {2, 4, 4, 1, 8, 4, 1, false, 2, true},   // 128 x 64, panel in LDS, three slabs (FP32)
    {2, 2, 4, 1, 4, 4, 1, false, 1, true},  // 128 x 32, panel in LDS, three slabs (FP64)
    {2, 2, 4, 1, 4, 8, 1, false, 1, true},  // 128 x 32, panel in LDS, seven slabs (FP64)
    {2, 8, 4, 1, 4, 4, 1, false, 3, true},  // 128 x 128, panel in LDS, three slabs
    {2, 8, 4, 1, 8, 4, 1, false, 2, true},  // 128 x 128, panel in LDS, 8 k per lane (FP32)
    {2, 4, 4, 1, 4, 4, 1, false, 1, true},  // 128 x 64, panel in LDS, three slabs (FP64)
};

template <typename T, int TM, int TN, int WM, int WN, int KV, int DEPTH = 2, bool LDSB = false>
hipError_t launch_one(const ChebStepArgs& a, hipStream_t s) {
    constexpr int BM = 16 * TM * WM, BN = 16 * TN * WN;
    if (a.Kp % BM || a.Bp % BN || a.Kp % (4 * DEPTH * KV)) return hipErrorInvalidValue;
    const dim3 grid((a.Kp / BM) * (a.Bp / BN));
    hipLaunchKernelGGL((cheb_step_kernel<T, TM, TN, WM, WN, KV, DEPTH, LDSB>), grid, dim3(64 * WM * WN), 0, s, a);
    return hipGetLastError();
}

template <typename T, int TM, int TN, int WM, int WN, int KV, int DEPTH, int NSPLIT, bool NT>
hipError_t launch_split(const ChebStepArgs& a, hipStream_t s) {
    constexpr int BM = 16 * TM * WM, BN = 16 * TN * WN;
    if (a.Kp % BM || a.Bp % BN || a.Bp > kSplitMaxCols || a.Kp % (NSPLIT * 4 * DEPTH * KV) || !a.work)
        return hipErrorInvalidValue;
    const dim3 grid(NSPLIT * (a.Kp / BM) * (a.Bp / BN));
    hipLaunchKernelGGL((cheb_partial_kernel<T, TM, TN, WM, WN, KV, DEPTH, NSPLIT, NT>), grid,
                       dim3(64 * WM * WN), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((cheb_combine_kernel<T, NSPLIT>), dim3((long)a.Kp * a.Bp / 1024), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cheb(const ChebStepArgs& a, int cfg, hipStream_t s) {
    switch (cfg) {
        case 0: return launch_one<T, 4, 4, 2, 2, 4>(a, s);
        case 1: return launch_one<T, 4, 2, 2, 2, 4>(a, s);
        case 2: return launch_one<T, 2, 2, 4, 1, 4>(a, s);
        case 3: return launch_one<T, 2, 2, 2, 2, 4>(a, s);
        case 4: return launch_one<T, 1, 2, 4, 1, 8>(a, s);
        case 5: return launch_one<T, 1, 4, 4, 1, 8>(a, s);
        case 6:
            if constexpr (sizeof(T) == 4) return launch_one<float, 1, 2, 4, 1, 16>(a, s);
            return hipErrorInvalidValue;
        case 7: return launch_one<T, 2, 2, 4, 1, 4, 4>(a, s);
        case 8: return launch_one<T, 4, 2, 2, 2, 4, 4>(a, s);
        case 9: return launch_one<T, 1, 2, 4, 1, 4, 4>(a, s);
        case 10: return launch_one<T, 4, 2, 2, 4, 4>(a, s);
        case 11: return launch_one<T, 2, 4, 4, 2, 4>(a, s);
        case 12: return launch_one<T, 4, 4, 2, 2, 4, 4>(a, s);
        case 13: return launch_split<T, 1, 2, 4, 1, 4, 4, 8, false>(a, s);
        case 14: return launch_split<T, 2, 2, 4, 1, 4, 4, 8, false>(a, s);
        case 15: return launch_split<T, 1, 2, 4, 1, 8, 2, 8, false>(a, s);
        case 16: return launch_split<T, 1, 2, 4, 1, 4, 4, 8, true>(a, s);
        case 17: return launch_split<T, 1, 4, 4, 1, 4, 4, 8, false>(a, s);
        case 18: return launch_split<T, 2, 4, 4, 1, 4, 4, 8, true>(a, s);
        case 19: return launch_split<T, 1, 2, 4, 1, 4, 4, 16, false>(a, s);
        case 20: return launch_one<T, 2, 2, 4, 1, 4, 8>(a, s);
        case 21: return launch_one<T, 1, 2, 4, 1, 4, 8>(a, s);
        case 22:
            if constexpr (sizeof(T) == 4) return launch_one<float, 2, 2, 4, 1, 8, 4>(a, s);
            return hipErrorInvalidValue;
        case 23:
            if constexpr (sizeof(T) == 4) return launch_one<float, 2, 2, 4, 1, 4, 16>(a, s);
            return hipErrorInvalidValue;
        case 24:
            if constexpr (sizeof(T) == 4) return launch_one<float, 4, 2, 2, 2, 4, 8>(a, s);
            return hipErrorInvalidValue;
        case 25:
            if constexpr (sizeof(T) == 4) return launch_one<float, 2, 2, 4, 1, 8, 8>(a, s);
            return hipErrorInvalidValue;
        case 26:
            if constexpr (sizeof(T) == 4) return launch_one<float, 1, 2, 8, 1, 8, 4>(a, s);
            return hipErrorInvalidValue;
        case 27:
            if constexpr (sizeof(T) == 4) return launch_one<float, 4, 4, 2, 2, 8, 4>(a, s);
            return hipErrorInvalidValue;
        case 28:
            if constexpr (sizeof(T) == 4) return launch_one<float, 4, 2, 2, 2, 8, 4>(a, s);
            return hipErrorInvalidValue;
        case 29:
            if constexpr (sizeof(T) == 4) return launch_one<float, 2, 2, 4, 1, 8, 8, true>(a, s);
            return hipErrorInvalidValue;
        case 30:
            if constexpr (sizeof(T) == 4) return launch_one<float, 2, 2, 4, 1, 8, 4, true>(a, s);
            return hipErrorInvalidValue;
        case 31:
            if constexpr (sizeof(T) == 4) return launch_one<float, 2, 4, 4, 1, 8, 4, true>(a, s);
            return hipErrorInvalidValue;
        case 32:
            if constexpr (sizeof(T) == 8) return launch_one<double, 2, 2, 4, 1, 4, 4, true>(a, s);
            return hipErrorInvalidValue;
        case 33:
            if constexpr (sizeof(T) == 8) return launch_one<double, 2, 2, 4, 1, 4, 8, true>(a, s);
            return hipErrorInvalidValue;
        case 34: return launch_one<T, 2, 8, 4, 1, 4, 4, true>(a, s);
        case 35:
            if constexpr (sizeof(T) == 4) return launch_one<float, 2, 8, 4, 1, 8, 4, true>(a, s);
            return hipErrorInvalidValue;
        case 36:
            if constexpr (sizeof(T) == 8) return launch_one<double, 2, 4, 4, 1, 4, 4, true>(a, s);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int TM, int TN, int WM, int WN, int KV, int DEPTH = 2>
hipError_t launch_batch_one(const BatchArgs& a, int grid, hipStream_t s, int* occ) {
    if (occ) {
        *occ = 0;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(
            occ, reinterpret_cast<const void*>(&cheb_batch_kernel<T, TM, TN, WM, WN, KV, DEPTH>), 64 * WM * WN, 0);
    }
    hipLaunchKernelGGL((cheb_batch_kernel<T, TM, TN, WM, WN, KV, DEPTH>), dim3(grid), dim3(64 * WM * WN), 0, s, a);
    return hipGetLastError();
}

// Tile shapes of the batch kernel, named by their index in kChebCfgs (the
// main loop and epilogue are the same code, so a batch run and a pinned
// single-operator run of the same shape agree bit for bit).
// occ != nullptr: report the occupancy instead of launching.
template <typename T>
hipError_t launch_batch(const BatchArgs& a, int cfg, int grid, hipStream_t s, int* occ) {
    switch (cfg) {
        case 0: return launch_batch_one<T, 4, 4, 2, 2, 4>(a, grid, s, occ);
        case 1: return launch_batch_one<T, 4, 2, 2, 2, 4>(a, grid, s, occ);
        case 2: return launch_batch_one<T, 2, 2, 4, 1, 4>(a, grid, s, occ);
        case 3: return launch_batch_one<T, 2, 2, 2, 2, 4>(a, grid, s, occ);
        case 7: return launch_batch_one<T, 2, 2, 4, 1, 4, 4>(a, grid, s, occ);
        case 8: return launch_batch_one<T, 4, 2, 2, 2, 4, 4>(a, grid, s, occ);
        case 12:  // the FP64 build of this ring spills in the persistent loop
            if constexpr (sizeof(T) == 4) return launch_batch_one<float, 4, 4, 2, 2, 4, 4>(a, grid, s, occ);
            return hipErrorInvalidValue;
        case 27:
            if constexpr (sizeof(T) == 4) return launch_batch_one<float, 4, 4, 2, 2, 8, 4>(a, grid, s, occ);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t cheb_batch(const BatchArgs& a, int cfg, int precision, int grid, hipStream_t s) {
    if (grid < 1) return hipErrorInvalidValue;
    return precision == 0 ? launch_batch<double>(a, cfg, grid, s, nullptr)
                          : launch_batch<float>(a, cfg, grid, s, nullptr);
}

int cheb_batch_num_cfgs() { return 8; }
int cheb_batch_cfg(int i, int precision) {
    static const int kBatch[] = {0, 1, 2, 3, 7, 8, 12, 27};
    if (i < 0 || i >= 8) return -1;
    const int cfg = kBatch[i];
    if (precision == 0 && cfg == 12) return -1;
    return cheb_cfg_supports(cfg, precision) ? cfg : -1;
}

int cheb_batch_occupancy(int cfg, int precision) {
    int occ = 0;
    hipError_t e = precision == 0 ? launch_batch<double>(BatchArgs{}, cfg, 1, nullptr, &occ)
                                  : launch_batch<float>(BatchArgs{}, cfg, 1, nullptr, &occ);
    return e == hipSuccess ? occ : 0;
}

int cheb_num_tile_configs() { return (int)(sizeof(kChebCfgs) / sizeof(kChebCfgs[0])); }
// Shapes built for the refined precision (FP32 storage, FP64 arithmetic).
constexpr int kW32Cfgs[] = {0, 2, 3, 7, 12, 20, 22, 29, 30};
bool cheb_cfg_supports(int cfg, int precision) {
    if (precision == 2) {
        for (int x : kW32Cfgs)
            if (x == cfg) return true;
        return false;
    }
    return (kChebCfgs[cfg].precs >> (precision == 0 ? 0 : 1)) & 1;
}
int cheb_tile_rows(int cfg) { return 16 * kChebCfgs[cfg].tm * kChebCfgs[cfg].wm; }
int cheb_tile_cols(int cfg) { return 16 * kChebCfgs[cfg].tn * kChebCfgs[cfg].wn; }
int cheb_cfg_split(int cfg) { return kChebCfgs[cfg].split; }
bool cheb_cfg_fits(int cfg, int precision, int Kp, int Bp) {
    if (cfg < 0 || cfg >= cheb_num_tile_configs() || !cheb_cfg_supports(cfg, precision)) return false;
    const CfgShape& c = kChebCfgs[cfg];
    if (Kp % cheb_tile_rows(cfg) || Bp % cheb_tile_cols(cfg)) return false;
    if (Kp % (c.split * 4 * c.depth * c.kv)) return false;
    return c.split == 1 || Bp <= kSplitMaxCols;
}
size_t cheb_work_bytes(int Kp, int Bp, int cfg, int precision) {
    const int sp = kChebCfgs[cfg].split;
    return sp == 1 ? 0 : (size_t)sp * Kp * Bp * (precision == 0 ? 8 : 4);
}
int cheb_num_tiles(int Kp, int Bp, int cfg) {
    if (kChebCfgs[cfg].split > 1) return (int)((long)Kp * Bp / 1024);
    return (Kp / cheb_tile_rows(cfg)) * (Bp / cheb_tile_cols(cfg));
}

hipError_t cheb_step_f64(const ChebStepArgs& a, int cfg, hipStream_t s) {
    return launch_cheb<double>(a, cfg, s);
}
hipError_t cheb_step_f32(const ChebStepArgs& a, int cfg, hipStream_t s) {
    return launch_cheb<float>(a, cfg, s);
}

// The refined precision: the shapes of kW32Cfgs with FP32 operands widened
// to FP64 in registers.
hipError_t cheb_step_w32(const ChebStepArgs& a, int cfg, hipStream_t s) {
    switch (cfg) {
        case 0: return launch_one<W32, 4, 4, 2, 2, 4>(a, s);
        case 2: return launch_one<W32, 2, 2, 4, 1, 4>(a, s);
        case 3: return launch_one<W32, 2, 2, 2, 2, 4>(a, s);
        case 7: return launch_one<W32, 2, 2, 4, 1, 4, 4>(a, s);
        case 12: return launch_one<W32, 4, 4, 2, 2, 4, 4>(a, s);
        case 20: return launch_one<W32, 2, 2, 4, 1, 4, 8>(a, s);
        case 22: return launch_one<W32, 2, 2, 4, 1, 8, 4>(a, s);
        case 29: return launch_one<W32, 2, 2, 4, 1, 8, 8, true>(a, s);
        case 30: return launch_one<W32, 2, 2, 4, 1, 8, 4, true>(a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t cheb_step(const ChebStepArgs& a, int cfg, int precision, hipStream_t s) {
    switch (precision) {
        case 0: return cheb_step_f64(a, cfg, s);
        case 1: return cheb_step_f32(a, cfg, s);
        case 2: return cheb_step_w32(a, cfg, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t gemm_nn_f64(int M, int N, int Kred, double alpha, const double* A, long lda, const double* B,
                       long ldb, double beta, double* C, long ldc, bool a_upper, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    if (M % 64 || N % 64 || Kred % 32 || Kred <= 0) return hipErrorInvalidValue;
    if (M % 128 == 0 && N % 128 == 0 && (long)(M / 128) * (N / 128) >= 256) {
        const dim3 grid((M / 128) * (N / 128));
        hipLaunchKernelGGL((gemm_nn_store_kernel<4, 4, 2, 2>), grid, dim3(256), 0, s, M, N, Kred, alpha, A, lda, B,
                           ldb, beta, C, ldc, (int)a_upper);
    } else {
        const dim3 grid((M / 64) * (N / 64));
        hipLaunchKernelGGL((gemm_nn_store_kernel<2, 2, 2, 2>), grid, dim3(256), 0, s, M, N, Kred, alpha, A, lda, B,
                           ldb, beta, C, ldc, (int)a_upper);
    }
    return hipGetLastError();
}

hipError_t gemm_tn_f64(int M, int N, int Kred, double alpha, const double* A, long lda,
                       const double* B, long ldb, double beta, double* C, long ldc,
                       bool upper_only, hipStream_t s, int a_upper_row0) {
    if (M <= 0 || N <= 0) return hipSuccess;
    if (M % 64 || N % 64 || Kred % 32 || Kred <= 0) return hipErrorInvalidValue;
    if (M % 128 == 0 && N % 128 == 0) {
        const dim3 grid((M / 128) * (N / 128));
        hipLaunchKernelGGL((gemm_tn_store_kernel<4, 4, 2, 2>), grid, dim3(256), 0, s, M, N, Kred,
                           alpha, A, lda, B, ldb, beta, C, ldc, (int)upper_only, a_upper_row0);
    } else {
        const dim3 grid((M / 64) * (N / 64));
        hipLaunchKernelGGL((gemm_tn_store_kernel<2, 2, 2, 2>), grid, dim3(256), 0, s, M, N, Kred,
                           alpha, A, lda, B, ldb, beta, C, ldc, (int)upper_only, a_upper_row0);
    }
    return hipGetLastError();
}

}  // namespace dm
