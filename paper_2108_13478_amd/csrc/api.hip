// Host runtime behind include/dm.h: argument checking, device memory, the
// operator setup sequence, the column-block passes of the recursion and the
// trace / chemical-potential calls.  Every arithmetic step on matrices and
// vectors runs in the HIP kernels of gemm.hip and kernels.hip; the host only
// orders launches and evaluates the k x k Lanczos tridiagonal.
#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <array>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/dm.h"
#include "dm_common.hpp"

using namespace dm;

namespace {

thread_local std::string g_init_error;

template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;  // elements
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
};

long long round_up(long long x, long long m) { return (x + m - 1) / m * m; }

// True for device memory (hipMalloc'ed, e.g. a torch tensor on the GPU);
// host memory, registered or not, is false.
bool is_device_ptr(const void* p) {
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice;
}

// Progress of long operator setups on stderr when the environment variable
// DM_LOG is set (minutes at K ~ 10^5): phase, elapsed seconds.
struct SetupLog {
    bool on = std::getenv("DM_LOG") != nullptr;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    void operator()(const char* fmt, ...) const {
        if (!on) return;
        const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        std::fprintf(stderr, "[dm setup %7.1f s] ", dt);
        va_list ap;
        va_start(ap, fmt);
        std::vfprintf(stderr, fmt, ap);
        va_end(ap);
        std::fputc('\n', stderr);
        std::fflush(stderr);
    }
};

}  // namespace

// Device memory of dm_chebyshev_block_noalloc: one array per GPU, resident
// from the moment the library's code object is loaded on that GPU until the
// process ends.  Host code never passes the array's name to a kernel or a
// copy: the name is a host-side stand-in.  The device address is looked up
// once per device, with that device current, by noalloc_register (called
// from dm_init) and kept in g_scratch_ptr.
constexpr size_t kScratchBytes = size_t(128) << 20;
static __device__ __align__(256) double dm_noalloc_scratch[kScratchBytes / 8];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};

// Called with `device` current.  Returns the lookup's status; on failure the
// device's pointer stays null and the allocation-free entry point refuses.
hipError_t noalloc_register(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_done[device]) return g_scratch_ptr[device] ? hipSuccess : hipErrorInvalidSymbol;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(dm_noalloc_scratch));
    g_scratch_done[device] = true;
    g_scratch_ptr[device] = (e == hipSuccess) ? ptr : nullptr;
    if (e != hipSuccess) (void)hipGetLastError();
    return e;
}

void* noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}
}  // namespace

// One loaded operator: the overlap in CSR, S^-1, H^T = (S^-1 F)^T and H_N in
// the recursion precision, all padded to Kp, and its spectral interval.
struct Op {
    long long K = 0;
    int Kp = 0;
    double emin = 0, emax = 0;
    double lz_emin = 0, lz_emax = 0, lz_resid_lo = 0, lz_resid_hi = 0;
    int lz_steps_done = 0;
    DevBuf<long long> S_rowptr;
    DevBuf<int> S_col;
    DevBuf<double> S_val;
    DevBuf<double> Sinv;   // Kp x Kp, S^-1
    DevBuf<double> HT;     // Kp x Kp, (S^-1 F)^T column-major = H row-major
    DevBuf<double> HNbuf;  // Kp x Kp of the recursion precision (FP64 slots reused for FP32)
    DevBuf<double> HN64;   // batch with FP64 moments under an FP32 recursion: H_N in FP64
    // symmetric form (DM_FORM_SYMMETRIC): S = U^T U; only X = U^-1 (upper,
    // FP64) is kept beside H~_N = (X^T F X - Ebar) / dE in HNbuf (F in CSR
    // below, to rebuild H~_N for other bounds or another precision).
    // sym_raw: HNbuf still holds H~ itself (between its panels and the
    // Lanczos interval)
    int form = DM_FORM_GENERAL;
    DevBuf<double> Xs;
    // F in groups of four rows (sym_panels' sparse products)
    DevBuf<long long> Fg_ptr;
    DevBuf<int> Fg_col;
    DevBuf<double> Fg_val;
    bool sym_raw = false;
    int hn_precision_raw = -1;
    double hn_lo = 0, hn_hi = 0;  // interval HNbuf was last normalised with
    // orthonormal basis (dm_set_fock_orthonormal): S = I, H = F kept in CSR
    // (S_* then hold the identity), no dense S^-1 / H^T
    bool orth = false;
    int hn_precision = -1;  // precision H_N was last built in
    DevBuf<long long> F_rowptr;
    DevBuf<int> F_col;
    DevBuf<double> F_val;
    // factored form (DM_FORM_FACTORED): sparse F, S and the FSAI factor G;
    // no dense arrays
    FactOp* fact = nullptr;
    void release() {
        if (fact) fact_destroy(fact);
        fact = nullptr;
        S_rowptr.release(); S_col.release(); S_val.release();
        Sinv.release(); HT.release(); HNbuf.release(); HN64.release();
        Xs.release();
        Fg_ptr.release(); Fg_col.release(); Fg_val.release();
        sym_raw = false;
        F_rowptr.release(); F_col.release(); F_val.release();
        K = 0; Kp = 0; form = DM_FORM_GENERAL; orth = false;
    }
};

struct BatchState;
struct MlpState;

// dm_density_on_grid: the per-function arrays and cell lists of the last
// call (they depend on the basis, the grid, eta and the columns, not on P),
// reused while those inputs are the same, and the staging buffers of P and n.
struct GridPlan {
    bool valid = false;
    long long K = 0;
    int dims[3] = {0, 0, 0};
    std::vector<double> key;         // centres, exponents, origin, h, eta
    std::vector<long long> key_cols;
    int ncx = 0, ncy = 0, ncz = 0;
    DevBuf<double> fx, fy, fz, fe, fn, fr, P, Pp, n;
    DevBuf<int> bp, bi, ap, ai, ac, perm;
    void release() {
        for (auto* x : {&fx, &fy, &fz, &fe, &fn, &fr, &P, &Pp, &n}) x->release();
        for (auto* x : {&bp, &bi, &ap, &ai, &ac, &perm}) x->release();
        valid = false;
    }
};

struct dm_ctx {
    dm_options opt{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool poisoned = false;
    std::string err;

    // operator
    bool have_fock = false;
    int precision = DM_FP64;
    Op op;
    // batch of independent operators (dm_batch_set_focks)
    std::vector<Op> batch;
    BatchState* bstate = nullptr;
    MlpState* mlp = nullptr;

    // moments
    DevBuf<double> mom;
    int mom_order = -1;
    long long ncols_done = 0;

    // pass width and tile shape chosen by dm_autotune (0 / -1: none)
    int tuned_width = 0;
    int tuned_cfg = -1;
    // operator form used by the next dm_set_fock
    int form = DM_FORM_GENERAL;
    // precision of the batch's moments pass for batches loaded afterwards
    // (-1: the recursion precision)
    int batch_mom_prec = -1;
    // factored form: solve tolerance and iteration limit, FSAI pattern
    double cg_tol = 1e-11;
    int cg_max_iter = 2000;
    double fsai_drop = 1e-5;
    int fsai_cap = 192;

    // workspace
    DevBuf<double> Ua, Ub, Z, P;  // sized in bytes via double slots
    DevBuf<double> part_start, part_steps;
    DevBuf<double> work;  // partial products of the split-reduction shapes (byte size via double slots)
    DevBuf<double> Pfin;  // symmetric form: P = L^T Q of one pass
    DevBuf<double> coef, coef_zero, fk, w, v, out;
    // dm_combine_sets: coefficient rows, cosine-sum nodes, the bound, and
    // device copies of blocks given in host memory (kept between calls)
    DevBuf<double> cs_coef, cs_fk, cs_out, cs_stage;
    DevBuf<int> flag;
    DevBuf<long long> cols;
    GridPlan grid;
};

// Device buffers and launch tables of a loaded batch.
struct BatchClusterBufs {
    DevBuf<double> Ua, Ub, Z, P, coef, partial, pstart, mom, w, v, out, fk;
    DevBuf<long long> cols;  // 0 .. K-1
    int Bp = 0;
};

// Rounds of one batch launch (see BatchRound) and the gang layout they were
// dealt to.
struct BatchTable {
    DevBuf<BatchRound> rounds;
    DevBuf<int> gang_start;
    int grid = 0, gmap = 1, ngangs = 0;
    void release() {
        rounds.release();
        gang_start.release();
    }
};

struct BatchState {
    std::vector<BatchClusterBufs> cl;
    DevBuf<BatchCluster> d_clusters;
    BatchTable tab;
    DevBuf<int> counter;  // barrier counters: one per gang and pass
    int cfg = 0;
    int table_cfg = -1, table_order = -1, table_prec = -1;
    // moments pass in FP64 under an FP32 recursion: its own tile shape,
    // cluster table (H_N in FP64) and item list
    int mom_prec = -1;  // precision of the moments pass (set at load)
    int cfg_m = -1;
    DevBuf<BatchCluster> d_clusters_m;
    BatchTable tab_m;
    // captured graph and the parameters it was captured with
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int g_order = -1, g_prec = -1, g_cfg = -1;
    double g_beta = 0, g_tol = 0;
    bool g_with_P = true;
    std::vector<double> g_ne;
    void drop_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        g_order = -1;
    }
    ~BatchState() {
        drop_graph();
        for (auto& b : cl)
            for (auto* x : {&b.Ua, &b.Ub, &b.Z, &b.P, &b.coef, &b.partial, &b.pstart, &b.mom, &b.w,
                            &b.v, &b.out, &b.fk})
                x->release();
        for (auto& b : cl) b.cols.release();
        d_clusters.release();
        tab.release();
        d_clusters_m.release();
        tab_m.release();
        counter.release();
    }
};

// Parameters (one flat FP32 buffer: W_0, b_0, W_1, b_1, ...), gradients,
// Adam moments and activations of the predictor network.
struct MlpState {
    std::vector<int> sizes;
    std::vector<long> w_off, b_off;
    long n_params = 0;
    int t = 0;
    DevBuf<float> params, grads, m, v;
    DevBuf<float> acts;  // H_0 (input) .. H_{L-1}, then Y: B x sizes[j] each
    std::vector<long> act_off;
    DevBuf<float> T, G0, G1, partial, loss;
    DevBuf<double> mom_in;  // dm_mlp_predict: device copy of the stochastic moments
    int cap_B = 0;
    ~MlpState() {
        for (auto* b : {&params, &grads, &m, &v, &acts, &T, &G0, &G1, &partial, &loss}) b->release();
        mom_in.release();
    }
};

namespace {

// A C++ exception (host allocation failure, no thread) caught at the ABI:
// no exception crosses it.
dm_status host_exception(dm_ctx* c) {
    if (c) c->err = "host allocation failed (C++ exception)";
    return DM_E_OOM;
}

dm_status set_err(dm_ctx* c, dm_status st, const std::string& msg) {
    c->err = msg;
    return st;
}

dm_status fail_hip(dm_ctx* c, hipError_t e, const char* what) {
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        return set_err(c, DM_E_OOM, std::string("out of device memory: ") + what);
    }
    c->poisoned = true;
    return set_err(c, DM_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPTRY(c, expr)                                   \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) return fail_hip(c, e_, #expr); \
    } while (0)

template <typename T>
hipError_t ensure(DevBuf<T>& b, size_t n) {
    if (b.n >= n && b.p) return hipSuccess;
    b.release();
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&b.p), std::max<size_t>(n, 1) * sizeof(T));
    if (e != hipSuccess) {
        b.p = nullptr;
        return e;
    }
    b.n = n;
    return hipSuccess;
}

dm_status enter(dm_ctx* c) {
    if (!c) return DM_E_ARG;
    if (c->poisoned) return set_err(c, DM_E_STATE, "context poisoned by an earlier HIP error");
    HIPTRY(c, hipSetDevice(c->opt.device));
    c->err.clear();
    return DM_OK;
}

template <typename T>
hipError_t to_host(std::vector<T>& dst, const T* src, size_t n) {
    dst.resize(n);
    if (n == 0) return hipSuccess;
    return hipMemcpy(dst.data(), src, n * sizeof(T), hipMemcpyDefault);
}

// Checks a CSR matrix copied to the host; returns an empty string when valid.
std::string check_csr(const char* name, long long K, const std::vector<long long>& rp,
                      const std::vector<int>& col, const std::vector<double>& val,
                      bool positive_diag) {
    if (rp[0] != 0) return std::string(name) + ": rowptr[0] != 0";
    for (long long r = 0; r < K; ++r) {
        if (rp[r + 1] < rp[r]) return std::string(name) + ": rowptr not monotone";
        bool diag = false;
        for (long long p = rp[r]; p < rp[r + 1]; ++p) {
            if (col[p] < 0 || col[p] >= K) return std::string(name) + ": column index out of range";
            if (p > rp[r] && col[p] <= col[p - 1])
                return std::string(name) + ": columns not sorted/unique within a row";
            if (!std::isfinite(val[p])) return std::string(name) + ": non-finite value";
            if (col[p] == r) {
                diag = true;
                if (positive_diag && !(val[p] > 0)) return std::string(name) + ": non-positive diagonal";
            }
        }
        if (positive_diag && !diag) return std::string(name) + ": missing diagonal entry";
    }
    return "";
}

// -------------------------------------------------------------- tridiagonal
// Number of eigenvalues of the symmetric tridiagonal (a, b) below x (Sturm count).
int sturm_count(const std::vector<double>& a, const std::vector<double>& b, double x) {
    int cnt = 0;
    double d = 1.0;
    for (size_t i = 0; i < a.size(); ++i) {
        const double bb = i ? b[i - 1] * b[i - 1] : 0.0;
        d = a[i] - x - (i ? bb / d : 0.0);
        if (d == 0.0) d = -1e-300;
        if (d < 0) ++cnt;
    }
    return cnt;
}

double tridiag_eig(const std::vector<double>& a, const std::vector<double>& b, int idx) {
    double lo = 1e300, hi = -1e300;
    for (size_t i = 0; i < a.size(); ++i) {
        const double r = (i ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < a.size() ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (sturm_count(a, b, mid) > idx)
            hi = mid;
        else
            lo = mid;
    }
    return 0.5 * (lo + hi);
}

// |last component| of the unit eigenvector of (a, b) for eigenvalue theta,
// by three steps of inverse iteration with a dense LU (k is at most a few
// hundred, so the k^3 host work is negligible).
double tridiag_last_component(const std::vector<double>& a, const std::vector<double>& b,
                              double theta) {
    const int n = (int)a.size();
    if (n == 1) return 1.0;
    const double shift = theta + 1e-10 * (std::fabs(theta) + 1.0);
    std::vector<double> LU((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) {
        LU[(size_t)i * n + i] = a[i] - shift;
        if (i + 1 < n) LU[(size_t)i * n + i + 1] = LU[(size_t)(i + 1) * n + i] = b[i];
    }
    std::vector<int> piv(n);
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i)
            if (std::fabs(LU[(size_t)i * n + k]) > std::fabs(LU[(size_t)p * n + k])) p = i;
        piv[k] = p;
        if (p != k)
            for (int j = 0; j < n; ++j) std::swap(LU[(size_t)k * n + j], LU[(size_t)p * n + j]);
        double d = LU[(size_t)k * n + k];
        if (d == 0.0) d = LU[(size_t)k * n + k] = 1e-300;
        for (int i = k + 1; i < n; ++i) {
            const double f = (LU[(size_t)i * n + k] /= d);
            if (f != 0.0)
                for (int j = k + 1; j < n; ++j) LU[(size_t)i * n + j] -= f * LU[(size_t)k * n + j];
        }
    }
    std::vector<double> y(n, 1.0);
    for (int rep = 0; rep < 3; ++rep) {
        for (int k = 0; k < n; ++k) std::swap(y[k], y[piv[k]]);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < i; ++j) y[i] -= LU[(size_t)i * n + j] * y[j];
        for (int i = n - 1; i >= 0; --i) {
            for (int j = i + 1; j < n; ++j) y[i] -= LU[(size_t)i * n + j] * y[j];
            y[i] /= LU[(size_t)i * n + i];
        }
        double nrm = 0;
        for (double x : y) nrm += x * x;
        nrm = std::sqrt(nrm);
        if (!(nrm > 0) || !std::isfinite(nrm)) return 1.0;
        for (double& x : y) x /= nrm;
    }
    return std::fabs(y[n - 1]);
}

// ------------------------------------------------------------------ Lanczos
dm_status lanczos_bounds(dm_ctx* c, Op& op) {
    const int K = (int)op.K, ld = op.Kp;
    const int ksteps = std::max(1, std::min<int>(c->opt.lanczos_steps > 0 ? c->opt.lanczos_steps : 100, K));
    hipStream_t s = c->stream;
    DevBuf<double> V, Q, wv, sw, cc, ab, sc;
    auto cleanup = [&]() {
        V.release(); Q.release(); wv.release(); sw.release(); cc.release(); ab.release(); sc.release();
    };
    hipError_t e = hipSuccess;
    if ((e = ensure(V, (size_t)ld * (ksteps + 1))) != hipSuccess ||
        (e = ensure(Q, (size_t)ld * (ksteps + 1))) != hipSuccess ||
        (e = ensure(wv, (size_t)ld)) != hipSuccess || (e = ensure(sw, (size_t)ld)) != hipSuccess ||
        (e = ensure(cc, (size_t)ksteps + 1)) != hipSuccess ||
        (e = ensure(ab, (size_t)2 * ksteps)) != hipSuccess || (e = ensure(sc, 4)) != hipSuccess) {
        cleanup();
        return fail_hip(c, e, "lanczos buffers");
    }
    double* alpha = ab.p;
    double* beta = ab.p + ksteps;
    const long long* rp = op.S_rowptr.p;
    const int* ci = op.S_col.p;
    const double* sv = op.S_val.p;
    // the symmetric form's H~ (in HNbuf, before normalisation) with the
    // standard inner product; every other form H = S^-1 F with the S one
    const bool ident = op.form == DM_FORM_SYMMETRIC;
    auto apply_s = [&](const double* x, double* y) -> hipError_t {
        if (ident) return hipMemcpyAsync(y, x, (size_t)K * 8, hipMemcpyDeviceToDevice, s);
        return csr_spmv(K, rp, ci, sv, x, y, s);
    };
#define LZ(expr)                          \
    do {                                  \
        if ((e = (expr)) != hipSuccess) { \
            cleanup();                    \
            return fail_hip(c, e, #expr); \
        }                                 \
    } while (0)
    LZ(random_vector(K, c->opt.seed, V.p, s));
    LZ(apply_s(V.p, Q.p));
    LZ(dots_cols(K, 1, V.p, ld, Q.p, sc.p, s));
    LZ(lanczos_normalize_start(K, V.p, Q.p, sc.p, s));
    for (int j = 0; j < ksteps; ++j) {
        double* vj = V.p + (size_t)j * ld;
        double* qj = Q.p + (size_t)j * ld;
        if (ident) {
            LZ(gemv_rows_t(K, c->precision, op.HNbuf.p, ld, vj, wv.p, s));
        } else if (op.orth) {
            LZ(csr_spmv(K, op.F_rowptr.p, op.F_col.p, op.F_val.p, vj, wv.p, s));
        } else if (op.fact) {
            // solves to at most 1e-8: the eigenvalue error this leaves (~1e-8
            // of the spectral radius) is far inside the widening margin
            int conv = 1;
            LZ(fact_apply(op.fact, vj, wv.p, std::max(c->cg_tol, 1e-8), c->cg_max_iter, &conv, s));
            if (!conv) {
                cleanup();
                return set_err(c, DM_E_NOCONV, "Lanczos: the solve with S did not converge within the iteration limit");
            }
        } else {
            LZ(gemv_rows(K, op.HT.p, ld, vj, wv.p, s));
        }
        LZ(dots_cols(K, 1, qj, ld, wv.p, alpha + j, s));
        LZ(lanczos_three_term(K, wv.p, vj, j ? vj - ld : nullptr, alpha + j, j ? beta + j - 1 : beta, s));
        for (int rep = 0; rep < 2; ++rep) {
            LZ(dots_cols(K, j + 1, Q.p, ld, wv.p, cc.p, s));
            LZ(lanczos_reorth(K, j + 1, wv.p, V.p, ld, cc.p, s));
        }
        LZ(apply_s(wv.p, sw.p));
        LZ(dots_cols(K, 1, wv.p, ld, sw.p, sc.p + 1, s));
        LZ(lanczos_next(K, wv.p, sw.p, sc.p + 1, beta + j, V.p + (size_t)(j + 1) * ld,
                        Q.p + (size_t)(j + 1) * ld, s));
    }
#undef LZ
    std::vector<double> h(2 * ksteps);
    e = hipMemcpyAsync(h.data(), ab.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    cleanup();
    if (e != hipSuccess) return fail_hip(c, e, "lanczos readback");
    std::vector<double> a(h.begin(), h.begin() + ksteps), b(h.begin() + ksteps, h.end());
    double scale = 0;
    for (double x : a) scale = std::max(scale, std::fabs(x));
    for (double x : a)
        if (!std::isfinite(x)) return set_err(c, DM_E_NOCONV, "Lanczos produced non-finite values");
    // truncate at an invariant subspace
    int k = ksteps;
    for (int j = 0; j < ksteps; ++j)
        if (!(b[j] > 1e-12 * (scale + 1e-300))) {
            k = j + 1;
            break;
        }
    a.resize(k);
    const double beta_last = b[k - 1];
    b.resize(k - 1);
    const double th_lo = tridiag_eig(a, b, 0), th_hi = tridiag_eig(a, b, k - 1);
    const double r_lo = beta_last * tridiag_last_component(a, b, th_lo);
    const double r_hi = beta_last * tridiag_last_component(a, b, th_hi);
    const double margin = c->opt.bound_margin > 0 ? c->opt.bound_margin : 0.01;
    const double width = std::max(th_hi - th_lo, 1e-12 * (std::fabs(th_hi) + 1.0));
    op.lz_emin = th_lo;
    op.lz_emax = th_hi;
    op.lz_resid_lo = r_lo;
    op.lz_resid_hi = r_hi;
    op.lz_steps_done = k;
    op.emin = th_lo - std::fabs(r_lo) - margin * width;
    op.emax = th_hi + std::fabs(r_hi) + margin * width;
    return DM_OK;
}

dm_status sym_panels(dm_ctx* c, Op& op, double ebar, double de, int precision, void* dst);

dm_status normalize(dm_ctx* c, Op& op) {
    const double ebar = 0.5 * (op.emax + op.emin), de = 0.5 * (op.emax - op.emin);
    if (op.form == DM_FORM_FACTORED) {  // H_N is applied, never formed
        op.hn_precision = c->precision;
        return DM_OK;
    }
    if (op.orth) {
        const size_t tsz = c->precision == DM_FP64 ? 8 : 4;
        HIPTRY(c, ensure(op.HNbuf, (size_t)op.Kp * op.Kp * tsz / 8));
        HIPTRY(c, csr_normalize((int)op.K, op.Kp, op.F_rowptr.p, op.F_col.p, op.F_val.p, ebar, de, c->precision,
                                op.HNbuf.p, c->stream));
        op.hn_precision = c->precision;
        return DM_OK;
    }
    if (op.form == DM_FORM_SYMMETRIC) {
        const size_t tsz = c->precision == DM_FP64 ? 8 : 4;
        const bool same_storage = (op.hn_precision == DM_FP64) == (c->precision == DM_FP64);
        if (!op.sym_raw && op.hn_precision >= 0 && same_storage && op.hn_lo == op.emin && op.hn_hi == op.emax) {
            // FP32 <-> refined FP32: the stored H~_N is the same array
        } else if (op.sym_raw && op.hn_precision_raw == c->precision) {
            // right after the panels: H~ -> H~_N in place
            HIPTRY(c, normalize_inplace((int)op.K, op.Kp, c->precision, op.HNbuf.p, ebar, de, c->stream));
        } else {
            // new bounds or precision: H~_N again from X and F (exact, no
            // second rounding of the stored H~_N)
            HIPTRY(c, ensure(op.HNbuf, (size_t)op.Kp * op.Kp * tsz / 8));
            dm_status st = sym_panels(c, op, ebar, de, c->precision, op.HNbuf.p);
            if (st != DM_OK) return st;
        }
        op.sym_raw = false;
        op.hn_precision = c->precision;
        op.hn_lo = op.emin;
        op.hn_hi = op.emax;
        return DM_OK;
    }
    HIPTRY(c, normalize_operator((int)op.K, op.Kp, op.HT.p, ebar, de, c->precision, op.HNbuf.p, c->stream));
    op.hn_precision = c->precision;
    return DM_OK;
}

// The batch keeps only H_N (its FP64 sources are released to save memory),
// so it can only run in the precision it was loaded with.
dm_status batch_precision_ok(dm_ctx* c) {
    for (const Op& o : c->batch)
        if (o.hn_precision != c->precision)
            return set_err(c, DM_E_STATE,
                           "the batch was loaded in the other precision; call dm_batch_set_focks again");
    return DM_OK;
}

dm_status reset_moments(dm_ctx* c) {
    c->mom_order = -1;
    c->ncols_done = 0;
    return DM_OK;
}

// Tile shape for a pass when nothing was tuned.  Shapes are tried in order
// of measured speed on MI355X (128 x 128 with three k-slabs in flight for
// wide passes; the LDS-shared panel shapes for 64- and 32-column passes);
// the first that fits, pads the pass by less than 32 columns and still
// gives 256 workgroups (one per CU) wins.  Narrow passes over small
// operators, which have too few row tiles, take a split-reduction shape.
int pick_cfg(int Kp, int ncols, int precision) {
    static const int kPrefF64[] = {12, 36, 33, 32, 1, 2, 3};
    static const int kPrefF32[] = {12, 31, 30, 29, 1, 2, 3};
    static const int kPrefW32[] = {12, 0, 22, 29, 30, 20, 7, 2, 3};
    static const int kSplit[] = {18, 14, 13};
    const int n = std::max(ncols, 1);
    const int n32 = (int)round_up(n, 32);
    const int* pref = precision == DM_FP64 ? kPrefF64 : precision == DM_FP32 ? kPrefF32 : kPrefW32;
    const int npref = precision == DM_FP64   ? (int)(sizeof(kPrefF64) / sizeof(int))
                      : precision == DM_FP32 ? (int)(sizeof(kPrefF32) / sizeof(int))
                                             : (int)(sizeof(kPrefW32) / sizeof(int));
    for (int i = 0; i < npref; ++i) {
        const int cfg = pref[i];
        const int Bp = (int)round_up(n, cheb_tile_cols(cfg));
        if (Bp > n32 || !cheb_cfg_fits(cfg, precision, Kp, Bp)) continue;
        if (cheb_num_tiles(Kp, Bp, cfg) >= 256) return cfg;
    }
    for (int cfg : kSplit) {
        const int Bp = (int)round_up(n, cheb_tile_cols(cfg));
        if (Bp <= n32 && cheb_cfg_fits(cfg, precision, Kp, Bp)) return cfg;
    }
    int best = 3, best_tiles = -1;
    for (int cfg : {2, 3}) {
        const int Bp = (int)round_up(n, cheb_tile_cols(cfg));
        const int t = cheb_num_tiles(Kp, Bp, cfg);
        if (Bp <= n32 && t > best_tiles) {
            best = cfg;
            best_tiles = t;
        }
    }
    return best;
}

}  // namespace

namespace {

struct HostCsr {
    std::vector<long long> rp;
    std::vector<int> col;
    std::vector<double> val;
};

// Copies a CSR pair (host or device pointers) to the host and validates it.
dm_status load_csr_pair(dm_ctx* c, long long K, const long long* F_rowptr, const int* F_col,
                        const double* F_val, const long long* S_rowptr, const int* S_col,
                        const double* S_val, HostCsr& F, HostCsr& S) {
    if (K <= 0 || K > (1LL << 30)) return set_err(c, DM_E_ARG, "K out of range");
    if (!F_rowptr || !F_col || !F_val || !S_rowptr || !S_col || !S_val)
        return set_err(c, DM_E_ARG, "null CSR array");
    HIPTRY(c, to_host(F.rp, F_rowptr, (size_t)K + 1));
    HIPTRY(c, to_host(S.rp, S_rowptr, (size_t)K + 1));
    if (F.rp[K] < 0 || S.rp[K] < 0 || F.rp[0] != 0 || S.rp[0] != 0)
        return set_err(c, DM_E_ARG, "malformed rowptr");
    HIPTRY(c, to_host(F.col, F_col, (size_t)F.rp[K]));
    HIPTRY(c, to_host(F.val, F_val, (size_t)F.rp[K]));
    HIPTRY(c, to_host(S.col, S_col, (size_t)S.rp[K]));
    HIPTRY(c, to_host(S.val, S_val, (size_t)S.rp[K]));
    std::string msg = check_csr("F", K, F.rp, F.col, F.val, false);
    if (msg.empty()) msg = check_csr("S", K, S.rp, S.col, S.val, true);
    if (!msg.empty()) return set_err(c, DM_E_ARG, msg);
    return DM_OK;
}

// Blocked right-looking Cholesky S = U^T U in place on the Kp x Kp
// column-major A (upper triangle; below it the entries are left stale).
// Block rows of kChol = 256: inside one, 64-wide steps factor the diagonal
// block (one workgroup, which also writes its inverse U_kk^-1 to V), solve
// the step's rows U12 = U_kk^-T A12 and update the remaining rows of the
// block row; the rows below then get one rank-256 update, which moves a
// quarter of the trailing-matrix bytes of rank-64 updates.
// V: Kp/64 blocks of 64 x 64; tmp: 64 x Kp.  Errors in flag (pivot + 1).
constexpr int kChol = 256;
hipError_t chol_upper(double* A, int Kp, double* V, double* tmp, int* flag, hipStream_t s) {
    const long ld = Kp;
    hipError_t e = hipSuccess;
    for (int K0 = 0; K0 < Kp && e == hipSuccess; K0 += kChol) {
        for (int k = K0; k < K0 + kChol && e == hipSuccess; k += kNb) {
            double* Vk = V + (size_t)(k / kNb) * kNb * kNb;
            e = potrf_diag(A + k + (long)k * ld, ld, Vk, flag, k, s);
            const int n2 = Kp - k - kNb;
            if (e != hipSuccess || n2 <= 0) continue;
            e = gemm_tn_f64(kNb, n2, kNb, 1.0, Vk, kNb, A + k + (long)(k + kNb) * ld, ld, 0.0, tmp, kNb, false, s);
            if (e == hipSuccess)
                e = hipMemcpy2DAsync(A + k + (long)(k + kNb) * ld, ld * 8, tmp, kNb * 8, kNb * 8, n2,
                                     hipMemcpyDeviceToDevice, s);
            const int r = K0 + kChol - k - kNb;  // rows of the block row still to update
            if (e == hipSuccess && r > 0)
                e = gemm_tn_f64(r, n2, kNb, -1.0, tmp, kNb, tmp, kNb, 1.0, A + (k + kNb) + (long)(k + kNb) * ld, ld,
                                true, s);
        }
        const int n3 = Kp - K0 - kChol;
        if (e == hipSuccess && n3 > 0) {
            const double* Ub = A + K0 + (long)(K0 + kChol) * ld;  // U[K0 : K0 + 256, K0 + 256 :]
            e = gemm_tn_f64(n3, n3, kChol, -1.0, Ub, ld, Ub, ld, 1.0, A + (K0 + kChol) + (long)(K0 + kChol) * ld, ld,
                            true, s);
        }
    }
    return e;
}

// Operator setup for one (F, S): S = U^T U, S^-1, H^T, Lanczos interval, H_N.
dm_status build_op(dm_ctx* c, Op& op, long long K, const HostCsr& Fh, const HostCsr& Sh, int form) {
    const std::vector<long long>& frp = Fh.rp;
    const std::vector<int>& fcol = Fh.col;
    const std::vector<double>& fval = Fh.val;
    const std::vector<long long>& srp = Sh.rp;
    const std::vector<int>& scol = Sh.col;
    const std::vector<double>& sval = Sh.val;
    hipStream_t s = c->stream;
    if (op.fact) fact_destroy(op.fact);
    op.fact = nullptr;
    op.K = K;
    op.Kp = (int)round_up(K, kRowPad);
    const int Kp = op.Kp;
    const size_t KK = (size_t)Kp * Kp;
    // ---- device copies of S (kept) and F (temporary)
    HIPTRY(c, ensure(op.S_rowptr, (size_t)K + 1));
    HIPTRY(c, ensure(op.S_col, sval.size()));
    HIPTRY(c, ensure(op.S_val, sval.size()));
    HIPTRY(c, hipMemcpyAsync(op.S_rowptr.p, srp.data(), srp.size() * 8, hipMemcpyHostToDevice, s));
    HIPTRY(c, hipMemcpyAsync(op.S_col.p, scol.data(), scol.size() * 4, hipMemcpyHostToDevice, s));
    HIPTRY(c, hipMemcpyAsync(op.S_val.p, sval.data(), sval.size() * 8, hipMemcpyHostToDevice, s));
    DevBuf<long long> Frp;
    DevBuf<int> Fci;
    DevBuf<double> Fv, Vblk, tmp;
    auto release_tmp = [&]() { Frp.release(); Fci.release(); Fv.release(); Vblk.release(); tmp.release(); };
    (void)form;
    op.form = DM_FORM_GENERAL;
    op.orth = false;
    op.F_rowptr.release();
    op.F_col.release();
    op.F_val.release();
    op.Xs.release();
    hipError_t e;
#define ST(expr)                          \
    do {                                  \
        if ((e = (expr)) != hipSuccess) { \
            release_tmp();                \
            return fail_hip(c, e, #expr); \
        }                                 \
    } while (0)
    ST(ensure(Frp, (size_t)K + 1));
    ST(ensure(Fci, fval.size()));
    ST(ensure(Fv, fval.size()));
    ST(hipMemcpyAsync(Frp.p, frp.data(), frp.size() * 8, hipMemcpyHostToDevice, s));
    ST(hipMemcpyAsync(Fci.p, fcol.data(), fcol.size() * 4, hipMemcpyHostToDevice, s));
    ST(hipMemcpyAsync(Fv.p, fval.data(), fval.size() * 8, hipMemcpyHostToDevice, s));
    // ---- dense buffers: A (S -> U -> F -> HN), X (U^-T -> H^T), Sinv
    ST(ensure(op.HNbuf, KK));
    ST(ensure(op.HT, KK));
    ST(ensure(op.Sinv, KK));
    ST(ensure(Vblk, (size_t)Kp * kNb));
    ST(ensure(tmp, (size_t)Kp * kNb));
    double* A = op.HNbuf.p;
    double* X = op.HT.p;
    const long ld = Kp;
    ST(fill_f64(A, 0.0, (long long)KK, s));
    ST(csr_to_dense((int)K, Kp, op.S_rowptr.p, op.S_col.p, op.S_val.p, 1.0, A, s));
    ST(fill_i32(c->flag.p, 0, 4, s));
    // ---- blocked Cholesky S = U^T U (upper)
    ST(chol_upper(A, Kp, Vblk.p, tmp.p, c->flag.p, s));
    int info[4] = {0, 0, 0, 0};
    ST(hipMemcpyAsync(info, c->flag.p, sizeof(info), hipMemcpyDeviceToHost, s));
    ST(hipStreamSynchronize(s));
    if (info[0] != 0) {
        release_tmp();
        return set_err(c, DM_E_NOTSPD, "overlap matrix is not positive definite (pivot " +
                                           std::to_string(info[0] - 1) + ")");
    }
    // ---- X = U^-T (lower) by block forward substitution
    ST(fill_f64(X, 0.0, (long long)KK, s));
    for (int k = 0; k < Kp; k += kNb) {
        const double* Vk = Vblk.p + (size_t)(k / kNb) * kNb * kNb;
        if (k > 0) {
            ST(gemm_tn_f64(kNb, k, k, -1.0, A + (long)k * ld, ld, X, ld, 0.0, tmp.p, kNb, false, s));
            ST(gemm_tn_f64(kNb, k, kNb, 1.0, Vk, kNb, tmp.p, kNb, 0.0, X + k, ld, false, s));
        }
        ST(copy_transpose_block(Vk, kNb, X + k + (long)k * ld, ld, s));
    }
    // ---- S^-1 = X^T X, then A := F and H^T = F S^-1
    ST(gemm_tn_f64(Kp, Kp, Kp, 1.0, X, ld, X, ld, 0.0, op.Sinv.p, ld, false, s));
    ST(fill_f64(A, 0.0, (long long)KK, s));
    ST(csr_to_dense((int)K, Kp, Frp.p, Fci.p, Fv.p, 0.0, A, s));
    ST(gemm_tn_f64(Kp, Kp, Kp, 1.0, A, ld, op.Sinv.p, ld, 0.0, X, ld, false, s));
    ST(hipStreamSynchronize(s));
    release_tmp();
#undef ST
    dm_status st = lanczos_bounds(c, op);
    if (st != DM_OK) return st;
    op.form = DM_FORM_GENERAL;
    return normalize(c, op);
}

// H~_N = (X^T F X - ebar I) / de (ebar = 0, de = 1: H~ itself) into dst in
// `precision`, by column panels J of width w: P = X[:, J] transposed to a
// row-major panel (X[:, J] is zero below row max J), Y = F P by the sparse
// product over groups of four rows, Y back to column-major, then the rows
// from j0 on of X^T Y on the MFMA (X upper: row tile r sums k <= r only) and
// the panel stored with the shift and scale; the upper triangle is then the
// mirror image of the lower one.
dm_status sym_panels(dm_ctx* c, Op& op, double ebar, double de, int precision, void* dst) {
    hipStream_t s = c->stream;
    const int Kp = op.Kp;
    const long ld = Kp;
    const int w = std::min(Kp, 1024);
    DevBuf<double> pa, pb;
    hipError_t e = ensure(pa, (size_t)Kp * w);
    if (e == hipSuccess) e = ensure(pb, (size_t)Kp * w);
    const SetupLog log;
    for (int j0 = 0; j0 < Kp && e == hipSuccess; j0 += w) {
        if (log.on && j0 > 0 && j0 % (16 * w) == 0) {
            e = hipStreamSynchronize(s);
            log("panel columns %d of %d", j0, Kp);
            if (e != hipSuccess) break;
        }
        // the last panel is narrower when Kp is not a multiple of w (Kp and
        // w are multiples of 256, so wj is too)
        const int wj = std::min(w, Kp - j0);
        const int kmax = j0 + wj;
        e = transpose_rect(kmax, wj, op.Xs.p + (long)j0 * ld, ld, pa.p, wj, s);
        if (e == hipSuccess)
            e = rg4_spmm_rm((int)op.K, op.Fg_ptr.p, op.Fg_col.p, op.Fg_val.p, wj, pa.p, kmax, pb.p, s);
        if (e == hipSuccess && Kp > op.K)
            e = fill_f64(pb.p + (size_t)op.K * wj, 0.0, (long long)(Kp - op.K) * wj, s);
        if (e == hipSuccess) e = transpose_rect(wj, Kp, pb.p, wj, pa.p, Kp, s);
        // rows j0 .. Kp of the panel only (H~ is symmetric; the rows above
        // come from earlier panels' columns, mirrored below)
        if (e == hipSuccess)
            e = gemm_tn_f64(Kp - j0, wj, Kp, 1.0, op.Xs.p + (long)j0 * ld, ld, pa.p, Kp, 0.0, pb.p + j0, Kp, false,
                            s, j0);
        if (e == hipSuccess) e = store_panel((int)op.K, Kp, wj, j0, j0, pb.p, ebar, 1.0 / de, precision, dst, s);
    }
    if (e == hipSuccess) e = mirror_lower(Kp, precision, dst, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    pa.release();
    pb.release();
    if (e != hipSuccess) return fail_hip(c, e, "symmetric operator panels");
    return DM_OK;
}

// Operator setup of the symmetric form, in place: S = U^T U is factored in
// the one FP64 K x K array op.Xs, which then becomes X = U^-1 (blocked
// left-looking inversion: with the leading block already inverted,
// X12 = -X11 U12 U22^-1, the diagonal blocks' inverses coming from the
// Cholesky).  H~ = X^T F X (= L F L^T with L = U^-T, the same spectrum as
// S^-1 F) is formed by sym_panels straight into the recursion-precision
// array HNbuf, the Lanczos interval comes from H~ with the standard inner
// product, and H~ is normalised in place.  Device memory: K^2 (8 + p) bytes
// (p = 8 or 4 for the recursion precision) plus panels and the CSR arrays.
dm_status build_sym(dm_ctx* c, Op& op, long long K, const HostCsr& Fh, const HostCsr& Sh) {
    hipStream_t s = c->stream;
    const SetupLog log;
    log("symmetric form, K = %lld: start", K);
    op.release();
    op.K = K;
    op.Kp = (int)round_up(K, kRowPad);
    const int Kp = op.Kp;
    const size_t KK = (size_t)Kp * Kp;
    const long ld = Kp;
    const size_t tsz = c->precision == DM_FP64 ? 8 : 4;
    HIPTRY(c, ensure(op.S_rowptr, (size_t)K + 1));
    HIPTRY(c, ensure(op.S_col, Sh.col.size()));
    HIPTRY(c, ensure(op.S_val, Sh.val.size()));
    HIPTRY(c, ensure(op.F_rowptr, (size_t)K + 1));
    HIPTRY(c, ensure(op.F_col, Fh.col.size()));
    HIPTRY(c, ensure(op.F_val, Fh.val.size()));
    HIPTRY(c, hipMemcpyAsync(op.S_rowptr.p, Sh.rp.data(), Sh.rp.size() * 8, hipMemcpyHostToDevice, s));
    HIPTRY(c, hipMemcpyAsync(op.S_col.p, Sh.col.data(), Sh.col.size() * 4, hipMemcpyHostToDevice, s));
    HIPTRY(c, hipMemcpyAsync(op.S_val.p, Sh.val.data(), Sh.val.size() * 8, hipMemcpyHostToDevice, s));
    HIPTRY(c, hipMemcpyAsync(op.F_rowptr.p, Fh.rp.data(), Fh.rp.size() * 8, hipMemcpyHostToDevice, s));
    HIPTRY(c, hipMemcpyAsync(op.F_col.p, Fh.col.data(), Fh.col.size() * 4, hipMemcpyHostToDevice, s));
    HIPTRY(c, hipMemcpyAsync(op.F_val.p, Fh.val.data(), Fh.val.size() * 8, hipMemcpyHostToDevice, s));
    {
        // F in groups of four rows: per group the sorted union of the rows'
        // columns, four values per column (zero where a row has none)
        const long long ng = (K + 3) / 4;
        std::vector<long long> gp((size_t)ng + 1, 0);
        std::vector<int> gc;
        std::vector<double> gv;
        gc.reserve(Fh.col.size() / 3);
        gv.reserve(Fh.col.size() * 4 / 3);
        for (long long g = 0; g < ng; ++g) {
            long long pos[4], end[4];
            for (int r = 0; r < 4; ++r) {
                const long long row = 4 * g + r;
                pos[r] = row < K ? Fh.rp[row] : 0;
                end[r] = row < K ? Fh.rp[row + 1] : 0;
            }
            for (;;) {
                int next = INT32_MAX;
                for (int r = 0; r < 4; ++r)
                    if (pos[r] < end[r]) next = std::min(next, Fh.col[pos[r]]);
                if (next == INT32_MAX) break;
                gc.push_back(next);
                for (int r = 0; r < 4; ++r)
                    gv.push_back(pos[r] < end[r] && Fh.col[pos[r]] == next ? Fh.val[pos[r]++] : 0.0);
            }
            gp[g + 1] = (long long)gc.size();
        }
        HIPTRY(c, ensure(op.Fg_ptr, gp.size()));
        HIPTRY(c, ensure(op.Fg_col, std::max<size_t>(gc.size(), 1)));
        HIPTRY(c, ensure(op.Fg_val, std::max<size_t>(gv.size(), 1)));
        HIPTRY(c, hipMemcpy(op.Fg_ptr.p, gp.data(), gp.size() * 8, hipMemcpyHostToDevice));
        if (!gc.empty()) HIPTRY(c, hipMemcpy(op.Fg_col.p, gc.data(), gc.size() * 4, hipMemcpyHostToDevice));
        if (!gv.empty()) HIPTRY(c, hipMemcpy(op.Fg_val.p, gv.data(), gv.size() * 8, hipMemcpyHostToDevice));
    }
    DevBuf<double> Vblk, tmp;
    auto release_tmp = [&]() { Vblk.release(); tmp.release(); };
    hipError_t e;
#define ST(expr)                          \
    do {                                  \
        if ((e = (expr)) != hipSuccess) { \
            release_tmp();                \
            return fail_hip(c, e, #expr); \
        }                                 \
    } while (0)
    ST(ensure(op.Xs, KK));
    ST(ensure(op.HNbuf, KK * tsz / 8));
    ST(ensure(Vblk, (size_t)Kp * kNb));
    ST(ensure(tmp, (size_t)Kp * kNb));
    double* A = op.Xs.p;
    ST(fill_f64(A, 0.0, (long long)KK, s));
    ST(csr_to_dense((int)K, Kp, op.S_rowptr.p, op.S_col.p, op.S_val.p, 1.0, A, s));
    ST(fill_i32(c->flag.p, 0, 4, s));
    // ---- blocked Cholesky S = U^T U (upper), as in build_op
    log("dense S built");
    ST(chol_upper(A, Kp, Vblk.p, tmp.p, c->flag.p, s));
    int info[4] = {0, 0, 0, 0};
    ST(hipMemcpyAsync(info, c->flag.p, sizeof(info), hipMemcpyDeviceToHost, s));
    ST(hipStreamSynchronize(s));
    log("Cholesky done");
    if (info[0] != 0) {
        release_tmp();
        return set_err(c, DM_E_NOTSPD,
                       "overlap matrix is not positive definite (pivot " + std::to_string(info[0] - 1) + ")");
    }
    // ---- X = U^-1 in place (the trailing updates left S below the diagonal),
    // by block columns of 256: the diagonal block D is inverted in place by
    // 64-wide steps (D12 := -D11^-1 D12 D22^-1 with the Cholesky's inverses
    // of the 64 x 64 blocks), then the block column above it becomes
    // X12 = -X11 U12 D^-1, two MFMA products 256 columns wide
    ST(zero_strict_lower(Kp, A, s));
    tmp.release();
    ST(ensure(tmp, (size_t)Kp * kChol));
    for (int K0 = 0; K0 < Kp; K0 += kChol) {
        double* D = A + K0 + (long)K0 * ld;
        for (int k = 0; k < kChol; k += kNb) {
            const double* Vk = Vblk.p + (size_t)((K0 + k) / kNb) * kNb * kNb;
            if (k > 0) {
                ST(gemm_nn_f64(k, kNb, k, 1.0, D, ld, D + (long)k * ld, ld, 0.0, tmp.p, Kp, true, s));
                ST(gemm_nn_f64(k, kNb, kNb, -1.0, tmp.p, Kp, Vk, kNb, 0.0, D + (long)k * ld, ld, false, s));
            }
            ST(set_upper_block(kNb, D + k + (long)k * ld, ld, Vk, s));
        }
        if (K0 > 0) {
            ST(gemm_nn_f64(K0, kChol, K0, 1.0, A, ld, A + (long)K0 * ld, ld, 0.0, tmp.p, Kp, true, s));
            ST(gemm_nn_f64(K0, kChol, kChol, -1.0, tmp.p, Kp, D, ld, 0.0, A + (long)K0 * ld, ld, false, s));
        }
    }
    ST(hipStreamSynchronize(s));
    release_tmp();
#undef ST
    log("X = U^-1 done");
    op.form = DM_FORM_SYMMETRIC;
    dm_status st = sym_panels(c, op, 0.0, 1.0, c->precision, op.HNbuf.p);
    if (st != DM_OK) return st;
    log("H~ = X^T F X done");
    op.sym_raw = true;
    op.hn_precision_raw = c->precision;
    st = lanczos_bounds(c, op);
    if (st != DM_OK) return st;
    log("Lanczos interval [%.4f, %.4f]", op.emin, op.emax);
    st = normalize(c, op);
    log("normalised");
    return st;
}

// Operator setup in an orthonormal basis (S = I): F in CSR on the device,
// the identity as S, the Lanczos interval of F, and H_N built from the CSR.
dm_status build_orth(dm_ctx* c, Op& op, long long K, const HostCsr& Fh) {
    hipStream_t s = c->stream;
    op.release();
    op.K = K;
    op.Kp = (int)round_up(K, kRowPad);
    std::vector<long long> irp((size_t)K + 1);
    std::vector<int> icol((size_t)K);
    std::vector<double> ival((size_t)K, 1.0);
    for (long long i = 0; i <= K; ++i) irp[i] = i;
    for (long long i = 0; i < K; ++i) icol[i] = (int)i;
    HIPTRY(c, ensure(op.S_rowptr, (size_t)K + 1));
    HIPTRY(c, ensure(op.S_col, (size_t)K));
    HIPTRY(c, ensure(op.S_val, (size_t)K));
    HIPTRY(c, ensure(op.F_rowptr, (size_t)K + 1));
    HIPTRY(c, ensure(op.F_col, Fh.col.size()));
    HIPTRY(c, ensure(op.F_val, Fh.val.size()));
    HIPTRY(c, hipMemcpyAsync(op.S_rowptr.p, irp.data(), irp.size() * 8, hipMemcpyHostToDevice, s));
    HIPTRY(c, hipMemcpyAsync(op.S_col.p, icol.data(), icol.size() * 4, hipMemcpyHostToDevice, s));
    HIPTRY(c, hipMemcpyAsync(op.S_val.p, ival.data(), ival.size() * 8, hipMemcpyHostToDevice, s));
    HIPTRY(c, hipMemcpyAsync(op.F_rowptr.p, Fh.rp.data(), Fh.rp.size() * 8, hipMemcpyHostToDevice, s));
    HIPTRY(c, hipMemcpyAsync(op.F_col.p, Fh.col.data(), Fh.col.size() * 4, hipMemcpyHostToDevice, s));
    HIPTRY(c, hipMemcpyAsync(op.F_val.p, Fh.val.data(), Fh.val.size() * 8, hipMemcpyHostToDevice, s));
    HIPTRY(c, hipStreamSynchronize(s));
    op.orth = true;
    dm_status st = lanczos_bounds(c, op);
    if (st != DM_OK) return st;
    return normalize(c, op);
}

// Operator setup in the factored form: S in CSR on the device (Lanczos
// products, start vectors), F, S and the FSAI factor G in row groups, the
// Lanczos interval of S^-1 F through solves with S.
dm_status build_fact(dm_ctx* c, Op& op, long long K, const HostCsr& Fh, const HostCsr& Sh) {
    hipStream_t s = c->stream;
    op.release();
    op.K = K;
    op.Kp = (int)round_up(K, kRowPad);
    HIPTRY(c, ensure(op.S_rowptr, (size_t)K + 1));
    HIPTRY(c, ensure(op.S_col, Sh.col.size()));
    HIPTRY(c, ensure(op.S_val, Sh.val.size()));
    HIPTRY(c, hipMemcpyAsync(op.S_rowptr.p, Sh.rp.data(), Sh.rp.size() * 8, hipMemcpyHostToDevice, s));
    HIPTRY(c, hipMemcpyAsync(op.S_col.p, Sh.col.data(), Sh.col.size() * 4, hipMemcpyHostToDevice, s));
    HIPTRY(c, hipMemcpyAsync(op.S_val.p, Sh.val.data(), Sh.val.size() * 8, hipMemcpyHostToDevice, s));
    op.fact = fact_create();
    if (!op.fact) return set_err(c, DM_E_OOM, "factored form: host allocation failed");
    int bad = 0;
    const hipError_t e = fact_setup(op.fact, (int)K, Fh.rp.data(), Fh.col.data(), Fh.val.data(), Sh.rp.data(),
                                    Sh.col.data(), Sh.val.data(), c->fsai_drop, c->fsai_cap, &bad, s);
    if (e == hipErrorInvalidValue)
        return set_err(c, DM_E_ARG, "factored form: more than 2^31 - 1 stored entries");
    if (e != hipSuccess) return fail_hip(c, e, "factored setup");
    if (bad)
        return set_err(c, DM_E_NOTSPD, "overlap matrix is not positive definite (FSAI block of row " +
                                           std::to_string(bad - 1) + ")");
    op.form = DM_FORM_FACTORED;
    dm_status st = lanczos_bounds(c, op);
    if (st != DM_OK) return st;
    HIPTRY(c, fact_reset_stats(op.fact, s));  // count the solves of the passes only
    return normalize(c, op);
}

}  // namespace

// =================================================================== C ABI
extern "C" {

void dm_default_options(dm_options* opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->device = 0;
    opt->stream = nullptr;
    opt->precision = DM_FP64;
    opt->block_width = 0;
    opt->spin = 2.0;
    opt->lanczos_steps = 100;
    opt->bound_margin = 0.01;
    opt->seed = 12345;
}

dm_status dm_init(dm_ctx** out, const dm_options* opt) try {
    if (!out) {
        g_init_error = "dm_init: out is NULL";
        return DM_E_ARG;
    }
    *out = nullptr;
    dm_options o;
    if (opt)
        o = *opt;
    else
        dm_default_options(&o);
    if ((o.precision != DM_FP64 && o.precision != DM_FP32 && o.precision != DM_FP32_ACC64) || o.block_width < 0 ||
        !(o.spin > 0) || o.lanczos_steps < 0 || o.device < 0) {
        g_init_error = "dm_init: invalid option";
        return DM_E_ARG;
    }
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || o.device >= ndev) {
        (void)hipGetLastError();
        g_init_error = std::string("dm_init: no HIP device ") + std::to_string(o.device);
        return DM_E_HIP;
    }
    e = hipSetDevice(o.device);
    if (e != hipSuccess) {
        g_init_error = std::string("dm_init: hipSetDevice: ") + hipGetErrorString(e);
        return DM_E_HIP;
    }
    dm_ctx* c = new (std::nothrow) dm_ctx();
    if (!c) {
        g_init_error = "dm_init: host allocation failed";
        return DM_E_OOM;
    }
    c->opt = o;
    c->precision = o.precision;
    if (o.stream) {
        c->stream = static_cast<hipStream_t>(o.stream);
    } else {
        e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete c;
            g_init_error = std::string("dm_init: stream: ") + hipGetErrorString(e);
            return DM_E_HIP;
        }
        c->own_stream = true;
    }
    if (ensure(c->flag, 4) != hipSuccess || ensure(c->out, 8) != hipSuccess) {
        dm_destroy(c);
        g_init_error = "dm_init: device allocation failed";
        return DM_E_OOM;
    }
    // the allocation-free entry point's device array (once per device; a
    // failed lookup only disables that entry point)
    (void)noalloc_register(o.device);
    *out = c;
    return DM_OK;
} catch (...) {
    g_init_error = "dm_init: host exception";
    return DM_E_OOM;
}

void dm_destroy(dm_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->opt.device);
    if (c->stream && !c->poisoned) (void)hipStreamSynchronize(c->stream);
    for (auto* b : {&c->op.Sinv, &c->op.HT, &c->op.HNbuf, &c->op.S_val, &c->mom, &c->Ua, &c->Ub, &c->Z, &c->P,
                    &c->part_start, &c->part_steps, &c->work, &c->Pfin, &c->coef, &c->coef_zero, &c->fk,
                    &c->w, &c->v, &c->out, &c->cs_coef, &c->cs_fk, &c->cs_out, &c->cs_stage})
        b->release();
    c->op.release();
    for (auto& o : c->batch) o.release();
    delete c->bstate;
    delete c->mlp;
    c->grid.release();
    c->flag.release();
    c->cols.release();
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char* dm_last_error(const dm_ctx* c) {
    if (!c) return g_init_error.c_str();
    return c->err.c_str();
}

dm_status dm_set_fock(dm_ctx* c, long long K, const long long* F_rowptr, const int* F_col,
                      const double* F_val, const long long* S_rowptr, const int* S_col,
                      const double* S_val, int atom_block) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (K <= 0 || K > (1LL << 30)) return set_err(c, DM_E_ARG, "K out of range");
    if (!F_rowptr || !F_col || !F_val || !S_rowptr || !S_col || !S_val)
        return set_err(c, DM_E_ARG, "null CSR array");
    if (atom_block < 1 || K % atom_block) return set_err(c, DM_E_ARG, "K not a multiple of atom_block");
    c->have_fock = false;
    c->tuned_width = 0;
    c->tuned_cfg = -1;
    reset_moments(c);
    HostCsr Fh, Sh;
    st = load_csr_pair(c, K, F_rowptr, F_col, F_val, S_rowptr, S_col, S_val, Fh, Sh);
    if (st != DM_OK) return st;
    st = c->form == DM_FORM_FACTORED    ? build_fact(c, c->op, K, Fh, Sh)
         : c->form == DM_FORM_SYMMETRIC ? build_sym(c, c->op, K, Fh, Sh)
                                        : build_op(c, c->op, K, Fh, Sh, c->form);
    if (st != DM_OK) return st;
    c->have_fock = true;
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

dm_status dm_set_fock_orthonormal(dm_ctx* c, long long K, const long long* F_rowptr, const int* F_col,
                                  const double* F_val) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (K <= 0 || K > (1LL << 30)) return set_err(c, DM_E_ARG, "K out of range");
    if (!F_rowptr || !F_col || !F_val) return set_err(c, DM_E_ARG, "null CSR array");
    c->have_fock = false;
    c->tuned_width = 0;
    c->tuned_cfg = -1;
    reset_moments(c);
    HostCsr Fh;
    HIPTRY(c, to_host(Fh.rp, F_rowptr, (size_t)K + 1));
    if (Fh.rp[0] != 0 || Fh.rp[K] < 0) return set_err(c, DM_E_ARG, "malformed rowptr");
    HIPTRY(c, to_host(Fh.col, F_col, (size_t)Fh.rp[K]));
    HIPTRY(c, to_host(Fh.val, F_val, (size_t)Fh.rp[K]));
    const std::string msg = check_csr("F", K, Fh.rp, Fh.col, Fh.val, false);
    if (!msg.empty()) return set_err(c, DM_E_ARG, msg);
    st = build_orth(c, c->op, K, Fh);
    if (st != DM_OK) return st;
    c->have_fock = true;
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

dm_status dm_get_bounds(dm_ctx* c, double* emin, double* emax) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (!c->have_fock) return set_err(c, DM_E_STATE, "no Fock matrix loaded");
    if (emin) *emin = c->op.emin;
    if (emax) *emax = c->op.emax;
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

dm_status dm_set_bounds(dm_ctx* c, double emin, double emax) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (!c->have_fock) return set_err(c, DM_E_STATE, "no Fock matrix loaded");
    if (!std::isfinite(emin) || !std::isfinite(emax) || !(emin < emax))
        return set_err(c, DM_E_ARG, "need finite emin < emax");
    c->op.emin = emin;
    c->op.emax = emax;
    reset_moments(c);
    return normalize(c, c->op);
} catch (...) {
    return host_exception(c);
}

dm_status dm_set_operator_form(dm_ctx* c, int form) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (form != DM_FORM_GENERAL && form != DM_FORM_SYMMETRIC && form != DM_FORM_FACTORED)
        return set_err(c, DM_E_ARG, "unknown operator form");
    c->form = form;
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

dm_status dm_set_factored_options(dm_ctx* c, double cg_tol, int cg_max_iter, double fsai_drop,
                                  int fsai_max_per_row) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (!(cg_tol > 0.0 && cg_tol < 1.0) || cg_max_iter < 1 || !(fsai_drop >= 0.0) || !std::isfinite(fsai_drop) ||
        fsai_max_per_row < 1 || fsai_max_per_row > 192)
        return set_err(c, DM_E_ARG, "need 0 < cg_tol < 1, cg_max_iter >= 1, fsai_drop >= 0, 1 <= max_per_row <= 192");
    c->cg_tol = cg_tol;
    c->cg_max_iter = cg_max_iter;
    c->fsai_drop = fsai_drop;
    c->fsai_cap = fsai_max_per_row;
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

dm_status dm_solve_overlap(dm_ctx* c, const double* B, long long nrhs, double* X) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (!c->have_fock || !c->op.fact) return set_err(c, DM_E_STATE, "no factored operator loaded");
    if (nrhs < 0 || nrhs > c->op.K * 64 || (nrhs > 0 && (!B || !X))) return set_err(c, DM_E_ARG, "bad right-hand sides");
    if (nrhs == 0) return DM_OK;
    int conv = 1;
    const hipError_t e = fact_solve(c->op.fact, (int)nrhs, B, c->op.K, X, c->op.K, c->cg_tol, c->cg_max_iter,
                                    1024, &conv, c->stream);
    if (e == hipErrorOutOfMemory) return set_err(c, DM_E_OOM, "solve: device allocation failed");
    if (e != hipSuccess) return fail_hip(c, e, "solve with S");
    if (!conv) return set_err(c, DM_E_NOCONV, "the conjugate-gradient solve with S did not converge within the iteration limit");
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

dm_status dm_get_preconditioner(dm_ctx* c, long long* nnz, long long* rowptr, int* col, double* val) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (!c->have_fock || !c->op.fact) return set_err(c, DM_E_STATE, "no factored operator loaded");
    if (nnz) *nnz = fact_precond_nnz(c->op.fact);
    HIPTRY(c, fact_precond_copy(c->op.fact, rowptr, col, val, c->stream));
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

dm_status dm_cg_stats(dm_ctx* c, long long* solves, long long* iterations, int* max_iterations) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (!c->have_fock || !c->op.fact) return set_err(c, DM_E_STATE, "no factored operator loaded");
    long long ns = 0, it = 0;
    int mx = 0;
    HIPTRY(c, fact_stats(c->op.fact, &ns, &it, &mx, c->stream));
    HIPTRY(c, fact_reset_stats(c->op.fact, c->stream));
    if (solves) *solves = ns;
    if (iterations) *iterations = it;
    if (max_iterations) *max_iterations = mx;
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

dm_status dm_cg_timing(dm_ctx* c, int enable, long long* launches, double* ms) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (!c->have_fock || !c->op.fact) return set_err(c, DM_E_STATE, "no factored operator loaded");
    long long n = 0;
    double t = 0.0;
    fact_take_timing(c->op.fact, &n, &t);
    fact_set_timing(c->op.fact, enable != 0);
    if (launches) *launches = n;
    if (ms) *ms = t;
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

dm_status dm_get_operator(dm_ctx* c, int which, double* out) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (!c->have_fock) return set_err(c, DM_E_STATE, "no Fock matrix loaded");
    if (!out || (which != DM_OP_SINV && which != DM_OP_H && which != DM_OP_HSYM))
        return set_err(c, DM_E_ARG, "bad operator request");
    if (which == DM_OP_HSYM && c->op.form != DM_FORM_SYMMETRIC)
        return set_err(c, DM_E_STATE, "the loaded operator was not built in the symmetric form");
    if (c->op.orth) return set_err(c, DM_E_STATE, "an orthonormal-basis operator keeps no dense setup products");
    if (c->op.fact) return set_err(c, DM_E_STATE, "a factored operator keeps no dense setup products");
    const size_t K = (size_t)c->op.K, Kp = (size_t)c->op.Kp;
    hipStream_t s = c->stream;
    if (c->op.form == DM_FORM_SYMMETRIC) {
        // formed on request from X = U^-1 and F: S^-1 = X X^T, H = X X^T F,
        // H~ = X^T F X (two K x K FP64 work arrays)
        const Op& op = c->op;
        const int kp = op.Kp;
        DevBuf<double> W, T;
        hipError_t e = ensure(W, Kp * Kp);
        if (e == hipSuccess) e = ensure(T, Kp * Kp);
        if (e == hipSuccess && which == DM_OP_SINV) {
            e = transpose_square(kp, op.Xs.p, W.p, s);
            if (e == hipSuccess) e = gemm_tn_f64(kp, kp, kp, 1.0, W.p, kp, W.p, kp, 0.0, T.p, kp, false, s);
        } else if (e == hipSuccess) {
            e = fill_f64(W.p, 0.0, (long long)(Kp * Kp), s);
            if (e == hipSuccess) e = csr_to_dense((int)K, kp, op.F_rowptr.p, op.F_col.p, op.F_val.p, 0.0, W.p, s);
            if (e == hipSuccess && which == DM_OP_H) {
                e = gemm_tn_f64(kp, kp, kp, 1.0, op.Xs.p, kp, W.p, kp, 0.0, T.p, kp, false, s, 0);
                if (e == hipSuccess) e = gemm_nn_f64(kp, kp, kp, 1.0, op.Xs.p, kp, T.p, kp, 0.0, W.p, kp, true, s);
                std::swap(W, T);
            } else if (e == hipSuccess) {
                e = gemm_nn_f64(kp, kp, kp, 1.0, W.p, kp, op.Xs.p, kp, 0.0, T.p, kp, false, s);
                if (e == hipSuccess) e = gemm_tn_f64(kp, kp, kp, 1.0, op.Xs.p, kp, T.p, kp, 0.0, W.p, kp, false, s, 0);
                std::swap(W, T);
            }
        }
        if (e == hipSuccess) e = hipMemcpy2DAsync(out, K * 8, T.p, Kp * 8, K * 8, K, hipMemcpyDefault, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        W.release();
        T.release();
        if (e != hipSuccess) return fail_hip(c, e, "symmetric-form operator on request");
        return DM_OK;
    }
    if (which == DM_OP_SINV || which == DM_OP_HSYM) {
        HIPTRY(c, hipMemcpy2DAsync(out, K * 8, c->op.Sinv.p, Kp * 8, K * 8, K, hipMemcpyDefault, s));
    } else {
        // HT holds H^T column-major; transpose through a device scratch buffer
        DevBuf<double> t;
        HIPTRY(c, ensure(t, K * K));
        HIPTRY(c, hipMemcpy2DAsync(t.p, K * 8, c->op.HT.p, Kp * 8, K * 8, K, hipMemcpyDeviceToDevice, s));
        std::vector<double> h(K * K), ht(K * K);
        hipError_t e = hipMemcpyAsync(ht.data(), t.p, K * K * 8, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        t.release();
        if (e != hipSuccess) return fail_hip(c, e, "operator readback");
        for (size_t i = 0; i < K; ++i)
            for (size_t j = 0; j < K; ++j) h[i + j * K] = ht[j + i * K];
        HIPTRY(c, hipMemcpy(out, h.data(), K * K * 8, hipMemcpyDefault));
    }
    HIPTRY(c, hipStreamSynchronize(s));
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

dm_status dm_set_precision(dm_ctx* c, int precision) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (precision != DM_FP64 && precision != DM_FP32 && precision != DM_FP32_ACC64)
        return set_err(c, DM_E_ARG, "bad precision");
    c->precision = precision;
    c->tuned_width = 0;  // shapes were timed (or fit) for the other precision
    c->tuned_cfg = -1;
    reset_moments(c);
    if (!c->have_fock) return DM_OK;
    return normalize(c, c->op);
} catch (...) {
    return host_exception(c);
}

// Start block of the symmetric form for the ncols columns `cols` (device)
// of a pass of width Bp (B64 = Bp rounded up to 64): the moment vectors
// Z[:, j] = U u_a = X^T s_a (S's column a, scattered into vbuf, then one
// MFMA product; X upper), V_0[:, j] = L u_a = X[a, :]^T into vbuf, then
// U_0 = V_0 in the recursion precision, P_q = a_0(q) V_0 and the moment
// partial sums of l = 0 as cheb_start does for the general form.  vbuf and
// Z are Kp x B64 FP64.
static hipError_t sym_start(const Op& op, int Bp, int B64, int ncols, const long long* cols, int precision,
                            void* U0, double* Z, double* P, double* vbuf, const double* coef, int nsets,
                            long long pstride, int cstride, double* partial, int* nts, hipStream_t s) {
    const int Kp = op.Kp;
    hipError_t e = fill_f64(vbuf, 0.0, (long long)Kp * B64, s);
    if (e == hipSuccess) e = scatter_s_columns(Kp, ncols, cols, op.S_rowptr.p, op.S_col.p, op.S_val.p, vbuf, s);
    if (e == hipSuccess) e = gemm_tn_f64(Kp, B64, Kp, 1.0, op.Xs.p, Kp, vbuf, Kp, 0.0, Z, Kp, false, s, 0);
    if (e == hipSuccess) e = gather_rows(Kp, ncols, cols, op.Xs.p, vbuf, s);
    if (e == hipSuccess)
        e = cheb_start((int)op.K, Kp, Bp, ncols, nullptr, vbuf, op.S_rowptr.p, op.S_col.p, op.S_val.p, precision, U0,
                       Z, P, coef, nsets, pstride, cstride, partial, nts, s, Z);
    return e;
}

// End of a pass: the moments accumulated so far must be finite and bounded.
static dm_status finish_pass(dm_ctx* c, int order, long long ncols) {
    hipStream_t s = c->stream;
    int flag = 0;
    HIPTRY(c, hipMemcpyAsync(&flag, c->flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
    std::vector<double> hm((size_t)order + 1);
    HIPTRY(c, hipMemcpyAsync(hm.data(), c->mom.p, hm.size() * 8, hipMemcpyDeviceToHost, s));
    HIPTRY(c, hipStreamSynchronize(s));
    c->ncols_done += ncols;
    const double lim = 1e8 * (double)(c->ncols_done + 1);
    bool bad = flag != 0;
    for (double x : hm)
        if (!std::isfinite(x) || std::fabs(x) > lim) bad = true;
    if (bad)
        return set_err(c, DM_E_BOUNDS,
                       "Chebyshev recursion diverged: the spectral interval does not enclose the spectrum");
    return DM_OK;
}

// Factored form: blocks of up to `bw` columns, each a full recursion with one
// solve with S per step (FP64).
static dm_status run_fact_blocks(dm_ctx* c, const std::vector<long long>& hc, long long ncols, int order,
                                 int nsets, int cstride, double ebar, double de, double* const* P_outs) {
    hipStream_t s = c->stream;
    const long long K = c->op.K;
    const long long Kr = round_up(K, 64);
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = 0;
    const size_t budget = std::max<size_t>((size_t)16 << 30, free_b / 2);
    const size_t per_col = (size_t)Kr * 8 * (13 + nsets);
    long long bw = c->opt.block_width > 0 ? c->opt.block_width : ncols;
    bw = std::min<long long>(bw, std::max<long long>(64, (long long)(budget / per_col) / 64 * 64));
    bw = std::min(bw, ncols);
    HIPTRY(c, ensure(c->cols, (size_t)bw));
    std::vector<double*> dst((size_t)nsets);
    for (long long off = 0; off < ncols; off += bw) {
        const int nc = (int)std::min<long long>(bw, ncols - off);
        HIPTRY(c, hipMemcpyAsync(c->cols.p, hc.data() + off, (size_t)nc * 8, hipMemcpyHostToDevice, s));
        for (int q = 0; q < nsets; ++q) dst[q] = (P_outs && P_outs[q]) ? P_outs[q] + off * K : nullptr;
        FactBlockArgs fa{};
        fa.nc = nc;
        fa.cols = c->cols.p;
        fa.order = order;
        fa.coef = c->coef.p;
        fa.cstride = cstride;
        fa.nsets = nsets;
        fa.ebar = ebar;
        fa.de = de;
        fa.tol = c->cg_tol;
        fa.max_iter = c->cg_max_iter;
        fa.mom = c->mom.p;
        fa.flag = c->flag.p;
        fa.P_out = dst.data();
        int conv = 1;
        const hipError_t e = fact_block(c->op.fact, fa, &conv, s);
        if (e == hipErrorOutOfMemory) return set_err(c, DM_E_OOM, "factored pass: device allocation failed");
        if (e != hipSuccess) return fail_hip(c, e, "factored pass");
        if (!conv)
            return set_err(c, DM_E_NOCONV,
                           "the conjugate-gradient solve with S did not converge within the iteration limit");
    }
    return DM_OK;
}

// One recursion pass over `cols` accumulating nsets density-matrix blocks,
// set q with the coefficients of (mus[q], betas[q]); the moments are shared.
static dm_status run_pass(dm_ctx* c, const long long* cols, long long ncols, int order, int nsets,
                          const double* mus, const double* betas, double* const* P_outs) {
    if (!c->have_fock) return set_err(c, DM_E_STATE, "no Fock matrix loaded");
    if (c->op.fact && c->precision != DM_FP64)
        return set_err(c, DM_E_STATE, "the factored form runs in FP64 only");
    if (order < 2 || order > (1 << 20)) return set_err(c, DM_E_ARG, "order must be >= 2");
    if (nsets < 1 || nsets > DM_MAX_SETS) return set_err(c, DM_E_ARG, "need 1 <= n_sets <= DM_MAX_SETS");
    for (int q = 0; q < nsets; ++q)
        if (!std::isfinite(mus[q]) || !std::isfinite(betas[q]) || !(betas[q] > 0))
            return set_err(c, DM_E_ARG, "need finite mu and beta > 0");
    if (ncols < 0 || ncols > c->op.K) return set_err(c, DM_E_ARG, "ncols out of range");
    if (ncols > 0 && !cols) return set_err(c, DM_E_ARG, "cols is NULL");
    const long long K = c->op.K;
    std::vector<long long> hc;
    HIPTRY(c, to_host(hc, cols, (size_t)ncols));
    {
        std::vector<char> seen((size_t)K, 0);
        for (long long x : hc) {
            if (x < 0 || x >= K) return set_err(c, DM_E_ARG, "column index out of range");
            if (seen[x]) return set_err(c, DM_E_ARG, "repeated column index");
            seen[x] = 1;
        }
    }
    hipStream_t s = c->stream;
    const int Kp = c->op.Kp;
    if (order != c->mom_order) {
        HIPTRY(c, ensure(c->mom, (size_t)order + 1));
        HIPTRY(c, fill_f64(c->mom.p, 0.0, order + 1, s));
        c->mom_order = order;
        c->ncols_done = 0;
    }
    if (ncols == 0) return DM_OK;
    const double ebar = 0.5 * (c->op.emax + c->op.emin), de = 0.5 * (c->op.emax - c->op.emin);
    const int M = 4 * order;
    const int cstride = order + 1;
    HIPTRY(c, ensure(c->coef, (size_t)cstride * nsets));
    HIPTRY(c, ensure(c->fk, (size_t)M));
    for (int q = 0; q < nsets; ++q)
        HIPTRY(c, cheb_coefficients(order, M, ebar, de, mus[q], betas[q], c->fk.p, c->coef.p + (size_t)q * cstride, s));
    HIPTRY(c, fill_i32(c->flag.p, 0, 4, s));
    if (c->op.fact) {
        const dm_status fs = run_fact_blocks(c, hc, ncols, order, nsets, cstride, ebar, de, P_outs);
        if (fs != DM_OK) {
            c->mom_order = -1;  // partial moments of a failed pass
            return fs;
        }
        return finish_pass(c, order, ncols);
    }

    // pass width
    const size_t tsz = c->precision == DM_FP64 ? 8 : 4;
    const bool tuned = c->opt.block_width == 0 && c->tuned_width > 0;
    long long bw = c->opt.block_width > 0 ? c->opt.block_width : (tuned ? c->tuned_width : ncols);
    // pass buffers may take half of the free HBM (at least 16 GiB)
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = 0;
    const size_t budget = std::max<size_t>((size_t)16 << 30, free_b / 2);
    const size_t per_col = (size_t)Kp * (2 * tsz + 8 + 8 * nsets);
    bw = std::min<long long>(bw, std::max<long long>(128, (long long)(budget / per_col) / 128 * 128));
    bw = std::min(bw, ncols);
    int cfg = pick_cfg(Kp, (int)bw, c->precision);
    if (tuned && cheb_cfg_fits(c->tuned_cfg, c->precision, Kp, (int)round_up(bw, cheb_tile_cols(c->tuned_cfg))))
        cfg = c->tuned_cfg;
    const int BN = cheb_tile_cols(cfg);
    const int Bp_max = (int)round_up(bw, std::max(BN, 16));
    const size_t wbytes = cheb_work_bytes(Kp, Bp_max, cfg, c->precision);
    if (wbytes) HIPTRY(c, ensure(c->work, (wbytes + 7) / 8));
    HIPTRY(c, ensure(c->Ua, (size_t)Kp * Bp_max * tsz / 8));
    HIPTRY(c, ensure(c->Ub, (size_t)Kp * Bp_max * tsz / 8));
    // symmetric form: the accumulated blocks are Q = p_N(H~) L u_a, and P = L^T Q
    // (L^T = X) is one FP64 product per pass, over columns padded to 64
    const bool sym = c->op.form == DM_FORM_SYMMETRIC;
    const int Bpad = sym ? (int)round_up(Bp_max, 64) : Bp_max;
    HIPTRY(c, ensure(c->Z, (size_t)Kp * Bpad));
    const long long pstride = (long long)Kp * Bpad;
    HIPTRY(c, ensure(c->P, (size_t)pstride * nsets));
    if (sym) HIPTRY(c, ensure(c->Pfin, (size_t)pstride));
    HIPTRY(c, ensure(c->cols, (size_t)Bp_max));
    const int nts_step = cheb_num_tiles(Kp, Bp_max, cfg);
    HIPTRY(c, ensure(c->part_steps, (size_t)(order + 1) * nts_step));
    HIPTRY(c, ensure(c->part_start, (size_t)(Kp / 64) * (Bp_max / 16)));

    for (long long off = 0; off < ncols; off += bw) {
        const int nc = (int)std::min<long long>(bw, ncols - off);
        const int Bp = (int)round_up(nc, std::max(BN, 16));
        HIPTRY(c, hipMemcpyAsync(c->cols.p, hc.data() + off, (size_t)nc * 8, hipMemcpyHostToDevice, s));
        int nts = 0;
        if (sym) {
            HIPTRY(c, sym_start(c->op, Bp, (int)round_up(Bp, 64), nc, c->cols.p, c->precision, c->Ua.p, c->Z.p,
                                c->P.p, c->Pfin.p, c->coef.p, nsets, pstride, cstride, c->part_start.p, &nts, s));
        } else {
            HIPTRY(c, fill_f64(c->Z.p, 0.0, (long long)Kp * Bp, s));
            const double* v0src = c->op.orth ? nullptr : c->op.Sinv.p;
            HIPTRY(c, cheb_start((int)K, Kp, Bp, nc, c->cols.p, v0src, c->op.S_rowptr.p, c->op.S_col.p,
                                 c->op.S_val.p, c->precision, c->Ua.p, c->Z.p, c->P.p, c->coef.p, nsets, pstride,
                                 cstride, c->part_start.p, &nts, s));
        }
        HIPTRY(c, reduce_moments(0, nts, c->part_start.p, c->mom.p, c->flag.p, s));
        void* ucur = c->Ua.p;
        void* uoth = c->Ub.p;
        ChebStepArgs a{};
        a.Kp = Kp;
        a.Bp = Bp;
        a.HN = c->op.HNbuf.p;
        a.coef = c->coef.p;
        a.P = c->P.p;
        a.Z = c->Z.p;
        a.partial = c->part_steps.p;
        a.work = c->work.p;
        a.nsets = nsets;
        a.cstride = cstride;
        a.pstride = pstride;
        const int ntl = cheb_num_tiles(Kp, Bp, cfg);
        for (int l = 1; l <= order; ++l) {
            a.Ucur = ucur;
            a.Uprev = (l == 1) ? nullptr : uoth;
            a.Unext = uoth;
            a.alpha = (l == 1) ? 1.0 : 2.0;
            a.has_prev = (l > 1);
            a.l = l;
            hipError_t e = cheb_step(a, cfg, c->precision, s);
            if (e != hipSuccess) return fail_hip(c, e, "cheb_step");
            std::swap(ucur, uoth);
        }
        HIPTRY(c, reduce_moments(order - 1, ntl, c->part_steps.p + ntl, c->mom.p + 1, c->flag.p, s));
        for (int q = 0; q < nsets; ++q) {
            if (!P_outs || !P_outs[q]) continue;
            const double* src = c->P.p + (size_t)q * pstride;
            if (sym) {
                const int B64 = (int)round_up(Bp, 64);
                double* Q = c->P.p + (size_t)q * pstride;
                if (B64 > Bp) HIPTRY(c, fill_f64(Q + (size_t)Kp * Bp, 0.0, (long long)Kp * (B64 - Bp), s));
                HIPTRY(c, gemm_nn_f64(Kp, B64, Kp, 1.0, c->op.Xs.p, Kp, Q, Kp, 0.0, c->Pfin.p, Kp, true, s));
                src = c->Pfin.p;
            }
            HIPTRY(c, hipMemcpy2DAsync(P_outs[q] + off * K, (size_t)K * 8, src, (size_t)Kp * 8, (size_t)K * 8, nc,
                                       hipMemcpyDefault, s));
        }
    }
    return finish_pass(c, order, ncols);
}

dm_status dm_chebyshev_block(dm_ctx* c, const long long* cols, long long ncols, int order,
                             double mu, double beta, double* P_out) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    return run_pass(c, cols, ncols, order, 1, &mu, &beta, &P_out);
} catch (...) {
    return host_exception(c);
}

dm_status dm_chebyshev_block_multi(dm_ctx* c, const long long* cols, long long ncols, int order,
                                   int n_sets, const double* mu, const double* beta, double* const* P_out) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (!mu || !beta) return set_err(c, DM_E_ARG, "mu or beta is NULL");
    if (n_sets < 1 || n_sets > DM_MAX_SETS) return set_err(c, DM_E_ARG, "need 1 <= n_sets <= DM_MAX_SETS");
    std::vector<double> hmu(n_sets), hbeta(n_sets);
    std::copy(mu, mu + n_sets, hmu.begin());
    std::copy(beta, beta + n_sets, hbeta.begin());
    return run_pass(c, cols, ncols, order, n_sets, hmu.data(), hbeta.data(), P_out);
} catch (...) {
    return host_exception(c);
}

dm_status dm_chebyshev_block_noalloc(dm_ctx* c, const long long* cols, long long ncols, int order, double mu,
                                     double beta, double* P_out, double* m_out) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (!c->have_fock) return set_err(c, DM_E_STATE, "no Fock matrix loaded");
    const Op& op = c->op;
    if (op.fact || op.form != DM_FORM_GENERAL)
        return set_err(c, DM_E_STATE, "the allocation-free pass runs on the general (or orthonormal) operator only");
    if (order < 2 || order > (1 << 20)) return set_err(c, DM_E_ARG, "order must be >= 2");
    if (!std::isfinite(mu) || !std::isfinite(beta) || !(beta > 0)) return set_err(c, DM_E_ARG, "need finite mu and beta > 0");
    if (ncols < 0 || ncols > op.K || (ncols > 0 && !cols)) return set_err(c, DM_E_ARG, "bad columns");
    char* base = static_cast<char*>(noalloc_scratch(c->opt.device));
    if (!base) return set_err(c, DM_E_STATE, "the allocation-free scratch array is not available on this device");
    hipStream_t s = c->stream;
    const long long K = op.K;
    const int Kp = op.Kp;
    const int prec = c->precision;
    const size_t tsz = prec == DM_FP64 ? 8 : 4;
    // the tile shape dm_chebyshev_block takes for one pass of ncols columns
    const long long nc = std::max<long long>(ncols, 1);
    int cfg = pick_cfg(Kp, (int)nc, prec);
    if (c->opt.block_width == 0 && c->tuned_width > 0 &&
        cheb_cfg_fits(c->tuned_cfg, prec, Kp, (int)round_up(nc, cheb_tile_cols(c->tuned_cfg))))
        cfg = c->tuned_cfg;
    const int BN = cheb_tile_cols(cfg);
    const int Bp = (int)round_up(nc, std::max(BN, 16));
    const size_t KB = (size_t)Kp * Bp;
    const int ntl = cheb_num_tiles(Kp, Bp, cfg);
    // regions of the scratch array, each 256-byte aligned
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    const size_t o_ua = take(KB * tsz), o_ub = take(KB * tsz), o_z = take(KB * 8), o_p = take(KB * 8);
    const size_t o_work = take(cheb_work_bytes(Kp, Bp, cfg, prec));
    const size_t o_steps = take((size_t)(order + 1) * ntl * 8);
    const size_t o_start = take((size_t)(Kp / 64) * (Bp / 16) * 8);
    const size_t o_coef = take((size_t)(order + 1) * 8), o_fk = take((size_t)4 * order * 8);
    const size_t o_mom = take((size_t)(order + 1) * 8), o_cols = take((size_t)Bp * 8);
    const size_t o_seen = take((size_t)K * 4), o_flag = take(16);
    if (off > kScratchBytes)
        return set_err(c, DM_E_ARG, "the allocation-free pass needs " + std::to_string(off) + " bytes of scratch for " +
                                        std::to_string(ncols) + " columns, order " + std::to_string(order) +
                                        " and K = " + std::to_string(K) + "; the array holds " +
                                        std::to_string(kScratchBytes));
    auto D = [&](size_t o) { return reinterpret_cast<double*>(base + o); };
    int* flag = reinterpret_cast<int*>(base + o_flag);
    long long* dcols = reinterpret_cast<long long*>(base + o_cols);
    double* mom = D(o_mom);
    int hflag = 0;
    HIPTRY(c, fill_i32(flag, 0, 4, s));
    HIPTRY(c, fill_f64(mom, 0.0, order + 1, s));
    if (ncols > 0) {
        // columns: copied in (host or device), checked on the device
        HIPTRY(c, hipMemcpyAsync(dcols, cols, (size_t)ncols * 8, hipMemcpyDefault, s));
        HIPTRY(c, fill_i32(reinterpret_cast<int*>(base + o_seen), 0, K, s));
        HIPTRY(c, check_columns(dcols, ncols, K, reinterpret_cast<int*>(base + o_seen), flag, s));
        HIPTRY(c, hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPTRY(c, hipStreamSynchronize(s));
        if (hflag & 2) return set_err(c, DM_E_ARG, "column index out of range");
        if (hflag & 4) return set_err(c, DM_E_ARG, "repeated column index");
        const double ebar = 0.5 * (op.emax + op.emin), de = 0.5 * (op.emax - op.emin);
        const int M = 4 * order;
        const long long pstride = (long long)KB;
        HIPTRY(c, cheb_coefficients(order, M, ebar, de, mu, beta, D(o_fk), D(o_coef), s));
        HIPTRY(c, fill_f64(D(o_z), 0.0, (long long)KB, s));
        int nts = 0;
        HIPTRY(c, cheb_start((int)K, Kp, Bp, (int)ncols, dcols, op.orth ? nullptr : op.Sinv.p, op.S_rowptr.p,
                             op.S_col.p, op.S_val.p, prec, base + o_ua, D(o_z), D(o_p), D(o_coef), 1, pstride,
                             order + 1, D(o_start), &nts, s));
        HIPTRY(c, reduce_moments(0, nts, D(o_start), mom, flag, s));
        void* ucur = base + o_ua;
        void* uoth = base + o_ub;
        ChebStepArgs a{};
        a.Kp = Kp;
        a.Bp = Bp;
        a.HN = op.HNbuf.p;
        a.coef = D(o_coef);
        a.P = D(o_p);
        a.Z = D(o_z);
        a.partial = D(o_steps);
        a.work = D(o_work);
        a.nsets = 1;
        a.cstride = order + 1;
        a.pstride = pstride;
        for (int l = 1; l <= order; ++l) {
            a.Ucur = ucur;
            a.Uprev = (l == 1) ? nullptr : uoth;
            a.Unext = uoth;
            a.alpha = (l == 1) ? 1.0 : 2.0;
            a.has_prev = (l > 1);
            a.l = l;
            const hipError_t e = cheb_step(a, cfg, prec, s);
            if (e != hipSuccess) return fail_hip(c, e, "cheb_step");
            std::swap(ucur, uoth);
        }
        HIPTRY(c, reduce_moments(order - 1, ntl, D(o_steps) + ntl, mom + 1, flag, s));
        HIPTRY(c, flag_large(mom, order + 1, 1e8 * (double)(ncols + 1), flag, s));
        if (P_out)
            HIPTRY(c, hipMemcpy2DAsync(P_out, (size_t)K * 8, D(o_p), (size_t)Kp * 8, (size_t)K * 8, (size_t)ncols,
                                       hipMemcpyDefault, s));
    }
    if (m_out) HIPTRY(c, hipMemcpyAsync(m_out, mom, (size_t)(order + 1) * 8, hipMemcpyDefault, s));
    HIPTRY(c, hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPTRY(c, hipStreamSynchronize(s));
    if (hflag & 1)
        return set_err(c, DM_E_BOUNDS, "Chebyshev recursion diverged: the spectral interval does not enclose the spectrum");
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

dm_status dm_combine_sets(dm_ctx* c, int n_sets, const double* mus, double beta, int order, double mu, long long n,
                          const double* const* P_in, double* P_out, double* bound) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (!c->have_fock) return set_err(c, DM_E_STATE, "no Fock matrix loaded (its interval sets the coefficients)");
    if (n_sets < 1 || n_sets > DM_MAX_SETS || !mus || order < 2 || order > (1 << 20) || !(beta > 0) ||
        !std::isfinite(beta) || !std::isfinite(mu) || n < 0 || (n > 0 && (!P_in || !P_out)))
        return set_err(c, DM_E_ARG, "bad set-combination arguments");
    for (int q = 0; q < n_sets; ++q) {
        if (!std::isfinite(mus[q])) return set_err(c, DM_E_ARG, "non-finite node");
        for (int r = 0; r < q; ++r)
            if (mus[r] == mus[q]) return set_err(c, DM_E_ARG, "repeated node");
    }
    // Lagrange weights of the nodes at mu
    CombineSets cs{};
    for (int q = 0; q < n_sets; ++q) {
        double wq = 1.0;
        for (int r = 0; r < n_sets; ++r)
            if (r != q) wq *= (mu - mus[r]) / (mus[q] - mus[r]);
        cs.w[q] = wq;
    }
    hipStream_t s = c->stream;
    const double ebar = 0.5 * (c->op.emax + c->op.emin), de = 0.5 * (c->op.emax - c->op.emin);
    const int M = 4 * order, stride = order + 1;
    DevBuf<double>& A = c->cs_coef;
    hipError_t e = ensure(A, (size_t)stride * (n_sets + 1));
    if (e == hipSuccess) e = ensure(c->cs_fk, (size_t)M);
    if (e == hipSuccess) e = ensure(c->cs_out, 1);
    for (int q = 0; q <= n_sets && e == hipSuccess; ++q)
        e = cheb_coefficients(order, M, ebar, de, q < n_sets ? mus[q] : mu, beta, c->cs_fk.p, A.p + (size_t)q * stride,
                              s);
    if (e == hipSuccess) e = interp_bound(order, n_sets, A.p, stride, cs, c->cs_out.p, s);
    double hb = 0.0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hb, c->cs_out.p, 8, hipMemcpyDeviceToHost, s);
    // blocks in host memory go through device copies
    DevBuf<double>& stage = c->cs_stage;
    if (e == hipSuccess && n > 0) {
        int nhost = 0;
        for (int q = 0; q < n_sets; ++q) nhost += !is_device_ptr(P_in[q]);
        const bool out_dev = is_device_ptr(P_out);
        e = ensure(stage, (size_t)n * (nhost + (out_dev ? 0 : 1)));
        int k = 0;
        for (int q = 0; q < n_sets && e == hipSuccess; ++q) {
            if (is_device_ptr(P_in[q])) {
                cs.p[q] = P_in[q];
            } else {
                double* d = stage.p + (size_t)n * k++;
                e = hipMemcpyAsync(d, P_in[q], (size_t)n * 8, hipMemcpyHostToDevice, s);
                cs.p[q] = d;
            }
        }
        double* dst = out_dev ? P_out : stage.p + (size_t)n * k;
        if (e == hipSuccess) e = combine_sets(n, n_sets, cs, dst, s);
        if (e == hipSuccess && !out_dev) e = hipMemcpyAsync(P_out, dst, (size_t)n * 8, hipMemcpyDeviceToHost, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail_hip(c, e, "set combination");
    if (bound) *bound = hb;
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

static dm_status eval_trace(dm_ctx* c, double beta, double target, double tol, double mu_in,
                            int max_iter, double out[5]) {
    if (!c->have_fock) return set_err(c, DM_E_STATE, "no Fock matrix loaded");
    if (c->mom_order < 2 || c->ncols_done == 0) return set_err(c, DM_E_STATE, "no accumulated moments");
    if (!std::isfinite(beta) || !(beta > 0)) return set_err(c, DM_E_ARG, "need beta > 0");
    hipStream_t s = c->stream;
    const int N = c->mom_order, M = 4 * N;
    const double ebar = 0.5 * (c->op.emax + c->op.emin), de = 0.5 * (c->op.emax - c->op.emin);
    HIPTRY(c, ensure(c->w, (size_t)M));
    HIPTRY(c, ensure(c->v, (size_t)M));
    HIPTRY(c, trace_weights(N, M, ebar, de, c->mom.p, c->w.p, c->v.p, s));
    HIPTRY(c, mu_bisect(M, ebar, de, beta, target, tol, c->op.emin, c->op.emax, mu_in, max_iter, c->w.p,
                        c->v.p, c->out.p, s));
    HIPTRY(c, hipMemcpyAsync(out, c->out.p, 5 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPTRY(c, hipStreamSynchronize(s));
    return DM_OK;
}

dm_status dm_trace(dm_ctx* c, double mu, double beta, double* tr_PS, double* e_band) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (!std::isfinite(mu)) return set_err(c, DM_E_ARG, "mu not finite");
    double out[5];
    st = eval_trace(c, beta, 0.0, 0.0, mu, 0, out);
    if (st != DM_OK) return st;
    if (tr_PS) *tr_PS = out[1];
    if (e_band) *e_band = c->opt.spin * out[2];
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

dm_status dm_solve_mu(dm_ctx* c, double n_e, double beta, double tol, double* mu) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (!mu || !std::isfinite(n_e) || !(tol > 0)) return set_err(c, DM_E_ARG, "bad n_e, tol or mu");
    double out[5];
    st = eval_trace(c, beta, n_e / c->opt.spin, tol / c->opt.spin, 0.0, 200, out);
    if (st != DM_OK) return st;
    *mu = out[0];
    if (out[3] == 0.0)
        return set_err(c, DM_E_NOCONV, "bisection bracket collapsed before reaching the tolerance");
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

dm_status dm_dos(dm_ctx* c, int kind, int n, const double* energies, double sigma, double* dos) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (n < 0 || (n > 0 && (!energies || !dos))) return set_err(c, DM_E_ARG, "bad energies or output");
    if (kind != DM_DOS_GAUSSIAN && kind != DM_DOS_KPM) return set_err(c, DM_E_ARG, "unknown DOS kind");
    if (kind == DM_DOS_GAUSSIAN && !(sigma > 0 && std::isfinite(sigma)))
        return set_err(c, DM_E_ARG, "need sigma > 0");
    if (!c->have_fock) return set_err(c, DM_E_STATE, "no Fock matrix loaded");
    if (c->mom_order < 2 || c->ncols_done == 0) return set_err(c, DM_E_STATE, "no accumulated moments");
    if (n == 0) return DM_OK;
    hipStream_t s = c->stream;
    const int N = c->mom_order, M = 4 * N;
    const double ebar = 0.5 * (c->op.emax + c->op.emin), de = 0.5 * (c->op.emax - c->op.emin);
    DevBuf<double> Ed, Od;
    auto rel = [&]() { Ed.release(); Od.release(); };
    hipError_t e;
#define DOS(expr)                         \
    do {                                  \
        if ((e = (expr)) != hipSuccess) { \
            rel();                        \
            return fail_hip(c, e, #expr); \
        }                                 \
    } while (0)
    DOS(ensure(Ed, (size_t)n));
    DOS(ensure(Od, (size_t)n));
    DOS(hipMemcpyAsync(Ed.p, energies, (size_t)n * 8, hipMemcpyDefault, s));
    if (kind == DM_DOS_GAUSSIAN) {
        DOS(ensure(c->w, (size_t)M));
        DOS(ensure(c->v, (size_t)M));
        DOS(trace_weights(N, M, ebar, de, c->mom.p, c->w.p, c->v.p, s));
        DOS(dos_gauss(n, Ed.p, M, ebar, de, sigma, c->opt.spin, c->w.p, Od.p, s));
    } else {
        DOS(dos_kpm(n, Ed.p, N, ebar, de, c->opt.spin, c->mom.p, Od.p, s));
    }
    DOS(hipMemcpyAsync(dos, Od.p, (size_t)n * 8, hipMemcpyDefault, s));
    DOS(hipStreamSynchronize(s));
#undef DOS
    rel();
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

// Window depth d = L sqrt(zeta) of an s-type Gaussian (grid-window section,
// eq. WindowLength): the window keeps the fraction 1 - eta of the function's
// one-dimensional integral, c(d, 0) = erf(d) = 1 - eta, i.e. erfc(d) = eta.
// Solved by Newton's method on ln erfc (convex and decreasing for d >= 0),
// which stays accurate for eta far below the rounding of 1 - eta.
static double window_depth_s(double eta) {
    const double two_over_sqrtpi = 1.1283791670955126;
    double d = eta < 0.5 ? std::sqrt(std::log(1.0 / eta)) : 0.5;
    for (int it = 0; it < 100; ++it) {
        const double q = std::erfc(d);
        const double g = std::log(q) - std::log(eta);
        const double dg = -two_over_sqrtpi * std::exp(-d * d) / q;
        const double nd = std::max(0.0, d - g / dg);
        if (std::fabs(nd - d) <= 1e-15 * std::max(1.0, d)) return nd;
        d = nd;
    }
    return d;
}

// Per-function arrays (spatial order) and per-cell function lists of
// dm_density_on_grid, uploaded into the context's grid plan; waits for the
// uploads, so the host arrays may go when it returns.  The inputs have been
// checked for sizes and columns by the caller.
static dm_status build_grid_plan(dm_ctx* c, long long K, const double* centres, const double* exponents,
                                 const double* origin, double h, int nx, int ny, int nz, double eta,
                                 const std::vector<long long>& hc) {
    std::vector<int> colpos((size_t)K, -1);
    for (size_t j = 0; j < hc.size(); ++j) colpos[(size_t)hc[j]] = (int)j;
    // per-function data and window half-widths (host arrays, K entries)
    std::vector<double> fx(K), fy(K), fz(K), fe(K), fn(K), fr(K);
    const double dwin = window_depth_s(eta);
    for (long long b = 0; b < K; ++b) {
        const double a = exponents[b];
        if (!(a > 0) || !std::isfinite(a)) return set_err(c, DM_E_ARG, "exponents must be > 0");
        fx[b] = centres[3 * b];
        fy[b] = centres[3 * b + 1];
        fz[b] = centres[3 * b + 2];
        fe[b] = a;
        fn[b] = std::pow(2.0 * a / 3.14159265358979323846, 0.75);
        fr[b] = dwin / std::sqrt(a);
        if (!std::isfinite(fx[b]) || !std::isfinite(fy[b]) || !std::isfinite(fz[b]))
            return set_err(c, DM_E_ARG, "centres must be finite");
    }
    // Functions in Morton (Z-curve) order of their centres, ties by index:
    // the functions that reach one cell are then a few runs of consecutive
    // indices, so the kernel reads a column of P in long runs instead of one
    // atom's rows here and there.  The per-function arrays, the column
    // positions and the rows of P are permuted alike (perm: new -> old); the
    // density does not depend on the order of the sum over functions.
    std::vector<int> perm((size_t)K);
    {
        double lo[3], hi[3];
        const std::vector<double>* axes[3] = {&fx, &fy, &fz};
        for (int d = 0; d < 3; ++d) {
            lo[d] = *std::min_element(axes[d]->begin(), axes[d]->end());
            hi[d] = *std::max_element(axes[d]->begin(), axes[d]->end());
        }
        const double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]});
        const double cell = ext > 0 ? ext / 1023.0 : 1.0;
        auto spread = [](unsigned long long v) {  // bit i of v -> bit 3 i
            v &= 0x3ffULL;
            v = (v | (v << 16)) & 0x30000ffULL;
            v = (v | (v << 8)) & 0x300f00fULL;
            v = (v | (v << 4)) & 0x30c30c3ULL;
            v = (v | (v << 2)) & 0x9249249ULL;
            return v;
        };
        std::vector<std::pair<unsigned long long, int>> key((size_t)K);
        for (long long b = 0; b < K; ++b) {
            unsigned long long q[3];
            for (int d = 0; d < 3; ++d)
                q[d] = (unsigned long long)std::min(1023.0, std::max(0.0, std::floor(((*axes[d])[b] - lo[d]) / cell)));
            key[b] = {spread(q[0]) | (spread(q[1]) << 1) | (spread(q[2]) << 2), (int)b};
        }
        std::sort(key.begin(), key.end());
        for (long long i = 0; i < K; ++i) perm[i] = key[i].second;
        auto apply = [&](auto& v) {
            std::remove_reference_t<decltype(v)> t(v.size());
            for (long long i = 0; i < K; ++i) t[i] = v[perm[i]];
            v.swap(t);
        };
        apply(fx);
        apply(fy);
        apply(fz);
        apply(fe);
        apply(fn);
        apply(fr);
        apply(colpos);
    }
    // cell lists: function b reaches the grid indices [lo, hi] along each axis
    const int ncx = (nx + 3) / 4, ncy = (ny + 3) / 4, ncz = (nz + 3) / 4;
    const long long ncell = (long long)ncx * ncy * ncz;
    if (ncell > (1LL << 31) - 1) return set_err(c, DM_E_ARG, "grid too large");
    // per-cell counts (each at most K), prefix sums in 64 bits: the number of
    // (function, cell) pairs can pass 2^31 on fine grids, and the kernel's
    // offsets are 32-bit, so such a call is refused below
    std::vector<long long> bcount((size_t)ncell + 1, 0), acount((size_t)ncell + 1, 0);
    // grid indices a window reaches, with one point of slack on each side (the
    // kernel tests every point exactly), clamped before the integer conversion
    auto range = [&](double ctr, double R, double o, int n, int& lo, int& hi) {
        const double l = std::ceil((ctr - R - o) / h) - 1, u = std::floor((ctr + R - o) / h) + 1;
        if (!(u >= 0) || !(l <= n - 1)) return false;
        lo = (int)std::max(0.0, l);
        hi = (int)std::min((double)n - 1, u);
        return lo <= hi;
    };
    std::vector<std::array<int, 6>> box((size_t)K);
    std::vector<char> reach((size_t)K, 0);
    for (long long b = 0; b < K; ++b) {
        int xl, xh, yl, yh, zl, zh;
        if (!range(fx[b], fr[b], origin[0], nx, xl, xh) || !range(fy[b], fr[b], origin[1], ny, yl, yh) ||
            !range(fz[b], fr[b], origin[2], nz, zl, zh))
            continue;
        box[b] = {xl / 4, xh / 4, yl / 4, yh / 4, zl / 4, zh / 4};
        reach[b] = 1;
    }
    // count and fill per slab of cell planes on host threads; every thread
    // walks the functions in ascending order, so each cell lists them in
    // ascending order whatever the number of threads
    const int nthr = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    auto slabs = [&](auto&& body) {
        std::vector<std::thread> th;
        th.reserve((size_t)nthr);
        int t = 0;
        for (; t < nthr; ++t) {
            const int z0 = (int)((long long)ncz * t / nthr), z1 = (int)((long long)ncz * (t + 1) / nthr);
            if (z0 >= z1) continue;
            try {
                th.emplace_back(body, z0, z1);
            } catch (...) {  // no thread available: this slab and the rest on the calling thread
                break;
            }
        }
        for (; t < nthr; ++t) {
            const int z0 = (int)((long long)ncz * t / nthr), z1 = (int)((long long)ncz * (t + 1) / nthr);
            if (z0 < z1) body(z0, z1);
        }
        for (auto& x : th) x.join();
    };
    slabs([&](int z0, int z1) {
        for (long long b = 0; b < K; ++b) {
            if (!reach[b]) continue;
            const auto& bx = box[b];
            for (int cz = std::max(bx[4], z0); cz <= std::min(bx[5], z1 - 1); ++cz)
                for (int cy = bx[2]; cy <= bx[3]; ++cy)
                    for (int cx = bx[0]; cx <= bx[1]; ++cx) {
                        const long long cell = cx + (long long)ncx * (cy + (long long)ncy * cz);
                        ++bcount[cell + 1];
                        if (colpos[b] >= 0) ++acount[cell + 1];
                    }
        }
    });
    for (long long i = 0; i < ncell; ++i) {
        bcount[i + 1] += bcount[i];
        acount[i + 1] += acount[i];
    }
    if (bcount[ncell] > (long long)INT32_MAX)
        return set_err(c, DM_E_ARG, "grid too fine for the windows: more than 2^31 - 1 (function, cell) pairs");
    std::vector<int> bidx((size_t)bcount[ncell]), aidx((size_t)acount[ncell]), acol((size_t)acount[ncell]);
    {
        std::vector<long long> bfill(bcount.begin(), bcount.end() - 1), afill(acount.begin(), acount.end() - 1);
        slabs([&](int z0, int z1) {
            for (long long b = 0; b < K; ++b) {
                if (!reach[b]) continue;
                const auto& bx = box[b];
                for (int cz = std::max(bx[4], z0); cz <= std::min(bx[5], z1 - 1); ++cz)
                    for (int cy = bx[2]; cy <= bx[3]; ++cy)
                        for (int cx = bx[0]; cx <= bx[1]; ++cx) {
                            const long long cell = cx + (long long)ncx * (cy + (long long)ncy * cz);
                            bidx[bfill[cell]++] = (int)b;
                            if (colpos[b] >= 0) {
                                aidx[afill[cell]] = (int)b;
                                acol[afill[cell]++] = colpos[b];
                            }
                        }
            }
        });
    }
    GridPlan& gp = c->grid;
    gp.ncx = ncx;
    gp.ncy = ncy;
    gp.ncz = ncz;
    hipStream_t s = c->stream;
    hipError_t e;
#define GR(expr)                          \
    do {                                  \
        if ((e = (expr)) != hipSuccess) { \
            gp.release();                 \
            return fail_hip(c, e, #expr); \
        }                                 \
    } while (0)
    auto up_d = [&](DevBuf<double>& d, const std::vector<double>& v) -> hipError_t {
        hipError_t r = ensure(d, v.size());
        if (r == hipSuccess) r = hipMemcpyAsync(d.p, v.data(), v.size() * 8, hipMemcpyHostToDevice, s);
        return r;
    };
    auto up_i = [&](DevBuf<int>& d, const std::vector<int>& v) -> hipError_t {
        hipError_t r = ensure(d, std::max<size_t>(v.size(), 1));
        if (r == hipSuccess && !v.empty()) r = hipMemcpyAsync(d.p, v.data(), v.size() * 4, hipMemcpyHostToDevice, s);
        return r;
    };
    const std::vector<int> bptr(bcount.begin(), bcount.end()), aptr(acount.begin(), acount.end());
    GR(up_d(gp.fx, fx));
    GR(up_d(gp.fy, fy));
    GR(up_d(gp.fz, fz));
    GR(up_d(gp.fe, fe));
    GR(up_d(gp.fn, fn));
    GR(up_d(gp.fr, fr));
    GR(up_i(gp.bp, bptr));
    GR(up_i(gp.bi, bidx));
    GR(up_i(gp.ap, aptr));
    GR(up_i(gp.ai, aidx));
    GR(up_i(gp.ac, acol));
    GR(up_i(gp.perm, perm));
    GR(hipStreamSynchronize(s));
#undef GR
    return DM_OK;
}

dm_status dm_density_on_grid(dm_ctx* c, long long K, const double* centres, const double* exponents,
                             const double* origin, double h, const int* dims, double eta, const long long* cols,
                             long long ncols, const double* P_cols, double* n_out) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (K <= 0 || K > (1LL << 30) || !centres || !exponents || !origin || !dims || !n_out)
        return set_err(c, DM_E_ARG, "bad basis or grid arguments");
    if (!(h > 0) || !std::isfinite(h) || !(eta > 0 && eta < 1)) return set_err(c, DM_E_ARG, "need h > 0 and 0 < eta < 1");
    if (ncols < 0 || ncols > K || (ncols > 0 && (!cols || !P_cols))) return set_err(c, DM_E_ARG, "bad columns");
    const int nx = dims[0], ny = dims[1], nz = dims[2];
    if (nx < 1 || ny < 1 || nz < 1) return set_err(c, DM_E_ARG, "grid dimensions must be >= 1");
    const long long G = (long long)nx * ny * nz;
    if (ncols == 0) return DM_OK;
    std::vector<long long> hc;
    HIPTRY(c, to_host(hc, cols, (size_t)ncols));
    std::vector<int> colpos((size_t)K, -1);
    for (long long j = 0; j < ncols; ++j) {
        if (hc[j] < 0 || hc[j] >= K) return set_err(c, DM_E_ARG, "column index out of range");
        if (colpos[hc[j]] >= 0) return set_err(c, DM_E_ARG, "repeated column index");
        colpos[hc[j]] = (int)j;
    }
    // The lists depend on the basis, the grid, eta and the columns only:
    // reuse those of the last call when all of them are the same.
    GridPlan& gp = c->grid;
    std::vector<double> key;
    key.reserve((size_t)(4 * K + 5));
    key.insert(key.end(), centres, centres + 3 * K);
    key.insert(key.end(), exponents, exponents + K);
    key.insert(key.end(), origin, origin + 3);
    key.push_back(h);
    key.push_back(eta);
    const bool reuse = gp.valid && gp.K == K && gp.dims[0] == nx && gp.dims[1] == ny && gp.dims[2] == nz &&
                       gp.key.size() == key.size() &&
                       std::memcmp(gp.key.data(), key.data(), key.size() * sizeof(double)) == 0 && gp.key_cols == hc;
    hipStream_t s = c->stream;
    hipError_t e;
#define GR(expr)                          \
    do {                                  \
        if ((e = (expr)) != hipSuccess) { \
            gp.release();                 \
            return fail_hip(c, e, #expr); \
        }                                 \
    } while (0)
    if (!reuse) {
        gp.valid = false;
        dm_status bs = build_grid_plan(c, K, centres, exponents, origin, h, nx, ny, nz, eta, hc);
        if (bs != DM_OK) return bs;
        gp.K = K;
        gp.dims[0] = nx;
        gp.dims[1] = ny;
        gp.dims[2] = nz;
        gp.key.swap(key);
        gp.key_cols = hc;
        gp.valid = true;
    }
    // P and n through the plan's device buffers (either may be host memory);
    // the rows of P in the functions' spatial order
    GR(ensure(gp.P, (size_t)K * ncols));
    GR(hipMemcpyAsync(gp.P.p, P_cols, (size_t)K * ncols * 8, hipMemcpyDefault, s));
    GR(ensure(gp.Pp, (size_t)K * ncols));
    GR(permute_rows((int)K, ncols, gp.perm.p, gp.P.p, gp.Pp.p, s));
    GR(ensure(gp.n, (size_t)G));
    GR(hipMemcpyAsync(gp.n.p, n_out, (size_t)G * 8, hipMemcpyDefault, s));
    GridArgs ga{};
    ga.nx = nx; ga.ny = ny; ga.nz = nz; ga.ncx = gp.ncx; ga.ncy = gp.ncy; ga.ncz = gp.ncz;
    ga.ox = origin[0]; ga.oy = origin[1]; ga.oz = origin[2]; ga.h = h;
    ga.cx = gp.fx.p; ga.cy = gp.fy.p; ga.cz = gp.fz.p; ga.ex = gp.fe.p; ga.norm = gp.fn.p; ga.R = gp.fr.p;
    ga.beta_ptr = gp.bp.p; ga.beta_idx = gp.bi.p; ga.alpha_ptr = gp.ap.p; ga.alpha_idx = gp.ai.p;
    ga.alpha_col = gp.ac.p;
    ga.P = gp.Pp.p;
    ga.ldp = K;
    ga.n = gp.n.p;
    GR(density_on_grid(ga, s));
    GR(hipMemcpyAsync(n_out, gp.n.p, (size_t)G * 8, hipMemcpyDefault, s));
    GR(hipStreamSynchronize(s));
#undef GR
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

dm_status dm_moments(dm_ctx* c, double* m, int n, long long* ncols_done) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (n < 0) return set_err(c, DM_E_ARG, "n < 0");
    if (ncols_done) *ncols_done = c->mom_order < 0 ? 0 : c->ncols_done;
    if (m && n > 0) {
        std::fill(m, m + n, 0.0);
        const int avail = c->mom_order < 0 ? 0 : std::min(n, c->mom_order + 1);
        if (avail > 0) {
            HIPTRY(c, hipMemcpyAsync(m, c->mom.p, (size_t)avail * 8, hipMemcpyDeviceToHost, c->stream));
            HIPTRY(c, hipStreamSynchronize(c->stream));
        }
    }
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

dm_status dm_reset_moments(dm_ctx* c) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    return reset_moments(c);
} catch (...) {
    return host_exception(c);
}

dm_status dm_set_pass_shape(dm_ctx* c, int width, int cfg) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (!c->have_fock) return set_err(c, DM_E_STATE, "no Fock matrix loaded");
    if (c->op.fact) return set_err(c, DM_E_STATE, "tile shapes do not apply to the factored form");
    if (width < 1 || cfg < 0 || cfg >= cheb_num_tile_configs() ||
        !cheb_cfg_fits(cfg, c->precision, c->op.Kp, (int)round_up(width, cheb_tile_cols(cfg))))
        return set_err(c, DM_E_ARG, "pass width must be >= 1 and the tile shape one that fits this operator and precision");
    c->tuned_width = width;
    c->tuned_cfg = cfg;
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

int dm_num_tile_shapes(void) { return cheb_num_tile_configs(); }

dm_status dm_tile_shape(int cfg, int* rows, int* cols, int* split) {
    if (cfg < 0 || cfg >= cheb_num_tile_configs()) return DM_E_ARG;
    if (rows) *rows = cheb_tile_rows(cfg);
    if (cols) *cols = cheb_tile_cols(cfg);
    if (split) *split = cheb_cfg_split(cfg);
    return DM_OK;
}

dm_status dm_autotune(dm_ctx* c, long long ncols, int steps, double* table, int* ntable,
                      int* best_width, int* best_cfg) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (!c->have_fock) return set_err(c, DM_E_STATE, "no Fock matrix loaded");
    if (c->op.fact) return set_err(c, DM_E_STATE, "tile shapes do not apply to the factored form");
    if (ncols < 1 || steps < 1) return set_err(c, DM_E_ARG, "need ncols >= 1 and steps >= 1");
    hipStream_t s = c->stream;
    const int K = (int)c->op.K, Kp = c->op.Kp;
    const size_t tsz = c->precision == DM_FP64 ? 8 : 4;
    const int wmax = (int)std::max<long long>(32, std::min<long long>(ncols, 256));
    struct Cand { int w, cfg; double ms; };
    std::vector<Cand> cands;
    std::vector<int> widths = {32, 64, 128, 256};
    // the full pass width as well, when the caller advances more columns
    const int wfull = (int)std::min<long long>(round_up(ncols, 128), 1 << 14);
    if (wfull > 256) widths.push_back(wfull);
    for (int w : widths) {
        if (w > wmax && w != wfull) continue;
        for (int cfg = 0; cfg < cheb_num_tile_configs(); ++cfg)
            if (cheb_cfg_fits(cfg, c->precision, Kp, w)) cands.push_back({w, cfg, 0.0});
    }
    const int W = std::max(256, wfull);
    DevBuf<double> U0, U1, Zb, Pb, part, pst, coef, work;
    DevBuf<long long> colsd;
    auto rel = [&]() { U0.release(); U1.release(); Zb.release(); Pb.release(); part.release(); pst.release(); coef.release(); work.release(); colsd.release(); };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e;
#define AT(expr)                                         \
    do {                                                 \
        if ((e = (expr)) != hipSuccess) {                \
            rel();                                       \
            if (e0) (void)hipEventDestroy(e0);           \
            if (e1) (void)hipEventDestroy(e1);           \
            return fail_hip(c, e, #expr);                \
        }                                                \
    } while (0)
    AT(hipEventCreate(&e0));
    AT(hipEventCreate(&e1));
    AT(ensure(U0, (size_t)Kp * W * tsz / 8));
    AT(ensure(U1, (size_t)Kp * W * tsz / 8));
    AT(ensure(Zb, (size_t)Kp * W));
    AT(ensure(Pb, (size_t)Kp * W));
    AT(ensure(pst, (size_t)(Kp / 64) * (W / 16)));
    AT(ensure(coef, (size_t)steps + 4));
    int max_tiles = 0;
    size_t max_work = 0;
    for (const Cand& cd : cands) {
        max_tiles = std::max(max_tiles, cheb_num_tiles(Kp, cd.w, cd.cfg));
        max_work = std::max(max_work, cheb_work_bytes(Kp, cd.w, cd.cfg, c->precision));
    }
    AT(ensure(part, (size_t)(steps + 4) * max_tiles));
    if (max_work) AT(ensure(work, (max_work + 7) / 8));
    std::vector<long long> hc(W);
    for (int j = 0; j < W; ++j) hc[j] = j % K;
    AT(ensure(colsd, (size_t)W));
    AT(hipMemcpyAsync(colsd.p, hc.data(), W * 8, hipMemcpyHostToDevice, s));
    AT(fill_f64(coef.p, 0.0, steps + 4, s));  // coefficient 0: the timing leaves P untouched
    for (Cand& cd : cands) {
        const int nc = std::min(cd.w, K);
        AT(fill_f64(Zb.p, 0.0, (long long)Kp * cd.w, s));
        int nts = 0;
        AT(cheb_start(K, Kp, cd.w, nc, colsd.p, c->op.orth ? nullptr : c->op.Sinv.p, c->op.S_rowptr.p, c->op.S_col.p, c->op.S_val.p,
                      c->precision, U0.p, Zb.p, Pb.p, coef.p, 1, 0, 0, pst.p, &nts, s));
        ChebStepArgs a{};
        a.Kp = Kp;
        a.Bp = cd.w;
        a.HN = c->op.HNbuf.p;
        a.coef = coef.p;
        a.P = Pb.p;
        a.Z = Zb.p;
        a.partial = part.p;
        a.work = work.p;
        a.nsets = 1;
        void* ucur = U0.p;
        void* uoth = U1.p;
        for (int l = 1; l <= steps + 2; ++l) {
            if (l == 3) AT(hipEventRecord(e0, s));
            a.Ucur = ucur;
            a.Uprev = (l == 1) ? nullptr : uoth;
            a.Unext = uoth;
            a.alpha = (l == 1) ? 1.0 : 2.0;
            a.has_prev = l > 1;
            a.l = l;
            AT(cheb_step(a, cd.cfg, c->precision, s));
            std::swap(ucur, uoth);
        }
        AT(hipEventRecord(e1, s));
        AT(hipEventSynchronize(e1));
        float ms = 0;
        AT(hipEventElapsedTime(&ms, e0, e1));
        cd.ms = ms / steps;
    }
    rel();
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
#undef AT
    int best = 0;
    for (size_t i = 0; i < cands.size(); ++i) {
        const double r = cands[i].w / cands[i].ms, rb = cands[best].w / cands[best].ms;
        if (r > rb) best = (int)i;
    }
    c->tuned_width = cands[best].w;
    c->tuned_cfg = cands[best].cfg;
    if (best_width) *best_width = c->tuned_width;
    if (best_cfg) *best_cfg = c->tuned_cfg;
    if (ntable) {
        const int cap = *ntable;
        if (table)
            for (int i = 0; i < (int)cands.size() && i < cap; ++i) {
                double* row = table + 6 * i;
                row[0] = cands[i].w;
                row[1] = cands[i].cfg;
                row[2] = cheb_tile_rows(cands[i].cfg);
                row[3] = cheb_tile_cols(cands[i].cfg);
                row[4] = cands[i].ms;
                row[5] = cands[i].w / (cands[i].ms * 1e-3);
            }
        *ntable = (int)cands.size();
    }
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

namespace {
dm_status stoch_moments_op(dm_ctx* c, Op& op, int n_mom, int n_vec, const double* xi, double* m_out);
}

dm_status dm_stoch_moments(dm_ctx* c, int n_mom, int n_vec, const double* xi, double* m_out) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (!c->have_fock) return set_err(c, DM_E_STATE, "no Fock matrix loaded");
    if (n_mom < 1 || n_vec < 1 || !xi || !m_out) return set_err(c, DM_E_ARG, "bad stochastic-moment arguments");
    if (c->op.fact) {
        if (c->precision != DM_FP64) return set_err(c, DM_E_STATE, "the factored form runs in FP64 only");
        hipStream_t s = c->stream;
        DevBuf<double> ms;
        HIPTRY(c, ensure(ms, (size_t)n_mom));
        HIPTRY(c, fill_f64(ms.p, 0.0, n_mom, s));
        HIPTRY(c, fill_i32(c->flag.p, 0, 4, s));
        const double ebar = 0.5 * (c->op.emax + c->op.emin), de = 0.5 * (c->op.emax - c->op.emin);
        int conv = 1;
        const hipError_t e = fact_stoch(c->op.fact, n_vec, xi, n_mom, ebar, de, c->cg_tol, c->cg_max_iter, ms.p,
                                        c->flag.p, &conv, s);
        std::vector<double> h((size_t)n_mom);
        hipError_t e2 = e == hipSuccess ? hipMemcpyAsync(h.data(), ms.p, (size_t)n_mom * 8, hipMemcpyDeviceToHost, s) : e;
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);
        ms.release();
        if (e2 == hipErrorOutOfMemory) return set_err(c, DM_E_OOM, "stochastic moments: device allocation failed");
        if (e2 != hipSuccess) return fail_hip(c, e2, "factored stochastic moments");
        if (!conv)
            return set_err(c, DM_E_NOCONV,
                           "the conjugate-gradient solve with S did not converge within the iteration limit");
        for (int l = 0; l < n_mom; ++l) m_out[l] = h[l] / n_vec;
        return DM_OK;
    }
    return stoch_moments_op(c, c->op, n_mom, n_vec, xi, m_out);
} catch (...) {
    return host_exception(c);
}

dm_status dm_batch_stoch_moments(dm_ctx* c, int n_mom, int n_vec, const double* const* xi, double* m_out) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (c->batch.empty()) return set_err(c, DM_E_STATE, "no batch loaded");
    if ((st = batch_precision_ok(c)) != DM_OK) return st;
    if (n_mom < 1 || n_vec < 1 || !xi || !m_out) return set_err(c, DM_E_ARG, "bad stochastic-moment arguments");
    for (size_t i = 0; i < c->batch.size(); ++i) {
        if (!xi[i]) return set_err(c, DM_E_ARG, "null probe block");
        st = stoch_moments_op(c, c->batch[i], n_mom, n_vec, xi[i], m_out + i * (size_t)n_mom);
        if (st != DM_OK) return st;
    }
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

}  // extern "C"

namespace {
dm_status stoch_moments_op(dm_ctx* c, Op& op, int n_mom, int n_vec, const double* xi, double* m_out) {
    hipStream_t s = c->stream;
    const int K = (int)op.K, Kp = op.Kp;
    const size_t tsz = c->precision == DM_FP64 ? 8 : 4;
    const int cfg = pick_cfg(Kp, n_vec, c->precision);
    const int BN = cheb_tile_cols(cfg);
    const int Bp = (int)round_up(n_vec, std::max(BN, 16));
    DevBuf<double> X, U0, U1, Zs, Pd, pst, pss, ms, cz, W;
    auto rel = [&]() { X.release(); U0.release(); U1.release(); Zs.release(); Pd.release(); pst.release(); pss.release(); ms.release(); cz.release(); W.release(); };
    hipError_t e;
#define SM(expr)                          \
    do {                                  \
        if ((e = (expr)) != hipSuccess) { \
            rel();                        \
            return fail_hip(c, e, #expr); \
        }                                 \
    } while (0)
    const int ntl = cheb_num_tiles(Kp, Bp, cfg);
    SM(ensure(X, (size_t)K * n_vec));
    SM(ensure(U0, (size_t)Kp * Bp * tsz / 8));
    SM(ensure(U1, (size_t)Kp * Bp * tsz / 8));
    SM(ensure(Zs, (size_t)Kp * Bp));
    SM(ensure(Pd, 4));
    SM(ensure(pst, (size_t)(Kp / 64) * (Bp / 16)));
    SM(ensure(pss, (size_t)std::max(n_mom, 1) * ntl));
    SM(ensure(ms, (size_t)n_mom));
    SM(ensure(cz, (size_t)n_mom + 1));
    const size_t wbytes = cheb_work_bytes(Kp, Bp, cfg, c->precision);
    if (wbytes) SM(ensure(W, (wbytes + 7) / 8));
    SM(hipMemcpyAsync(X.p, xi, (size_t)K * n_vec * 8, hipMemcpyDefault, s));
    SM(fill_f64(ms.p, 0.0, n_mom, s));
    SM(fill_f64(cz.p, 0.0, n_mom + 1, s));
    SM(fill_i32(c->flag.p, 0, 4, s));
    int nts = 0;
    SM(cheb_start_vectors(K, Kp, Bp, n_vec, X.p, 1.0 / n_vec, c->precision, U0.p, Zs.p, pst.p, &nts, s));
    SM(reduce_moments(0, nts, pst.p, ms.p, c->flag.p, s));
    void* ucur = U0.p;
    void* uoth = U1.p;
    ChebStepArgs a{};
    a.Kp = Kp;
    a.Bp = Bp;
    a.HN = op.HNbuf.p;
    a.coef = cz.p;
    a.P = Pd.p;
    a.Z = Zs.p;
    a.partial = pss.p;
    a.work = W.p;
    a.nsets = 1;
    for (int l = 1; l < n_mom; ++l) {
        a.Ucur = ucur;
        a.Uprev = (l == 1) ? nullptr : uoth;
        a.Unext = uoth;
        a.alpha = (l == 1) ? 1.0 : 2.0;
        a.has_prev = (l > 1);
        a.l = l;
        SM(cheb_step(a, cfg, c->precision, s));
        std::swap(ucur, uoth);
    }
    if (n_mom > 1) SM(reduce_moments(n_mom - 2, ntl, pss.p + ntl, ms.p + 1, c->flag.p, s));
    SM(hipMemcpyAsync(m_out, ms.p, (size_t)n_mom * 8, hipMemcpyDeviceToHost, s));
    SM(hipStreamSynchronize(s));
#undef SM
    rel();
    return DM_OK;
}
}  // namespace

extern "C" {

}  // extern "C"

// ------------------------------------------------------------------- batch

namespace {

// Tile shape of the FP64 moments pass that goes with the recursion shape
// cfg: the FP64 batch shape with the same tile rows and columns, else the
// first FP64 batch shape.
int batch_mom_cfg(int cfg) {
    int first = -1;
    for (int i = 0; i < cheb_batch_num_cfgs(); ++i) {
        const int m = cheb_batch_cfg(i, DM_FP64);
        if (m < 0) continue;
        if (first < 0) first = m;
        if (cheb_tile_rows(m) == cheb_tile_rows(cfg) && cheb_tile_cols(m) == cheb_tile_cols(cfg)) return m;
    }
    return first;
}

// Polls after which a gang barrier of the batch kernel gives up: 2^20, or
// the environment variable DM_BATCH_BARRIER_POLLS (>= 0) read when a batch
// launch sequence is built (so tests can make the give-up path run).
int batch_barrier_polls() {
    const char* v = std::getenv("DM_BATCH_BARRIER_POLLS");
    if (v && *v) {
        char* end = nullptr;
        const long x = std::strtol(v, &end, 10);
        if (end && *end == '\0' && x >= 0 && x <= (1L << 30)) return (int)x;
    }
    return 1 << 20;
}

// Items of at least this many operator rows are shared by a gang (its
// members split the row tiles and meet after every step); smaller ones run
// on one workgroup each, kGang of similar size to a round.
constexpr int kGangSplitRows = 2048;

// Workgroups of the batch kernel for tile shape cfg: every CU filled, in
// whole gangs; gmap = 8 when the grid deals whole gangs to each of the 8
// XCDs, else 1 (members then need not share an XCD).
void batch_launch_shape(dm_ctx* c, int cfg, int precision, BatchTable& t) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->opt.device) != hipSuccess || cus < 1)
        cus = 256;
    const int resident = cus * std::max(1, cheb_batch_occupancy(cfg, precision));
    if (resident >= 8 * kGang) {
        t.gmap = 8;
        t.ngangs = resident / (8 * kGang) * 8;
    } else {
        t.gmap = 1;
        t.ngangs = std::max(1, resident / kGang);
    }
    t.grid = t.ngangs * kGang;
}

// Cluster table and the gangs' round lists of one pass with tile shape cfg,
// reading H_N from HN64 (FP64 moments pass) or HNbuf.  Rounds are dealt
// longest first to the gang with the least work so far (work of a round:
// Kp^2 x its columns, divided among the members of a shared item).
dm_status batch_pass_table(dm_ctx* c, int cfg, bool fp64_copy, int precision, DevBuf<BatchCluster>& dcl,
                           BatchTable& tab) {
    BatchState& bs = *c->bstate;
    const int BN = cheb_tile_cols(cfg);
    const int n = (int)c->batch.size();
    std::vector<BatchCluster> hcl(n);
    std::vector<std::pair<double, BatchRound>> rounds;
    std::vector<std::pair<int, BatchItem>> solo;  // (Kp, item)
    for (int i = 0; i < n; ++i) {
        const Op& op = c->batch[i];
        BatchClusterBufs& b = bs.cl[i];
        BatchCluster& h = hcl[i];
        h.Kp = op.Kp;
        h.Kt = (int)round_up(op.K, 128);
        h.Bp = b.Bp;
        h.nblocks = b.Bp / BN;
        h.HN = fp64_copy ? op.HN64.p : op.HNbuf.p;
        h.Ua = b.Ua.p;
        h.Ub = b.Ub.p;
        h.P = b.P.p;
        h.Z = b.Z.p;
        h.coef = b.coef.p;
        h.partial = b.partial.p;
        for (int blk = 0; blk < h.nblocks; ++blk) {
            if (op.Kp >= kGangSplitRows) {
                BatchRound r{};
                r.split = 1;
                r.n = 1;
                r.item[0] = BatchItem{i, blk};
                rounds.push_back({(double)op.Kp * op.Kp / kGang, r});
            } else {
                solo.push_back({op.Kp, BatchItem{i, blk}});
            }
        }
    }
    std::stable_sort(solo.begin(), solo.end(),
                     [](const std::pair<int, BatchItem>& x, const std::pair<int, BatchItem>& y) {
                         return x.first > y.first;
                     });
    for (size_t k = 0; k < solo.size(); k += kGang) {
        BatchRound r{};
        r.split = 0;
        r.n = (int)std::min<size_t>(kGang, solo.size() - k);
        for (int m = 0; m < r.n; ++m) r.item[m] = solo[k + m].second;
        rounds.push_back({(double)solo[k].first * solo[k].first, r});
    }
    std::stable_sort(rounds.begin(), rounds.end(),
                     [](const std::pair<double, BatchRound>& x, const std::pair<double, BatchRound>& y) {
                         return x.first > y.first;
                     });
    batch_launch_shape(c, cfg, precision, tab);
    const int G = tab.ngangs;
    std::vector<double> load(G, 0.0);
    std::vector<std::vector<BatchRound>> per(G);
    for (const auto& r : rounds) {
        const int g = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[g] += r.first;
        per[g].push_back(r.second);
    }
    // in each gang the shared rounds first: its members then start every
    // shared round together, and wait at a barrier at most about one row
    // tile for each other
    std::vector<BatchRound> hr;
    std::vector<int> gstart(G + 1, 0);
    for (int g = 0; g < G; ++g) {
        gstart[g] = (int)hr.size();
        std::stable_partition(per[g].begin(), per[g].end(), [](const BatchRound& r) { return r.split != 0; });
        hr.insert(hr.end(), per[g].begin(), per[g].end());
    }
    gstart[G] = (int)hr.size();
    HIPTRY(c, ensure(dcl, (size_t)n));
    HIPTRY(c, ensure(tab.rounds, std::max<size_t>(hr.size(), 1)));
    HIPTRY(c, ensure(tab.gang_start, gstart.size()));
    HIPTRY(c, hipMemcpy(dcl.p, hcl.data(), n * sizeof(BatchCluster), hipMemcpyHostToDevice));
    if (!hr.empty())
        HIPTRY(c, hipMemcpy(tab.rounds.p, hr.data(), hr.size() * sizeof(BatchRound), hipMemcpyHostToDevice));
    HIPTRY(c, hipMemcpy(tab.gang_start.p, gstart.data(), gstart.size() * sizeof(int), hipMemcpyHostToDevice));
    return DM_OK;
}

// Precision of the batch's moments pass.
int batch_mom_precision(const dm_ctx* c) {
    return c->bstate && c->bstate->mom_prec >= 0 ? c->bstate->mom_prec : c->precision;
}

// (Re)builds the per-cluster buffers and the device tables of the batch
// kernel for tile shape cfg and `order` steps.  Rebuilding invalidates any
// captured graph (buffer addresses may change).
dm_status batch_tables(dm_ctx* c, int cfg, int order) {
    BatchState& bs = *c->bstate;
    if (bs.table_cfg == cfg && bs.table_order == order && bs.table_prec == c->precision) return DM_OK;
    bs.drop_graph();
    const int mprec = batch_mom_precision(c);
    const bool split_mom = mprec != c->precision;
    const size_t tsz = (c->precision == DM_FP64 || mprec == DM_FP64) ? 8 : 4;
    const int n = (int)c->batch.size();
    const int M = 4 * order;
    for (int i = 0; i < n; ++i) {
        const Op& op = c->batch[i];
        BatchClusterBufs& b = bs.cl[i];
        const size_t KB = (size_t)op.Kp * b.Bp;
        HIPTRY(c, ensure(b.Ua, KB * tsz / 8));
        HIPTRY(c, ensure(b.Ub, KB * tsz / 8));
        HIPTRY(c, ensure(b.Z, KB));
        HIPTRY(c, ensure(b.P, KB));
        HIPTRY(c, ensure(b.coef, (size_t)order + 1));
        HIPTRY(c, ensure(b.partial, (size_t)(order + 1) * (b.Bp / 32) * kGang));
        HIPTRY(c, ensure(b.pstart, (size_t)(op.Kp / 64) * (b.Bp / 16)));
        HIPTRY(c, ensure(b.mom, (size_t)order + 1));
        HIPTRY(c, ensure(b.w, (size_t)M));
        HIPTRY(c, ensure(b.v, (size_t)M));
        HIPTRY(c, ensure(b.fk, (size_t)M));
        HIPTRY(c, ensure(b.out, 8));
    }
    dm_status st = batch_pass_table(c, cfg, false, c->precision, bs.d_clusters, bs.tab);
    if (st != DM_OK) return st;
    int ng = bs.tab.ngangs;
    if (split_mom) {
        bs.cfg_m = batch_mom_cfg(cfg);
        if (bs.cfg_m < 0) return set_err(c, DM_E_STATE, "no FP64 batch tile shape");
        st = batch_pass_table(c, bs.cfg_m, true, mprec, bs.d_clusters_m, bs.tab_m);
        if (st != DM_OK) return st;
        ng = std::max(ng, bs.tab_m.ngangs);
    }
    HIPTRY(c, ensure(bs.counter, (size_t)2 * ng));
    bs.table_cfg = cfg;
    bs.table_order = order;
    bs.table_prec = c->precision;
    return DM_OK;
}


// Start blocks of every cluster (U_0 = S^-1 columns into U_a in `precision`,
// Z = S, P = a_0 U_0).
hipError_t batch_start(dm_ctx* c, bool zero_moments, int precision) {
    BatchState& bs = *c->bstate;
    hipStream_t s = c->stream;
    hipError_t e;
    for (size_t i = 0; i < c->batch.size(); ++i) {
        const Op& op = c->batch[i];
        BatchClusterBufs& b = bs.cl[i];
        int nts = 0;
        if (op.form == DM_FORM_SYMMETRIC) {
            // V_0 staged in P (cheb_start reads and writes each element in one thread)
            if ((e = sym_start(op, b.Bp, b.Bp, (int)op.K, b.cols.p, precision, b.Ua.p, b.Z.p, b.P.p, b.P.p,
                               b.coef.p, 1, 0, 0, b.pstart.p, &nts, s)) != hipSuccess)
                return e;
        } else {
            if ((e = fill_f64(b.Z.p, 0.0, (long long)op.Kp * b.Bp, s)) != hipSuccess) return e;
            if ((e = cheb_start((int)op.K, op.Kp, b.Bp, (int)op.K, b.cols.p, op.Sinv.p, op.S_rowptr.p, op.S_col.p,
                                op.S_val.p, precision, b.Ua.p, b.Z.p, b.P.p, b.coef.p, 1, 0, 0, b.pstart.p, &nts,
                                s)) != hipSuccess)
                return e;
        }
        if (zero_moments) {
            if ((e = fill_f64(b.mom.p, 0.0, bs.table_order + 1, s)) != hipSuccess) return e;
            if ((e = reduce_moments(0, nts, b.pstart.p, b.mom.p, c->flag.p, s)) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

// The whole batch sequence on c->stream (also recorded under graph capture).
// grid1, grid2: workgroups of the moments and the P pass (batch_grid),
// taken before a capture starts.
hipError_t batch_enqueue(dm_ctx* c, int order, double beta, const std::vector<double>& ne, double tol,
                         bool with_P) {
    BatchState& bs = *c->bstate;
    hipStream_t s = c->stream;
    const int n = (int)c->batch.size();
    const int M = 4 * order;
    const double g = c->opt.spin;
    const int mprec = batch_mom_precision(c);
    const bool split_mom = mprec != c->precision;
    hipError_t e;
#define BQ(x)                                 \
    do {                                      \
        if ((e = (x)) != hipSuccess) return e; \
    } while (0)
    BQ(fill_i32(c->flag.p, 0, 4, s));
    const int ngm = split_mom ? bs.tab_m.ngangs : bs.tab.ngangs;
    BQ(fill_i32(bs.counter.p, 0, ngm + bs.tab.ngangs, s));
    for (int i = 0; i < n; ++i) BQ(fill_f64(bs.cl[i].coef.p, 0.0, order + 1, s));
    // pass 1: moments of every column (coefficients zero: P is not touched),
    // in FP64 from the FP64 copy of H_N when the batch was loaded so
    const int cfg1 = split_mom ? bs.cfg_m : bs.cfg;
    const BatchTable& t1 = split_mom ? bs.tab_m : bs.tab;
    BQ(batch_start(c, true, mprec));
    const int polls = batch_barrier_polls();
    BatchArgs a{split_mom ? bs.d_clusters_m.p : bs.d_clusters.p, t1.rounds.p, t1.gang_start.p, bs.counter.p,
                c->flag.p, order, 0, t1.gmap, polls};
    BQ(cheb_batch(a, cfg1, mprec, t1.grid, s));
    const int BN = cheb_tile_cols(cfg1);
    for (int i = 0; i < n; ++i) {
        const Op& op = c->batch[i];
        BatchClusterBufs& b = bs.cl[i];
        const int nb = b.Bp / BN;
        BQ(reduce_moments(order - 1, nb * kGang, b.partial.p + (size_t)nb * kGang, b.mom.p + 1, c->flag.p, s));
        const double ebar = 0.5 * (op.emax + op.emin), de = 0.5 * (op.emax - op.emin);
        // mu_c from the exact moments, then the coefficients at mu_c
        BQ(trace_weights(order, M, ebar, de, b.mom.p, b.w.p, b.v.p, s));
        BQ(mu_bisect(M, ebar, de, beta, ne[i] / g, tol / g, op.emin, op.emax, 0.0, 200, b.w.p, b.v.p,
                     b.out.p, s));
        BQ(cheb_coefficients_devmu(order, M, ebar, de, b.out.p, beta, b.fk.p, b.coef.p, s));
    }
    if (!with_P) return hipSuccess;
    // pass 2: P at mu_c
    BQ(batch_start(c, false, c->precision));
    BatchArgs a2{bs.d_clusters.p, bs.tab.rounds.p, bs.tab.gang_start.p, bs.counter.p + ngm, c->flag.p, order, 1,
                 bs.tab.gmap, polls};
    BQ(cheb_batch(a2, bs.cfg, c->precision, bs.tab.grid, s));
    // symmetric form: P = L^T Q into the Z buffer (Z is not read after the pass)
    for (int i = 0; i < n; ++i) {
        const Op& op = c->batch[i];
        if (op.form != DM_FORM_SYMMETRIC) continue;
        BatchClusterBufs& b = bs.cl[i];
        BQ(gemm_nn_f64(op.Kp, b.Bp, op.Kp, 1.0, op.Xs.p, op.Kp, b.P.p, op.Kp, 0.0, b.Z.p, op.Kp, true, s));
    }
#undef BQ
    return hipSuccess;
}

}  // namespace

extern "C" {

dm_status dm_batch_set_focks(dm_ctx* c, int n, const dm_csr_pair* cl) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (n < 1 || !cl) return set_err(c, DM_E_ARG, "need n >= 1 clusters");
    if (c->precision == DM_FP32_ACC64)
        return set_err(c, DM_E_STATE, "the batch runs in DM_FP64 or DM_FP32");
    if (c->form == DM_FORM_FACTORED)
        return set_err(c, DM_E_STATE, "the batch runs in the general or symmetric form");
    delete c->bstate;
    c->bstate = nullptr;
    for (auto& o : c->batch) o.release();
    c->batch.clear();
    c->batch.resize(n);
    for (int i = 0; i < n; ++i) {
        HostCsr Fh, Sh;
        st = load_csr_pair(c, cl[i].K, cl[i].F_rowptr, cl[i].F_col, cl[i].F_val, cl[i].S_rowptr,
                           cl[i].S_col, cl[i].S_val, Fh, Sh);
        if (st == DM_OK)
            st = c->form == DM_FORM_SYMMETRIC ? build_sym(c, c->batch[i], cl[i].K, Fh, Sh)
                                              : build_op(c, c->batch[i], cl[i].K, Fh, Sh, c->form);
        if (st != DM_OK) {
            const std::string m = "cluster " + std::to_string(i) + ": " + c->err;
            for (auto& o : c->batch) o.release();
            c->batch.clear();
            return set_err(c, st, m);
        }
        // FP64 moments under an FP32 recursion: an FP64 H_N beside the FP32 one
        if (c->batch_mom_prec == DM_FP64 && c->precision == DM_FP32) {
            Op& op = c->batch[i];
            const double ebar = 0.5 * (op.emax + op.emin), de = 0.5 * (op.emax - op.emin);
            hipError_t e = ensure(op.HN64, (size_t)op.Kp * op.Kp);
            dm_status st2 = DM_OK;
            if (e == hipSuccess && op.form == DM_FORM_SYMMETRIC)
                st2 = sym_panels(c, op, ebar, de, DM_FP64, op.HN64.p);
            else if (e == hipSuccess)
                e = normalize_operator((int)op.K, op.Kp, op.HT.p, ebar, de, DM_FP64, op.HN64.p, c->stream);
            if (e != hipSuccess || st2 != DM_OK) {
                const std::string m = c->err;
                for (auto& o : c->batch) o.release();
                c->batch.clear();
                return e != hipSuccess ? fail_hip(c, e, "FP64 copy of a batch operator") : set_err(c, st2, m);
            }
        }
        // H^T is only needed to renormalise, F only to rebuild H~_N; the
        // batch keeps H_N (and X or S^-1 for its start blocks)
        c->batch[i].HT.release();
        c->batch[i].F_rowptr.release();
        c->batch[i].F_col.release();
        c->batch[i].F_val.release();
        c->batch[i].Fg_ptr.release();
        c->batch[i].Fg_col.release();
        c->batch[i].Fg_val.release();
    }
    c->bstate = new BatchState();
    c->bstate->cl.resize(n);
    c->bstate->mom_prec = (c->batch_mom_prec == DM_FP64 && c->precision == DM_FP32) ? DM_FP64 : -1;
    for (int i = 0; i < n; ++i) {
        BatchClusterBufs& b = c->bstate->cl[i];
        const long long K = c->batch[i].K;
        b.Bp = (int)round_up(K, kColPad);
        std::vector<long long> ar((size_t)K);
        for (long long j = 0; j < K; ++j) ar[j] = j;
        HIPTRY(c, ensure(b.cols, (size_t)K));
        HIPTRY(c, hipMemcpy(b.cols.p, ar.data(), (size_t)K * 8, hipMemcpyHostToDevice));
    }
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

dm_status dm_set_moments_precision(dm_ctx* c, int precision) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (precision != DM_FP64 && precision != DM_FP32 && precision != -1)
        return set_err(c, DM_E_ARG, "precision must be DM_FP64, DM_FP32 or -1");
    c->batch_mom_prec = precision;
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

dm_status dm_batch_run(dm_ctx* c, int order, double beta, const double* n_e, double tol,
                       double* mu_out, double* const* P_out, int flags) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (!c->bstate || c->batch.empty()) return set_err(c, DM_E_STATE, "no batch loaded");
    if ((st = batch_precision_ok(c)) != DM_OK) return st;
    if (order < 2 || !(beta > 0) || !std::isfinite(beta) || !(tol > 0) || !n_e)
        return set_err(c, DM_E_ARG, "need order >= 2, beta > 0, tol > 0 and n_e");
    BatchState& bs = *c->bstate;
    const int n = (int)c->batch.size();
    std::vector<double> ne(n_e, n_e + n);
    for (double x : ne)
        if (!std::isfinite(x)) return set_err(c, DM_E_ARG, "non-finite n_e");
    st = batch_tables(c, bs.cfg, order);
    if (st != DM_OK) return st;
    const int mprec = batch_mom_precision(c);
    const bool split_mom = mprec != c->precision;
    const bool with_P = !(flags & DM_BATCH_MOMENTS_ONLY);
    hipStream_t s = c->stream;
    if (flags & DM_BATCH_EAGER) {
        HIPTRY(c, batch_enqueue(c, order, beta, ne, tol, with_P));
    } else {
        const bool same = bs.exec && bs.g_order == order && bs.g_beta == beta && bs.g_tol == tol &&
                          bs.g_prec == c->precision && bs.g_cfg == bs.cfg && bs.g_ne == ne &&
                          bs.g_with_P == with_P;
        if (!same) {
            bs.drop_graph();
            HIPTRY(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            const hipError_t e1 = batch_enqueue(c, order, beta, ne, tol, with_P);
            hipGraph_t g = nullptr;
            const hipError_t e2 = hipStreamEndCapture(s, &g);
            if (e1 != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return fail_hip(c, e1, "batch capture");
            }
            HIPTRY(c, e2);
            bs.graph = g;
            HIPTRY(c, hipGraphInstantiate(&bs.exec, bs.graph, nullptr, nullptr, 0));
            bs.g_order = order;
            bs.g_beta = beta;
            bs.g_tol = tol;
            bs.g_prec = c->precision;
            bs.g_cfg = bs.cfg;
            bs.g_ne = ne;
            bs.g_with_P = with_P;
        }
        HIPTRY(c, hipGraphLaunch(bs.exec, s));
    }
    std::vector<double> outs((size_t)n * 8);
    for (int i = 0; i < n; ++i)
        HIPTRY(c, hipMemcpyAsync(outs.data() + 8 * i, bs.cl[i].out.p, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
    if (P_out && with_P)
        for (int i = 0; i < n; ++i)
            if (P_out[i]) {
                const size_t K = (size_t)c->batch[i].K, Kp = (size_t)c->batch[i].Kp;
                const double* src = c->batch[i].form == DM_FORM_SYMMETRIC ? bs.cl[i].Z.p : bs.cl[i].P.p;
                HIPTRY(c, hipMemcpy2DAsync(P_out[i], K * 8, src, Kp * 8, K * 8, K, hipMemcpyDefault, s));
            }
    int flag = 0;
    HIPTRY(c, hipMemcpyAsync(&flag, c->flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPTRY(c, hipStreamSynchronize(s));
    bool conv = true;
    for (int i = 0; i < n; ++i) {
        if (mu_out) mu_out[i] = outs[8 * i];
        if (outs[8 * i + 3] == 0.0) conv = false;
    }
    if (flag & 8) return set_err(c, DM_E_STATE, "a batch workgroup waited too long for its gang (too few resident)");
    if (flag) return set_err(c, DM_E_BOUNDS, "batch recursion diverged");
    if (!conv) return set_err(c, DM_E_NOCONV, "a cluster's mu bisection stopped before the tolerance");
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

dm_status dm_batch_get_bounds(dm_ctx* c, int i, double* emin, double* emax) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (i < 0 || i >= (int)c->batch.size()) return set_err(c, DM_E_ARG, "no such batch cluster");
    if (emin) *emin = c->batch[i].emin;
    if (emax) *emax = c->batch[i].emax;
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

dm_status dm_batch_autotune(dm_ctx* c, int steps, double* table, int* ntable, int* best_cfg) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (!c->bstate || c->batch.empty()) return set_err(c, DM_E_STATE, "no batch loaded");
    if ((st = batch_precision_ok(c)) != DM_OK) return st;
    if (steps < 2) return set_err(c, DM_E_ARG, "steps must be >= 2");
    BatchState& bs = *c->bstate;
    hipStream_t s = c->stream;
    hipEvent_t e0, e1;
    HIPTRY(c, hipEventCreate(&e0));
    HIPTRY(c, hipEventCreate(&e1));
    std::vector<std::pair<int, double>> res;
    for (int ci = 0; ci < cheb_batch_num_cfgs(); ++ci) {
        const int cfg = cheb_batch_cfg(ci, c->precision);
        if (cfg < 0) continue;
        st = batch_tables(c, cfg, steps);
        if (st != DM_OK) break;
        for (size_t i = 0; i < c->batch.size(); ++i) HIPTRY(c, fill_f64(bs.cl[i].coef.p, 0.0, steps + 1, s));
        HIPTRY(c, batch_start(c, false, c->precision));
        HIPTRY(c, fill_i32(bs.counter.p, 0, bs.tab.ngangs, s));
        HIPTRY(c, fill_i32(c->flag.p, 0, 4, s));
        BatchArgs a{bs.d_clusters.p, bs.tab.rounds.p, bs.tab.gang_start.p, bs.counter.p, c->flag.p, steps, 0,
                    bs.tab.gmap, batch_barrier_polls()};
        HIPTRY(c, hipEventRecord(e0, s));
        HIPTRY(c, cheb_batch(a, cfg, c->precision, bs.tab.grid, s));
        HIPTRY(c, hipEventRecord(e1, s));
        HIPTRY(c, hipEventSynchronize(e1));
        float ms = 0;
        HIPTRY(c, hipEventElapsedTime(&ms, e0, e1));
        int hflag = 0;
        HIPTRY(c, hipMemcpy(&hflag, c->flag.p, sizeof(int), hipMemcpyDeviceToHost));
        if (hflag & 8) {
            st = set_err(c, DM_E_STATE, "a batch workgroup waited too long for its gang (too few resident)");
            break;
        }
        res.push_back({cfg, ms});
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != DM_OK) return st;
    int best = 0;
    for (size_t i = 1; i < res.size(); ++i)
        if (res[i].second < res[best].second) best = (int)i;
    bs.cfg = res[best].first;
    if (best_cfg) *best_cfg = bs.cfg;
    if (ntable) {
        if (table)
            for (int i = 0; i < (int)res.size() && i < *ntable; ++i) {
                table[4 * i] = res[i].first;
                table[4 * i + 1] = cheb_tile_rows(res[i].first);
                table[4 * i + 2] = cheb_tile_cols(res[i].first);
                table[4 * i + 3] = res[i].second;
            }
        *ntable = (int)res.size();
    }
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

}  // extern "C"

// --------------------------------------------------------------------- MLP
namespace {

dm_status mlp_reserve(dm_ctx* c, int B) {
    MlpState& M = *c->mlp;
    if (B <= M.cap_B) return DM_OK;
    const int L = (int)M.sizes.size() - 1;
    M.act_off.assign(L + 2, 0);
    long tot = 0;
    int wmax = 0;
    for (int j = 0; j <= L; ++j) {
        M.act_off[j] = tot;
        tot += (long)B * M.sizes[j];
        wmax = std::max(wmax, M.sizes[j]);
    }
    M.act_off[L + 1] = tot;
    HIPTRY(c, ensure(M.acts, (size_t)tot));
    HIPTRY(c, ensure(M.T, (size_t)B * M.sizes[L]));
    HIPTRY(c, ensure(M.G0, (size_t)B * wmax));
    HIPTRY(c, ensure(M.G1, (size_t)B * wmax));
    HIPTRY(c, ensure(M.partial, (size_t)(B * M.sizes[L] + 255) / 256 + 1));
    HIPTRY(c, ensure(M.loss, 1));
    M.cap_B = B;
    return DM_OK;
}

// forward pass of B rows of X (host or device) into the activation buffers
dm_status mlp_fwd(dm_ctx* c, const float* X, int B) {
    MlpState& M = *c->mlp;
    dm_status st = mlp_reserve(c, B);
    if (st != DM_OK) return st;
    hipStream_t s = c->stream;
    const int L = (int)M.sizes.size() - 1;
    HIPTRY(c, hipMemcpyAsync(M.acts.p, X, (size_t)B * M.sizes[0] * 4, hipMemcpyDefault, s));
    for (int j = 0; j < L; ++j)
        HIPTRY(c, mlp_linear_fwd(B, M.sizes[j], M.sizes[j + 1], M.acts.p + M.act_off[j],
                                 M.params.p + M.w_off[j], M.params.p + M.b_off[j], j < L - 1,
                                 M.acts.p + M.act_off[j + 1], s));
    return DM_OK;
}

// loss and gradients of the batch (X, T) into M.grads
dm_status mlp_grad(dm_ctx* c, const float* X, const float* T, int B) {
    MlpState& M = *c->mlp;
    dm_status st = mlp_fwd(c, X, B);
    if (st != DM_OK) return st;
    hipStream_t s = c->stream;
    const int L = (int)M.sizes.size() - 1;
    const int nout = M.sizes[L];
    HIPTRY(c, hipMemcpyAsync(M.T.p, T, (size_t)B * nout * 4, hipMemcpyDefault, s));
    HIPTRY(c, mlp_mse_grad(B * nout, M.acts.p + M.act_off[L], M.T.p, M.G0.p, M.partial.p, M.loss.p, s));
    float* G = M.G0.p;
    float* Gn = M.G1.p;
    for (int j = L - 1; j >= 0; --j) {
        HIPTRY(c, mlp_linear_bwd(B, M.sizes[j], M.sizes[j + 1], G, M.acts.p + M.act_off[j],
                                 M.params.p + M.w_off[j], M.grads.p + M.w_off[j], M.grads.p + M.b_off[j],
                                 j > 0 ? Gn : nullptr, s));
        std::swap(G, Gn);
    }
    return DM_OK;
}

dm_status mlp_ready(dm_ctx* c) {
    if (!c->mlp) return set_err(c, DM_E_STATE, "no network: call dm_mlp_init first");
    return DM_OK;
}

}  // namespace

extern "C" {

dm_status dm_mlp_init(dm_ctx* c, int n_layers, const int* sizes, unsigned long long seed) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (n_layers < 1 || n_layers > 16 || !sizes) return set_err(c, DM_E_ARG, "need 1..16 layers");
    for (int j = 0; j <= n_layers; ++j)
        if (sizes[j] < 1 || sizes[j] > 4096) return set_err(c, DM_E_ARG, "layer width out of range");
    delete c->mlp;
    c->mlp = new MlpState();
    MlpState& M = *c->mlp;
    M.sizes.assign(sizes, sizes + n_layers + 1);
    long off = 0;
    for (int j = 0; j < n_layers; ++j) {
        M.w_off.push_back(off);
        off += (long)sizes[j] * sizes[j + 1];
        M.b_off.push_back(off);
        off += sizes[j + 1];
    }
    M.n_params = off;
    HIPTRY(c, ensure(M.params, (size_t)off));
    HIPTRY(c, ensure(M.grads, (size_t)off));
    HIPTRY(c, ensure(M.m, (size_t)off));
    HIPTRY(c, ensure(M.v, (size_t)off));
    for (int j = 0; j < n_layers; ++j)
        HIPTRY(c, mlp_init_layer(sizes[j], sizes[j + 1], seed * 1315423911ull + (unsigned long long)j,
                                 M.params.p + M.w_off[j], M.params.p + M.b_off[j], c->stream));
    HIPTRY(c, hipMemsetAsync(M.m.p, 0, (size_t)off * 4, c->stream));
    HIPTRY(c, hipMemsetAsync(M.v.p, 0, (size_t)off * 4, c->stream));
    HIPTRY(c, hipStreamSynchronize(c->stream));
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

dm_status dm_mlp_num_params(dm_ctx* c, long long* n) try {
    if (!c || !n) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if ((st = mlp_ready(c)) != DM_OK) return st;
    *n = c->mlp->n_params;
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

dm_status dm_mlp_get_params(dm_ctx* c, float* out) try {
    if (!c || !out) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if ((st = mlp_ready(c)) != DM_OK) return st;
    HIPTRY(c, hipMemcpyAsync(out, c->mlp->params.p, (size_t)c->mlp->n_params * 4, hipMemcpyDefault, c->stream));
    HIPTRY(c, hipStreamSynchronize(c->stream));
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

dm_status dm_mlp_set_params(dm_ctx* c, const float* in) try {
    if (!c || !in) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if ((st = mlp_ready(c)) != DM_OK) return st;
    HIPTRY(c, hipMemcpyAsync(c->mlp->params.p, in, (size_t)c->mlp->n_params * 4, hipMemcpyDefault, c->stream));
    HIPTRY(c, hipStreamSynchronize(c->stream));
    c->mlp->t = 0;
    HIPTRY(c, hipMemsetAsync(c->mlp->m.p, 0, (size_t)c->mlp->n_params * 4, c->stream));
    HIPTRY(c, hipMemsetAsync(c->mlp->v.p, 0, (size_t)c->mlp->n_params * 4, c->stream));
    HIPTRY(c, hipStreamSynchronize(c->stream));
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

dm_status dm_mlp_forward(dm_ctx* c, const float* X, int batch, float* Y) try {
    if (!c || !X || !Y || batch < 1) return c ? set_err(c, DM_E_ARG, "bad forward arguments") : DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if ((st = mlp_ready(c)) != DM_OK) return st;
    if ((st = mlp_fwd(c, X, batch)) != DM_OK) return st;
    MlpState& M = *c->mlp;
    const int L = (int)M.sizes.size() - 1;
    HIPTRY(c, hipMemcpyAsync(Y, M.acts.p + M.act_off[L], (size_t)batch * M.sizes[L] * 4, hipMemcpyDefault, c->stream));
    HIPTRY(c, hipStreamSynchronize(c->stream));
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

dm_status dm_mlp_gradients(dm_ctx* c, const float* X, const float* T, int batch, float* loss,
                           float* grads) try {
    if (!c || !X || !T || batch < 1) return c ? set_err(c, DM_E_ARG, "bad gradient arguments") : DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if ((st = mlp_ready(c)) != DM_OK) return st;
    if ((st = mlp_grad(c, X, T, batch)) != DM_OK) return st;
    if (loss) HIPTRY(c, hipMemcpyAsync(loss, c->mlp->loss.p, 4, hipMemcpyDefault, c->stream));
    if (grads)
        HIPTRY(c, hipMemcpyAsync(grads, c->mlp->grads.p, (size_t)c->mlp->n_params * 4, hipMemcpyDefault, c->stream));
    HIPTRY(c, hipStreamSynchronize(c->stream));
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

dm_status dm_mlp_train_step(dm_ctx* c, const float* X, const float* T, int batch, float lr,
                            float* loss) try {
    if (!c || !X || !T || batch < 1 || !(lr > 0)) return c ? set_err(c, DM_E_ARG, "bad training arguments") : DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if ((st = mlp_ready(c)) != DM_OK) return st;
    if ((st = mlp_grad(c, X, T, batch)) != DM_OK) return st;
    MlpState& M = *c->mlp;
    M.t += 1;
    HIPTRY(c, mlp_adam(M.n_params, M.params.p, M.grads.p, M.m.p, M.v.p, lr, M.t, c->stream));
    if (loss) {
        HIPTRY(c, hipMemcpyAsync(loss, M.loss.p, 4, hipMemcpyDefault, c->stream));
        HIPTRY(c, hipStreamSynchronize(c->stream));
    }
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

dm_status dm_mlp_features(dm_ctx* c, const double* m_stoch, int n_mom, double emin, double emax,
                          double beta, double n_e, long long K, float* x) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (!m_stoch || !x || n_mom < 1 || n_mom > 1020 || !(emax > emin) || !(beta > 0) || K < 1)
        return set_err(c, DM_E_ARG, "bad feature arguments");
    DevBuf<double> md;
    DevBuf<float> xd;
    HIPTRY(c, ensure(md, (size_t)n_mom));
    HIPTRY(c, ensure(xd, (size_t)n_mom + 4));
    hipError_t e = hipMemcpyAsync(md.p, m_stoch, (size_t)n_mom * 8, hipMemcpyDefault, c->stream);
    if (e == hipSuccess)
        e = mlp_features(n_mom, md.p, emin, emax, beta, n_e, c->opt.spin, (double)K, xd.p, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(x, xd.p, (size_t)(n_mom + 4) * 4, hipMemcpyDefault, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    md.release();
    xd.release();
    if (e != hipSuccess) return fail_hip(c, e, "features");
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

}  // extern "C"

extern "C" {

dm_status dm_cheb_order(dm_ctx* c, double emin, double emax, double mu, double beta, double tol,
                        int max_order, int* order) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if (!order || !(emax > emin) || !std::isfinite(mu) || !(beta > 0) || !(tol > 0) || max_order < 2 ||
        max_order > (1 << 16))
        return set_err(c, DM_E_ARG, "bad order-estimate arguments");
    // twice as many coefficients as the cap, so the tail beyond the cap is seen
    const int n = 2 * max_order, M = 4 * n;
    DevBuf<double> a, fk;
    DevBuf<int> o;
    hipError_t e = ensure(a, (size_t)n + 1);
    if (e == hipSuccess) e = ensure(fk, (size_t)M);
    if (e == hipSuccess) e = ensure(o, 1);
    if (e == hipSuccess)
        e = cheb_coefficients(n, M, 0.5 * (emax + emin), 0.5 * (emax - emin), mu, beta, fk.p, a.p, c->stream);
    if (e == hipSuccess) e = coef_tail_order(n, max_order, a.p, tol, o.p, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(order, o.p, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    a.release();
    fk.release();
    o.release();
    if (e != hipSuccess) return fail_hip(c, e, "order estimate");
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

dm_status dm_cheb_order_rule(double emin, double emax, double beta, int min_order, int max_order,
                             int* order) {
    if (!order || !std::isfinite(emin) || !std::isfinite(emax) || !(emax > emin) || !(beta > 0) ||
        !std::isfinite(beta) || min_order < 2 || max_order < min_order)
        return DM_E_ARG;
    const double n = std::ceil(2.0 * 0.5 * (emax - emin) * beta);
    *order = n >= (double)max_order ? max_order : std::max(min_order, (int)n);
    return DM_OK;
}

dm_status dm_mlp_encode_targets(double mu, double emin, double emax, int order, float* y) {
    if (!y || !std::isfinite(mu) || !std::isfinite(emin) || !std::isfinite(emax) || !(emax > emin) || order < 1)
        return DM_E_ARG;
    const double ebar = 0.5 * (emax + emin), de = 0.5 * (emax - emin);
    y[0] = (float)(10.0 * (mu - ebar) / de);
    y[1] = (float)(std::log2((double)order) / 10.0 - 1.0);
    return DM_OK;
}

dm_status dm_mlp_predict(dm_ctx* c, const double* m_stoch, int n_mom, double beta, double n_e,
                         int max_order, double* mu, int* order) try {
    if (!c) return DM_E_ARG;
    dm_status st = enter(c);
    if (st != DM_OK) return st;
    if ((st = mlp_ready(c)) != DM_OK) return st;
    if (!c->have_fock) return set_err(c, DM_E_STATE, "no Fock matrix loaded");
    MlpState& M = *c->mlp;
    if (!m_stoch || !mu || !order || n_mom < 1 || M.sizes.front() != n_mom + 4 || M.sizes.back() != 2 ||
        max_order < 16)
        return set_err(c, DM_E_ARG, "network shape does not match n_mom + 4 -> 2, or bad arguments");
    if ((st = mlp_reserve(c, 1)) != DM_OK) return st;
    HIPTRY(c, ensure(M.mom_in, (size_t)n_mom));
    hipError_t e = hipMemcpyAsync(M.mom_in.p, m_stoch, (size_t)n_mom * 8, hipMemcpyDefault, c->stream);
    if (e == hipSuccess)
        e = mlp_features(n_mom, M.mom_in.p, c->op.emin, c->op.emax, beta, n_e, c->opt.spin, (double)c->op.K,
                         M.acts.p, c->stream);
    if (e != hipSuccess) return fail_hip(c, e, "predict features");
    const int L = (int)M.sizes.size() - 1;
    for (int j = 0; j < L && e == hipSuccess; ++j)
        e = mlp_linear_fwd(1, M.sizes[j], M.sizes[j + 1], M.acts.p + M.act_off[j], M.params.p + M.w_off[j],
                           M.params.p + M.b_off[j], j < L - 1, M.acts.p + M.act_off[j + 1], c->stream);
    float y[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(y, M.acts.p + M.act_off[L], 2 * sizeof(float), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail_hip(c, e, "predict");
    const double ebar = 0.5 * (c->op.emax + c->op.emin), de = 0.5 * (c->op.emax - c->op.emin);
    *mu = ebar + de * (double)y[0] / 10.0;
    const double N = std::pow(2.0, 10.0 * ((double)y[1] + 1.0));
    *order = (int)std::lround(std::min<double>(std::max<double>(N, 16.0), (double)max_order));
    return DM_OK;
} catch (...) {
    return host_exception(c);
}

}  // extern "C"
