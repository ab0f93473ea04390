// C ABI of the vectorized PSDP library (include/psdp.h): validation,
// workspace, and the host loop that drives the per-sweep kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "launch.hpp"

using namespace psdp;

namespace {

thread_local std::string g_err;
std::mutex g_lock;

psdp_status fail(psdp_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

psdp_status hipfail(hipError_t e, const char *where) {
    g_err = std::string(where) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? PSDP_E_NOMEM : PSDP_E_DEVICE;
}

#define HIPCHK(expr)                                   \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) return hipfail(e_, #expr); \
    } while (0)

// Leading dimension of every operand copy: a multiple of the GEMM K chunk
// (32), zero padded, so that 16-byte loads of whole chunks stay in bounds.
int64_t padld(int64_t n) { return (n + 31) / 32 * 32; }

// Single-instance solves from this n on read Q from its packed upper tiles
// (psdp_params.gemv_sym = -1).
constexpr int64_t kSymAutoN = 4096;
// Group solves read the Q_i from their packed upper tiles once the stored
// matrices together reach the size of the Infinity Cache, or an instance
// reaches kSymAutoN (gemv_sym = -1).
constexpr int64_t kSymAutoGroupBytes = 256ll << 20;

// Batched integer-product solves with at least this many columns run them as
// two lanes (psdp_params.lanes = 0); at most kMaxLanes lanes.
constexpr int kLaneAutoCols = 512;
constexpr int kMaxLanes = 4;

// Every list and every operand buffer that the product kernels read through
// a list holds zero_col + 1 columns: an empty list slot names zero_col.
bool plan_holds_zero_col(const psdp_column_plan &p) {
    const int64_t need = (int64_t)p.zero_col + 1;
    return p.ncol >= 1 && p.zero_col >= p.ncol && p.list_len >= need && (p.digit_cols == 0 || p.digit_cols >= need) &&
           (p.word_cols == 0 || p.word_cols >= need);
}

// Column bookkeeping of a solve of B starts on n variables (see
// psdp_column_plan); the allocations below take their sizes from it.
psdp_column_plan plan_columns(int64_t n, int32_t B, const psdp_params &prm, bool sparse_copy) {
    psdp_column_plan p{};
    const bool i8 = prm.qx_dtype == PSDP_I8;  // exact integer products, any B
    const bool batched = B > 1 || i8;
    // columns advanced together: every start, or prm.slots of them with the
    // other starts queued (a column takes the next start when its own ends)
    p.ncol = (batched && prm.slots > 0 && prm.slots < B) ? prm.slots : B;
    p.ld = i8 ? (n + 63) / 64 * 64 : padld(n);
    p.zero_col = p.ncol;
    p.list_len = p.ncol + 1;
    p.digit_cols = i8 ? p.ncol + 1 : 0;
    p.word_cols = (i8 && sparse_copy) ? p.ncol + 1 : 0;
    p.ok = plan_holds_zero_col(p) ? 1 : 0;
    return p;
}

// Settings of the exact integer product (layout and K slices) per live
// column estimate, for one n and one digit count, installed by
// psdp_set_digit_table (written by the package's autotuner). Every setting
// yields the same integers, so a table changes the speed only.
struct DigitTableEntry {
    int max_cols, layout, ks;
};
std::map<std::pair<int64_t, int>, std::vector<DigitTableEntry>> g_digit_tables;

// Layouts and K slices of the two products of one launch (est4 subproblem
// columns, est8 lambda_min / CG columns; an estimate of 0 means no product):
// a product with a table for (n, D) takes the entry of the first bucket
// holding its estimate (the last bucket beyond); otherwise the layout comes
// from the live count and the K slices from both products' block count.
struct DigitChoice {
    int mt4, ks4, mt8, ks8;
};
DigitChoice digit_choice(int64_t n, int64_t ld, int est4, int est8) {
    DigitChoice c{1, 1, 1, 1};
    int b4 = 0, b8 = 0;
    if (est4 > 0) digit_layout(est4, 4, ld, &c.mt4, &b4);
    if (est8 > 0) digit_layout(est8, 8, ld, &c.mt8, &b8);
    c.ks4 = digit_slices(c.mt4, b4 + b8);
    c.ks8 = digit_slices(c.mt8, b4 + b8);
    auto table = [&](int D, int est, int *mt, int *ks) {
        auto it = g_digit_tables.find({n, D});
        if (est <= 0 || it == g_digit_tables.end() || it->second.empty()) return;
        const DigitTableEntry *e = &it->second.back();
        for (const DigitTableEntry &t : it->second)
            if (est <= t.max_cols) {
                e = &t;
                break;
            }
        *mt = e->layout;
        *ks = e->ks;
    };
    table(4, est4, &c.mt4, &c.ks4);
    table(8, est8, &c.mt8, &c.ks8);
    return c;
}

// The plan of a group launch: one column per instance, no integer operands.
psdp_column_plan plan_group(int32_t count) {
    psdp_column_plan p{};
    p.ncol = count;
    p.zero_col = count;
    p.list_len = count + 1;
    p.ok = plan_holds_zero_col(p) ? 1 : 0;
    return p;
}

// Device allocations released in reverse order when the solve returns.
struct Arena {
    std::vector<void *> ptrs;
    ~Arena() {
        for (auto it = ptrs.rbegin(); it != ptrs.rend(); ++it) (void)hipFree(*it);
    }
    hipError_t get(void **p, size_t bytes) {
        *p = nullptr;
        if (bytes == 0) bytes = 256;
        hipError_t e = hipMalloc(p, (bytes + 255) / 256 * 256);
        if (e == hipSuccess) ptrs.push_back(*p);
        return e;
    }
};

size_t esize(int dtype) { return dtype == PSDP_F64 ? 8 : dtype == PSDP_F32 ? 4 : dtype == PSDP_I8 ? 1 : 2; }

psdp_status check_params(const psdp_params &p) {
    if (p.inner != PSDP_INNER_PABB && p.inner != PSDP_INNER_PPA) return fail(PSDP_E_INVALID, "params.inner");
    if (p.qx_dtype < PSDP_F64 || p.qx_dtype > PSDP_I8) return fail(PSDP_E_INVALID, "params.qx_dtype");
    if (p.perturb < PSDP_PERTURB_NONE || p.perturb > PSDP_PERTURB_DIAG)
        return fail(PSDP_E_INVALID, "params.perturb");
    if (p.max_inner < 1 || p.max_outer < 0 || p.stall_outer < 1 || p.eig_maxit < 1 || p.cg_maxit < 1 ||
        p.poll_sweeps < 1)
        return fail(PSDP_E_INVALID, "params: iteration caps must be positive");
    if (!(p.eta > 0.0 && p.eta < 1.0)) return fail(PSDP_E_INVALID, "params.eta must be in (0,1)");
    if (!(p.tol_kkt > 0.0) || !(p.tol_binary >= 0.0) || !(p.eps_hp > 0.0) || !(p.eig_tol > 0.0) ||
        !(p.cg_tol > 0.0) || !(p.alpha_min > 0.0) || !(p.alpha_max >= p.alpha_min) ||
        !(p.lambda_floor_rel >= 0.0) || !(p.sigma >= 0.0) || !std::isfinite(p.sigma))
        return fail(PSDP_E_INVALID, "params: tolerance out of range");
    if (p.sparse < -1 || p.sparse > 1) return fail(PSDP_E_INVALID, "params.sparse must be -1, 0 or 1");
    if (p.gemv_sym < -1 || p.gemv_sym > 1) return fail(PSDP_E_INVALID, "params.gemv_sym must be -1, 0 or 1");
    if (p.lanes < 0 || p.lanes > kMaxLanes) return fail(PSDP_E_INVALID, "params.lanes must be 0 (automatic) to 4");
    if (p.lambda_reuse < 0 || p.lambda_reuse > 1) return fail(PSDP_E_INVALID, "params.lambda_reuse must be 0 or 1");
    if (p.slots < 0) return fail(PSDP_E_INVALID, "params.slots must be >= 0");
    if (p.sparse == 1 && p.qx_dtype != PSDP_I8)
        return fail(PSDP_E_UNSUPPORTED, "sparse products need I8 operands");
    return PSDP_OK;
}

// Row starts of the compressed sparse rows of Q_off from per-row counts;
// false when there are 2^31 or more nonzeros (int32 row starts).
bool csr_rowptr(const std::vector<int64_t> &rownnz, std::vector<int32_t> *rowptr, int64_t *nnz) {
    rowptr->assign(rownnz.size() + 1, 0);
    int64_t s = 0;
    for (size_t i = 0; i < rownnz.size(); ++i) {
        s += rownnz[i];
        if (s > 2147483647ll) return false;
        (*rowptr)[i + 1] = (int32_t)s;
    }
    *nnz = s;
    return true;
}

// When the sparse products pay (measured on gfx950 against the digit
// products, whole solves): never at n <= 3000, even at 1% density (5-10%
// slower per sweep: the digit products of Q with under 10^7 entries are
// latency-bound and so are the gathers); at n = 8000 and 0.5% density 7%
// faster with one start and 21% with 16. Automatic use therefore needs
// n >= 4096 and a density of at most 1/64, and then takes a batch whose
// nonzeros x 2 x live columns (every live column counted as a two-half
// lambda_min column) stay within n^2 / 4.
constexpr int64_t kSparseMinN = 4096;
bool sparse_worth_building(int64_t n, int64_t nnz) { return n >= kSparseMinN && 64 * nnz <= n * n; }
bool sparse_batch(int64_t n, int64_t nnz, int live) { return (double)nnz * 2.0 * live <= 0.25 * (double)n * (double)n; }

// What the device checks found about one instance, in host terms. For
// integer data the magnitudes are integers; for real data they come back as
// the bit patterns of non-negative doubles.
struct InstFacts {
    bool real = false;
    double qmax = 0.0, offmax = 0.0, bmax = 0.0;
    uint64_t nonint_off = 0, non32_off = 0, non16_off = 0;
};

double bits_to_double(uint64_t u) {
    double d;
    std::memcpy(&d, &u, sizeof d);
    return d;
}

// Limits of one instance from its largest magnitudes: the objective bound
// and what each operand type represents exactly.
psdp_status check_limits(int64_t n, const InstFacts &f, const psdp_params &p) {
    const bool full = p.perturb == PSDP_PERTURB_FULL && p.sigma > 0.0;
    const long double bound = (long double)n * n * f.qmax + (long double)n * f.bmax;
    if (!f.real) {
        // |f(x)| <= n^2 max|Q| + n max|b| must stay below 2^62
        if (bound >= 4.611686018427388e18L) return fail(PSDP_E_OVERFLOW, "n^2 max|Q| + n max|b| >= 2^62");
        if (p.qx_dtype == PSDP_BF16 && full)
            return fail(PSDP_E_UNSUPPORTED, "FULL perturbation is not exact in bfloat16 operands");
        if (p.qx_dtype == PSDP_BF16 && f.offmax > 256)
            return fail(PSDP_E_UNSUPPORTED, "bfloat16 operands need |Q_ij| <= 256 off the diagonal");
        if (p.qx_dtype == PSDP_F32 && f.offmax > (double)(1u << 24))
            return fail(PSDP_E_UNSUPPORTED, "float operands need |Q_ij| <= 2^24 off the diagonal");
        if (p.qx_dtype == PSDP_I8 && f.offmax > 127)
            return fail(PSDP_E_UNSUPPORTED, "int8 operands need |Q_ij| <= 127 off the diagonal");
    } else {
        // every partial sum of the objective (and of the products) stays finite
        if (!(bound < 1e300L)) return fail(PSDP_E_OVERFLOW, "n^2 max|Q| + n max|b| >= 1e300");
        if (p.qx_dtype == PSDP_BF16 && (full || f.non16_off))
            return fail(PSDP_E_UNSUPPORTED, "bfloat16 operands need Q~ off the diagonal exact in bfloat16");
        if (p.qx_dtype == PSDP_F32 && f.non32_off)
            return fail(PSDP_E_UNSUPPORTED, "float operands need Q off the diagonal exact in float");
        if (p.qx_dtype == PSDP_I8 && f.nonint_off)
            return fail(PSDP_E_UNSUPPORTED, "int8 operands need integral |Q_ij| <= 127 off the diagonal");
    }
    if (p.qx_dtype == PSDP_I8 && full)
        return fail(PSDP_E_UNSUPPORTED, "FULL perturbation is not integer (int8 operands)");
    return PSDP_OK;
}

// Checks of one instance (integer or real data) on the device (device
// pointers, stream st), in this order: finite entries (real data), exact
// symmetry of Q, the limits above, X0 (nx entries, nullable) in [0,1], p0
// (nullable) finite. rownnz (optional): the off-diagonal nonzeros of every row.
template <typename T>
psdp_status check_instance(const T *Q, const T *b, int64_t n, const double *X0, int64_t nx, const double *p0,
                           const psdp_params &p, hipStream_t st, InstFacts *facts_out = nullptr,
                           std::vector<int64_t> *rownnz = nullptr) {
    constexpr bool kReal = std::is_same<T, double>::value;
    Arena ar;
    CheckOut *o;
    int32_t *rn = nullptr;
    HIPCHK(ar.get((void **)&o, sizeof(CheckOut)));
    if (rownnz) {
        HIPCHK(ar.get((void **)&rn, n * sizeof(int32_t)));
        HIPCHK(hipMemsetAsync(rn, 0, n * sizeof(int32_t), st));
    }
    HIPCHK(launch_check(Q, b, n, X0, nx, p0, o, rn, st));
    CheckOut h;
    HIPCHK(hipMemcpyAsync(&h, o, sizeof h, hipMemcpyDeviceToHost, st));
    std::vector<int32_t> hr;
    if (rownnz) {
        hr.resize(n);
        HIPCHK(hipMemcpyAsync(hr.data(), rn, n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    if (h.nonfinite) return fail(PSDP_E_NONFINITE, "Q and b must be finite");
    if (h.first_asym != ~0ull) {
        const long long i = (long long)(h.first_asym / (uint64_t)n), j = (long long)(h.first_asym % (uint64_t)n);
        char buf[128];
        snprintf(buf, sizeof buf, "Q[%lld][%lld] != Q[%lld][%lld]", i, j, j, i);
        return fail(PSDP_E_NOT_SYMMETRIC, buf);
    }
    InstFacts f;
    f.real = kReal;
    f.qmax = kReal ? bits_to_double(h.qmax) : (double)h.qmax;
    f.offmax = kReal ? bits_to_double(h.offmax) : (double)h.offmax;
    f.bmax = kReal ? bits_to_double(h.bmax) : (double)h.bmax;
    f.nonint_off = h.nonint_off;
    f.non32_off = h.non32_off;
    f.non16_off = h.non16_off;
    if (psdp_status s = check_limits(n, f, p)) return s;
    if (h.x0_bad) return fail(PSDP_E_NONFINITE, "X0 entries must lie in [0,1]");
    if (h.p0_bad) return fail(PSDP_E_NONFINITE, "p0 must be finite");
    if (facts_out) *facts_out = f;
    if (rownnz) rownnz->assign(hr.begin(), hr.end());
    return PSDP_OK;
}

__global__ void fill_p_kernel(double *p, const double *p0, int64_t n, int64_t ld, int ncol) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ld * ncol) return;
    const int64_t i = idx % ld;
    p[idx] = (p0 && i < n) ? p0[i] : 0.0;
}

constexpr int kMaxSplit = 8;

// Floating-point Q.X kernel for a batch: up to 64 columns the wave-streaming
// kernel (needs the FP32 copy of Q), above that the LDS-tiled GEMM with
// enough split-K for ~512 tiles. ncols: columns of the list; live: the live
// count of the last poll (est bounds the grid); MT: 64-row tiles of Q.
struct Pick { bool stream; int nt; int ks; int est; };
Pick pick_product(int B, int ncols, int live, int gemm_dtype, int gemm_variant, int64_t MT) {
    Pick pk{false, 4, 1, std::min({B, ncols + 16, live})};
    if (gemm_variant > 0) {
        pk.ks = std::min(kMaxSplit, gemm_variant & 0xff);
        pk.stream = (gemm_variant & 0x100) != 0 && gemm_dtype != PSDP_F64;
        pk.nt = 4;
        return pk;
    }
    if (ncols <= 64 && gemm_dtype != PSDP_F64) {
        pk.stream = true;
        pk.nt = ncols <= 16 ? 1 : (ncols <= 32 ? 2 : 4);
        pk.ks = 4;
        return pk;
    }
    const int tiles = (int)MT * std::max(1, (ncols + 63) / 64);
    pk.ks = std::max(1, std::min(kMaxSplit, (512 + tiles - 1) / tiles));
    return pk;
}

// Operand columns of a product from X (n x B, leading dimension n): entry
// converted to the operand type, padded with zeros to ld.
template <typename OpT>
__global__ void pack_operand_kernel(const double *X, int64_t n, int64_t ld, int B, OpT *op) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ld * B) return;
    const int64_t c = idx / ld, i = idx % ld;
    op[idx] = i < n ? from_f64<OpT>(X[c * n + i]) : from_f64<OpT>(0.0);
}

// Y = the K slices of U summed in slice order in FP64, as the column kernel
// reads them.
template <typename UT>
__global__ void sum_slices_kernel(const UT *U, int64_t slice, int ks, int64_t n, int64_t ld, int B, double *Y) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * B) return;
    const int64_t c = idx / n, i = idx % n;
    double u = to_f64<UT>(U[c * ld + i]);
    for (int t = 1; t < ks; ++t) u += to_f64<UT>(U[t * slice + c * ld + i]);
    Y[idx] = u;
}

__global__ void iota_list_kernel(int32_t *a, int B) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < B) a[i] = i;
    if (i == 0) a[B] = B;
}

struct Solver {
    Arena ar;
    Work w{};
    std::function<void(int, int)> repick;  // adapts the product kernels to the live counts
    std::function<int64_t()> config_key;   // identifies the current product configuration
    // enqueued before each batch of sweeps, after the configuration of the
    // batch is chosen (nullable)
    std::function<hipError_t(hipStream_t)> before_batch;
    bool sym_gemv = false;  // the single-instance product reads the packed upper tiles
    // when set, each poll also copies the first list_cap entries of the main
    // live list, and relist receives the list and its count (a superset of the
    // columns still live when it runs)
    std::function<hipError_t(const int32_t *, int)> relist;
    int32_t list_cap = 0;
    int optype = PSDP_F64, utype = PSDP_F64;
    int64_t *sweeps = nullptr;
    int64_t nmax = 0;  // largest column length (selects the per-thread unroll)
    int64_t rounds = 1;  // starts per column (queued starts run one after another)
    // live-list buffers by sweep parity and their counters
    // (cnt[2 p] main, cnt[2 p + 1] aux)
    int32_t *act[2] = {nullptr, nullptr}, *act_aux[2] = {nullptr, nullptr};
    int32_t *cnt = nullptr;
    // sparse copy of Q_off (I8) and whether the current batch uses it
    const int32_t *rowptr = nullptr;
    const uint32_t *pk = nullptr;
    int64_t nnz = 0;
    bool sparse_now = false;
    int64_t sparse_sweeps = 0;
};

// Points the work record at the lists of a sweep of parity p: the products
// read the lists of p, the column kernel fills those of 1 - p and clears the
// counters of p.
void set_parity(Solver &S, int p) {
    Work &w = S.w;
    w.active = S.act[p];
    w.active_aux = S.act_aux[p];
    w.nactive = S.cnt + 2 * p;
    w.nactive_aux = w.nactive + 1;
    w.next_active = S.act[1 - p];
    w.next_active_aux = S.act_aux[1 - p];
    w.next_cnt = S.cnt + 2 * (1 - p);
    w.clear_cnt = S.cnt + 2 * p;
}

// One default-priority stream per device for the solve work: the caller's
// stream may be the null stream, which cannot be captured into a graph.
// Created under the library lock and kept until the process ends.
hipError_t solve_stream(hipStream_t *out, int index = 0) {
    static std::map<std::pair<int, int>, hipStream_t> streams;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    auto it = streams.find({dev, index});
    if (it == streams.end()) {
        hipStream_t s;
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
        it = streams.emplace(std::make_pair(dev, index), s).first;
    }
    *out = it->second;
    return hipSuccess;
}

void fill_work_params(Work &w, const psdp_params &p) {
    w.clear_main = 1;
    w.clear_aux = 1;
    w.inner = p.inner;
    w.max_inner = p.max_inner;
    w.max_outer = p.max_outer;
    w.stall_outer = p.stall_outer;
    w.eig_maxit = p.eig_maxit;
    w.cg_maxit = p.cg_maxit;
    w.lambda_reuse = p.lambda_reuse;
    w.tol_kkt = p.tol_kkt;
    w.tol_binary = p.tol_binary;
    w.eta = p.eta;
    w.eps_hp = p.eps_hp;
    w.lambda_floor_rel = p.lambda_floor_rel;
    w.alpha_min = p.alpha_min;
    w.alpha_max = p.alpha_max;
    w.eig_tol = p.eig_tol;
    w.cg_tol = p.cg_tol;
}

// Allocates the per-column vectors for `total` doubles of column storage.
// Every buffer is cleared on the solve stream: that stream does not wait for
// the null stream, so a plain hipMemset could land after the first kernels.
psdp_status alloc_columns(Solver &S, int64_t total, const psdp_column_plan &pl, int64_t ksplit, hipStream_t st) {
    if (!pl.ok || !plan_holds_zero_col(pl))
        return fail(PSDP_E_INTERNAL, "a list-indexed buffer lacks the all-zero column");
    Work &w = S.w;
    const int ncol = pl.ncol;
    const int64_t ld = pl.ld;
    double **vecs[] = {&w.x, &w.xp, &w.g, &w.gp, &w.p, &w.v, &w.Av, &w.P, &w.AP, &w.w, &w.zx};
    for (double **v : vecs) {
        HIPCHK(S.ar.get((void **)v, total * sizeof(double)));
        HIPCHK(hipMemsetAsync(*v, 0, total * sizeof(double), st));
    }
    // integer path: int64 product slices; the operands are digit planes
    const size_t oe = w.i8 ? 0 : esize(S.optype), ue = w.i8 ? sizeof(int64_t) : esize(S.utype);
    if (oe) {
        HIPCHK(S.ar.get(&w.op, total * oe));
        HIPCHK(hipMemsetAsync(w.op, 0, total * oe, st));
    }
    w.ksplit = 1;
    w.slice = total;
    HIPCHK(S.ar.get(&w.U, ksplit * total * ue));
    HIPCHK(hipMemsetAsync(w.U, 0, ksplit * total * ue, st));
    if (w.i8) {
        // one extra all-zero column stands in for the unused rows of a digit tile
        if (pl.digit_cols < pl.zero_col + 1) return fail(PSDP_E_INTERNAL, "digit planes lack the all-zero column");
        const int64_t plane = (int64_t)pl.digit_cols * ld;
        HIPCHK(S.ar.get((void **)&w.dig, 4 * plane));
        HIPCHK(hipMemsetAsync(w.dig, 0, 4 * plane, st));
        HIPCHK(S.ar.get((void **)&w.dig_aux, 8 * plane));
        HIPCHK(hipMemsetAsync(w.dig_aux, 0, 8 * plane, st));
        HIPCHK(S.ar.get((void **)&w.U_lo, ksplit * total * sizeof(int64_t)));
        HIPCHK(hipMemsetAsync(w.U_lo, 0, ksplit * total * sizeof(int64_t), st));
    }
    for (int p = 0; p < 2; ++p) HIPCHK(S.ar.get((void **)&S.act[p], (size_t)pl.list_len * sizeof(int32_t)));
    HIPCHK(S.ar.get((void **)&S.cnt, 64));
    HIPCHK(hipMemsetAsync(S.cnt, 0, 64, st));
    HIPCHK(S.ar.get((void **)&S.sweeps, 64));
    HIPCHK(hipMemsetAsync(S.sweeps, 0, 64, st));
    w.sweeps = S.sweeps;
    w.ncol = ncol;
    w.col_base = 0;
    w.col_count = ncol;
    if (S.w.split) {
        w.ksplit_aux = 1;
        w.slice_aux = total;
        HIPCHK(S.ar.get((void **)&w.op_aux, total * sizeof(double)));
        HIPCHK(hipMemsetAsync(w.op_aux, 0, total * sizeof(double), st));
        HIPCHK(S.ar.get((void **)&w.U_aux, ksplit * total * sizeof(double)));
        HIPCHK(hipMemsetAsync(w.U_aux, 0, ksplit * total * sizeof(double), st));
        for (int p = 0; p < 2; ++p) HIPCHK(S.ar.get((void **)&S.act_aux[p], (size_t)pl.list_len * sizeof(int32_t)));
    } else {
        w.ksplit_aux = w.ksplit;
        w.slice_aux = w.slice;
        S.act_aux[0] = S.act[0];
        S.act_aux[1] = S.act[1];
    }
    set_parity(S, 0);
    return PSDP_OK;
}

// Timing of Q.X launches with HIP events on the solve stream.
struct QxTimer {
    bool on = false;
    std::vector<hipEvent_t> ev;
    size_t used = 0;
    double seconds = 0.0;
    int64_t launches = 0;
    ~QxTimer() {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
    hipError_t begin(hipStream_t st) {
        if (!on) return hipSuccess;
        if (used + 2 > ev.size()) {
            for (int q = 0; q < 64; ++q) {
                hipEvent_t e;
                hipError_t r = hipEventCreate(&e);
                if (r != hipSuccess) return r;
                ev.push_back(e);
            }
        }
        return hipEventRecord(ev[used], st);
    }
    hipError_t end(hipStream_t st) {
        if (!on) return hipSuccess;
        hipError_t r = hipEventRecord(ev[used + 1], st);
        used += 2;
        return r;
    }
    // Accumulates every recorded pair; call after the stream is synchronized.
    void add(const QxTimer &o) {
        seconds += o.seconds;
        launches += o.launches;
    }
    hipError_t collect() {
        for (size_t q = 0; q + 1 < used; q += 2) {
            float ms = 0.f;
            hipError_t r = hipEventElapsedTime(&ms, ev[q], ev[q + 1]);
            if (r != hipSuccess) return r;
            seconds += ms * 1e-3;
            launches += 1;
        }
        used = 0;
        return hipSuccess;
    }
};

// The sweeps of one launch sequence until no column is live: `apply`
// enqueues the Q.X product of the main live list, `apply_aux` (split
// precision only) the FP64 product of the lambda_min / CG list. Batches of
// poll_sweeps sweeps are replayed as graphs (one per product configuration:
// the kernels' arguments are fixed inside a graph); the live counts are read
// back after every batch and consumed one batch later (the next batch is
// queued first), and the product configuration is re-chosen from them.
// advance() queues one batch and processes the previous one's counts; a
// solve runs one loop to the end, or several loops (one per stream) in turn,
// so that their kernels overlap.
template <typename Apply, typename ApplyAux>
struct SweepLoop {
    Solver &S;
    const psdp_params &prm;
    QxTimer &tm, &ta, &ts;
    hipStream_t st;
    const Apply &apply;
    const ApplyAux &apply_aux;
    int32_t *host_cnt = nullptr, *host_list = nullptr;
    hipEvent_t evs[2] = {nullptr, nullptr};
    int64_t cap = 0, done_sweeps = 0;
    int batch = 0;
    bool finished = false, graphs = false;
    std::map<int64_t, hipGraphExec_t> execs;

    SweepLoop(Solver &S_, const psdp_params &prm_, QxTimer &tm_, QxTimer &ta_, QxTimer &ts_, hipStream_t st_,
              const Apply &apply_, const ApplyAux &apply_aux_)
        : S(S_), prm(prm_), tm(tm_), ta(ta_), ts(ts_), st(st_), apply(apply_), apply_aux(apply_aux_) {}
    ~SweepLoop() {
        for (auto &kv : execs) (void)hipGraphExecDestroy(kv.second);
        for (hipEvent_t e : evs)
            if (e) (void)hipEventDestroy(e);
        if (host_cnt) (void)hipHostFree(host_cnt);
        if (host_list) (void)hipHostFree(host_list);
    }

    psdp_status init() {
        HIPCHK(hipHostMalloc((void **)&host_cnt, 4 * sizeof(int32_t), hipHostMallocDefault));
        if (S.relist)
            HIPCHK(hipHostMalloc((void **)&host_list, 2 * (size_t)S.list_cap * sizeof(int32_t), hipHostMallocDefault));
        HIPCHK(hipEventCreateWithFlags(&evs[0], hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&evs[1], hipEventDisableTiming));
        // hard bound from the per-column caps (every sweep advances every live column)
        cap = ((int64_t)prm.cg_maxit + (int64_t)(prm.max_outer + 1) * ((int64_t)prm.eig_maxit + prm.max_inner + 2) + 2) *
              S.rounds;
        graphs = prm.graph != 0 && !tm.on;
        return PSDP_OK;
    }

    // sweep s reads the lists of parity s % 2 (the initial lists are parity 0)
    hipError_t enqueue_sweeps(int nb) {
        Work &w = S.w;
        for (int q = 0; q < nb; ++q) {
            set_parity(S, (int)((done_sweeps + q) & 1));
            hipError_t e;
            if ((e = tm.begin(st)) != hipSuccess) return e;
            if ((e = apply()) != hipSuccess) return e;
            if ((e = tm.end(st)) != hipSuccess) return e;
            if (w.split) {
                if ((e = ta.begin(st)) != hipSuccess) return e;
                if ((e = apply_aux()) != hipSuccess) return e;
                if ((e = ta.end(st)) != hipSuccess) return e;
            }
            if ((e = ts.begin(st)) != hipSuccess) return e;
            if ((e = launch_solver_step(S.optype, S.utype, w, S.nmax, st)) != hipSuccess) return e;
            if ((e = ts.end(st)) != hipSuccess) return e;
        }
        return hipSuccess;
    }

    psdp_status advance() {
        Work &w = S.w;
        const int nb = (int)std::min<int64_t>(prm.poll_sweeps, cap - done_sweeps);
        if (nb <= 0) return fail(PSDP_E_DEVICE, "sweep bound exceeded");
        if (S.before_batch) HIPCHK(S.before_batch(st));
        if (graphs && nb == prm.poll_sweeps) {
            const int64_t key = (S.config_key ? S.config_key() : 0) * 2 + (done_sweeps & 1);
            auto it = execs.find(key);
            if (it == execs.end()) {
                hipGraph_t g;
                HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                hipError_t ce = enqueue_sweeps(nb);
                hipError_t ee = hipStreamEndCapture(st, &g);
                if (ce != hipSuccess) return hipfail(ce, "graph capture");
                if (ee != hipSuccess) return hipfail(ee, "hipStreamEndCapture");
                hipGraphExec_t ex;
                hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (ie != hipSuccess) return hipfail(ie, "hipGraphInstantiate");
                it = execs.emplace(key, ex).first;
            }
            HIPCHK(hipGraphLaunch(it->second, st));
        } else {
            HIPCHK(enqueue_sweeps(nb));
        }
        done_sweeps += nb;
        if (S.sparse_now) S.sparse_sweeps += nb;
        set_parity(S, (int)(done_sweeps & 1));  // the lists the next sweep would read
        const int slot = batch & 1;
        HIPCHK(hipMemcpyAsync(host_cnt + 2 * slot, w.nactive, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        if (host_list)
            HIPCHK(hipMemcpyAsync(host_list + (size_t)slot * S.list_cap, w.active, (size_t)S.list_cap * sizeof(int32_t),
                                  hipMemcpyDeviceToHost, st));
        HIPCHK(hipEventRecord(evs[slot], st));
        if (batch > 0) {
            const int prev = slot ^ 1;
            HIPCHK(hipEventSynchronize(evs[prev]));
            if (host_cnt[2 * prev] + host_cnt[2 * prev + 1] == 0) finished = true;
            else {
                if (S.repick) S.repick(host_cnt[2 * prev], host_cnt[2 * prev + 1]);
                if (host_list) HIPCHK(S.relist(host_list + (size_t)prev * S.list_cap, host_cnt[2 * prev]));
            }
        }
        if ((tm.on && tm.used > 4096) || (ta.on && ta.used > 4096) || (ts.on && ts.used > 4096)) {
            HIPCHK(hipEventSynchronize(evs[slot]));
            HIPCHK(tm.collect());
            HIPCHK(ta.collect());
            HIPCHK(ts.collect());
        }
        ++batch;
        return PSDP_OK;
    }

    psdp_status finish() {
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(tm.collect());
        HIPCHK(ta.collect());
        HIPCHK(ts.collect());
        return PSDP_OK;
    }
};

template <typename Apply, typename ApplyAux>
psdp_status run_sweeps(Solver &S, const psdp_params &prm, QxTimer &tm, QxTimer &ta, QxTimer &ts, hipStream_t st,
                       const Apply &apply, const ApplyAux &apply_aux) {
    SweepLoop<Apply, ApplyAux> L(S, prm, tm, ta, ts, st, apply, apply_aux);
    if (psdp_status e = L.init()) return e;
    while (!L.finished)
        if (psdp_status e = L.advance()) return e;
    return L.finish();
}

void fill_stats(const std::vector<Col> &cols, int64_t sweeps, const QxTimer &tm, double flops_total,
                const QxTimer &ta, double aux_flops, const QxTimer &ts, psdp_stats *stats) {
    int64_t colsteps = 0;
    for (const Col &c : cols) colsteps += c.evals + c.aux;
    for (size_t c = 0; c < cols.size(); ++c) {
        psdp_stats &s = stats[c];
        std::memset(&s, 0, sizeof s);
        s.exit_reason = cols[c].exit_reason;
        s.outer_iters = cols[c].s;
        s.inner_iters = cols[c].evals;
        s.aux_matvecs = cols[c].aux;
        s.final_cret_rel = cols[c].final_rel;
        s.final_binary_gap = cols[c].final_bg;
        s.sweeps = sweeps;
        s.qx_seconds = tm.seconds;
        s.qx_flops = flops_total;
        s.qx_launches = tm.launches;
        s.aux_seconds = ta.seconds;
        s.aux_flops = aux_flops;
        s.step_seconds = ts.seconds;
        s.step_launches = ts.launches;
        s.column_steps = colsteps;
    }
}

// Algorithm 3 on B starts of one instance with integer (T = int32_t, obj
// int64) or real (T = double, obj FP64) data.
template <typename T, typename ObjT>
psdp_status solve_impl(const T *Q, const T *b, int64_t n, const double *X0, const double *p0, int32_t B,
                       const psdp_params *prm_in, uint8_t *xhat, ObjT *obj, double *X_out, int32_t *best,
                       psdp_stats *stats, double *trace, int32_t trace_cap, const double *alpha_in,
                       int32_t alpha_cap, hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_lock);
    g_err.clear();
    psdp_params prm;
    psdp_params_default(&prm);
    if (prm_in) {
        if (prm_in->struct_size != sizeof(psdp_params)) return fail(PSDP_E_INVALID, "params.struct_size");
        prm = *prm_in;
    }
    if (psdp_status s = check_params(prm)) return s;
    if (!Q || !b || !xhat || !obj) return fail(PSDP_E_INVALID, "null required pointer");
    if (n < 1 || B < 1) return fail(PSDP_E_INVALID, "n and B must be >= 1");
    if (!X0 && B != 1) return fail(PSDP_E_INVALID, "X0 = NULL needs B = 1");
    if (trace && trace_cap < 1) return fail(PSDP_E_INVALID, "trace_cap");
    if (alpha_in && alpha_cap < 1) return fail(PSDP_E_INVALID, "alpha_cap");
    if (alpha_in)
        for (int64_t q = 0; q < (int64_t)B * alpha_cap; ++q)
            if (!(std::isfinite(alpha_in[q]) && alpha_in[q] > 0.0))
                return fail(PSDP_E_INVALID, "alpha_in entries must be finite and positive");
    if (n > 65536) return fail(PSDP_E_UNSUPPORTED, "n > 65536");
    // validation on the device; a few words come back (the caller's stream is
    // synchronized, so the inputs are ready for the solve stream too)
    InstFacts facts;
    std::vector<int64_t> rownnz;
    const bool want_counts = prm.qx_dtype == PSDP_I8 && prm.sparse != 0;
    if (psdp_status s = check_instance(Q, b, n, X0, X0 ? n * B : 0, p0, prm, st, &facts,
                                       want_counts ? &rownnz : nullptr))
        return s;
    std::vector<int32_t> hrowptr;
    bool csr = false;
    int64_t csr_nnz = 0;
    if (want_counts) {
        int64_t nnz = 0;
        const bool fits = csr_rowptr(rownnz, &hrowptr, &nnz);
        if (!fits && prm.sparse == 1) return fail(PSDP_E_UNSUPPORTED, "sparse Q needs fewer than 2^31 nonzeros");
        csr = fits && (prm.sparse == 1 || sparse_worth_building(n, nnz));
        if (csr) csr_nnz = nnz;
    }
    if (B > 1 && prm.qx_dtype == PSDP_BF16)
        return fail(PSDP_E_UNSUPPORTED, "batched starts support F64 and F32 operands");
    // the inputs are ready (the stream was synchronized above); the solve runs
    // on the library's own stream and is synchronized before returning
    HIPCHK(solve_stream(&st));

    Solver S;
    const bool i8 = prm.qx_dtype == PSDP_I8;  // exact integer products, any B
    const bool batched = B > 1 || i8;
    const psdp_column_plan plan = plan_columns(n, B, prm, csr);
    const int32_t ncol = plan.ncol;
    const bool queued = ncol < B;
    const int64_t ld = plan.ld;
    S.optype = batched ? prm.qx_dtype : PSDP_F64;  // single instance: FP64 x, Q in qx_dtype
    S.utype = batched ? prm.qx_dtype : PSDP_F64;
    Work &w = S.w;
    S.nmax = n;
    fill_work_params(w, prm);
    // batched lower-precision products: lambda_min and CG keep FP64 operands
    w.split = (batched && prm.qx_dtype != PSDP_F64) ? 1 : 0;
    w.i8 = i8 ? 1 : 0;
    // Q~ off the diagonal is exact in FP32 for integers up to 2^24 unless a
    // FULL perturbation adds 2^-16-grid values to entries of 2^8 or more
    // (real data: every off-diagonal entry a float, and no FULL perturbation)
    const bool no_full = prm.perturb != PSDP_PERTURB_FULL || prm.sigma == 0.0;
    const bool q32_exact = facts.real ? (facts.non32_off == 0 && no_full)
                                      : (facts.offmax <= (double)(1 << 24) &&
                                         (no_full || facts.offmax + 3.5 * prm.sigma < 256.0));
    // Qop: operand of the main product; Qaux: operand of the FP64 products
    // (the exact FP32 copy widened in the kernel, or an FP64 copy)
    const int qtype = i8 ? PSDP_I8
                         : batched ? ((prm.qx_dtype == PSDP_F32 || q32_exact) ? PSDP_F32 : PSDP_F64) : prm.qx_dtype;
    int main_gemm = PSDP_F64, aux_gemm = PSDP_F64;
    if (batched) {
        main_gemm = prm.qx_dtype == PSDP_F32 ? PSDP_F32 : (q32_exact ? kGemmF32QF64 : PSDP_F64);
        aux_gemm = q32_exact ? kGemmF32QF64 : PSDP_F64;
    }
    void *Qop = nullptr;
    if (i8) {
        // int8 rows up to a multiple of kDigitRowsAlign: the digit kernel's row
        // blocks may run past ld into these zero rows
        const int64_t rows = (ld + kDigitRowsAlign - 1) / kDigitRowsAlign * kDigitRowsAlign;
        HIPCHK(S.ar.get(&Qop, rows * ld));
        HIPCHK(hipMemsetAsync(Qop, 0, rows * ld, st));
    } else {
        HIPCHK(S.ar.get(&Qop, ld * ld * esize(qtype)));
    }
    double *bd, *gam, *R, *dq;
    HIPCHK(S.ar.get((void **)&bd, ld * 8));
    HIPCHK(S.ar.get((void **)&gam, ld * 8));
    HIPCHK(S.ar.get((void **)&R, ld * 8));
    HIPCHK(S.ar.get((void **)&dq, ld * 8));
    HIPCHK(launch_prep_q(qtype, Q, n, ld, prm.perturb, prm.sigma, prm.seed, Qop, R, dq, st));
    if (csr) {
        // sparse rows of Q_off from the int8 copy (row starts counted on the host)
        int32_t *drp;
        uint32_t *dpk;
        HIPCHK(S.ar.get((void **)&drp, (n + 1) * sizeof(int32_t)));
        HIPCHK(S.ar.get((void **)&dpk, std::max<int64_t>(1, csr_nnz) * sizeof(uint32_t)));
        HIPCHK(hipMemcpyAsync(drp, hrowptr.data(), (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice, st));
        HIPCHK(launch_csr_fill((const int8_t *)Qop, ld, n, drp, dpk, st));
        S.rowptr = drp;
        S.pk = dpk;
        S.nnz = csr_nnz;
    }
    void *Qaux = Qop;
    if (w.split && !i8 && aux_gemm == PSDP_F64) {
        HIPCHK(S.ar.get(&Qaux, ld * ld * sizeof(double)));
        HIPCHK(launch_prep_q(PSDP_F64, Q, n, ld, prm.perturb, prm.sigma, prm.seed, Qaux, R, dq, st));
    }
    double *dgi, *lni;
    HIPCHK(S.ar.get((void **)&dgi, ld * 8));
    HIPCHK(S.ar.get((void **)&lni, ld * 8));
    HIPCHK(launch_gamma(b, R, dq, n, ld, bd, gam, dgi, lni, st));
    w.b = bd;
    w.gam = gam;
    w.R = R;
    w.dq = dq;
    w.dgi = dgi;
    w.lni = lni;
    Inst hin{n, ld, 0, Qop};
    HIPCHK(S.ar.get((void **)&w.inst, sizeof(Inst)));
    HIPCHK(hipMemcpyAsync(w.inst, &hin, sizeof(Inst), hipMemcpyHostToDevice, st));
    // column data
    const int kmax = (batched && !i8) ? kMaxSplit : 1;  // integer slices add into one buffer
    if (psdp_status s2 = alloc_columns(S, ld * ncol, plan, kmax, st)) return s2;
    if (S.rowptr) {
        // the operands' grid values as words, for the sparse products; like
        // the digit planes they hold one extra all-zero column (index ncol),
        // which empty list slots and the slots past the count name
        if (plan.word_cols < plan.zero_col + 1) return fail(PSDP_E_INTERNAL, "operand words lack the all-zero column");
        for (int32_t **pw : {&w.tw, &w.tw_hi, &w.tw_lo}) {
            HIPCHK(S.ar.get((void **)pw, ld * plan.word_cols * sizeof(int32_t)));
            HIPCHK(hipMemsetAsync(*pw, 0, ld * plan.word_cols * sizeof(int32_t), st));
        }
    }
    const int MT = (int)((ld + 63) / 64);
    // Product kernel per live count (the count comes from the last host poll,
    // so it is an estimate; every kernel covers all ncol columns regardless).
    // Columns move between the two lists from sweep to sweep but never come
    // back to life, so neither list outgrows the total live count of the
    // poll: the estimate is the list's count plus 16, at most that total.
    // up to 64 live columns the wave-streaming kernel (needs the FP32 copy of
    // Q), above that the LDS-tiled GEMM with enough split-K for ~512 tiles.
    auto pick = [&](int ncols, int live, int gemm_dtype) {
        if (!batched) return Pick{false, 4, 1, std::min({ncol, ncols + 16, live})};
        return pick_product(ncol, ncols, live, gemm_dtype, prm.gemm_variant, MT);
    };
    // Integer path: the columns may run as up to four lanes, concurrent
    // launch sequences on as many streams, each over its share of the columns
    // and of the starts with its own live lists, counters and queue (the step
    // kernels of one lane then overlap the products of another). Every start performs
    // the same arithmetic in any lane. Each lane picks its products' layouts
    // from its estimated live counts and their K slices from the blocks of
    // both products (they share one launch).
    struct Pick8 { int mt; int ks; int est; };
    struct Lane {
        Solver *S = nullptr;
        int ncols = 0;
        Pick8 p8m{}, p8a{};
        bool dirty_m = false, dirty_a = false;
        hipStream_t st = nullptr;
        QxTimer tm, ta, ts;
        // staging of the sparse products' operands (lanes run concurrently)
        int32_t *stg = nullptr, *stg_aux = nullptr;
        int64_t stg_passes = 0, stg_passes_aux = 0;
    };
    const int want = prm.lanes == 0 ? (ncol >= kLaneAutoCols ? 2 : 1) : prm.lanes;
    const int nlanes = i8 ? std::max(1, std::min({want, kMaxLanes, ncol})) : 1;
    // lane l runs columns [cb[l], cb[l + 1]) over starts [sb[l], sb[l + 1]):
    // start ranges in proportion to the columns, each holding at least its
    // lane's columns
    std::vector<int32_t> cb(nlanes + 1), sb(nlanes + 1);
    for (int l = 0; l <= nlanes; ++l) cb[l] = (int32_t)((int64_t)ncol * l / nlanes);
    sb[0] = 0;
    sb[nlanes] = B;
    for (int l = 1; l < nlanes; ++l) {
        const int32_t lo = sb[l - 1] + (cb[l] - cb[l - 1]), hi = B - (ncol - cb[l]);
        const int32_t prop = (int32_t)(((int64_t)B * cb[l] + ncol / 2) / ncol);
        sb[l] = std::max(lo, std::min(hi, prop));
    }
    const int32_t nc0 = cb[1];
    std::vector<std::unique_ptr<Solver>> extra;
    std::vector<std::unique_ptr<Lane>> lanes;
    for (int l = 0; l < nlanes; ++l) {
        if (l > 0) {
            extra.emplace_back(new Solver());
            extra.back()->rowptr = S.rowptr;
            extra.back()->pk = S.pk;
            extra.back()->nnz = S.nnz;
        }
        lanes.emplace_back(new Lane());
        lanes[l]->S = l == 0 ? &S : extra.back().get();
        lanes[l]->ncols = cb[l + 1] - cb[l];
        if (S.rowptr) {
            Lane &L = *lanes[l];
            L.stg_passes = sparse_stage_passes(L.ncols, 1);
            L.stg_passes_aux = sparse_stage_passes(L.ncols, 2);
            HIPCHK(S.ar.get((void **)&L.stg, L.stg_passes * ld * 16 * (int64_t)sizeof(int32_t)));
            HIPCHK(S.ar.get((void **)&L.stg_aux, L.stg_passes_aux * ld * 16 * (int64_t)sizeof(int32_t)));
        }
    }
    auto pick8 = [&](Lane &L, int cm, int ca) {
        L.p8m.est = std::min({L.ncols, cm + 16, cm + ca});
        L.p8a.est = std::min({L.ncols, ca + 16, cm + ca});
        const DigitChoice dc = digit_choice(n, ld, L.p8m.est, L.p8a.est);
        L.p8m.mt = dc.mt4;
        L.p8m.ks = dc.ks4;
        L.p8a.mt = dc.mt8;
        L.p8a.ks = dc.ks8;
        // sparse products while they cost less than the digit products; the
        // bound takes every live column as a two-half lambda_min column
        const int live = std::min(L.ncols, cm + ca);
        L.S->sparse_now = L.S->rowptr != nullptr && (prm.sparse == 1 || sparse_batch(n, L.S->nnz, live));
    };
    for (auto &L : lanes) pick8(*L, L->ncols, L->ncols);
    Pick pm = pick(ncol, ncol, main_gemm), pa = pick(ncol, ncol, aux_gemm);
    // integer path: the column kernel reads one buffer, whatever the
    // product's K slices
    w.ksplit = i8 ? 1 : pm.ks;
    w.ksplit_aux = i8 ? 1 : (w.split ? pa.ks : w.ksplit);
    std::vector<Col> hcol(ncol);
    for (int c = 0; c < ncol; ++c) {
        Col &cc = hcol[c];
        std::memset(&cc, 0, sizeof cc);
        cc.inst = 0;
        cc.n = n;
        cc.ld = ld;
        cc.off = (int64_t)c * ld;
        cc.ioff = 0;
        cc.id = c;
        int l = 0;
        while (c >= cb[l + 1]) ++l;
        cc.start = sb[l] + (c - cb[l]);
        cc.phase = PH_INNER;  // placeholder, set by the init kernel
    }
    HIPCHK(S.ar.get((void **)&w.col, ncol * sizeof(Col)));
    HIPCHK(hipMemcpyAsync(w.col, hcol.data(), ncol * sizeof(Col), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(fill_p_kernel, dim3((unsigned)((ld * ncol + 255) / 256)), dim3(256), 0, st, w.p, p0, n,
                       ld, ncol);
    if (queued) {
        S.rounds = (sb[1] + nc0 - 1) / nc0;
        int32_t *q;
        HIPCHK(S.ar.get((void **)&q, 64));
        HIPCHK(hipMemcpyAsync(q, &nc0, sizeof(int32_t), hipMemcpyHostToDevice, st));
        HIPCHK(S.ar.get((void **)&w.xfin, (size_t)n * B * sizeof(double)));
        HIPCHK(S.ar.get((void **)&w.fin, (size_t)B * sizeof(Col)));
        w.queue = q;
        w.nstart = sb[1];
        w.X0 = X0;
        w.p0 = p0;
    }
    HIPCHK(hipGetLastError());
    if (trace) {
        // seeded with the caller's records, so that the unused ones come back untouched
        HIPCHK(S.ar.get((void **)&w.trace, (size_t)B * trace_cap * 6 * sizeof(double)));
        HIPCHK(hipMemcpyAsync(w.trace, trace, (size_t)B * trace_cap * 6 * sizeof(double), hipMemcpyHostToDevice,
                              st));
        w.trace_cap = trace_cap;
    }
    if (alpha_in) {
        double *da;
        HIPCHK(S.ar.get((void **)&da, (size_t)B * alpha_cap * sizeof(double)));
        HIPCHK(hipMemcpyAsync(da, alpha_in, (size_t)B * alpha_cap * sizeof(double), hipMemcpyHostToDevice, st));
        w.alpha_in = da;
        w.alpha_cap = alpha_cap;
    }
    // optional per-phase timing of the column kernel (diagnostics, env PSDP_PHASE_PROFILE=1)
    const bool phase_prof = getenv("PSDP_PHASE_PROFILE") != nullptr;
    if (phase_prof) {
        HIPCHK(S.ar.get((void **)&w.phase_prof, 16 * sizeof(unsigned long long)));
        HIPCHK(hipMemsetAsync(w.phase_prof, 0, 16 * sizeof(unsigned long long), st));
    }
    lanes[0]->st = st;
    for (int l = 1; l < nlanes; ++l) {
        // lane l: the shared buffers and parameters, its own lists,
        // counters, sweep counter and queue, and columns [cb[l], cb[l + 1])
        Solver &LS = *lanes[l]->S;
        const int32_t ncl = cb[l + 1] - cb[l];
        LS.w = w;
        LS.optype = S.optype;
        LS.utype = S.utype;
        LS.nmax = S.nmax;
        for (int p = 0; p < 2; ++p) {
            HIPCHK(S.ar.get((void **)&LS.act[p], (size_t)plan.list_len * sizeof(int32_t)));
            if (w.split) HIPCHK(S.ar.get((void **)&LS.act_aux[p], (size_t)plan.list_len * sizeof(int32_t)));
            else LS.act_aux[p] = LS.act[p];
        }
        HIPCHK(S.ar.get((void **)&LS.cnt, 64));
        HIPCHK(hipMemsetAsync(LS.cnt, 0, 64, st));
        HIPCHK(S.ar.get((void **)&LS.sweeps, 64));
        HIPCHK(hipMemsetAsync(LS.sweeps, 0, 64, st));
        LS.w.sweeps = LS.sweeps;
        set_parity(LS, 0);
        LS.w.col_base = cb[l];
        LS.w.col_count = ncl;
        if (queued) {
            const int32_t qv = sb[l] + ncl;
            int32_t *ql;
            HIPCHK(S.ar.get((void **)&ql, 64));
            HIPCHK(hipMemcpyAsync(ql, &qv, sizeof(int32_t), hipMemcpyHostToDevice, st));
            LS.w.queue = ql;
            LS.w.nstart = sb[l + 1];
            LS.rounds = (sb[l + 1] - sb[l] + ncl - 1) / ncl;
        }
        HIPCHK(solve_stream(&lanes[l]->st, l));
    }
    w.col_count = nc0;
    for (auto &L : lanes) {
        HIPCHK(launch_solver_init(S.optype, L->S->w, X0, X0 ? 0 : 1, st));
        HIPCHK(launch_compact(L->S->w, st));
        L->tm.on = L->ta.on = L->ts.on = prm.timing != 0;
    }
    if (nlanes > 1) {
        // the other lanes start once the set-up on the first stream is done
        hipEvent_t ready;
        HIPCHK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
        hipError_t e = hipEventRecord(ready, st);
        for (int l = 1; l < nlanes && e == hipSuccess; ++l) e = hipStreamWaitEvent(lanes[l]->st, ready, 0);
        (void)hipEventDestroy(ready);
        HIPCHK(e);
    }
    QxTimer tm, ta, ts;
    tm.on = ta.on = ts.on = prm.timing != 0;
    auto none = []() { return hipSuccess; };
    psdp_status rs;
    if (i8) {
        const int8_t *Q8 = (const int8_t *)Qop;
        for (auto &Lp : lanes) {
            Lane *L = Lp.get();
            Solver &LS = *L->S;
            LS.config_key = [&LS, L]() {
                return ((int64_t)L->p8m.mt | ((int64_t)L->p8m.ks << 5) | ((int64_t)L->p8a.mt << 9) |
                        ((int64_t)L->p8a.ks << 14) | ((int64_t)L->p8m.est << 18) | ((int64_t)L->p8a.est << 38)) * 2 +
                       (LS.sparse_now ? 1 : 0);
            };
            LS.repick = [&pick8, L](int cm, int ca) { pick8(*L, cm, ca); };
            // a product written by one K slice overwrites its outputs, so the
            // column kernel clears what it read only when the next product of
            // that kind adds its slices (K slices > 1); before such a batch the
            // lane's columns of the buffers are cleared here if the previous
            // batch left values in them
            LS.before_batch = [&LS, L, ld](hipStream_t s) -> hipError_t {
                Work &lw = LS.w;
                const bool zm = !LS.sparse_now && L->p8m.ks > 1, za = !LS.sparse_now && L->p8a.ks > 1;
                lw.clear_main = zm ? 1 : 0;
                lw.clear_aux = za ? 1 : 0;
                hipError_t e = hipSuccess;
                const int64_t off = (int64_t)lw.col_base * ld;
                const size_t bytes = (size_t)ld * lw.col_count * sizeof(int64_t);
                if (zm && L->dirty_m) e = hipMemsetAsync((int64_t *)lw.U + off, 0, bytes, s);
                if (e == hipSuccess && za && L->dirty_a) e = hipMemsetAsync(lw.U_aux + off, 0, bytes, s);
                if (e == hipSuccess && za && L->dirty_a) e = hipMemsetAsync(lw.U_lo + off, 0, bytes, s);
                L->dirty_m = !zm;
                L->dirty_a = !za;
                return e;
            };
        }
        // both products of a lane's sweep in one launch (timed as one launch
        // when timing = 1)
        auto make_apply = [&](Lane *L) {
            return [&, L]() -> hipError_t {
                Solver &LS = *L->S;
                const Work &lw = LS.w;
                if (LS.sparse_now) {
                    const SparseJob sm{L->p8m.est > 0, LS.rowptr, LS.pk, n, lw.tw, nullptr, ld, lw.active, lw.nactive,
                                       ncol, (int64_t *)lw.U, nullptr, ld, L->stg, L->stg_passes, L->ncols};
                    const SparseJob sa{L->p8a.est > 0, LS.rowptr, LS.pk, n, lw.tw_hi, lw.tw_lo, ld, lw.active_aux,
                                       lw.nactive_aux, ncol, (int64_t *)lw.U_aux, lw.U_lo, ld,
                                       L->stg_aux, L->stg_passes_aux, L->ncols};
                    return launch_sparse(&sm, &sa, L->st);
                }
                const DigitJob jm{lw.dig, lw.active, lw.nactive, (int64_t *)lw.U, nullptr, ncol,
                                  L->p8m.ks, L->p8m.mt, L->p8m.est};
                const DigitJob ja{lw.dig_aux, lw.active_aux, lw.nactive_aux, (int64_t *)lw.U_aux, lw.U_lo, ncol,
                                  L->p8a.ks, L->p8a.mt, L->p8a.est};
                return launch_digit(Q8, ld, n, ld, &jm, &ja, L->st);
            };
        };
        using ApplyT = decltype(make_apply(nullptr));
        using LoopT = SweepLoop<ApplyT, decltype(none)>;
        std::vector<ApplyT> applies;
        applies.reserve(lanes.size());
        std::vector<std::unique_ptr<LoopT>> loops;
        rs = PSDP_OK;
        for (auto &L : lanes) {
            applies.push_back(make_apply(L.get()));
            loops.emplace_back(new LoopT(*L->S, prm, L->tm, L->ta, L->ts, L->st, applies.back(), none));
            if (rs == PSDP_OK) rs = loops.back()->init();
        }
        // the lanes in turn, one batch each: a lane's next batch is queued
        // before its previous batch's counts are waited for
        for (bool more = true; rs == PSDP_OK && more;) {
            more = false;
            for (auto &L : loops) {
                if (L->finished) continue;
                rs = L->advance();
                if (rs != PSDP_OK) break;
                more = more || !L->finished;
            }
        }
        for (auto &L : loops) {
            const psdp_status f = L->finish();
            if (rs == PSDP_OK) rs = f;
        }
        for (auto &L : lanes) {
            tm.add(L->tm);
            ta.add(L->ta);
            ts.add(L->ts);
        }
    } else if (!batched) {
        // one column: the row-by-row GEMV, or the product from the unique
        // half of Q (packed upper tiles) once Q outgrows the caches
        const bool sym = prm.gemv_sym == 1 || (prm.gemv_sym == -1 && n >= kSymAutoN);
        SymTiles sy{};
        if (sym) {
            sy.nb = symv_blocks(n);
            sy.ntiles = (int64_t)sy.nb * (sy.nb + 1) / 2;
            const std::vector<int32_t> tl = symv_tile_list(sy.nb);
            void *P;
            int2 *tiles;
            HIPCHK(S.ar.get(&P, symv_packed_elems(sy.nb) * esize(qtype)));
            HIPCHK(S.ar.get((void **)&tiles, tl.size() * sizeof(int32_t)));
            HIPCHK(hipMemcpyAsync(tiles, tl.data(), tl.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
            HIPCHK(S.ar.get((void **)&sy.D, sy.ntiles * 128 * sizeof(double)));
            HIPCHK(S.ar.get((void **)&sy.T, sy.ntiles * 128 * sizeof(double)));
            sy.P = P;
            sy.tiles = tiles;
            HIPCHK(launch_symv_pack(qtype, Qop, ld, sy, st));
            S.sym_gemv = true;
        }
        rs = run_sweeps(
            S, prm, tm, ta, ts, st,
            [&]() {
                if (!sym) return launch_gemv(prm.qx_dtype, &hin, 1, w, 1, st);
                sy.live = w.nactive;
                return launch_symv(prm.qx_dtype, sy, (const double *)w.op, ld, n, (double *)w.U, st);
            },
            none);
    } else {
        const bool merge = w.split && prm.timing == 0 && main_gemm == PSDP_F32 && aux_gemm == kGemmF32QF64;
        S.config_key = [&]() {
            return (int64_t)pm.stream | ((int64_t)pm.nt << 1) | ((int64_t)pm.ks << 4) | ((int64_t)pa.stream << 9) |
                   ((int64_t)pa.nt << 10) | ((int64_t)pa.ks << 13) | ((int64_t)pm.est << 20) |
                   ((int64_t)pa.est << 32);
        };
        S.repick = [&](int cm, int ca) {
            pm = pick(cm, cm + ca, main_gemm);
            pa = pick(ca, cm + ca, aux_gemm);
            w.ksplit = pm.ks;
            w.ksplit_aux = w.split ? pa.ks : w.ksplit;
        };
        rs = run_sweeps(
            S, prm, tm, ta, ts, st,
            [&]() {
                // split precision with both lists on the streaming kernel: one
                // launch for both products (kept apart when every launch is timed)
                if (merge && pm.stream && pa.stream)
                    return launch_stream2(Qop, ld, w.op, w.U, w.active, w.nactive, w.slice, w.ksplit, pm.nt,
                                          w.op_aux, w.U_aux, w.active_aux, w.nactive_aux, w.slice_aux,
                                          w.ksplit_aux, pa.nt, pm.est, pa.est, st);
                if (pm.stream)
                    return launch_stream(main_gemm, Qop, ld, w.op, w.U, w.active, w.nactive, w.slice, w.ksplit,
                                         pm.est, pm.nt, st);
                return launch_gemm(main_gemm, Qop, ld, w.op, w.U, w.active, w.nactive, w.slice, w.ksplit, ncol, st);
            },
            [&]() {
                if (merge && pm.stream && pa.stream) return hipSuccess;
                if (pa.stream)
                    return launch_stream(aux_gemm, Qaux, ld, w.op_aux, w.U_aux, w.active_aux, w.nactive_aux,
                                         w.slice_aux, w.ksplit_aux, pa.est, pa.nt, st);
                return launch_gemm(aux_gemm, Qaux, ld, w.op_aux, w.U_aux, w.active_aux, w.nactive_aux,
                                   w.slice_aux, w.ksplit_aux, ncol, st);
            });
    }
    if (rs != PSDP_OK) return rs;
    if (phase_prof) {
        unsigned long long hp[16];
        HIPCHK(hipMemcpyAsync(hp, w.phase_prof, sizeof hp, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        int rate_khz = 100000;
        (void)hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, 0);
        const char *nm[5] = {"done", "cg", "eig0", "eig", "inner"};
        for (int q = 1; q < 5; ++q)
            if (hp[3 * q + 1])
                fprintf(stderr, "phase %-5s n=%llu avg %.2f us max %.2f us\n", nm[q], hp[3 * q + 1],
                        1e3 * (double)hp[3 * q] / hp[3 * q + 1] / rate_khz, 1e3 * (double)hp[3 * q + 2] / rate_khz);
    }
    // rounding and exact objective on the original data; with queued starts
    // the final iterates and records were saved per start as each one ended
    const double *Xf = queued ? w.xfin : w.x;
    const int64_t ldf = queued ? n : ld;
    if constexpr (std::is_same<T, double>::value) {
        int64_t *acc;
        HIPCHK(S.ar.get((void **)&acc, (size_t)B * kObjAccWords * sizeof(int64_t)));
        HIPCHK(hipMemsetAsync(acc, 0, (size_t)B * kObjAccWords * sizeof(int64_t), st));
        HIPCHK(launch_round_objective(Q, b, n, Xf, ldf, B, xhat, n, obj, acc, st));
    } else {
        int64_t *partial;
        const int64_t nblk = (n + 15) / 16;
        HIPCHK(S.ar.get((void **)&partial, nblk * B * sizeof(int64_t)));
        HIPCHK(launch_round_objective(Q, b, n, Xf, ldf, B, xhat, n, obj, partial, st));
    }
    if (X_out)
        HIPCHK(hipMemcpy2DAsync(X_out, n * sizeof(double), Xf, ldf * sizeof(double), n * sizeof(double), B,
                                hipMemcpyDeviceToDevice, st));
    hcol.resize(B);
    HIPCHK(hipMemcpyAsync(hcol.data(), queued ? w.fin : w.col, B * sizeof(Col), hipMemcpyDeviceToHost, st));
    std::vector<int64_t> lane_sweeps(1 + extra.size(), 0);
    HIPCHK(hipMemcpyAsync(&lane_sweeps[0], S.sweeps, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    for (size_t l = 0; l < extra.size(); ++l)
        HIPCHK(hipMemcpyAsync(&lane_sweeps[l + 1], extra[l]->sweeps, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    std::vector<ObjT> hobj;
    if (best) {
        hobj.resize(B);
        HIPCHK(hipMemcpyAsync(hobj.data(), obj, B * sizeof(ObjT), hipMemcpyDeviceToHost, st));
    }
    if (trace)
        HIPCHK(hipMemcpyAsync(trace, w.trace, (size_t)B * trace_cap * 6 * sizeof(double),
                              hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const int64_t nsweeps = *std::max_element(lane_sweeps.begin(), lane_sweeps.end());
    if (best) {
        int32_t bi = 0;
        for (int c = 1; c < B; ++c)
            if (hobj[c] < hobj[bi]) bi = c;
        *best = bi;
    }
    if (stats) {
        double flops = 0.0, aflops = 0.0;
        for (const Col &cc : hcol) {
            // the integer path times both products in one launch
            const bool apart = w.split && !w.i8;
            flops += 2.0 * (double)n * (double)n * (double)(apart ? cc.evals : cc.evals + cc.aux);
            aflops += apart ? 2.0 * (double)n * (double)n * (double)cc.aux : 0.0;
        }
        fill_stats(hcol, nsweeps, tm, flops, ta, aflops, ts, stats);
        int64_t ssw = S.sparse_sweeps;
        for (const auto &X : extra) ssw = std::max(ssw, X->sparse_sweeps);
        for (int64_t c = 0; c < B; ++c) stats[c].sparse_sweeps = ssw;
    }
    return PSDP_OK;
}

}  // namespace

namespace psdp {
// The thread-local error detail of psdp_last_error, for the entry points of
// other translation units.
psdp_status set_error(psdp_status s, const char *msg) {
    g_err = msg ? msg : "";
    return s;
}
}  // namespace psdp

// ===========================================================================

extern "C" {

void psdp_params_default(psdp_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->struct_size = sizeof(psdp_params);
    p->inner = PSDP_INNER_PABB;
    p->qx_dtype = PSDP_F64;
    p->perturb = PSDP_PERTURB_NONE;
    p->max_inner = 10000;
    p->max_outer = 1000;
    p->stall_outer = 2;
    p->eig_maxit = 500;
    p->cg_maxit = 500;
    p->timing = 0;
    p->poll_sweeps = 64;
    p->gemm_variant = -1;
    p->graph = 1;
    p->sparse = -1;
    p->gemv_sym = -1;
    p->lanes = 0;
    p->lambda_reuse = 1;
    p->slots = 0;
    p->tol_kkt = 1e-5;
    p->tol_binary = 1e-5;
    p->eta = 0.999;
    p->eps_hp = 1e-8;
    p->lambda_floor_rel = 1e-8;
    p->alpha_min = 1e-30;
    p->alpha_max = 1e30;
    p->sigma = 0.0;
    p->eig_tol = 1e-7;
    p->cg_tol = 1e-12;
    p->seed = 0;
}

const char *psdp_status_string(psdp_status s) {
    switch (s) {
        case PSDP_OK: return "ok";
        case PSDP_E_INVALID: return "invalid argument";
        case PSDP_E_NOT_SYMMETRIC: return "Q is not symmetric";
        case PSDP_E_NONFINITE: return "non-finite or out-of-range input";
        case PSDP_E_OVERFLOW: return "objective bound overflows int64";
        case PSDP_E_DEVICE: return "HIP device error";
        case PSDP_E_NOMEM: return "out of device memory";
        case PSDP_E_UNSUPPORTED: return "unsupported combination";
        case PSDP_E_INTERNAL: return "internal bookkeeping check failed";
    }
    return "unknown status";
}

const char *psdp_last_error(void) { return g_err.c_str(); }

int32_t psdp_version(void) { return 10000; }

psdp_status psdp_plan_columns(int64_t n, int32_t B, const psdp_params *prm_in, int32_t sparse_copy,
                              psdp_column_plan *out) {
    g_err.clear();
    if (!out) return fail(PSDP_E_INVALID, "null out");
    if (n < 1 || n > 65536 || B < 1) return fail(PSDP_E_INVALID, "n must be in [1, 65536] and B >= 1");
    psdp_params prm;
    psdp_params_default(&prm);
    if (prm_in) {
        if (prm_in->struct_size != sizeof(psdp_params)) return fail(PSDP_E_INVALID, "params.struct_size");
        prm = *prm_in;
    }
    if (psdp_status s = check_params(prm)) return s;
    *out = plan_columns(n, B, prm, sparse_copy != 0);
    return PSDP_OK;
}

psdp_status psdp_solve_i32_ex(const int32_t *Q, const int32_t *b, int64_t n, const double *X0,
                              const double *p0, int32_t B, const psdp_params *prm, uint8_t *xhat,
                              int64_t *obj, double *X_out, int32_t *best, psdp_stats *stats,
                              double *trace, int32_t trace_cap, const double *alpha_in, int32_t alpha_cap,
                              hipStream_t st) {
    return solve_impl<int32_t, int64_t>(Q, b, n, X0, p0, B, prm, xhat, obj, X_out, best, stats, trace,
                                        trace_cap, alpha_in, alpha_cap, st);
}

psdp_status psdp_solve_i32(const int32_t *Q, const int32_t *b, int64_t n, const double *X0,
                           const double *p0, int32_t B, const psdp_params *prm, uint8_t *xhat,
                           int64_t *obj, double *X_out, int32_t *best, psdp_stats *stats,
                           hipStream_t st) {
    return solve_impl<int32_t, int64_t>(Q, b, n, X0, p0, B, prm, xhat, obj, X_out, best, stats, nullptr, 0,
                                        nullptr, 0, st);
}

psdp_status psdp_solve_f64_ex(const double *Q, const double *b, int64_t n, const double *X0,
                              const double *p0, int32_t B, const psdp_params *prm, uint8_t *xhat,
                              double *obj, double *X_out, int32_t *best, psdp_stats *stats,
                              double *trace, int32_t trace_cap, const double *alpha_in, int32_t alpha_cap,
                              hipStream_t st) {
    return solve_impl<double, double>(Q, b, n, X0, p0, B, prm, xhat, obj, X_out, best, stats, trace,
                                      trace_cap, alpha_in, alpha_cap, st);
}

psdp_status psdp_solve_f64(const double *Q, const double *b, int64_t n, const double *X0,
                           const double *p0, int32_t B, const psdp_params *prm, uint8_t *xhat,
                           double *obj, double *X_out, int32_t *best, psdp_stats *stats,
                           hipStream_t st) {
    return solve_impl<double, double>(Q, b, n, X0, p0, B, prm, xhat, obj, X_out, best, stats, nullptr, 0,
                                      nullptr, 0, st);
}

psdp_status psdp_solve_group_i32(int32_t count, const int64_t *n, const int32_t *const *Q,
                                 const int32_t *const *b, const uint64_t *seeds, const double *sigmas,
                                 const psdp_params *prm_in, uint8_t *const *xhat, int64_t *obj,
                                 psdp_stats *stats, hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_lock);
    g_err.clear();
    psdp_params prm;
    psdp_params_default(&prm);
    if (prm_in) {
        if (prm_in->struct_size != sizeof(psdp_params)) return fail(PSDP_E_INVALID, "params.struct_size");
        prm = *prm_in;
    }
    if (psdp_status s = check_params(prm)) return s;
    if (count < 1 || !n || !Q || !b || !xhat || !obj) return fail(PSDP_E_INVALID, "null or empty group");
    if (prm.qx_dtype == PSDP_I8) return fail(PSDP_E_UNSUPPORTED, "the group solve takes F64, F32 or BF16 operands");
    for (int i = 0; i < count; ++i) {
        if (n[i] < 1 || n[i] > 65536) return fail(PSDP_E_INVALID, "instance size out of range");
        if (!Q[i] || !b[i] || !xhat[i]) return fail(PSDP_E_INVALID, "null instance pointer");
    }
    // per-instance perturbation scale (sigmas) or the parameters' one
    auto sigma_of = [&](int i) { return sigmas ? sigmas[i] : prm.sigma; };
    for (int i = 0; i < count; ++i)
        if (!(sigma_of(i) >= 0.0) || !std::isfinite(sigma_of(i)))
            return fail(PSDP_E_INVALID, "instance " + std::to_string(i) + ": sigma must be finite and >= 0");
    for (int i = 0; i < count; ++i) {
        psdp_params pi = prm;
        pi.sigma = sigma_of(i);
        if (psdp_status s = check_instance(Q[i], b[i], n[i], nullptr, 0, nullptr, pi, st)) {
            g_err = "instance " + std::to_string(i) + ": " + g_err;
            return s;
        }
    }
    HIPCHK(solve_stream(&st));
    Solver S;
    S.optype = PSDP_F64;
    S.utype = PSDP_F64;
    Work &w = S.w;
    fill_work_params(w, prm);
    for (int i = 0; i < count; ++i) S.nmax = std::max<int64_t>(S.nmax, n[i]);
    std::vector<int64_t> ld(count), off(count + 1, 0), rowstart(count + 1, 0);
    for (int i = 0; i < count; ++i) {
        ld[i] = padld(n[i]);
        off[i + 1] = off[i] + ld[i];
        rowstart[i + 1] = rowstart[i] + (n[i] + 3) / 4;  // units of 4 rows of the group product
    }
    const int64_t total = off[count];
    double *bd, *gam, *R, *dq, *dgi, *lni;
    HIPCHK(S.ar.get((void **)&bd, total * 8));
    HIPCHK(S.ar.get((void **)&gam, total * 8));
    HIPCHK(S.ar.get((void **)&R, total * 8));
    HIPCHK(S.ar.get((void **)&dq, total * 8));
    HIPCHK(S.ar.get((void **)&dgi, total * 8));
    HIPCHK(S.ar.get((void **)&lni, total * 8));
    std::vector<Inst> hin(count);
    for (int i = 0; i < count; ++i) {
        void *Qop;
        HIPCHK(S.ar.get(&Qop, ld[i] * ld[i] * esize(prm.qx_dtype)));
        const uint64_t seed = seeds ? seeds[i] : prm.seed;
        HIPCHK(launch_prep_q(prm.qx_dtype, Q[i], n[i], ld[i], prm.perturb, sigma_of(i), seed, Qop, R + off[i],
                             dq + off[i], st));
        HIPCHK(launch_gamma(b[i], R + off[i], dq + off[i], n[i], ld[i], bd + off[i], gam + off[i], dgi + off[i],
                            lni + off[i], st));
        hin[i] = Inst{n[i], ld[i], off[i], Qop};
    }
    w.b = bd;
    w.gam = gam;
    w.R = R;
    w.dq = dq;
    w.dgi = dgi;
    w.lni = lni;
    HIPCHK(S.ar.get((void **)&w.inst, count * sizeof(Inst)));
    HIPCHK(hipMemcpyAsync(w.inst, hin.data(), count * sizeof(Inst), hipMemcpyHostToDevice, st));
    if (psdp_status s2 = alloc_columns(S, total, plan_group(count), 1, st)) return s2;
    std::vector<Col> hcol(count);
    for (int i = 0; i < count; ++i) {
        Col &cc = hcol[i];
        std::memset(&cc, 0, sizeof cc);
        cc.inst = i;
        cc.n = n[i];
        cc.ld = ld[i];
        cc.off = off[i];
        cc.ioff = off[i];
        cc.id = i;
        cc.start = i;
        cc.phase = PH_INNER;
    }
    HIPCHK(S.ar.get((void **)&w.col, count * sizeof(Col)));
    HIPCHK(hipMemcpyAsync(w.col, hcol.data(), count * sizeof(Col), hipMemcpyHostToDevice, st));
    int64_t *drow;
    HIPCHK(S.ar.get((void **)&drow, (count + 1) * sizeof(int64_t)));
    HIPCHK(hipMemcpyAsync(drow, rowstart.data(), (count + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
    std::vector<int32_t> unitcol(rowstart[count]);  // the column of every unit of 4 rows
    for (int i = 0; i < count; ++i)
        std::fill(unitcol.begin() + rowstart[i], unitcol.begin() + rowstart[i + 1], i);
    int32_t *dunit;
    HIPCHK(S.ar.get((void **)&dunit, unitcol.size() * sizeof(int32_t)));
    HIPCHK(hipMemcpyAsync(dunit, unitcol.data(), unitcol.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    // The product from the unique halves of the Q_i (packed 128 x 128 upper
    // tiles, each read once for its row and column parts; the same tile and
    // reduction order as the single-instance product, so each instance's
    // result equals its single-instance tile product) by the rule above or
    // when asked for (psdp_params.gemv_sym); otherwise the row-by-row group
    // GEMV.
    int64_t stored = 0;
    for (int i = 0; i < count; ++i) stored += ld[i] * ld[i] * esize(prm.qx_dtype);
    std::vector<int64_t> tbase(count + 1, 0);
    for (int i = 0; i < count; ++i) {
        const int64_t nb = symv_blocks(n[i]);
        tbase[i + 1] = tbase[i] + nb * (nb + 1) / 2;
    }
    const bool sym = (prm.gemv_sym == 1 ||
                      (prm.gemv_sym == -1 && (stored >= kSymAutoGroupBytes || S.nmax >= kSymAutoN))) &&
                     tbase[count] < INT32_MAX;
    SymGroup sg{};
    std::vector<SymGroupTile> hlist;
    std::vector<SymGroupRow> hrows;
    std::map<int, std::vector<int32_t>> tile_lists;  // per tile-row count; kept until the copies are done
    auto build_sym = [&](const std::vector<int32_t> &ids) {
        hlist.clear();
        hrows.clear();
        for (int32_t id : ids) {
            const int nb = symv_blocks(n[id]);
            int32_t t = (int32_t)tbase[id];
            for (int bi = 0; bi < nb; ++bi) {
                for (int bj = bi; bj < nb; ++bj) hlist.push_back(SymGroupTile{t++, id, bi, bj, off[id], ld[id]});
                hrows.push_back(SymGroupRow{id, bi, off[id], n[id], tbase[id]});
            }
        }
    };
    SymGroupTile *dlist = nullptr;
    SymGroupRow *drows = nullptr;
    if (sym) {
        const int64_t ntot = tbase[count];
        void *P;
        HIPCHK(S.ar.get(&P, ntot * 128 * 128 * esize(prm.qx_dtype)));
        HIPCHK(S.ar.get((void **)&sg.D, ntot * 128 * sizeof(double)));
        HIPCHK(S.ar.get((void **)&sg.T, ntot * 128 * sizeof(double)));
        std::map<int, int2 *> dtiles;
        for (int i = 0; i < count; ++i) {
            const int nb = symv_blocks(n[i]);
            if (!dtiles.count(nb)) {
                std::vector<int32_t> &tl = tile_lists[nb];
                tl = symv_tile_list(nb);
                int2 *d;
                HIPCHK(S.ar.get((void **)&d, tl.size() * sizeof(int32_t)));
                HIPCHK(hipMemcpyAsync(d, tl.data(), tl.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
                dtiles[nb] = d;
            }
            SymTiles ti{};
            ti.P = (const char *)P + tbase[i] * 128 * 128 * esize(prm.qx_dtype);
            ti.tiles = dtiles[nb];
            ti.nb = nb;
            ti.ntiles = (int64_t)nb * (nb + 1) / 2;
            HIPCHK(launch_symv_pack(prm.qx_dtype, hin[i].Qop, ld[i], ti, st));
        }
        std::vector<int32_t> all(count);
        for (int i = 0; i < count; ++i) all[i] = i;
        build_sym(all);
        HIPCHK(S.ar.get((void **)&dlist, hlist.size() * sizeof(SymGroupTile)));
        HIPCHK(S.ar.get((void **)&drows, hrows.size() * sizeof(SymGroupRow)));
        HIPCHK(hipMemcpyAsync(dlist, hlist.data(), hlist.size() * sizeof(SymGroupTile), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(drows, hrows.data(), hrows.size() * sizeof(SymGroupRow), hipMemcpyHostToDevice, st));
        sg.P = P;
        sg.list = dlist;
        sg.nlist = (int64_t)hlist.size();
        sg.rows = drows;
        sg.nrows = (int64_t)hrows.size();
    }
    HIPCHK(launch_solver_init(S.optype, w, nullptr, 1, st));
    HIPCHK(launch_compact(w, st));
    // Work list of the live instances only: once a poll finds at most 3/4 of
    // the instances of the last list live, the units of the live ones are laid
    // out again (rowstart stays indexed by column) and later batches launch
    // over those units alone. Which rows a live column gets, and how each row
    // is summed, do not change.
    int64_t live_units = rowstart[count], list_gen = 0;
    int last_live = count;
    S.list_cap = count;
    S.relist = [&](const int32_t *list, int cnt) -> hipError_t {
        if (cnt < 1 || cnt > count || 4 * (int64_t)cnt > 3 * (int64_t)last_live) return hipSuccess;
        std::vector<int32_t> ids(list, list + cnt);
        std::sort(ids.begin(), ids.end());
        std::vector<int64_t> rsv(count + 1, 0);
        int64_t u = 0;
        for (int32_t id : ids) {
            if (id < 0 || id >= count) return hipErrorInvalidValue;
            rsv[id] = u;
            u += (n[id] + 3) / 4;
        }
        unitcol.resize(u);
        for (int32_t id : ids) std::fill(unitcol.begin() + rsv[id], unitcol.begin() + rsv[id] + (n[id] + 3) / 4, id);
        // the batch in flight still reads the old list: the copies queue behind it
        hipError_t e = hipMemcpyAsync(drow, rsv.data(), (count + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(dunit, unitcol.data(), u * sizeof(int32_t), hipMemcpyHostToDevice, st);
        if (sym) {
            build_sym(ids);
            if (e == hipSuccess)
                e = hipMemcpyAsync(dlist, hlist.data(), hlist.size() * sizeof(SymGroupTile), hipMemcpyHostToDevice,
                                   st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(drows, hrows.data(), hrows.size() * sizeof(SymGroupRow), hipMemcpyHostToDevice,
                                   st);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(st);  // the host vectors are consumed
        if (e != hipSuccess) return e;
        sg.nlist = (int64_t)hlist.size();
        sg.nrows = (int64_t)hrows.size();
        live_units = u;
        last_live = cnt;
        ++list_gen;
        return hipSuccess;
    };
    S.config_key = [&]() { return list_gen; };
    QxTimer tm, ta, ts;
    tm.on = ts.on = prm.timing != 0;
    psdp_status rs = run_sweeps(
        S, prm, tm, ta, ts, st,
        [&]() {
            return sym ? launch_symv_group(prm.qx_dtype, sg, w, st)
                       : launch_gemv_group(prm.qx_dtype, w, drow, dunit, live_units, st);
        },
        []() { return hipSuccess; });
    if (rs != PSDP_OK) return rs;
    int64_t maxblk = 0;
    for (int i = 0; i < count; ++i) maxblk = std::max<int64_t>(maxblk, (n[i] + 15) / 16);
    int64_t *partial;
    HIPCHK(S.ar.get((void **)&partial, maxblk * sizeof(int64_t) * 2));
    for (int i = 0; i < count; ++i)
        HIPCHK(launch_round_objective(Q[i], b[i], n[i], w.x + off[i], ld[i], 1, xhat[i], n[i], obj + i,
                                      partial, st));
    HIPCHK(hipMemcpyAsync(hcol.data(), w.col, count * sizeof(Col), hipMemcpyDeviceToHost, st));
    int64_t nsweeps = 0;
    HIPCHK(hipMemcpyAsync(&nsweeps, S.sweeps, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (stats) {
        double flops = 0.0;
        for (const Col &cc : hcol) flops += 2.0 * (double)cc.n * (double)cc.n * (double)(cc.evals + cc.aux);
        fill_stats(hcol, nsweeps, tm, flops, ta, 0.0, ts, stats);
    }
    return PSDP_OK;
}

psdp_status psdp_eval_penalty_grad(int32_t dtype, int32_t vtype, const void *Q, int64_t ldq,
                                   const void *b, const void *p, const void *X, int64_t n, int64_t B,
                                   void *h, void *G, hipStream_t st) {
    g_err.clear();
    if (dtype < PSDP_F64 || dtype > PSDP_BF16) return fail(PSDP_E_INVALID, "dtype");
    if (vtype != PSDP_F64 && vtype != PSDP_F32) return fail(PSDP_E_INVALID, "vtype");
    if (!Q || !b || !p || !X || !h) return fail(PSDP_E_INVALID, "null required pointer");
    if (n < 1 || B < 1 || ldq < n) return fail(PSDP_E_INVALID, "sizes");
    if (B > 65535) return fail(PSDP_E_UNSUPPORTED, "B > 65535");
    double *ws = nullptr;
    const size_t bytes = (size_t)n * B * sizeof(double) + (B + 16) * sizeof(int32_t) + 256;
    HIPCHK(hipMallocAsync((void **)&ws, bytes, st));
    hipError_t e = launch_eval(dtype, vtype, Q, ldq, b, p, X, n, B, h, G, ws, st);
    hipError_t e2 = hipFreeAsync(ws, st);
    if (e != hipSuccess) return hipfail(e, "eval");
    if (e2 != hipSuccess) return hipfail(e2, "hipFreeAsync");
    return PSDP_OK;
}

psdp_status psdp_penalty_adjoint(int32_t dtype, int32_t vtype, const void *X, const void *G,
                                 const void *w, int64_t n, int64_t B, void *dX, void *dQ, void *db,
                                 void *dp, hipStream_t st) {
    g_err.clear();
    if (dtype != PSDP_F64 && dtype != PSDP_F32) {
        if (dtype == PSDP_BF16) return fail(PSDP_E_UNSUPPORTED, "adjoint supports F32 and F64");
        return fail(PSDP_E_INVALID, "dtype");
    }
    if (vtype != PSDP_F64 && vtype != PSDP_F32) return fail(PSDP_E_INVALID, "vtype");
    if (!X || !w || (dX && !G)) return fail(PSDP_E_INVALID, "null required pointer");
    if (n < 1 || B < 1) return fail(PSDP_E_INVALID, "sizes");
    if (n > 65535 * 64) return fail(PSDP_E_UNSUPPORTED, "n too large");
    hipError_t e = launch_adjoint(dtype, vtype, X, G, w, n, B, dX, dQ, db, dp, st);
    if (e != hipSuccess) return hipfail(e, "adjoint");
    return PSDP_OK;
}

psdp_status psdp_round_objective_i32(const int32_t *Q, const int32_t *b, int64_t n, const double *X,
                                     int64_t B, uint8_t *xhat, int64_t *obj, hipStream_t st) {
    g_err.clear();
    if (!Q || !b || !X || !xhat || !obj) return fail(PSDP_E_INVALID, "null required pointer");
    if (n < 1 || B < 1 || B > 65535) return fail(PSDP_E_INVALID, "sizes");
    int64_t *partial = nullptr;
    const int64_t nblk = (n + 15) / 16;
    HIPCHK(hipMallocAsync((void **)&partial, nblk * B * sizeof(int64_t), st));
    hipError_t e = launch_round_objective(Q, b, n, X, n, B, xhat, n, obj, partial, st);
    hipError_t e2 = hipFreeAsync(partial, st);
    if (e != hipSuccess) return hipfail(e, "round_objective");
    if (e2 != hipSuccess) return hipfail(e2, "hipFreeAsync");
    return PSDP_OK;
}

psdp_status psdp_perturbation(int64_t n, double sigma, uint64_t seed, int32_t mode, double *mu,
                              hipStream_t st) {
    g_err.clear();
    if (n < 1 || !mu) return fail(PSDP_E_INVALID, "sizes");
    if (mode < PSDP_PERTURB_NONE || mode > PSDP_PERTURB_DIAG) return fail(PSDP_E_INVALID, "mode");
    if (!(sigma >= 0.0) || !std::isfinite(sigma)) return fail(PSDP_E_INVALID, "sigma");
    hipError_t e = launch_perturbation(n, sigma, seed, mode, mu, st);
    if (e != hipSuccess) return hipfail(e, "perturbation");
    return PSDP_OK;
}

// Checks of the stand-alone integer products; rownnz gets the off-diagonal
// nonzeros of every row.
psdp_status qx_int_checks(const int32_t *Q, int64_t n, const double *X, int32_t B, int32_t digits, double *Y,
                          hipStream_t st, std::vector<int64_t> *rownnz) {
    if (!Q || !X || !Y) return fail(PSDP_E_INVALID, "null pointer");
    if (n < 1 || n > 65536 || B < 1) return fail(PSDP_E_INVALID, "n must be in [1, 65536] and B >= 1");
    if (digits != 4 && digits != 8) return fail(PSDP_E_INVALID, "digits must be 4 or 8");
    std::vector<int32_t> hQ(n * n);
    std::vector<double> hX(n * B);
    HIPCHK(hipMemcpyAsync(hQ.data(), Q, n * n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hX.data(), X, n * B * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    rownnz->assign(n, 0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            const int32_t v = hQ[i * n + j];
            if (i == j) continue;
            if (std::llabs((long long)v) > 127)
                return fail(PSDP_E_UNSUPPORTED, "int8 operands need |Q_ij| <= 127 off the diagonal");
            if (v != 0) ++(*rownnz)[i];
        }
    for (double v : hX) {
        if (!std::isfinite(v)) return fail(PSDP_E_NONFINITE, "X must be finite");
        if (digits == 4 && !(v >= 0.0 && v <= 1.0)) return fail(PSDP_E_NONFINITE, "digits 4 needs X in [0,1]");
    }
    return PSDP_OK;
}

psdp_status psdp_qx_digits(const int32_t *Q, int64_t n, const double *X, int32_t B, int32_t digits, double *Y,
                           hipStream_t st) {
    return psdp_qx_digits_ex(Q, n, X, B, digits, 0, 0, 0, nullptr, Y, st);
}

psdp_status psdp_qx_digits_ex(const int32_t *Q, int64_t n, const double *X, int32_t B, int32_t digits,
                              int32_t layout, int32_t slices, int32_t reps, double *us, double *Y, hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_lock);
    g_err.clear();
    if (layout != 0 && !digit_layout_valid(layout)) return fail(PSDP_E_INVALID, "layout must be 0, 1, 2, 4, 8 or 16");
    if (slices < 0 || slices > 8) return fail(PSDP_E_INVALID, "slices must be in [0, 8]");
    if (reps < 0 || (reps > 0 && !us)) return fail(PSDP_E_INVALID, "reps >= 0, and us given when reps > 0");
    std::vector<int64_t> rownnz;
    if (psdp_status s = qx_int_checks(Q, n, X, B, digits, Y, st, &rownnz)) return s;
    Arena ar;
    psdp_params prm;
    psdp_params_default(&prm);
    prm.qx_dtype = PSDP_I8;
    const psdp_column_plan plan = plan_columns(n, B, prm, false);
    if (!plan.ok) return fail(PSDP_E_INTERNAL, "a list-indexed buffer lacks the all-zero column");
    const int64_t ld = plan.ld;
    const int64_t rows = (ld + kDigitRowsAlign - 1) / kDigitRowsAlign * kDigitRowsAlign;
    const int D = digits;
    const DigitChoice dc = digit_choice(n, ld, D == 4 ? B : 0, D == 8 ? B : 0);
    const int mt = layout ? layout : (D == 4 ? dc.mt4 : dc.mt8);
    const int ks = slices ? slices : (D == 4 ? dc.ks4 : dc.ks8);
    int8_t *Q8, *dig;
    double *R, *dq;
    int64_t *U0, *U1 = nullptr;
    int32_t *act, *cnt, *esc;
    HIPCHK(ar.get((void **)&Q8, rows * ld));
    HIPCHK(hipMemsetAsync(Q8, 0, rows * ld, st));
    HIPCHK(ar.get((void **)&R, ld * 8));
    HIPCHK(ar.get((void **)&dq, ld * 8));
    HIPCHK(launch_prep_q(PSDP_I8, Q, n, ld, PSDP_PERTURB_NONE, 0.0, 0, Q8, R, dq, st));
    HIPCHK(ar.get((void **)&dig, (int64_t)plan.digit_cols * D * ld));
    HIPCHK(hipMemsetAsync(dig, 0, (int64_t)plan.digit_cols * D * ld, st));
    HIPCHK(ar.get((void **)&esc, (int64_t)B * sizeof(int32_t)));
    HIPCHK(launch_digits_from_vectors(X, n, n, B, D, dig, ld, esc, st));
    // the K slices add into one zeroed product buffer (two for 8 digits)
    const int64_t slice = (int64_t)B * ld;
    HIPCHK(ar.get((void **)&U0, slice * sizeof(int64_t)));
    HIPCHK(hipMemsetAsync(U0, 0, slice * sizeof(int64_t), st));
    if (D == 8) {
        HIPCHK(ar.get((void **)&U1, slice * sizeof(int64_t)));
        HIPCHK(hipMemsetAsync(U1, 0, slice * sizeof(int64_t), st));
    }
    // the live list: every column, then the count at index B = zero_col
    std::vector<int32_t> iota(plan.list_len);
    for (int c = 0; c < B; ++c) iota[c] = c;
    iota[B] = B;  // live count
    HIPCHK(ar.get((void **)&act, (size_t)plan.list_len * sizeof(int32_t)));
    HIPCHK(hipMemcpyAsync(act, iota.data(), (size_t)plan.list_len * sizeof(int32_t), hipMemcpyHostToDevice, st));
    cnt = act + B;
    const DigitJob job{dig, act, cnt, U0, U1, B, ks, mt, B};
    HIPCHK(launch_digit(Q8, ld, n, ld, D == 4 ? &job : nullptr, D == 8 ? &job : nullptr, st));
    HIPCHK(launch_digit_combine(U0, U1, n, ld, B, D, esc, Y, st));
    if (reps > 0) {
        // the same product again, reps times between two events (the result
        // is already in Y; with several K slices these launches add further
        // parts into the product buffers, which nothing reads afterwards)
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        hipError_t r = hipEventRecord(e0, st);
        for (int q = 0; q < reps && r == hipSuccess; ++q)
            r = launch_digit(Q8, ld, n, ld, D == 4 ? &job : nullptr, D == 8 ? &job : nullptr, st);
        if (r == hipSuccess) r = hipEventRecord(e1, st);
        if (r == hipSuccess) r = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (r == hipSuccess) r = hipEventElapsedTime(&ms, e0, e1);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        HIPCHK(r);
        *us = (double)ms * 1e3 / reps;
    }
    HIPCHK(hipStreamSynchronize(st));
    return PSDP_OK;
}

psdp_status psdp_set_digit_table(int64_t n, int32_t digits, int32_t count, const int32_t *max_cols,
                                 const int32_t *layout, const int32_t *slices) {
    std::lock_guard<std::mutex> lk(g_lock);
    g_err.clear();
    if (n < 1 || n > 65536) return fail(PSDP_E_INVALID, "n must be in [1, 65536]");
    if (digits != 4 && digits != 8) return fail(PSDP_E_INVALID, "digits must be 4 or 8");
    if (count < 0 || (count > 0 && (!max_cols || !layout || !slices))) return fail(PSDP_E_INVALID, "entries");
    std::vector<DigitTableEntry> t;
    for (int32_t q = 0; q < count; ++q) {
        if (max_cols[q] < 1 || (q > 0 && max_cols[q] <= max_cols[q - 1]))
            return fail(PSDP_E_INVALID, "max_cols must be positive and increasing");
        if (!digit_layout_valid(layout[q])) return fail(PSDP_E_INVALID, "layout must be 1, 2, 4, 8 or 16");
        if (slices[q] < 1 || slices[q] > 8) return fail(PSDP_E_INVALID, "slices must be in [1, 8]");
        t.push_back(DigitTableEntry{max_cols[q], layout[q], slices[q]});
    }
    if (t.empty()) g_digit_tables.erase({n, digits});
    else g_digit_tables[{n, digits}] = t;
    return PSDP_OK;
}

psdp_status psdp_digit_choice(int64_t n, int32_t est4, int32_t est8, int32_t *choice) {
    std::lock_guard<std::mutex> lk(g_lock);
    g_err.clear();
    if (n < 1 || n > 65536 || est4 < 0 || est8 < 0 || !choice) return fail(PSDP_E_INVALID, "arguments");
    const DigitChoice c = digit_choice(n, (n + 63) / 64 * 64, est4, est8);
    choice[0] = c.mt4;
    choice[1] = c.ks4;
    choice[2] = c.mt8;
    choice[3] = c.ks8;
    return PSDP_OK;
}

psdp_status psdp_qx_single(int32_t dtype, const int32_t *Q, int64_t n, const double *x, int32_t sym, double *y,
                           hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_lock);
    g_err.clear();
    if (dtype != PSDP_F64 && dtype != PSDP_F32 && dtype != PSDP_BF16)
        return fail(PSDP_E_INVALID, "dtype must be F64, F32 or BF16");
    if (sym != 0 && sym != 1) return fail(PSDP_E_INVALID, "sym must be 0 or 1");
    if (!Q || !x || !y) return fail(PSDP_E_INVALID, "null pointer");
    if (n < 1 || n > 65536) return fail(PSDP_E_INVALID, "n must be in [1, 65536]");
    psdp_params prm;
    psdp_params_default(&prm);
    prm.qx_dtype = dtype;
    InstFacts facts;
    if (psdp_status s = check_instance(Q, Q, n, nullptr, 0, nullptr, prm, st, &facts)) return s;
    Arena ar;
    const int64_t ld = padld(n);
    void *Qop;
    double *R, *dq, *op, *U;
    int32_t *act;
    HIPCHK(ar.get(&Qop, ld * ld * esize(dtype)));
    HIPCHK(ar.get((void **)&R, ld * 8));
    HIPCHK(ar.get((void **)&dq, ld * 8));
    HIPCHK(launch_prep_q(dtype, Q, n, ld, PSDP_PERTURB_NONE, 0.0, 0, Qop, R, dq, st));
    HIPCHK(ar.get((void **)&op, ld * sizeof(double)));
    HIPCHK(hipMemsetAsync(op, 0, ld * sizeof(double), st));
    HIPCHK(hipMemcpyAsync(op, x, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIPCHK(ar.get((void **)&U, ld * sizeof(double)));
    HIPCHK(ar.get((void **)&act, 2 * sizeof(int32_t)));
    hipLaunchKernelGGL(iota_list_kernel, dim3(1), dim3(256), 0, st, act, 1);
    HIPCHK(hipGetLastError());
    if (sym) {
        SymTiles sy{};
        sy.nb = symv_blocks(n);
        sy.ntiles = (int64_t)sy.nb * (sy.nb + 1) / 2;
        const std::vector<int32_t> tl = symv_tile_list(sy.nb);
        void *P;
        int2 *tiles;
        HIPCHK(ar.get(&P, symv_packed_elems(sy.nb) * esize(dtype)));
        HIPCHK(ar.get((void **)&tiles, tl.size() * sizeof(int32_t)));
        HIPCHK(hipMemcpyAsync(tiles, tl.data(), tl.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
        HIPCHK(ar.get((void **)&sy.D, sy.ntiles * 128 * sizeof(double)));
        HIPCHK(ar.get((void **)&sy.T, sy.ntiles * 128 * sizeof(double)));
        sy.P = P;
        sy.tiles = tiles;
        sy.live = act + 1;
        HIPCHK(launch_symv_pack(dtype, Qop, ld, sy, st));
        HIPCHK(launch_symv(dtype, sy, op, ld, n, U, st));
    } else {
        Work w{};
        w.op = op;
        w.U = U;
        w.active = act;
        w.nactive = act + 1;
        Inst hin{n, ld, 0, Qop};
        HIPCHK(launch_gemv(dtype, &hin, 1, w, 1, st));
    }
    HIPCHK(hipMemcpyAsync(y, U, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return PSDP_OK;
}

psdp_status psdp_qx_dense(int32_t dtype, const int32_t *Q, int64_t n, const double *X, int32_t B, double *Y,
                          hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_lock);
    g_err.clear();
    if (dtype != PSDP_F32 && dtype != PSDP_F64) return fail(PSDP_E_INVALID, "dtype must be F32 or F64");
    if (!Q || !X || !Y) return fail(PSDP_E_INVALID, "null pointer");
    if (n < 1 || n > 65536 || B < 1) return fail(PSDP_E_INVALID, "n must be in [1, 65536] and B >= 1");
    psdp_params prm;
    psdp_params_default(&prm);
    prm.qx_dtype = dtype;
    InstFacts facts;
    if (psdp_status s = check_instance(Q, Q, n, nullptr, 0, nullptr, prm, st, &facts)) return s;
    const bool q32 = facts.offmax <= (double)(1 << 24);
    if (!q32) return fail(PSDP_E_UNSUPPORTED, "the products read an FP32 copy of Q: |Q_ij| <= 2^24 needed");
    Arena ar;
    const int64_t ld = padld(n), MT = (ld + 63) / 64;
    const int gemm_dtype = dtype == PSDP_F32 ? PSDP_F32 : kGemmF32QF64;
    const Pick pk = pick_product(B, B, B, gemm_dtype, -1, MT);
    void *Qop, *op, *U;
    double *R, *dq;
    int32_t *act;
    const size_t oe = dtype == PSDP_F32 ? 4 : 8;
    const int64_t slice = ld * B;
    HIPCHK(ar.get(&Qop, ld * ld * sizeof(float)));
    HIPCHK(ar.get((void **)&R, ld * 8));
    HIPCHK(ar.get((void **)&dq, ld * 8));
    HIPCHK(launch_prep_q(PSDP_F32, Q, n, ld, PSDP_PERTURB_NONE, 0.0, 0, Qop, R, dq, st));
    HIPCHK(ar.get(&op, slice * oe));
    HIPCHK(ar.get(&U, slice * oe * pk.ks));
    HIPCHK(ar.get((void **)&act, (B + 1) * sizeof(int32_t)));
    const unsigned g = (unsigned)((slice + 255) / 256), gy = (unsigned)((n * B + 255) / 256);
    if (dtype == PSDP_F32)
        hipLaunchKernelGGL(pack_operand_kernel<float>, dim3(g), dim3(256), 0, st, X, n, ld, B, (float *)op);
    else
        hipLaunchKernelGGL(pack_operand_kernel<double>, dim3(g), dim3(256), 0, st, X, n, ld, B, (double *)op);
    hipLaunchKernelGGL(iota_list_kernel, dim3((unsigned)((B + 256) / 256)), dim3(256), 0, st, act, B);
    HIPCHK(hipGetLastError());
    if (pk.stream)
        HIPCHK(launch_stream(gemm_dtype, Qop, ld, op, U, act, act + B, slice, pk.ks, pk.est, pk.nt, st));
    else
        HIPCHK(launch_gemm(gemm_dtype, Qop, ld, op, U, act, act + B, slice, pk.ks, B, st));
    if (dtype == PSDP_F32)
        hipLaunchKernelGGL(sum_slices_kernel<float>, dim3(gy), dim3(256), 0, st, (const float *)U, slice, pk.ks, n,
                           ld, B, Y);
    else
        hipLaunchKernelGGL(sum_slices_kernel<double>, dim3(gy), dim3(256), 0, st, (const double *)U, slice, pk.ks,
                           n, ld, B, Y);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return PSDP_OK;
}

psdp_status psdp_qx_sparse(const int32_t *Q, int64_t n, const double *X, int32_t B, int32_t digits, double *Y,
                           hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_lock);
    g_err.clear();
    std::vector<int64_t> rownnz;
    if (psdp_status s = qx_int_checks(Q, n, X, B, digits, Y, st, &rownnz)) return s;
    std::vector<int32_t> hrowptr;
    int64_t nnz = 0;
    if (!csr_rowptr(rownnz, &hrowptr, &nnz)) return fail(PSDP_E_UNSUPPORTED, "sparse Q needs fewer than 2^31 nonzeros");
    Arena ar;
    psdp_params prm;
    psdp_params_default(&prm);
    prm.qx_dtype = PSDP_I8;
    const psdp_column_plan plan = plan_columns(n, B, prm, true);
    if (!plan.ok) return fail(PSDP_E_INTERNAL, "a list-indexed buffer lacks the all-zero column");
    const int64_t ld = plan.ld;
    const int D = digits;
    int8_t *Q8;
    double *R, *dq;
    int32_t *rowptr, *w0, *w1 = nullptr, *act, *esc;
    uint32_t *pk;
    int64_t *U0, *U1 = nullptr;
    HIPCHK(ar.get((void **)&Q8, ld * ld));
    HIPCHK(hipMemsetAsync(Q8, 0, ld * ld, st));
    HIPCHK(ar.get((void **)&R, ld * 8));
    HIPCHK(ar.get((void **)&dq, ld * 8));
    HIPCHK(launch_prep_q(PSDP_I8, Q, n, ld, PSDP_PERTURB_NONE, 0.0, 0, Q8, R, dq, st));
    HIPCHK(ar.get((void **)&rowptr, (n + 1) * sizeof(int32_t)));
    HIPCHK(ar.get((void **)&pk, std::max<int64_t>(1, nnz) * sizeof(uint32_t)));
    HIPCHK(hipMemcpyAsync(rowptr, hrowptr.data(), (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice, st));
    HIPCHK(launch_csr_fill(Q8, ld, n, rowptr, pk, st));
    const int64_t slice = (int64_t)B * ld, wslice = (int64_t)plan.word_cols * ld;
    HIPCHK(ar.get((void **)&w0, wslice * sizeof(int32_t)));
    HIPCHK(hipMemsetAsync(w0, 0, wslice * sizeof(int32_t), st));
    if (D == 8) {
        HIPCHK(ar.get((void **)&w1, wslice * sizeof(int32_t)));
        HIPCHK(hipMemsetAsync(w1, 0, wslice * sizeof(int32_t), st));
    }
    HIPCHK(ar.get((void **)&esc, (int64_t)B * sizeof(int32_t)));
    HIPCHK(launch_words_from_vectors(X, n, n, B, D, w0, w1, ld, esc, st));
    HIPCHK(ar.get((void **)&U0, slice * sizeof(int64_t)));
    if (D == 8) HIPCHK(ar.get((void **)&U1, slice * sizeof(int64_t)));
    std::vector<int32_t> iota(plan.list_len);
    for (int c = 0; c < B; ++c) iota[c] = c;
    iota[B] = B;  // live count
    HIPCHK(ar.get((void **)&act, (size_t)plan.list_len * sizeof(int32_t)));
    HIPCHK(hipMemcpyAsync(act, iota.data(), (size_t)plan.list_len * sizeof(int32_t), hipMemcpyHostToDevice, st));
    int32_t *stage;
    const int64_t passes = sparse_stage_passes(B, D == 4 ? 1 : 2);
    HIPCHK(ar.get((void **)&stage, passes * ld * 16 * (int64_t)sizeof(int32_t)));
    const SparseJob job{1, rowptr, pk, n, w0, w1, ld, act, act + B, B, U0, U1, ld, stage, passes, B};
    HIPCHK(launch_sparse(D == 4 ? &job : nullptr, D == 8 ? &job : nullptr, st));
    HIPCHK(launch_digit_combine(U0, U1, n, ld, B, D, esc, Y, st));
    HIPCHK(hipStreamSynchronize(st));
    return PSDP_OK;
}

psdp_status psdp_round_objective_f64(const double *Q, const double *b, int64_t n, const double *X,
                                     int64_t B, uint8_t *xhat, double *obj, hipStream_t st) {
    g_err.clear();
    if (!Q || !b || !X || !xhat || !obj) return fail(PSDP_E_INVALID, "null required pointer");
    if (n < 1 || B < 1 || B > 65535 || n > 65536) return fail(PSDP_E_INVALID, "sizes");
    int64_t *acc = nullptr;
    const size_t bytes = (size_t)B * kObjAccWords * sizeof(int64_t);
    HIPCHK(hipMallocAsync((void **)&acc, bytes, st));
    hipError_t e = hipMemsetAsync(acc, 0, bytes, st);
    if (e == hipSuccess) e = launch_round_objective(Q, b, n, X, n, B, xhat, n, obj, acc, st);
    hipError_t e2 = hipFreeAsync(acc, st);
    if (e != hipSuccess) return hipfail(e, "round_objective");
    if (e2 != hipSuccess) return hipfail(e2, "hipFreeAsync");
    return PSDP_OK;
}

}  // extern "C"

namespace {

// Host-pointer form of the solve: device copies of the inputs, the device
// entry point on the null stream, the outputs copied back.
template <typename T, typename ObjT>
psdp_status solve_host(const T *Q, const T *b, int64_t n, const double *X0, const double *p0, int32_t B,
                       const psdp_params *prm, uint8_t *xhat, ObjT *obj, double *X_out, int32_t *best,
                       psdp_stats *stats) {
    g_err.clear();
    if (!Q || !b || !xhat || !obj) return fail(PSDP_E_INVALID, "null required pointer");
    if (n < 1 || B < 1) return fail(PSDP_E_INVALID, "n and B must be >= 1");
    if (n > 65536) return fail(PSDP_E_UNSUPPORTED, "n > 65536");
    Arena ar;
    T *dQ, *db;
    double *dX0 = nullptr, *dp0 = nullptr, *dX = nullptr;
    uint8_t *dxh;
    ObjT *dobj;
    HIPCHK(ar.get((void **)&dQ, (size_t)n * n * sizeof(T)));
    HIPCHK(ar.get((void **)&db, (size_t)n * sizeof(T)));
    HIPCHK(hipMemcpy(dQ, Q, (size_t)n * n * sizeof(T), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(db, b, (size_t)n * sizeof(T), hipMemcpyHostToDevice));
    if (X0) {
        HIPCHK(ar.get((void **)&dX0, (size_t)n * B * sizeof(double)));
        HIPCHK(hipMemcpy(dX0, X0, (size_t)n * B * sizeof(double), hipMemcpyHostToDevice));
    }
    if (p0) {
        HIPCHK(ar.get((void **)&dp0, (size_t)n * sizeof(double)));
        HIPCHK(hipMemcpy(dp0, p0, (size_t)n * sizeof(double), hipMemcpyHostToDevice));
    }
    HIPCHK(ar.get((void **)&dxh, (size_t)n * B));
    HIPCHK(ar.get((void **)&dobj, (size_t)B * sizeof(ObjT)));
    if (X_out) HIPCHK(ar.get((void **)&dX, (size_t)n * B * sizeof(double)));
    psdp_status s = solve_impl<T, ObjT>(dQ, db, n, dX0, dp0, B, prm, dxh, dobj, dX, best, stats, nullptr, 0,
                                        nullptr, 0, nullptr);
    if (s != PSDP_OK) return s;
    HIPCHK(hipMemcpy(xhat, dxh, (size_t)n * B, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(obj, dobj, (size_t)B * sizeof(ObjT), hipMemcpyDeviceToHost));
    if (X_out) HIPCHK(hipMemcpy(X_out, dX, (size_t)n * B * sizeof(double), hipMemcpyDeviceToHost));
    return PSDP_OK;
}

}  // namespace

extern "C" {

psdp_status psdp_solve_host_i32(const int32_t *Q, const int32_t *b, int64_t n, const double *X0,
                                const double *p0, int32_t B, const psdp_params *prm, uint8_t *xhat,
                                int64_t *obj, double *X_out, int32_t *best, psdp_stats *stats) {
    return solve_host<int32_t, int64_t>(Q, b, n, X0, p0, B, prm, xhat, obj, X_out, best, stats);
}

psdp_status psdp_solve_host_f64(const double *Q, const double *b, int64_t n, const double *X0,
                                const double *p0, int32_t B, const psdp_params *prm, uint8_t *xhat,
                                double *obj, double *X_out, int32_t *best, psdp_stats *stats) {
    return solve_host<double, double>(Q, b, n, X0, p0, B, prm, xhat, obj, X_out, best, stats);
}

void psdp_release(void) {}

}  // extern "C"
