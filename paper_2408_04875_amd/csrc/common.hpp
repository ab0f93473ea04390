// Shared definitions of the gfx950 vectorized-PSDP library: device state
// layout, dtype helpers and deterministic block reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include "../../include/psdp.h"

namespace psdp {

constexpr int kBlock = 256;          // threads of the generic kernels
constexpr int kWaves = kBlock / 64;  // wave64
constexpr int kSB = 512;             // threads of the per-column solver kernel
constexpr int kSWaves = kSB / 64;

// Column phases of the solver state machine. Each sweep applies Q to exactly
// one vector per live column; the phase says what that vector was.
enum Phase : int32_t {
    PH_DONE = 0,
    PH_CG = 1,     // x^0 linear solve (eq. (gamma)): operand = search direction
    PH_EIG0 = 2,   // lambda_min: operand = first basis vector
    PH_EIG = 3,    // lambda_min: operand = preconditioned residual
    PH_INNER = 4,  // subproblem: operand = current iterate x^k
};

// Per-instance data (one problem Q, b); the vectors live at `off` in the
// instance arrays, padded to `ld` entries (ld multiple of 16, pads are 0).
struct Inst {
    int64_t n;
    int64_t ld;
    int64_t off;         // offset into b, gamma, R, dq arrays
    const void *Qop;     // operand copy of Q with zero diagonal, ld x ld row-major
};

// Per-column state (one start of one instance).
struct Col {
    int32_t inst;
    int32_t phase;
    int64_t n;
    int64_t ld;
    int64_t off;         // offset of this column's vectors (stride ld)
    int32_t k;           // inner iteration index within the current subproblem
    int32_t s;           // penalty updates done
    int32_t stall;       // consecutive subproblems that did not move x
    int32_t it;          // lambda_min / CG iteration counter
    int32_t hasP;        // LOBPCG search direction present
    int32_t exit_reason;
    int32_t ntrace;      // trace records written
    int32_t id;          // column index (digit planes of the integer path)
    double rho;          // rho at the current p (Section 3.3)
    double rho_outer;    // rho at the p of the current penalty update
    double lam;          // current Ritz value
    double rz;           // CG: r^T M^-1 r
    double r0;           // CG: ||r_0||
    double final_rel;    // cret/rho of the last evaluation
    double final_bg;     // binary gap of the final iterate
    double alpha;        // penalty step of the current update (eq. (alpha1))
    int64_t evals;       // penalty-gradient evaluations
    int64_t aux;         // lambda_min and CG products
    int64_t inner_start; // evals at the start of the current subproblem
    int32_t nI;          // |I| of the current penalty update
    int32_t escale;      // integer path: lambda_min / CG operand scaled by 2^-escale
    int64_t ioff;        // offset of the instance vectors (Inst::off), so that
                         // the column kernel reads no Inst record
    int32_t start;       // the start this column holds (its trace, replayed steps
                         // and outputs); equals id unless starts are queued
    int32_t pad_;
};

// Flat solver workspace (device pointers), passed to every solver kernel.
struct Work {
    int32_t ncol;         // columns of the solve (index ncol: the all-zero operand column)
    // the columns this launch sequence advances, [col_base, col_base + col_count)
    // (a solve may run its columns as several concurrent sequences, each with
    // its own live lists, counters and queue)
    int32_t col_base, col_count;
    int32_t ksplit;      // number of U slices to sum (split-K)
    int64_t slice;       // elements per U slice
    Inst *inst;
    Col *col;
    // instance vectors; dgi = Q_ii + gamma_i and lni = b_i - gamma_i, so that
    // a column's diagonal of Q_r - Diag p is dgi_i - p_i and its linear term
    // b_r + p is lni_i + p_i (the instance vectors are shared by all the
    // columns of an instance and stay in the caches)
    double *b, *gam, *R, *dq, *dgi, *lni;
    // column vectors
    double *x, *xp, *g, *gp, *p, *v, *Av, *P, *AP, *w;
    // zx = x_i - x_i^2 (written at every outer-loop head, constant while
    // lambda_min runs)
    double *zx;
    void *op;            // operand buffer (OpT), column layout as the vectors
    void *U;             // Q.X output (UT): ksplit slices; the integer path keeps one
                         // int64 buffer that its K slices add into
    int32_t *active;     // live column list for the next sweep (split: PH_INNER only)
    int32_t *nactive;
    // split precision: lambda_min and CG products use their own FP64 operand
    // and product buffers and their own live list; otherwise these alias the
    // main ones
    int32_t split;
    int32_t ksplit_aux;
    int64_t slice_aux;
    double *op_aux;
    double *U_aux;
    int32_t *active_aux;
    int32_t *nactive_aux;
    // exact integer products (I8): digit planes of the subproblem operands
    // ([ncol + 1][4][ld] int8) and of the lambda_min / CG operands
    // ([ncol + 1][8][ld]); U holds int64 slices, U_aux the high halves and
    // U_lo the low halves of the 8-digit products
    int32_t i8;
    // integer path: whether the column kernel clears the int64 product
    // values it reads (the next product of that kind adds K slices into
    // them); a product written by a single slice overwrites its outputs, and
    // the host clears the buffers itself before a batch whose product adds
    // onto values left by a batch that did not clear them
    int32_t clear_main, clear_aux;
    int8_t *dig;
    int8_t *dig_aux;
    int64_t *U_lo;
    // integer path with a sparse copy of Q: the operands' grid values as
    // int32 words too (tw: T of a subproblem iterate; tw_hi, tw_lo: the two
    // halves of a lambda_min / CG vector), column layout as the vectors;
    // null when no sparse copy exists
    int32_t *tw, *tw_hi, *tw_lo;
    // live lists of the next sweep: the column kernel appends every live
    // column (slot claimed with an atomic on next_cnt[0] for the main list,
    // next_cnt[1] for the aux list) and clears clear_cnt[0..1], the counters
    // of the lists this sweep's products consumed (they are filled again in
    // the sweep after). The lists alternate between two buffers by sweep.
    int32_t *next_active;
    int32_t *next_active_aux;
    int32_t *next_cnt;
    int32_t *clear_cnt;
    int64_t *sweeps;      // sweep counter (nullable)
    unsigned long long *phase_prof;  // optional per-phase {sum, count, max} of step ticks
    double *trace;       // per column trace_cap records of 6 doubles, or null
    int32_t trace_cap;
    // prescribed penalty steps (a parity hook): update s < alpha_cap of the
    // start c takes alpha_in[c * alpha_cap + s]; null: computed
    const double *alpha_in;
    int32_t alpha_cap;
    // queued starts (null queue: every start has its own column). A column
    // whose start ends writes the final iterate to xfin (n x nstart, leading
    // dimension n) and its record to fin, then takes the next start from the
    // counter *queue (x from X0, n x nstart; the penalty from p0 or 0)
    int32_t *queue;
    int32_t nstart;
    const double *X0;
    const double *p0;
    double *xfin;
    Col *fin;
    // parameters
    int32_t inner;       // psdp_inner
    int32_t max_inner, max_outer, stall_outer, eig_maxit, cg_maxit;
    int32_t lambda_reuse;  // shift-law lambda_min after a subproblem that left x unchanged
    double tol_kkt, tol_binary, eta, eps_hp, lambda_floor_rel, alpha_min, alpha_max;
    double eig_tol, cg_tol;
};

// ---------------------------------------------------------------------------
// dtype helpers

template <typename T> __device__ __forceinline__ double to_f64(T v);
template <> __device__ __forceinline__ double to_f64<double>(double v) { return v; }
template <> __device__ __forceinline__ double to_f64<float>(float v) { return (double)v; }
template <> __device__ __forceinline__ double to_f64<__hip_bfloat16>(__hip_bfloat16 v) {
    return (double)__bfloat162float(v);
}

template <typename T> __device__ __forceinline__ T from_f64(double v);
template <> __device__ __forceinline__ double from_f64<double>(double v) { return v; }
template <> __device__ __forceinline__ float from_f64<float>(double v) { return __double2float_rn(v); }
// int8 operand of the integer path: callers pass integers in [-127, 127]
template <> __device__ __forceinline__ int8_t from_f64<int8_t>(double v) { return (int8_t)__double2int_rn(v); }
template <> __device__ __forceinline__ __hip_bfloat16 from_f64<__hip_bfloat16>(double v) {
    // double -> float is exact for every value the callers pass (vectors in
    // [0,1] or preconditioned residuals); float -> bf16 rounds to nearest even
    return __float2bfloat16(__double2float_rn(v));
}

// ---------------------------------------------------------------------------
// Integer operands of the exact product path: an integer T with
// |T| <= 2^27 as four signed base-128 digits, most significant first,
// T = d0 2^21 + d1 2^14 + d2 2^7 + d3 with every d in [-64, 64]
// (each step keeps the nearest multiple of the next power, ties upward).
// Digit t of element i goes to p[t * plane + i].
constexpr double kMainScale = 134217728.0;  // 2^27: iterate grid of the 4-digit operand
constexpr int kAuxBits = 55;                // 8-digit operand: v 2^(55 - e) rounded
// The plane pointers are formed before the element offset is added, so with
// a uniform p and plane every store takes a scalar base and one 32-bit
// offset. The digit arithmetic is 32-bit (|T| + 2^20 < 2^31).
__device__ __forceinline__ void put_digits4(int8_t *p, int64_t plane, uint32_t i, int32_t T) {
    const int32_t d0 = (T + (1 << 20)) >> 21;
    T -= d0 << 21;
    const int32_t d1 = (T + (1 << 13)) >> 14;
    T -= d1 << 14;
    const int32_t d2 = (T + (1 << 6)) >> 7;
    T -= d2 << 7;
    int8_t *p1 = p + plane, *p2 = p + 2 * plane, *p3 = p + 3 * plane;
    p[i] = (int8_t)d0;
    p1[i] = (int8_t)d1;
    p2[i] = (int8_t)d2;
    p3[i] = (int8_t)T;
}

// Eight digits of v scaled by 2^-e (|v| < 2^e): T = rint(v 2^(55 - e)),
// split as T = T_hi 2^28 + T_lo with |T_hi|, |T_lo| <= 2^27 (split8), each in
// four digits (planes 0-3 and 4-7).
__device__ __forceinline__ void split8(double v, int e, int32_t *hi, int32_t *lo) {
    const int64_t T = __double2ll_rn(ldexp(v, kAuxBits - e));
    const int64_t h = (T + (1ll << 27)) >> 28;
    *hi = (int32_t)h;
    *lo = (int32_t)(T - (h << 28));
}
__device__ __forceinline__ void put_digits8(int8_t *p, int64_t plane, uint32_t i, double v, int e) {
    int32_t hi, lo;
    split8(v, e, &hi, &lo);
    put_digits4(p, plane, i, hi);
    put_digits4(p + 4 * plane, plane, i, lo);
}

// Value of an 8-digit product from its summed halves: (hi 2^28 + lo) 2^(e - 55),
// both halves exact in FP64 (|hi|, |lo| < 2^51), one rounding in the sum.
__device__ __forceinline__ double digits8_value(int64_t hi, int64_t lo, int e) {
    return ldexp((double)hi * 268435456.0 + (double)lo, e - kAuxBits);
}

// Least e with |m| < 2^e for m > 0 (0 for m = 0): the 8-digit operand scale.
__device__ __forceinline__ int digits8_exponent(double maxabs) {
    int e = 0;
    if (maxabs > 0.0) (void)frexp(maxabs, &e);
    return e;
}

// ---------------------------------------------------------------------------
// Deterministic block reductions over NT threads. Inside a wave the values
// move with DPP row shifts and row broadcasts (plain VALU moves, no LDS
// traffic) in a fixed pattern that leaves the wave's total in lane 63:
// each row of 16 lanes forms prefix sums over shifts of 1, 2, 4 and 8, then
// lane 15 of rows 0 and 2 joins rows 1 and 3, and lane 31 joins row 3. The
// wave totals are then combined in wave order through shared memory, so
// every thread gets the same value. `scratch` must hold N * NT / 64 doubles
// of shared memory and is free again when the call returns. The max
// reductions take 0 as identity: their inputs must be non-negative.

// A double moved across lanes by DPP control CTRL on the rows in ROWMASK;
// lanes whose source lies outside the row, or whose row is masked off, get 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_f64(double v) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u & 0xffffffffull), CTRL, ROWMASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, ROWMASK, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;

__device__ __forceinline__ double wave_sum_to_63(double v) {
    v += dpp_f64<kDppRowShr1, 0xf>(v);
    v += dpp_f64<kDppRowShr2, 0xf>(v);
    v += dpp_f64<kDppRowShr4, 0xf>(v);
    v += dpp_f64<kDppRowShr8, 0xf>(v);
    v += dpp_f64<kDppRowBcast15, 0xa>(v);
    v += dpp_f64<kDppRowBcast31, 0xc>(v);
    return v;
}

__device__ __forceinline__ double wave_max_to_63(double v) {
    v = fmax(v, dpp_f64<kDppRowShr1, 0xf>(v));
    v = fmax(v, dpp_f64<kDppRowShr2, 0xf>(v));
    v = fmax(v, dpp_f64<kDppRowShr4, 0xf>(v));
    v = fmax(v, dpp_f64<kDppRowShr8, 0xf>(v));
    v = fmax(v, dpp_f64<kDppRowBcast15, 0xa>(v));
    v = fmax(v, dpp_f64<kDppRowBcast31, 0xc>(v));
    return v;
}

// Max-reduction of mx and sum-reduction of sm in one shared-memory round.
template <int NM, int NS, int NT>
__device__ __forceinline__ void block_maxsum(double (&mx)[NM], double (&sm)[NS], double *scratch) {
    constexpr int kWaves = NT / 64;
#pragma unroll
    for (int j = 0; j < NM; ++j) mx[j] = wave_max_to_63(mx[j]);
#pragma unroll
    for (int j = 0; j < NS; ++j) sm[j] = wave_sum_to_63(sm[j]);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 63) {
#pragma unroll
        for (int j = 0; j < NM; ++j) scratch[j * kWaves + wv] = mx[j];
#pragma unroll
        for (int j = 0; j < NS; ++j) scratch[(NM + j) * kWaves + wv] = sm[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NM; ++j) {
        double v = scratch[j * kWaves];
#pragma unroll
        for (int q = 1; q < kWaves; ++q) v = fmax(v, scratch[j * kWaves + q]);
        mx[j] = v;
    }
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        double v = scratch[(NM + j) * kWaves];
#pragma unroll
        for (int q = 1; q < kWaves; ++q) v += scratch[(NM + j) * kWaves + q];
        sm[j] = v;
    }
    __syncthreads();
}

// Double-double sums (Ogita, Rump and Oishi, "Accurate sum and dot
// product", 2005: Sum2 / Dot2): a pair (h, l) carries a value h + l; every
// addition keeps the rounding error of the high part exactly (TwoSum) and a
// product enters as its exact pair (a b rounded, and the fma residual). The
// result h + l, rounded once, is the exact sum rounded to nearest unless the
// exact sum lies within about n^2 2^-106 of the summed magnitudes of a
// rounding boundary, so it agrees with an exact reference in practice and does
// not depend on the order of the terms. Needs fp-contraction off (the build
// sets it) so that no TwoSum is fused.
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}
__device__ __forceinline__ void dd_add(double &h, double &l, double h2, double l2) {
    double s, e;
    two_sum(h, h2, s, e);
    h = s;
    l = (l + l2) + e;
}
__device__ __forceinline__ void dd_add_prod(double &h, double &l, double a, double b) {
    const double p = a * b;
    const double pe = fma(a, b, -p);
    double s, e;
    two_sum(h, p, s, e);
    h = s;
    l = l + (e + pe);
}

// The DPP pattern of wave_sum_to_63 on pairs: lane 63 ends with the wave's pair.
__device__ __forceinline__ void wave_ddsum_to_63(double &h, double &l) {
    dd_add(h, l, dpp_f64<kDppRowShr1, 0xf>(h), dpp_f64<kDppRowShr1, 0xf>(l));
    dd_add(h, l, dpp_f64<kDppRowShr2, 0xf>(h), dpp_f64<kDppRowShr2, 0xf>(l));
    dd_add(h, l, dpp_f64<kDppRowShr4, 0xf>(h), dpp_f64<kDppRowShr4, 0xf>(l));
    dd_add(h, l, dpp_f64<kDppRowShr8, 0xf>(h), dpp_f64<kDppRowShr8, 0xf>(l));
    dd_add(h, l, dpp_f64<kDppRowBcast15, 0xa>(h), dpp_f64<kDppRowBcast15, 0xa>(l));
    dd_add(h, l, dpp_f64<kDppRowBcast31, 0xc>(h), dpp_f64<kDppRowBcast31, 0xc>(l));
}

// Max-reduction of mx and double-double sum-reduction of the pairs (h, l) in
// one shared-memory round; on return h[j] holds the sum rounded once (and
// l[j] zero). scratch: (NM + 2 NS) * NT / 64 doubles.
template <int NM, int NS, int NT>
__device__ __forceinline__ void block_maxsum_dd(double (&mx)[NM], double (&h)[NS], double (&l)[NS],
                                                double *scratch) {
    constexpr int kWaves = NT / 64;
#pragma unroll
    for (int j = 0; j < NM; ++j) mx[j] = wave_max_to_63(mx[j]);
#pragma unroll
    for (int j = 0; j < NS; ++j) wave_ddsum_to_63(h[j], l[j]);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 63) {
#pragma unroll
        for (int j = 0; j < NM; ++j) scratch[j * kWaves + wv] = mx[j];
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            scratch[(NM + 2 * j) * kWaves + wv] = h[j];
            scratch[(NM + 2 * j + 1) * kWaves + wv] = l[j];
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NM; ++j) {
        double v = scratch[j * kWaves];
#pragma unroll
        for (int q = 1; q < kWaves; ++q) v = fmax(v, scratch[j * kWaves + q]);
        mx[j] = v;
    }
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        double H = scratch[(NM + 2 * j) * kWaves], L = scratch[(NM + 2 * j + 1) * kWaves];
#pragma unroll
        for (int q = 1; q < kWaves; ++q)
            dd_add(H, L, scratch[(NM + 2 * j) * kWaves + q], scratch[(NM + 2 * j + 1) * kWaves + q]);
        h[j] = H + L;
        l[j] = 0.0;
    }
    __syncthreads();
}

template <int N, int NT = kBlock>
__device__ __forceinline__ void block_sum(double (&v)[N], double *scratch) {
    constexpr int kWaves = NT / 64;
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] = wave_sum_to_63(v[j]);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 63) {
#pragma unroll
        for (int j = 0; j < N; ++j) scratch[j * kWaves + wv] = v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < N; ++j) {
        double s = scratch[j * kWaves];
#pragma unroll
        for (int q = 1; q < kWaves; ++q) s += scratch[j * kWaves + q];
        v[j] = s;
    }
    __syncthreads();
}

template <int N, int NT = kBlock>
__device__ __forceinline__ void block_max(double (&v)[N], double *scratch) {
    constexpr int kWaves = NT / 64;
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] = wave_max_to_63(v[j]);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 63) {
#pragma unroll
        for (int j = 0; j < N; ++j) scratch[j * kWaves + wv] = v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < N; ++j) {
        double s = scratch[j * kWaves];
#pragma unroll
        for (int q = 1; q < kWaves; ++q) s = fmax(s, scratch[j * kWaves + q]);
        v[j] = s;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Sets the thread-local detail returned by psdp_last_error (an empty string
// for msg = nullptr) and returns s.
psdp_status set_error(psdp_status s, const char *msg);

}  // namespace psdp
