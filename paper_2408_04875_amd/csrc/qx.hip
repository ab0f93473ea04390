// Q.X products of the vectorized PSDP solver: the O(n^2) part of every
// penalty-gradient evaluation grad h = 2 (Q - Diag p) x + (b + p) (eq. (kkt1)),
// of every lambda_min matvec (eq. (alpha)) and every x^0 CG matvec
// (eq. (gamma)). All kernels compute U[:, c] = Qop X[:, c] for the live
// columns c listed in `active` (Qop: zero-diagonal operand copy, row-major,
// leading dimension ld, a multiple of 16 with zero padding).
//
//  gemv_kernel        one instance, few columns: one wave per row (four
//                     from n = 8192), 16-byte coalesced loads of Q, FP64
//                     accumulation, x in FP64.
//  gemv_group_kernel  uneven instances: the rows of every instance form one
//                     flat work list of four-row units (one wave per unit).
//  gemm_*_kernel      one instance, many columns: MFMA tiles (FP32 16x16x4 or
//                     FP64 16x16x4) staged through LDS, split over K into
//                     separate output slices that the solver sums in order.
#include <algorithm>

#include "launch.hpp"

namespace psdp {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

// Four consecutive Q entries as doubles (16-byte aligned for float, 32 for double).
__device__ __forceinline__ void load4(const double *q, double (&o)[4]) {
    const double2 a = *(const double2 *)q, b = *(const double2 *)(q + 2);
    o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
}
__device__ __forceinline__ void load4(const float *q, double (&o)[4]) {
    const float4 a = *(const float4 *)q;
    o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w;
}
__device__ __forceinline__ void load4(const __hip_bfloat16 *q, double (&o)[4]) {
    const uint2 a = *(const uint2 *)q;
    o[0] = (double)__uint_as_float(a.x << 16);
    o[1] = (double)__uint_as_float(a.x & 0xffff0000u);
    o[2] = (double)__uint_as_float(a.y << 16);
    o[3] = (double)__uint_as_float(a.y & 0xffff0000u);
}

template <typename QT>
__device__ __forceinline__ double row_dot(const QT *q, const double *x, int64_t ld, int lane) {
    double acc0 = 0.0, acc1 = 0.0;
    for (int64_t j = (int64_t)lane * 4; j < ld; j += 256) {
        double qv[4], xv[4];
        load4(q + j, qv);
        load4(x + j, xv);
        acc0 = fma(qv[0], xv[0], acc0);
        acc1 = fma(qv[1], xv[1], acc1);
        acc0 = fma(qv[2], xv[2], acc0);
        acc1 = fma(qv[3], xv[3], acc1);
    }
    double acc = acc0 + acc1;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    return acc;
}

// R rows of Q against one x per wave: the lane's x entries are loaded once
// per K step and feed all R rows, so that x (FP64, two to four times the
// bytes of a Q entry) is not read again for every row. Each row keeps the
// summation of row_dot (same lanes, same two accumulators, same order), so
// the result does not depend on R.
template <typename QT, int R>
__device__ __forceinline__ void rows_dot(const QT *q, const double *x, int64_t ld, int lane, double (&out)[R]) {
    double acc0[R], acc1[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc0[r] = acc1[r] = 0.0;
    for (int64_t j = (int64_t)lane * 4; j < ld; j += 256) {
        double xv[4];
        load4(x + j, xv);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            double qv[4];
            load4(q + r * ld + j, qv);
            acc0[r] = fma(qv[0], xv[0], acc0[r]);
            acc1[r] = fma(qv[1], xv[1], acc1[r]);
            acc0[r] = fma(qv[2], xv[2], acc0[r]);
            acc1[r] = fma(qv[3], xv[3], acc1[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        double acc = acc0[r] + acc1[r];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
        out[r] = acc;
    }
}

// grid (ceil(n / (4 R)), ncol_max): block = 4 waves, R consecutive rows each,
// of one column; a wave with fewer than R rows left takes them one by one.
template <typename QT, int R>
__global__ void __launch_bounds__(kBlock) gemv_kernel(const QT *Qop, int64_t n, int64_t ld,
                                                      const double *op, double *U,
                                                      const int32_t *active,
                                                      const int32_t *nactive) {
    const int slot = blockIdx.y;
    if (slot >= *nactive) return;
    const int64_t ci = active[slot];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t row0 = ((int64_t)blockIdx.x * kWaves + wv) * R;
    if (row0 >= n) return;
    if (R == 1 || row0 + R <= n) {
        double acc[R];
        rows_dot<QT, R>(Qop + row0 * ld, op + ci * ld, ld, lane, acc);
        if (lane == 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) U[ci * ld + row0 + r] = acc[r];
        }
    } else {  // fewer than R rows left: one at a time
        for (int64_t row = row0; row < n; ++row) {
            double acc[1];
            rows_dot<QT, 1>(Qop + row * ld, op + ci * ld, ld, lane, acc);
            if (lane == 0) U[ci * ld + row] = acc[0];
        }
    }
}

// Flat work list of all columns in units of 4 rows: units rowstart[c] ..
// rowstart[c+1]-1 belong to column c (ceil(n_c / 4) of them), and unitcol
// names the column of every unit (one load instead of a search, which
// matters late in a solve, when most units belong to finished columns and
// only look up their column and leave); a wave takes one unit, rows_dot
// over its rows (per-row sums as in row_dot).
template <typename QT>
__global__ void __launch_bounds__(kBlock) gemv_group_kernel(const Col *col, const Inst *inst,
                                                            const int64_t *rowstart, const int32_t *unitcol,
                                                            int64_t total, const double *op, double *U) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t r = (int64_t)blockIdx.x * kWaves + wv;
    if (r >= total) return;
    const int lo = unitcol[r];
    const Col &c = col[lo];
    if (c.phase == PH_DONE) return;
    const Inst &in = inst[c.inst];
    const int64_t row0 = (r - rowstart[lo]) * 4;
    const QT *Q = (const QT *)in.Qop;
    if (row0 + 4 <= in.n) {
        double acc[4];
        rows_dot<QT, 4>(Q + row0 * in.ld, op + c.off, in.ld, lane, acc);
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) U[c.off + row0 + k] = acc[k];
        }
    } else {
        for (int64_t row = row0; row < in.n; ++row) {
            double acc[1];
            rows_dot<QT, 1>(Q + row * in.ld, op + c.off, in.ld, lane, acc);
            if (lane == 0) U[c.off + row] = acc[0];
        }
    }
}

// ---------------------------------------------------------------------------
// MFMA GEMM, U[:, c] = Q X[:, c] for the live columns c (block tile 64 x 64,
// 4 waves of 32 x 32, each 2 x 2 MFMA 16x16x4 tiles).
//
// LDS holds the Q tile row-major (row m, contiguous k) and the X tile column
// by column (column n, contiguous k): both are straight copies of global
// memory. The MFMA 16x16x4 operand layout gives lane l the entries
// A[l % 16][k] and B[k][l % 16] with k = l / 16; over four instructions the
// lane group g = l / 16 instead reads the 16-byte run k = 4 g .. 4 g + 3 of
// its row once and feeds one element to each instruction, so the four
// instructions together cover 16 consecutive k (the sum is the same set of
// products in another order). The accumulator rows differ between the FP32
// and FP64 instructions (Mfma<T>::row, measured on gfx950).
//
// TA is the storage type of Q (float or double), T the MFMA type (float, or
// double with Q widened exactly while staging). The K range is split into
// ksplit slices written to separate outputs; blocks are ordered so that the
// column tiles sharing one Q block run on the same XCD (same L2).

template <typename T> struct Mfma;
template <> struct Mfma<float> {
    typedef floatx4 acc_t;
    static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // accumulator register r of lane l holds row 4 (l / 16) + r, column l % 16
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <> struct Mfma<double> {
    typedef doublex4 acc_t;
    static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // accumulator register r of lane l holds row l / 16 + 4 r, column l % 16
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

constexpr int kGM = 64, kGN = 64, kGK = 32;

template <typename T> struct GemmLds {
    static constexpr int PAD = sizeof(T) == 4 ? 4 : 2;  // conflict-free 16-byte row reads
    static constexpr int LDK = kGK + PAD;
};

// Loads one 64 x 32 tile row-slice per thread group: thread t covers row
// t / 4 and k = (t % 4) * 8 .. + 7 (8 elements).
template <typename TA>
__device__ __forceinline__ void load8(const TA *src, bool ok, TA (&v)[8]) {
    if (!ok) {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (TA)0;
        return;
    }
    if constexpr (sizeof(TA) == 4) {
        const float4 a = *(const float4 *)src, b = *(const float4 *)(src + 4);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double2 a = *(const double2 *)(src + 2 * q);
            v[2 * q] = a.x;
            v[2 * q + 1] = a.y;
        }
    }
}

template <typename T, typename TA>
__device__ __forceinline__ void store8(T *dst, const TA (&v)[8]) {
    if constexpr (sizeof(T) == 4) {
        *(float4 *)dst = make_float4(v[0], v[1], v[2], v[3]);
        *(float4 *)(dst + 4) = make_float4(v[4], v[5], v[6], v[7]);
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) *(double2 *)(dst + 2 * q) = make_double2((double)v[2 * q], (double)v[2 * q + 1]);
    }
}

template <typename T>
__device__ __forceinline__ void lds4(const T *src, T (&v)[4]) {
    if constexpr (sizeof(T) == 4) {
        const float4 a = *(const float4 *)src;
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    } else {
        const double2 a = *(const double2 *)src, b = *(const double2 *)(src + 2);
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    }
}

template <typename T, typename TA>
__global__ void __launch_bounds__(kBlock) gemm_kernel(const TA *Q, int64_t ld, const T *X,
                                                      const int32_t *active,
                                                      const int32_t *nactive, T *U,
                                                      int64_t slice, int64_t kchunk, int MT,
                                                      int NT, int KS) {
    typedef typename Mfma<T>::acc_t acc_t;
    constexpr int LDK = GemmLds<T>::LDK;
    __shared__ __attribute__((aligned(16))) T As[2][kGM * LDK];
    __shared__ __attribute__((aligned(16))) T Bs[2][kGN * LDK];
    // XCD-aware order: consecutive tile ids (same Q block, different column
    // tiles) go to blocks dispatched on the same XCD
    const int total = MT * NT * KS;
    const int per = (total + 7) / 8;
    const int L = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (L >= total) return;
    const int nt = L % NT, mt = (L / NT) % MT, kz = L / (NT * MT);
    const int nact = *nactive;
    const int n0 = nt * kGN;
    if (n0 >= nact) return;
    const int64_t m0 = (int64_t)mt * kGM;
    const int64_t kbeg = (int64_t)kz * kchunk;
    const int64_t kend = min(ld, kbeg + kchunk);
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
    const int lrow = t >> 2, lk = (t & 3) * 8;
    const int64_t grow = m0 + lrow;
    const bool arow_ok = grow < ld;
    const TA *Ap = Q + (arow_ok ? grow : 0) * ld + lk;
    const int bslot = n0 + lrow;
    const bool bcol_ok = bslot < nact;
    const T *Bp = X + (bcol_ok ? (int64_t)active[bslot] : 0) * ld + lk;
    acc_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
    TA ra[8];
    T rb[8];
    int buf = 0;
    if (kbeg < kend) {
        load8<TA>(Ap + kbeg, arow_ok, ra);
        load8<T>(Bp + kbeg, bcol_ok, rb);
        store8<T, TA>(&As[0][lrow * LDK + lk], ra);
        store8<T, T>(&Bs[0][lrow * LDK + lk], rb);
    }
    __syncthreads();
    const int cc = lane & 15, g = lane >> 4;
    for (int64_t k0 = kbeg; k0 < kend; k0 += kGK) {
        const bool more = k0 + kGK < kend;
        if (more) {  // prefetch the next chunk into registers
            load8<TA>(Ap + k0 + kGK, arow_ok, ra);
            load8<T>(Bp + k0 + kGK, bcol_ok, rb);
        }
        const T *as = As[buf], *bs = Bs[buf];
#pragma unroll
        for (int sc = 0; sc < kGK; sc += 16) {
            T a0[4], a1[4], b0[4], b1[4];
            lds4<T>(as + (wm + cc) * LDK + sc + 4 * g, a0);
            lds4<T>(as + (wm + 16 + cc) * LDK + sc + 4 * g, a1);
            lds4<T>(bs + (wn + cc) * LDK + sc + 4 * g, b0);
            lds4<T>(bs + (wn + 16 + cc) * LDK + sc + 4 * g, b1);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                acc[0][0] = Mfma<T>::run(a0[e], b0[e], acc[0][0]);
                acc[0][1] = Mfma<T>::run(a0[e], b1[e], acc[0][1]);
                acc[1][0] = Mfma<T>::run(a1[e], b0[e], acc[1][0]);
                acc[1][1] = Mfma<T>::run(a1[e], b1[e], acc[1][1]);
            }
        }
        if (more) {
            store8<T, TA>(&As[buf ^ 1][lrow * LDK + lk], ra);
            store8<T, T>(&Bs[buf ^ 1][lrow * LDK + lk], rb);
        }
        __syncthreads();
        buf ^= 1;
    }
    T *Us = U + (int64_t)kz * slice;
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) {
        const int slot = n0 + wn + ni * 16 + cc;
        if (slot >= nact) continue;
        const int64_t c = active[slot];
#pragma unroll
        for (int mi = 0; mi < 2; ++mi) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = m0 + wm + mi * 16 + Mfma<T>::row(lane, r);
                if (row < ld) Us[c * ld + row] = acc[mi][ni][r];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Wave-streaming MFMA product for few columns (the common case of the sweep
// loop): no LDS and no barriers. Each wave owns 16 rows of Q, one K range and
// one group of up to 64 live columns (NT tiles of 16). Lane l = m + 16 g
// loads the 16-byte run k = k0 + 4 g .. + 3 of Q row m and of live column
// 16 t + m, and feeds one element to each of four MFMA 16x16x4 (the same
// K permutation as the tiled kernel). The K loop is unrolled UNR times so
// that several chunks of Q are in flight per wave.

template <typename T> struct Vec4;
template <> struct Vec4<float> {
    static __device__ __forceinline__ void load(const float *p, float (&v)[4]) {
        const float4 a = *(const float4 *)p;
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    }
};
template <> struct Vec4<double> {
    static __device__ __forceinline__ void load(const double *p, double (&v)[4]) {
        const double2 a = *(const double2 *)p, b = *(const double2 *)(p + 2);
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    }
};

template <typename T> struct StreamArgs {
    const float *Q;
    int64_t ld;
    const T *X;
    const int32_t *active;
    const int32_t *nactive;
    T *U;
    int64_t slice, kchunk;
    int MT, KS, NG;
};

template <typename T, int NT, int UNR>
__device__ __forceinline__ void stream_body(const StreamArgs<T> &sa, int gb) {
    typedef typename Mfma<T>::acc_t acc_t;
    __shared__ acc_t part[kWaves - 1][NT][64];
    const float *Q = sa.Q;
    const int64_t ld = sa.ld;
    const T *X = sa.X;
    const int32_t *active = sa.active;
    T *U = sa.U;
    const int64_t slice = sa.slice, kchunk = sa.kchunk;
    const int MT = sa.MT, KS = sa.KS, NG = sa.NG;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (gb >= MT * KS * NG) return;
    const int mt = gb % MT, kz = (gb / MT) % KS, ng0 = gb / (MT * KS);
    const int nact = *sa.nactive;
    const int m = lane & 15, g = lane >> 4;
    const int64_t m0 = (int64_t)mt * 16;
    // the block's K range, split into kWaves contiguous parts (multiples of 16)
    const int64_t kb = (int64_t)kz * kchunk;
    const int64_t ke = min(ld, kb + kchunk);
    const int64_t nchunks = ke > kb ? (ke - kb) / 16 : 0;
    const int64_t per = (nchunks + kWaves - 1) / kWaves;
    const int64_t kbeg = kb + 16 * min(nchunks, per * wv);
    const int64_t kend = kb + 16 * min(nchunks, per * (wv + 1));
    const float *qrow = Q + (m0 + m) * ld + 4 * g;
    T *Us = U + (int64_t)kz * slice;
    // column groups ng0, ng0 + NG, ...: the grid may be sized from an
    // estimate of the live count; the loop covers the actual one
    for (int c0 = ng0 * 16 * NT; c0 < nact; c0 += NG * 16 * NT) {  // uniform over the block
        const T *xcol[NT];
        bool ok[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int slot = c0 + 16 * t + m;
            ok[t] = slot < nact;
            xcol[t] = X + (ok[t] ? (int64_t)active[slot] : 0) * ld + 4 * g;
        }
        acc_t acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = acc_t{0, 0, 0, 0};
        int64_t k0 = kbeg;
        for (; k0 + 16 * UNR <= kend; k0 += 16 * UNR) {
            float a[UNR][4];
            T b[UNR][NT][4];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                Vec4<float>::load(qrow + k0 + 16 * u, a[u]);
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    if (ok[t]) Vec4<T>::load(xcol[t] + k0 + 16 * u, b[u][t]);
                    else b[u][t][0] = b[u][t][1] = b[u][t][2] = b[u][t][3] = (T)0;
                }
            }
#pragma unroll
            for (int u = 0; u < UNR; ++u)
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int t = 0; t < NT; ++t) acc[t] = Mfma<T>::run((T)a[u][e], b[u][t][e], acc[t]);
        }
        for (; k0 < kend; k0 += 16) {
            float a[4];
            Vec4<float>::load(qrow + k0, a);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                T b[4] = {(T)0, (T)0, (T)0, (T)0};
                if (ok[t]) Vec4<T>::load(xcol[t] + k0, b);
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[t] = Mfma<T>::run((T)a[e], b[e], acc[t]);
            }
        }
        // deterministic reduction of the four K parts: wave 0 adds waves 1..3 in order
        __syncthreads();  // the previous group's partials have been read
        if (wv > 0) {
#pragma unroll
            for (int t = 0; t < NT; ++t) part[wv - 1][t][lane] = acc[t];
        }
        __syncthreads();
        if (wv == 0) {
#pragma unroll
            for (int q = 0; q < kWaves - 1; ++q)
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const acc_t o = part[q][t][lane];
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[t][r] += o[r];
                }
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                if (!ok[t]) continue;
                const int64_t c = active[c0 + 16 * t + m];
#pragma unroll
                for (int r = 0; r < 4; ++r) Us[c * ld + m0 + Mfma<T>::row(lane, r)] = acc[t][r];
            }
        }
    }
}

template <typename T, int NT, int UNR>
__global__ void __launch_bounds__(kBlock) stream_kernel(StreamArgs<T> sa) {
    stream_body<T, NT, UNR>(sa, blockIdx.x);
}

// Both products of a split-precision sweep in one launch: the first nb1
// blocks compute the FP32 product of the subproblem columns, the rest the
// FP64 product (exactly widened FP32 Q) of the lambda_min / CG columns.
template <int NT1, int UNR1, int NT2, int UNR2>
__global__ void __launch_bounds__(kBlock) stream2_kernel(StreamArgs<float> a, StreamArgs<double> b,
                                                         int nb1) {
    if ((int)blockIdx.x < nb1) stream_body<float, NT1, UNR1>(a, blockIdx.x);
    else stream_body<double, NT2, UNR2>(b, blockIdx.x - nb1);
}

// Wave-streaming product from an FP32 copy of Q: dtype PSDP_F32 (FP32 MFMA)
// or kGemmF32QF64 (FP64 MFMA on the exactly widened entries). nt (1, 2 or 4)
// is the number of 16-column tiles per block; the grid is sized for ncol
// columns (an estimate) and blocks loop over further groups, so neither nt
// nor ncol affects the result, only the speed.
// ncol is the number of columns the grid is sized for (an estimate of the
// live count is enough: blocks loop over further column groups).
template <typename T>
static StreamArgs<T> stream_args(const void *Qop, int64_t ld, const void *op, void *U,
                                 const int32_t *active, const int32_t *nactive, int64_t slice,
                                 int ksplit, int ncol, int nt) {
    int64_t kchunk = (ld + ksplit - 1) / ksplit;
    kchunk = (kchunk + 15) / 16 * 16;
    StreamArgs<T> a;
    a.Q = (const float *)Qop;
    a.ld = ld;
    a.X = (const T *)op;
    a.active = active;
    a.nactive = nactive;
    a.U = (T *)U;
    a.slice = slice;
    a.kchunk = kchunk;
    a.MT = (int)(ld / 16);
    a.KS = ksplit;
    a.NG = std::max(1, (ncol + 16 * nt - 1) / (16 * nt));
    return a;
}

template <typename T, int NT, int UNR>
static void stream_go(const StreamArgs<T> &a, hipStream_t st) {
    hipLaunchKernelGGL((stream_kernel<T, NT, UNR>), dim3((unsigned)(a.MT * a.KS * a.NG)), dim3(kBlock), 0, st, a);
}

hipError_t launch_stream(int dtype, const void *Qop, int64_t ld, const void *op, void *U,
                         const int32_t *active, const int32_t *nactive, int64_t slice, int ksplit,
                         int ncol_max, int nt, hipStream_t st) {
    if (dtype == PSDP_F32) {
        auto a = stream_args<float>(Qop, ld, op, U, active, nactive, slice, ksplit, ncol_max, nt <= 1 ? 1 : (nt == 2 ? 2 : 4));
        if (nt <= 1) stream_go<float, 1, 8>(a, st);
        else if (nt == 2) stream_go<float, 2, 8>(a, st);
        else stream_go<float, 4, 4>(a, st);
    } else if (dtype == kGemmF32QF64) {
        auto a = stream_args<double>(Qop, ld, op, U, active, nactive, slice, ksplit, ncol_max, nt <= 1 ? 1 : (nt == 2 ? 2 : 4));
        if (nt <= 1) stream_go<double, 1, 8>(a, st);
        else if (nt == 2) stream_go<double, 2, 4>(a, st);
        else stream_go<double, 4, 2>(a, st);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int NT1, int UNR1, int NT2, int UNR2>
static void stream2_go(const StreamArgs<float> &a, const StreamArgs<double> &b, hipStream_t st) {
    const int nb1 = a.MT * a.KS * a.NG, nb2 = b.MT * b.KS * b.NG;
    hipLaunchKernelGGL((stream2_kernel<NT1, UNR1, NT2, UNR2>), dim3((unsigned)(nb1 + nb2)), dim3(kBlock), 0, st,
                       a, b, nb1);
}

template <int NT1, int UNR1>
static void stream2_second(const StreamArgs<float> &a, const StreamArgs<double> &b, int nt2, hipStream_t st) {
    if (nt2 <= 1) stream2_go<NT1, UNR1, 1, 8>(a, b, st);
    else if (nt2 == 2) stream2_go<NT1, UNR1, 2, 4>(a, b, st);
    else stream2_go<NT1, UNR1, 4, 2>(a, b, st);
}

// FP32 product (subproblem columns) and FP64 product (lambda_min / CG
// columns) of one sweep, both from the FP32 copy of Q, in one launch.
hipError_t launch_stream2(const void *Qop, int64_t ld, const void *op1, void *U1, const int32_t *active1,
                          const int32_t *nactive1, int64_t slice1, int ks1, int nt1, const void *op2,
                          void *U2, const int32_t *active2, const int32_t *nactive2, int64_t slice2,
                          int ks2, int nt2, int ncol1, int ncol2, hipStream_t st) {
    nt1 = nt1 <= 1 ? 1 : (nt1 == 2 ? 2 : 4);
    nt2 = nt2 <= 1 ? 1 : (nt2 == 2 ? 2 : 4);
    auto a = stream_args<float>(Qop, ld, op1, U1, active1, nactive1, slice1, ks1, ncol1, nt1);
    auto b = stream_args<double>(Qop, ld, op2, U2, active2, nactive2, slice2, ks2, ncol2, nt2);
    if (nt1 == 1) stream2_second<1, 8>(a, b, nt2, st);
    else if (nt1 == 2) stream2_second<2, 8>(a, b, nt2, st);
    else stream2_second<4, 4>(a, b, nt2, st);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Launchers.

// Four rows per wave once Q no longer fits the caches (n >= 8192: 256 MB in
// FP32), one row per wave below (more blocks for the smaller grids).
template <typename QT, int R>
static void gemv_go(const Inst *in, const Work &w, int ncol_max, hipStream_t st) {
    const dim3 grid((unsigned)((in->n + kWaves * R - 1) / (kWaves * R)), (unsigned)ncol_max);
    hipLaunchKernelGGL((gemv_kernel<QT, R>), grid, dim3(kBlock), 0, st, (const QT *)in->Qop, in->n, in->ld,
                       (const double *)w.op, (double *)w.U, w.active, w.nactive);
}

template <typename QT>
static void gemv_pick(const Inst *in, const Work &w, int ncol_max, hipStream_t st) {
    if (in->n >= 8192) gemv_go<QT, 4>(in, w, ncol_max, st);
    else gemv_go<QT, 1>(in, w, ncol_max, st);
}

hipError_t launch_gemv(int dtype, const Inst *in, int, const Work &w, int ncol_max,
                       hipStream_t st) {
    if (dtype == PSDP_F64) gemv_pick<double>(in, w, ncol_max, st);
    else if (dtype == PSDP_F32) gemv_pick<float>(in, w, ncol_max, st);
    else gemv_pick<__hip_bfloat16>(in, w, ncol_max, st);
    return hipGetLastError();
}

hipError_t launch_gemv_group(int dtype, const Work &w, const int64_t *rowstart, const int32_t *unitcol,
                             int64_t total_rows, hipStream_t st) {
    // total_rows counts units of 4 rows (rowstart in the same units)
    const dim3 grid((unsigned)((total_rows + kWaves - 1) / kWaves));
    const double *op = (const double *)w.op;
    double *U = (double *)w.U;
    if (dtype == PSDP_F64)
        hipLaunchKernelGGL(gemv_group_kernel<double>, grid, dim3(kBlock), 0, st, w.col, w.inst,
                           rowstart, unitcol, total_rows, op, U);
    else if (dtype == PSDP_F32)
        hipLaunchKernelGGL(gemv_group_kernel<float>, grid, dim3(kBlock), 0, st, w.col, w.inst,
                           rowstart, unitcol, total_rows, op, U);
    else
        hipLaunchKernelGGL(gemv_group_kernel<__hip_bfloat16>, grid, dim3(kBlock), 0, st, w.col,
                           w.inst, rowstart, unitcol, total_rows, op, U);
    return hipGetLastError();
}

// dtype: PSDP_F32 (FP32 Q and X, FP32 MFMA), PSDP_F64 (FP64 Q and X, FP64
// MFMA) or kGemmF32QF64 (FP32-stored Q widened exactly, FP64 X, FP64 MFMA).
hipError_t launch_gemm(int dtype, const void *Qop, int64_t ld, const void *op, void *U,
                       const int32_t *active, const int32_t *nactive, int64_t slice, int ksplit,
                       int ncol_max, hipStream_t st) {
    int64_t kchunk = (ld + ksplit - 1) / ksplit;
    kchunk = (kchunk + kGK - 1) / kGK * kGK;
    const int MT = (int)((ld + kGM - 1) / kGM), NT = (ncol_max + kGN - 1) / kGN;
    const int total = MT * NT * ksplit;
    const dim3 grid((unsigned)((total + 7) / 8 * 8));
    if (dtype == PSDP_F32)
        hipLaunchKernelGGL((gemm_kernel<float, float>), grid, dim3(kBlock), 0, st, (const float *)Qop, ld,
                           (const float *)op, active, nactive, (float *)U, slice, kchunk, MT, NT, ksplit);
    else if (dtype == PSDP_F64)
        hipLaunchKernelGGL((gemm_kernel<double, double>), grid, dim3(kBlock), 0, st, (const double *)Qop,
                           ld, (const double *)op, active, nactive, (double *)U, slice, kchunk, MT, NT,
                           ksplit);
    else if (dtype == kGemmF32QF64)
        hipLaunchKernelGGL((gemm_kernel<double, float>), grid, dim3(kBlock), 0, st, (const float *)Qop,
                           ld, (const double *)op, active, nactive, (double *)U, slice, kchunk, MT, NT,
                           ksplit);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace psdp
