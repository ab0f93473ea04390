// Q.X products of the vectorized PSDP solver: the O(n^2) part of every
// penalty-gradient evaluation grad h = 2 (Q - Diag p) x + (b + p) (eq. (kkt1)),
// of every lambda_min matvec (eq. (alpha)) and every x^0 CG matvec
// (eq. (gamma)). All kernels compute U[:, c] = Qop X[:, c] for the live
// columns c listed in `active` (Qop: zero-diagonal operand copy, row-major,
// leading dimension ld, a multiple of 16 with zero padding).
//
//  gemv_kernel        one instance, few columns: one wave per row, 16-byte
//                     coalesced loads of Q, FP64 accumulation, x in FP64.
//  gemv_group_kernel  uneven instances: the rows of every live instance form
//                     one flat work list (one wave per row).
//  gemm_*_kernel      one instance, many columns: MFMA tiles (FP32 16x16x4 or
//                     FP64 16x16x4) staged through LDS, split over K into
//                     separate output slices that the solver sums in order.
#include "common.hpp"

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

// grid (ceil(n / 4), ncol_max): block = 4 waves = 4 rows of one column.
template <typename QT>
__global__ void __launch_bounds__(kBlock) gemv_kernel(const QT *Qop, int64_t n, int64_t ld,
                                                      const double *op, double *U,
                                                      const int32_t *active,
                                                      const int32_t *nactive) {
    const int slot = blockIdx.y;
    if (slot >= *nactive) return;
    const int64_t ci = active[slot];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t row = (int64_t)blockIdx.x * kWaves + wv;
    if (row >= n) return;
    const double acc = row_dot<QT>(Qop + row * ld, op + ci * ld, ld, lane);
    if (lane == 0) U[ci * ld + row] = acc;
}

// Flat rows of all columns: rowstart[c] .. rowstart[c+1]-1 belong to column c.
template <typename QT>
__global__ void __launch_bounds__(kBlock) gemv_group_kernel(const Col *col, const Inst *inst,
                                                            const int64_t *rowstart, int ncol,
                                                            int64_t total, const double *op,
                                                            double *U) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t r = (int64_t)blockIdx.x * kWaves + wv;
    if (r >= total) return;
    int lo = 0, hi = ncol - 1;  // last c with rowstart[c] <= r
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (rowstart[mid] <= r) lo = mid;
        else hi = mid - 1;
    }
    const Col &c = col[lo];
    if (c.phase == PH_DONE) return;
    const Inst &in = inst[c.inst];
    const int64_t row = r - rowstart[lo];
    const double acc = row_dot<QT>((const QT *)in.Qop + row * in.ld, op + c.off, in.ld, lane);
    if (lane == 0) U[c.off + row] = acc;
}

// ---------------------------------------------------------------------------
// MFMA GEMM: block tile BM x BN (BM = BN = 64), 4 waves each 32 x 32 made of
// 2 x 2 MFMA 16x16 tiles. MFMA 16x16x4 operand layout (wave64): lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; the accumulator rows differ
// between the FP32 and FP64 instructions (Mfma<T>::row, measured on gfx950).

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

template <typename T, int BK>
__global__ void __launch_bounds__(kBlock) gemm_kernel(const T *Q, int64_t ld, const T *X,
                                                      const int32_t *active,
                                                      const int32_t *nactive, T *U,
                                                      int64_t slice, int64_t kchunk) {
    constexpr int BM = 64, BN = 64, PAD = 16;
    constexpr int VEC = 16 / sizeof(T);           // elements per 16-byte load
    constexpr int LOADS = BK / 4 / VEC;           // 16-byte loads per thread per tile row quarter
    typedef typename Mfma<T>::acc_t acc_t;
    const int nact = *nactive;
    const int n0 = blockIdx.y * BN;
    if (n0 >= nact) return;
    const int64_t m0 = (int64_t)blockIdx.x * BM;
    const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
    const int64_t kend = min(ld, kbeg + kchunk);
    __shared__ T As[BK][BM + PAD];
    __shared__ T Bs[BK][BN + PAD];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
    acc_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
    // each thread stages BK/4 consecutive k of one A row and one B column
    const int lrow = t >> 2, lk = (t & 3) * (BK / 4);
    const int64_t grow = m0 + lrow;
    const bool arow_ok = grow < ld;
    const T *Ap = Q + (arow_ok ? grow : 0) * ld;
    const int bslot = n0 + lrow;
    const bool bcol_ok = bslot < nact;
    const T *Bp = X + (bcol_ok ? (int64_t)active[bslot] : 0) * ld;
    for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
        T av[BK / 4], bv[BK / 4];
#pragma unroll
        for (int q = 0; q < LOADS; ++q) {
            typedef T vec_t __attribute__((ext_vector_type(VEC)));
            vec_t a = arow_ok ? *(const vec_t *)(Ap + k0 + lk + q * VEC) : vec_t{};
            vec_t b = bcol_ok ? *(const vec_t *)(Bp + k0 + lk + q * VEC) : vec_t{};
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                av[q * VEC + e] = a[e];
                bv[q * VEC + e] = b[e];
            }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < BK / 4; ++e) {
            As[lk + e][lrow] = av[e];
            Bs[lk + e][lrow] = bv[e];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            const int kr = kk + (lane >> 4), cc = lane & 15;
            const T a0 = As[kr][wm + cc], a1 = As[kr][wm + 16 + cc];
            const T b0 = Bs[kr][wn + cc], b1 = Bs[kr][wn + 16 + cc];
            acc[0][0] = Mfma<T>::run(a0, b0, acc[0][0]);
            acc[0][1] = Mfma<T>::run(a0, b1, acc[0][1]);
            acc[1][0] = Mfma<T>::run(a1, b0, acc[1][0]);
            acc[1][1] = Mfma<T>::run(a1, b1, acc[1][1]);
        }
    }
    T *Us = U + (int64_t)blockIdx.z * slice;
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) {
        const int slot = n0 + wn + ni * 16 + (lane & 15);
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
// Launchers.

hipError_t launch_gemv(int dtype, const Inst *in, int, const Work &w, int ncol_max,
                       hipStream_t st) {
    const dim3 grid((unsigned)((in->n + kWaves - 1) / kWaves), (unsigned)ncol_max);
    const double *op = (const double *)w.op;
    double *U = (double *)w.U;
    if (dtype == PSDP_F64)
        hipLaunchKernelGGL(gemv_kernel<double>, grid, dim3(kBlock), 0, st, (const double *)in->Qop,
                           in->n, in->ld, op, U, w.active, w.nactive);
    else if (dtype == PSDP_F32)
        hipLaunchKernelGGL(gemv_kernel<float>, grid, dim3(kBlock), 0, st, (const float *)in->Qop,
                           in->n, in->ld, op, U, w.active, w.nactive);
    else
        hipLaunchKernelGGL(gemv_kernel<__hip_bfloat16>, grid, dim3(kBlock), 0, st,
                           (const __hip_bfloat16 *)in->Qop, in->n, in->ld, op, U, w.active,
                           w.nactive);
    return hipGetLastError();
}

hipError_t launch_gemv_group(int dtype, const Work &w, const int64_t *rowstart, int64_t total_rows,
                             hipStream_t st) {
    const dim3 grid((unsigned)((total_rows + kWaves - 1) / kWaves));
    const double *op = (const double *)w.op;
    double *U = (double *)w.U;
    if (dtype == PSDP_F64)
        hipLaunchKernelGGL(gemv_group_kernel<double>, grid, dim3(kBlock), 0, st, w.col, w.inst,
                           rowstart, w.ncol, total_rows, op, U);
    else if (dtype == PSDP_F32)
        hipLaunchKernelGGL(gemv_group_kernel<float>, grid, dim3(kBlock), 0, st, w.col, w.inst,
                           rowstart, w.ncol, total_rows, op, U);
    else
        hipLaunchKernelGGL(gemv_group_kernel<__hip_bfloat16>, grid, dim3(kBlock), 0, st, w.col,
                           w.inst, rowstart, w.ncol, total_rows, op, U);
    return hipGetLastError();
}

hipError_t launch_gemm(int dtype, const void *Qop, int64_t ld, const void *op, void *U,
                       const int32_t *active, const int32_t *nactive, int64_t slice, int ksplit,
                       int ncol_max, hipStream_t st) {
    int64_t kchunk = (ld + ksplit - 1) / ksplit;
    kchunk = (kchunk + 15) / 16 * 16;
    const dim3 grid((unsigned)((ld + 63) / 64), (unsigned)((ncol_max + 63) / 64), (unsigned)ksplit);
    if (dtype == PSDP_F32)
        hipLaunchKernelGGL((gemm_kernel<float, 16>), grid, dim3(kBlock), 0, st, (const float *)Qop, ld,
                           (const float *)op, active, nactive, (float *)U, slice, kchunk);
    else if (dtype == PSDP_F64)
        hipLaunchKernelGGL((gemm_kernel<double, 16>), grid, dim3(kBlock), 0, st, (const double *)Qop,
                           ld, (const double *)op, active, nactive, (double *)U, slice, kchunk);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace psdp
