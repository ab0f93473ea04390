// Penalty value/gradient evaluation and its adjoint.
//
// eval:    h(x_c, p) = x_c^T Q x_c + b^T x_c + sum_i p_i (x_ci - x_ci^2)
//          (eq. (p1)) and G[:, c] = 2 (Q - Diag p) x_c + (b + p) (eq. (kkt1)),
//          from U = Q X computed by the MFMA GEMM (F32/F64, aligned shapes)
//          or by a plain FP64-accumulating GEMV (any shape, any dtype).
// adjoint: for L = sum_c w_c h(x_c, p) (h linear in Q, b, p):
//          dX = G Diag(w), dQ = X Diag(w) X^T (MFMA, operands read straight
//          from the columns of X), db = X w, dp = (X - X o X) w.
#include "launch.hpp"

namespace psdp {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename T> __device__ __forceinline__ double ld64(const T *p, int64_t i) {
    return to_f64<T>(p[i]);
}

// U[c * n + i] = sum_j Q[i * ldq + j] X[c * n + j], one wave per (row, column).
template <typename QT>
__global__ void __launch_bounds__(kBlock) eval_gemv_kernel(const QT *Q, int64_t ldq, const QT *X,
                                                           int64_t n, int64_t B, double *U) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t r = (int64_t)blockIdx.x * kWaves + wv;
    const int64_t c = blockIdx.y;
    if (r >= n || c >= B) return;
    const QT *q = Q + r * ldq;
    const QT *x = X + c * n;
    double a0 = 0.0, a1 = 0.0;
    int64_t j = lane;
    for (; j + 64 < n; j += 128) {
        a0 = fma(ld64(q, j), ld64(x, j), a0);
        a1 = fma(ld64(q, j + 64), ld64(x, j + 64), a1);
    }
    if (j < n) a0 = fma(ld64(q, j), ld64(x, j), a0);
    double acc = a0 + a1;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) U[c * n + r] = acc;
}

// h and G for column c from U (type UT), X (type XT), b, p (type VT).
template <typename UT, typename XT, typename VT>
__global__ void __launch_bounds__(kBlock) eval_epilogue_kernel(const UT *U, int64_t ldu,
                                                               const XT *X, const VT *b,
                                                               const VT *p, int64_t n, VT *h,
                                                               VT *G) {
    const int64_t c = blockIdx.x;
    __shared__ double red[kWaves];
    double acc[1] = {0.0};
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
        const double x = to_f64<XT>(X[c * n + i]);
        const double u = to_f64<UT>(U[c * ldu + i]);
        const double bi = to_f64<VT>(b[i]), pi = to_f64<VT>(p[i]);
        acc[0] += x * u + bi * x + pi * (x - x * x);
        if (G) G[c * n + i] = from_f64<VT>(2.0 * (u - pi * x) + (bi + pi));
    }
    block_sum<1>(acc, red);
    if (threadIdx.x == 0) h[c] = from_f64<VT>(acc[0]);
}

__global__ void iota_kernel(int32_t *a, int32_t *cnt, int B) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < B) a[i] = i;
    if (i == 0) *cnt = B;
}

// ---------------------------------------------------------------------------
// Adjoint.

template <typename T> struct MfmaA;
template <> struct MfmaA<float> {
    typedef floatx4 acc_t;
    static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <> struct MfmaA<double> {
    typedef doublex4 acc_t;
    static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

// dQ[i][j] = sum_c w_c X[c n + i] X[c n + j]; block tile 64 x 64, K = columns.
template <typename T, typename VT>
__global__ void __launch_bounds__(kBlock) outer_gemm_kernel(const T *X, const VT *w, int64_t n,
                                                            int64_t B, T *dQ) {
    constexpr int BM = 64, BN = 64, BK = 16, PAD = 16;
    typedef typename MfmaA<T>::acc_t acc_t;
    const int64_t m0 = (int64_t)blockIdx.x * BM, n0 = (int64_t)blockIdx.y * BN;
    __shared__ T As[BK][BM + PAD];
    __shared__ T Bs[BK][BN + PAD];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
    acc_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
    const int lrow = t & 63, lk = (t >> 6) * 4;  // 64 rows x 4 k per thread group
    for (int64_t k0 = 0; k0 < B; k0 += BK) {
        T av[4], bv[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t c = k0 + lk + e;
            const int64_t i = m0 + lrow, j = n0 + lrow;
            const bool cok = c < B;
            const double wc = cok ? to_f64<VT>(w[c]) : 0.0;
            av[e] = (cok && i < n) ? (T)(wc * (double)X[c * n + i]) : (T)0;
            bv[e] = (cok && j < n) ? X[c * n + j] : (T)0;
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            As[lk + e][lrow] = av[e];
            Bs[lk + e][lrow] = bv[e];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            const int kr = kk + (lane >> 4), cc = lane & 15;
            const T a0 = As[kr][wm + cc], a1 = As[kr][wm + 16 + cc];
            const T b0 = Bs[kr][wn + cc], b1 = Bs[kr][wn + 16 + cc];
            acc[0][0] = MfmaA<T>::run(a0, b0, acc[0][0]);
            acc[0][1] = MfmaA<T>::run(a0, b1, acc[0][1]);
            acc[1][0] = MfmaA<T>::run(a1, b0, acc[1][0]);
            acc[1][1] = MfmaA<T>::run(a1, b1, acc[1][1]);
        }
    }
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) {
        const int64_t j = n0 + wn + ni * 16 + (lane & 15);
        if (j >= n) continue;
#pragma unroll
        for (int mi = 0; mi < 2; ++mi) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = m0 + wm + mi * 16 + MfmaA<T>::row(lane, r);
                if (i < n) dQ[i * n + j] = acc[mi][ni][r];
            }
        }
    }
}

// dX[c n + i] = w_c G[c n + i]; db_i = sum_c w_c x_ci; dp_i = sum_c w_c (x_ci - x_ci^2).
template <typename T, typename VT>
__global__ void adjoint_vec_kernel(const T *X, const VT *G, const VT *w, int64_t n, int64_t B,
                                   VT *dX, VT *db, VT *dp) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double sb = 0.0, sp = 0.0;
    for (int64_t c = 0; c < B; ++c) {
        const double wc = to_f64<VT>(w[c]);
        const double x = to_f64<T>(X[c * n + i]);
        sb += wc * x;
        sp += wc * (x - x * x);
        if (dX) dX[c * n + i] = from_f64<VT>(wc * to_f64<VT>(G[c * n + i]));
    }
    if (db) db[i] = from_f64<VT>(sb);
    if (dp) dp[i] = from_f64<VT>(sp);
}

// ---------------------------------------------------------------------------

template <typename QT, typename VT>
static hipError_t eval_typed(const QT *Q, int64_t ldq, const VT *b, const VT *p, const QT *X,
                             int64_t n, int64_t B, VT *h, VT *G, double *ws, hipStream_t st) {
    // ws holds U as doubles (n x B)
    const dim3 grid((unsigned)((n + kWaves - 1) / kWaves), (unsigned)B);
    hipLaunchKernelGGL(eval_gemv_kernel<QT>, grid, dim3(kBlock), 0, st, Q, ldq, X, n, B, ws);
    hipLaunchKernelGGL((eval_epilogue_kernel<double, QT, VT>), dim3(B), dim3(kBlock), 0, st,
                       (const double *)ws, n, X, b, p, n, h, G);
    return hipGetLastError();
}

// MFMA path for aligned F32/F64 shapes: U slices in the operand type.
template <typename T, typename VT>
static hipError_t eval_mfma(const T *Q, int64_t n, const VT *b, const VT *p, const T *X,
                            int64_t B, VT *h, VT *G, double *ws, hipStream_t st) {
    // ws layout: [U (n x B of T)] [active (B int32)] [nactive]
    T *U = (T *)ws;
    int32_t *active = (int32_t *)(U + n * B);
    int32_t *nact = active + B;
    hipLaunchKernelGGL(iota_kernel, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, st, active, nact,
                       (int)B);
    hipError_t e = launch_gemm(sizeof(T) == 4 ? PSDP_F32 : PSDP_F64, Q, n, X, U, active, nact, n * B, 1,
                               (int)B, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((eval_epilogue_kernel<T, T, VT>), dim3(B), dim3(kBlock), 0, st, (const T *)U,
                       n, X, b, p, n, h, G);
    return hipGetLastError();
}

hipError_t launch_eval(int dtype, int vtype, const void *Q, int64_t ldq, const void *b,
                       const void *p, const void *X, int64_t n, int64_t B, void *h, void *G,
                       double *ws, hipStream_t st) {
    const bool aligned = (n % 32 == 0) && (ldq == n) && ((uintptr_t)Q % 16 == 0) &&
                         ((uintptr_t)X % 16 == 0);
#define EVAL_V(QT, VT)                                                                          \
    return (aligned && dtype != PSDP_BF16)                                                      \
               ? eval_mfma<QT, VT>((const QT *)Q, n, (const VT *)b, (const VT *)p,              \
                                   (const QT *)X, B, (VT *)h, (VT *)G, ws, st)                  \
               : eval_typed<QT, VT>((const QT *)Q, ldq, (const VT *)b, (const VT *)p,           \
                                    (const QT *)X, n, B, (VT *)h, (VT *)G, ws, st);
    if (dtype == PSDP_F64 && vtype == PSDP_F64) { EVAL_V(double, double) }
    if (dtype == PSDP_F64 && vtype == PSDP_F32) { EVAL_V(double, float) }
    if (dtype == PSDP_F32 && vtype == PSDP_F64) { EVAL_V(float, double) }
    if (dtype == PSDP_F32 && vtype == PSDP_F32) { EVAL_V(float, float) }
#undef EVAL_V
    if (dtype == PSDP_BF16 && vtype == PSDP_F64)
        return eval_typed<__hip_bfloat16, double>((const __hip_bfloat16 *)Q, ldq, (const double *)b,
                                                  (const double *)p, (const __hip_bfloat16 *)X, n,
                                                  B, (double *)h, (double *)G, ws, st);
    if (dtype == PSDP_BF16 && vtype == PSDP_F32)
        return eval_typed<__hip_bfloat16, float>((const __hip_bfloat16 *)Q, ldq, (const float *)b,
                                                 (const float *)p, (const __hip_bfloat16 *)X, n, B,
                                                 (float *)h, (float *)G, ws, st);
    return hipErrorInvalidValue;
}

template <typename T, typename VT>
static hipError_t adjoint_typed(const T *X, const VT *G, const VT *w, int64_t n, int64_t B, VT *dX,
                                T *dQ, VT *db, VT *dp, hipStream_t st) {
    if (dX || db || dp)
        hipLaunchKernelGGL((adjoint_vec_kernel<T, VT>), dim3((unsigned)((n + 255) / 256)), dim3(256),
                           0, st, X, G, w, n, B, dX, db, dp);
    if (dQ) {
        const dim3 grid((unsigned)((n + 63) / 64), (unsigned)((n + 63) / 64));
        hipLaunchKernelGGL((outer_gemm_kernel<T, VT>), grid, dim3(kBlock), 0, st, X, w, n, B, dQ);
    }
    return hipGetLastError();
}

hipError_t launch_adjoint(int dtype, int vtype, const void *X, const void *G, const void *w,
                          int64_t n, int64_t B, void *dX, void *dQ, void *db, void *dp,
                          hipStream_t st) {
    if (dtype == PSDP_F32 && vtype == PSDP_F32)
        return adjoint_typed<float, float>((const float *)X, (const float *)G, (const float *)w, n, B,
                                           (float *)dX, (float *)dQ, (float *)db, (float *)dp, st);
    if (dtype == PSDP_F32 && vtype == PSDP_F64)
        return adjoint_typed<float, double>((const float *)X, (const double *)G, (const double *)w,
                                            n, B, (double *)dX, (float *)dQ, (double *)db,
                                            (double *)dp, st);
    if (dtype == PSDP_F64 && vtype == PSDP_F64)
        return adjoint_typed<double, double>((const double *)X, (const double *)G,
                                             (const double *)w, n, B, (double *)dX, (double *)dQ,
                                             (double *)db, (double *)dp, st);
    if (dtype == PSDP_F64 && vtype == PSDP_F32)
        return adjoint_typed<double, float>((const double *)X, (const float *)G, (const float *)w, n,
                                            B, (float *)dX, (double *)dQ, (float *)db, (float *)dp,
                                            st);
    return hipErrorInvalidValue;
}

}  // namespace psdp
