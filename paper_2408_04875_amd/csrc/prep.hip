// Instance preparation and finalization kernels.
//
//  - prep_q: Q~ = Q + mu (Section 3.5, "Random Perturbation") written as the
//    Q.X operand with a zero diagonal (the diagonal, its reformation shift
//    gamma and the penalty stay in FP64 on the solver side), plus the FP64
//    row data R_i = sum_{j != i} |Q~_ij| and dq_i = Q~_ii used by the
//    reformation gamma (Section 3.5, "Reformation"), rho (Section 3.3) and
//    H_p (Section 3.1).
//  - perturbation: the perturbation matrix alone (test hook).
//  - round_objective: x^_i = [x_i > 1/2] and f(x^) = x^T Q x^ + b^T x^ on the
//    original data (Section 2, eq. (bqp)): exact integer arithmetic for
//    integer data, the exact sum rounded once to FP64 for real data.
#include "launch.hpp"

namespace psdp {

__device__ __forceinline__ uint64_t splitmix64(uint64_t state) {
    uint64_t z = state + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// mu_ij for i <= j: Irwin-Hall(4) sum of 53-bit uniforms from a counter-based
// SplitMix64 stream keyed by the mixed seed, rescaled to unit variance, times
// sigma, rounded to the 2^-16 grid with ties to even.
__device__ __forceinline__ double perturb_entry(uint64_t key, int64_t n, int64_t i, int64_t j,
                                                double sigma) {
    uint64_t S = 0;
    const uint64_t base = ((uint64_t)i * (uint64_t)n + (uint64_t)j) * 4ull;
#pragma unroll
    for (int t = 0; t < 4; ++t) S += splitmix64(key ^ (base + (uint64_t)t)) >> 11;
    const double N = (__ull2double_rn(S) * 0x1p-53 - 2.0) * 1.7320508075688772;
    return rint((N * sigma) * 65536.0) / 65536.0;
}

template <typename QIn>
__device__ __forceinline__ double perturbed(const QIn *Q, int64_t n, int64_t i, int64_t j,
                                            int perturb, double sigma, uint64_t key) {
    double q = (double)Q[i * n + j];
    if (perturb == PSDP_PERTURB_FULL || (perturb == PSDP_PERTURB_DIAG && i == j)) {
        const int64_t a = i < j ? i : j, c = i < j ? j : i;
        q = q + perturb_entry(key, n, a, c, sigma);
    }
    return q;
}

// One block per operand row i < ld (rows n..ld-1 are zero padding). For
// real data the perturbed entry is Q_ij + mu_ij rounded once to FP64, and R_i
// sums in the block's fixed order (integer data sums exactly).
template <typename QT, typename QIn>
__global__ void __launch_bounds__(kBlock) prep_q_kernel(const QIn *Q, int64_t n, int64_t ld,
                                                        int perturb, double sigma, uint64_t key,
                                                        QT *Qop, double *R, double *dq) {
    const int64_t i = blockIdx.x;
    __shared__ double red[kWaves];
    double acc[1] = {0.0};
    for (int64_t j = threadIdx.x; j < ld; j += kBlock) {
        double q = 0.0;
        if (i < n && j < n) q = perturbed(Q, n, i, j, perturb, sigma, key);
        if (j == i) {
            Qop[i * ld + j] = from_f64<QT>(0.0);
        } else {
            acc[0] += fabs(q);
            Qop[i * ld + j] = from_f64<QT>(q);
        }
    }
    block_sum<1>(acc, red);
    if (threadIdx.x == 0) {
        R[i] = acc[0];
        dq[i] = i < n ? perturbed(Q, n, i, i, perturb, sigma, key) : 0.0;
    }
}

__global__ void perturbation_kernel(int64_t n, double sigma, uint64_t key, int mode, double *mu) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * n) return;
    const int64_t i = idx / n, j = idx % n;
    double v = 0.0;
    if (mode == PSDP_PERTURB_FULL || (mode == PSDP_PERTURB_DIAG && i == j)) {
        const int64_t a = i < j ? i : j, c = i < j ? j : i;
        v = perturb_entry(key, n, a, c, sigma);
    }
    mu[idx] = v;
}

// x^ = [X > 1/2], column-major outputs.
__global__ void round_kernel(const double *X, int64_t ldx, int64_t n, int64_t B, uint8_t *xhat,
                             int64_t ldh) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * B) return;
    const int64_t c = idx / n, i = idx % n;
    xhat[c * ldh + i] = X[c * ldx + i] > 0.5 ? 1 : 0;
}

// partial[c * nblk + blk] = sum over the block's rows i with x^_i = 1 of
// sum_j Q_ij x^_j, in int64 (exact). One wave per row.
constexpr int kObjRows = 16;
__global__ void __launch_bounds__(kBlock) objective_partial_kernel(const int32_t *Q, int64_t n,
                                                                   const uint8_t *xhat, int64_t ldh,
                                                                   int64_t nblk, int64_t *partial) {
    const int64_t c = blockIdx.y;
    const int64_t blk = blockIdx.x;
    const uint8_t *xh = xhat + c * ldh;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __shared__ long long red[kWaves];
    long long acc = 0;
    for (int r = wv; r < kObjRows; r += kWaves) {
        const int64_t i = blk * kObjRows + r;
        if (i >= n || !xh[i]) continue;
        const int32_t *row = Q + i * n;
        for (int64_t j = lane; j < n; j += 64)
            if (xh[j]) acc += (long long)row[j];
    }
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) red[wv] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long s = 0;
        for (int q = 0; q < kWaves; ++q) s += red[q];
        partial[c * nblk + blk] = (int64_t)s;
    }
}

__global__ void __launch_bounds__(kBlock) objective_final_kernel(const int32_t *b, int64_t n,
                                                                 const uint8_t *xhat, int64_t ldh,
                                                                 int64_t nblk,
                                                                 const int64_t *partial,
                                                                 int64_t *obj) {
    const int64_t c = blockIdx.x;
    const uint8_t *xh = xhat + c * ldh;
    __shared__ long long red[kWaves];
    long long acc = 0;
    for (int64_t i = threadIdx.x; i < n; i += kBlock)
        if (xh[i]) acc += (long long)b[i];
    for (int64_t t = threadIdx.x; t < nblk; t += kBlock) acc += (long long)partial[c * nblk + t];
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long s = 0;
        for (int q = 0; q < kWaves; ++q) s += red[q];
        obj[c] = (int64_t)s;
    }
}

// ---------------------------------------------------------------------------
// Real data: the objective as the exact sum of its terms, rounded once.
//
// Every finite double is v = (-1)^s M 2^(e - 1075) with an integer
// mantissa M < 2^53 and e = max(biased exponent, 1), so v 2^1074 is the
// integer +-M 2^(e - 1). The terms of one column are accumulated exactly in
// integers bucketed by e: acc[e] collects the signed high parts M >> 26
// (< 2^27) and acc[2048 + e] the low parts M mod 2^26. With at most
// 2^32 + 2^16 terms no bucket leaves int64. The final kernel expands the
// buckets into a big integer N = sum_e (hi_e 2^26 + lo_e) 2^(e - 1) of
// 32-bit limbs, normalizes it and rounds N 2^-1074 to the nearest double
// (ties to even). The result is independent of the order of the terms.

__device__ __forceinline__ void obj_term(double v, long long *hi, long long *lo) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const int E = (int)((u >> 52) & 0x7ff);
    uint64_t M = u & 0xfffffffffffffull;
    if (E != 0) M |= 1ull << 52;
    if (M == 0) return;
    const int e = E == 0 ? 1 : E;
    const long long h = (long long)(M >> 26), l = (long long)(M & 0x3ffffffull);
    const bool neg = (u >> 63) != 0;
    atomicAdd((unsigned long long *)&hi[e], (unsigned long long)(neg ? -h : h));
    atomicAdd((unsigned long long *)&lo[e], (unsigned long long)(neg ? -l : l));
}

// Block (blk, c): rows blk * kObjRowsReal .. of column c; block 0 adds b.
constexpr int kObjRowsReal = 64;
__global__ void __launch_bounds__(kBlock) objective_real_partial_kernel(const double *Q, const double *b, int64_t n,
                                                                        const uint8_t *xhat, int64_t ldh,
                                                                        int64_t *acc) {
    __shared__ long long bk[2 * 2048];
    const int64_t c = blockIdx.y, blk = blockIdx.x;
    const uint8_t *xh = xhat + c * ldh;
    for (int t = threadIdx.x; t < 2 * 2048; t += kBlock) bk[t] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int r = wv; r < kObjRowsReal; r += kWaves) {
        const int64_t i = blk * kObjRowsReal + r;
        if (i >= n || !xh[i]) continue;
        const double *row = Q + i * n;
        for (int64_t j = lane; j < n; j += 64)
            if (xh[j]) obj_term(row[j], bk, bk + 2048);
    }
    if (blk == 0)
        for (int64_t i = threadIdx.x; i < n; i += kBlock)
            if (xh[i]) obj_term(b[i], bk, bk + 2048);
    __syncthreads();
    int64_t *a = acc + c * kObjAccWords;
    for (int t = threadIdx.x; t < 2 * 2048; t += kBlock)
        if (bk[t] != 0) atomicAdd((unsigned long long *)&a[t], (unsigned long long)bk[t]);
}

constexpr int kLimbs = 72;  // 32-bit limbs (in int64 slots) of N: bits up to 2^2304

// adds t 2^sh to the limbs (t signed, |t| < 2^61); every addend is below
// 2^32 in magnitude, so the limbs absorb all 4096 buckets without overflow
__device__ __forceinline__ void limb_add(long long *L, long long t, int sh) {
    const int q = sh >> 5, r = sh & 31;
    const unsigned long long a0 = (unsigned long long)t & 0xffffffffull;
    const long long t1 = t >> 32;
    const unsigned long long A = a0 << r;
    const long long T1 = (long long)((unsigned long long)t1 << r);
    atomicAdd((unsigned long long *)&L[q], A & 0xffffffffull);
    atomicAdd((unsigned long long *)&L[q + 1], (A >> 32) + ((unsigned long long)T1 & 0xffffffffull));
    atomicAdd((unsigned long long *)&L[q + 2], (unsigned long long)(T1 >> 32));
}

// limbs normalized to [0, 2^32) below the top, which keeps the sign
__device__ void limb_carry(long long *L) {
    for (int k = 0; k + 1 < kLimbs; ++k) {
        const long long cy = L[k] >> 32;
        L[k] -= cy << 32;
        L[k + 1] += cy;
    }
}

// 64 bits of N >> pos (pos >= 0) from normalized limbs
__device__ __forceinline__ unsigned long long limb_window(const long long *L, int pos) {
    const int q = pos >> 5, r = pos & 31;
    const unsigned long long lo = (unsigned long long)L[q] | ((unsigned long long)L[q + 1] << 32);
    const unsigned long long hi = (unsigned long long)L[q + 2];
    return r ? (lo >> r) | (hi << (64 - r)) : lo;
}

__global__ void __launch_bounds__(kBlock) objective_real_final_kernel(int64_t *acc, double *obj) {
    __shared__ long long L[kLimbs];
    const int64_t c = blockIdx.x;
    int64_t *a = acc + c * kObjAccWords;
    for (int t = threadIdx.x; t < kLimbs; t += kBlock) L[t] = 0;
    __syncthreads();
    for (int e = threadIdx.x; e < 2048; e += kBlock) {
        const long long h = a[e], l = a[2048 + e];
        if (h) limb_add(L, h, e - 1 + 26);
        if (l) limb_add(L, l, e - 1);
        a[e] = 0;  // leave the scratch zero for the next use
        a[2048 + e] = 0;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    limb_carry(L);
    const bool neg = L[kLimbs - 1] < 0;
    if (neg) {
        for (int k = 0; k < kLimbs; ++k) L[k] = -L[k];
        limb_carry(L);
    }
    int top = kLimbs - 1;
    while (top >= 0 && L[top] == 0) --top;
    double v = 0.0;
    if (top >= 0) {
        const int p = 32 * top + (31 - __clz((unsigned)L[top]));  // highest set bit of N
        if (p <= 52) {
            v = ldexp((double)((unsigned long long)L[0] | ((unsigned long long)L[1] << 32)), -1074);
        } else {
            // m = bits p-52 .. p; then the round bit and the sticky bits below
            unsigned long long w;
            bool sticky;
            if (p < 63) {
                w = limb_window(L, 0) << (63 - p);
                sticky = false;
            } else {
                const int pos = p - 63;
                w = limb_window(L, pos);
                sticky = false;
                const int q = pos >> 5, r = pos & 31;
                for (int k = 0; k < q; ++k) sticky |= L[k] != 0;
                if (r) sticky |= (L[q] & ((1ll << r) - 1)) != 0;
            }
            unsigned long long m = w >> 11;
            const bool rbit = (w >> 10) & 1;
            sticky |= (w & 0x3ffull) != 0;
            if (rbit && (sticky || (m & 1))) ++m;
            v = ldexp((double)m, p - 52 - 1074);
        }
    }
    obj[c] = neg ? -v : v;
}

// Host-side mixing of the seed into the stream key (same function on the host).
static uint64_t splitmix64_host(uint64_t state) {
    uint64_t z = state + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <typename QIn>
static hipError_t prep_typed(int dtype, const QIn *Q, int64_t n, int64_t ld, int perturb, double sigma,
                             uint64_t seed, void *Qop, double *R, double *dq, hipStream_t st) {
    const uint64_t key = splitmix64_host(seed);
    if (sigma == 0.0) perturb = PSDP_PERTURB_NONE;
    if (dtype == PSDP_F64)
        hipLaunchKernelGGL((prep_q_kernel<double, QIn>), dim3(ld), dim3(kBlock), 0, st, Q, n, ld, perturb,
                           sigma, key, (double *)Qop, R, dq);
    else if (dtype == PSDP_F32)
        hipLaunchKernelGGL((prep_q_kernel<float, QIn>), dim3(ld), dim3(kBlock), 0, st, Q, n, ld, perturb,
                           sigma, key, (float *)Qop, R, dq);
    else if (dtype == PSDP_I8)
        hipLaunchKernelGGL((prep_q_kernel<int8_t, QIn>), dim3(ld), dim3(kBlock), 0, st, Q, n, ld, perturb,
                           sigma, key, (int8_t *)Qop, R, dq);
    else
        hipLaunchKernelGGL((prep_q_kernel<__hip_bfloat16, QIn>), dim3(ld), dim3(kBlock), 0, st, Q, n, ld,
                           perturb, sigma, key, (__hip_bfloat16 *)Qop, R, dq);
    return hipGetLastError();
}

hipError_t launch_prep_q(int dtype, const int32_t *Q, int64_t n, int64_t ld, int perturb,
                         double sigma, uint64_t seed, void *Qop, double *R, double *dq,
                         hipStream_t st) {
    return prep_typed<int32_t>(dtype, Q, n, ld, perturb, sigma, seed, Qop, R, dq, st);
}

hipError_t launch_prep_q(int dtype, const double *Q, int64_t n, int64_t ld, int perturb,
                         double sigma, uint64_t seed, void *Qop, double *R, double *dq,
                         hipStream_t st) {
    return prep_typed<double>(dtype, Q, n, ld, perturb, sigma, seed, Qop, R, dq, st);
}

// gamma_i = 2 sum_j |Q~_ij| + |b_i| + 1 (Section 3.5, strict margin 1), b
// as FP64, and the reformulated data's diagonal dgi_i = Q~_ii + gamma_i and
// linear term lni_i = b_i - gamma_i (Algorithm 3, reformation); zero in the
// padding up to ld.
template <typename BT>
__global__ void gamma_kernel(const BT *b, const double *R, const double *dq, int64_t n, int64_t ld, double *bd,
                             double *gam, double *dgi, double *lni) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ld) return;
    if (i < n) {
        const double bi = (double)b[i];
        const double g = 2.0 * (R[i] + fabs(dq[i])) + fabs(bi) + 1.0;
        bd[i] = bi;
        gam[i] = g;
        dgi[i] = dq[i] + g;
        lni[i] = bi - g;
    } else {
        bd[i] = 0.0;
        gam[i] = 0.0;
        dgi[i] = 0.0;
        lni[i] = 0.0;
    }
}

hipError_t launch_gamma(const int32_t *b, const double *R, const double *dq, int64_t n, int64_t ld,
                        double *bd, double *gam, double *dgi, double *lni, hipStream_t st) {
    hipLaunchKernelGGL(gamma_kernel<int32_t>, dim3((unsigned)((ld + 255) / 256)), dim3(256), 0, st, b, R, dq, n,
                       ld, bd, gam, dgi, lni);
    return hipGetLastError();
}

hipError_t launch_gamma(const double *b, const double *R, const double *dq, int64_t n, int64_t ld,
                        double *bd, double *gam, double *dgi, double *lni, hipStream_t st) {
    hipLaunchKernelGGL(gamma_kernel<double>, dim3((unsigned)((ld + 255) / 256)), dim3(256), 0, st, b, R, dq, n,
                       ld, bd, gam, dgi, lni);
    return hipGetLastError();
}

hipError_t launch_perturbation(int64_t n, double sigma, uint64_t seed, int mode, double *mu,
                               hipStream_t st) {
    const int64_t tot = n * n;
    const int64_t blocks = (tot + kBlock - 1) / kBlock;
    if (sigma == 0.0) mode = PSDP_PERTURB_NONE;
    hipLaunchKernelGGL(perturbation_kernel, dim3(blocks), dim3(kBlock), 0, st, n, sigma,
                       splitmix64_host(seed), mode, mu);
    return hipGetLastError();
}

hipError_t launch_round_objective(const int32_t *Q, const int32_t *b, int64_t n,
                                  const double *X, int64_t ldx, int64_t B, uint8_t *xhat,
                                  int64_t ldh, int64_t *obj, int64_t *partial, hipStream_t st) {
    const int64_t tot = n * B;
    hipLaunchKernelGGL(round_kernel, dim3((tot + kBlock - 1) / kBlock), dim3(kBlock), 0, st, X, ldx,
                       n, B, xhat, ldh);
    const int64_t nblk = (n + kObjRows - 1) / kObjRows;
    hipLaunchKernelGGL(objective_partial_kernel, dim3(nblk, B), dim3(kBlock), 0, st, Q, n, xhat, ldh,
                       nblk, partial);
    hipLaunchKernelGGL(objective_final_kernel, dim3(B), dim3(kBlock), 0, st, b, n, xhat, ldh, nblk,
                       partial, obj);
    return hipGetLastError();
}

}  // namespace psdp

namespace psdp {

hipError_t launch_round_objective(const double *Q, const double *b, int64_t n, const double *X, int64_t ldx,
                                  int64_t B, uint8_t *xhat, int64_t ldh, double *obj, int64_t *acc, hipStream_t st) {
    const int64_t tot = n * B;
    hipLaunchKernelGGL(round_kernel, dim3((tot + kBlock - 1) / kBlock), dim3(kBlock), 0, st, X, ldx, n, B, xhat, ldh);
    const int64_t nblk = (n + kObjRowsReal - 1) / kObjRowsReal;
    hipLaunchKernelGGL(objective_real_partial_kernel, dim3(nblk, B), dim3(kBlock), 0, st, Q, b, n, xhat, ldh, acc);
    hipLaunchKernelGGL(objective_real_final_kernel, dim3(B), dim3(kBlock), 0, st, acc, obj);
    return hipGetLastError();
}

}  // namespace psdp
