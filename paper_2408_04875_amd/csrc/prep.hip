// Instance preparation and finalization kernels.
//
//  - prep_q: Q~ = Q + mu (Section 3.5, "Random Perturbation") written as the
//    Q.X operand with a zero diagonal (the diagonal, its reformation shift
//    gamma and the penalty stay in FP64 on the solver side), plus the FP64
//    row data R_i = sum_{j != i} |Q~_ij| and dq_i = Q~_ii used by the
//    reformation gamma (Section 3.5, "Reformation"), rho (Section 3.3) and
//    H_p (Section 3.1).
//  - perturbation: the perturbation matrix alone (test hook).
//  - round_objective: x^_i = [x_i > 1/2] and f(x^) = x^T Q x^ + b^T x^ in
//    exact integer arithmetic on the original data (Section 2, eq. (bqp)).
#include "common.hpp"

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

__device__ __forceinline__ double perturbed(const int32_t *Q, int64_t n, int64_t i, int64_t j,
                                            int perturb, double sigma, uint64_t key) {
    double q = (double)Q[i * n + j];
    if (perturb == PSDP_PERTURB_FULL || (perturb == PSDP_PERTURB_DIAG && i == j)) {
        const int64_t a = i < j ? i : j, c = i < j ? j : i;
        q = q + perturb_entry(key, n, a, c, sigma);
    }
    return q;
}

// One block per operand row i < ld (rows n..ld-1 are zero padding).
template <typename QT>
__global__ void __launch_bounds__(kBlock) prep_q_kernel(const int32_t *Q, int64_t n, int64_t ld,
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

// Host-side mixing of the seed into the stream key (same function on the host).
static uint64_t splitmix64_host(uint64_t state) {
    uint64_t z = state + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

hipError_t launch_prep_q(int dtype, const int32_t *Q, int64_t n, int64_t ld, int perturb,
                         double sigma, uint64_t seed, void *Qop, double *R, double *dq,
                         hipStream_t st) {
    const uint64_t key = splitmix64_host(seed);
    if (sigma == 0.0) perturb = PSDP_PERTURB_NONE;
    if (dtype == PSDP_F64)
        hipLaunchKernelGGL(prep_q_kernel<double>, dim3(ld), dim3(kBlock), 0, st, Q, n, ld, perturb,
                           sigma, key, (double *)Qop, R, dq);
    else if (dtype == PSDP_F32)
        hipLaunchKernelGGL(prep_q_kernel<float>, dim3(ld), dim3(kBlock), 0, st, Q, n, ld, perturb,
                           sigma, key, (float *)Qop, R, dq);
    else if (dtype == PSDP_I8)
        hipLaunchKernelGGL(prep_q_kernel<int8_t>, dim3(ld), dim3(kBlock), 0, st, Q, n, ld, perturb,
                           sigma, key, (int8_t *)Qop, R, dq);
    else
        hipLaunchKernelGGL(prep_q_kernel<__hip_bfloat16>, dim3(ld), dim3(kBlock), 0, st, Q, n, ld,
                           perturb, sigma, key, (__hip_bfloat16 *)Qop, R, dq);
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
