// Input checks of an integer instance on the device (the problem statement of
// Section 2 takes Q symmetric; the solve entry points reject anything else
// before they start): exact symmetry with the first offending entry, the
// largest |Q_ij| overall and off the diagonal, the largest |b_i|, the
// off-diagonal nonzeros of every row (for the sparse-row products), starts
// X0 in [0,1] and a finite p0. One pass over Q in 32 x 32 tiles: a block
// compares its tile with the transposed tile through LDS. The host reads a
// few words back instead of the whole matrix.
#include <algorithm>

#include "common.hpp"

namespace psdp {

constexpr int kCT = 32;  // tile edge; blocks of kCT x 8 threads, 4 rows each

__global__ void __launch_bounds__(256) check_q_kernel(const int32_t *Q, int64_t n, CheckOut *o,
                                                      int32_t *rownnz) {
    __shared__ int32_t tB[kCT][kCT + 1];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int64_t i0 = (int64_t)blockIdx.y * kCT, j0 = (int64_t)blockIdx.x * kCT;
    // tile B = Q[j0.., i0..], stored so that tB[c][r] = Q[j0 + r][i0 + c]
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int r = ty + 8 * k;
        const int64_t gi = j0 + r, gj = i0 + tx;
        tB[tx][r] = (gi < n && gj < n) ? Q[gi * n + gj] : 0;
    }
    __syncthreads();
    uint64_t amax = 0, omax = 0, bad = ~0ull;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int r = ty + 8 * k;
        const int64_t i = i0 + r, j = j0 + tx;
        const bool in = i < n && j < n;
        const int32_t v = in ? Q[i * n + j] : 0;
        if (in) {
            // Q[j][i] is tB[r][tx] (= Q[j0 + tx][i0 + r])
            if (v != tB[r][tx]) bad = min(bad, (uint64_t)(i * n + j));
            const uint64_t a = (uint64_t)(v < 0 ? -(int64_t)v : (int64_t)v);
            amax = max(amax, a);
            if (i != j) omax = max(omax, a);
        }
        if (rownnz) {
            // the 32 lanes of this row sit in one half of the wave
            const uint64_t m = __ballot(in && i != j && v != 0);
            const int cnt = __popcll((threadIdx.x & 32) ? (m >> 32) : (m & 0xffffffffull));
            if (tx == 0 && i < n && cnt) atomicAdd(&rownnz[i], cnt);
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        amax = max(amax, (uint64_t)__shfl_xor((long long)amax, off, 64));
        omax = max(omax, (uint64_t)__shfl_xor((long long)omax, off, 64));
        bad = min(bad, (uint64_t)__shfl_xor((long long)bad, off, 64));
    }
    // lane 0 of every wave updates the totals, and only where it would
    // change them (a relaxed read filters the contended atomics: the totals
    // only grow, so a stale read costs at most one atomic more)
    if ((threadIdx.x & 63) == 0) {
        if (amax > __hip_atomic_load(&o->qmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax((unsigned long long *)&o->qmax, (unsigned long long)amax);
        if (omax > __hip_atomic_load(&o->offmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax((unsigned long long *)&o->offmax, (unsigned long long)omax);
        if (bad != ~0ull) atomicMin((unsigned long long *)&o->first_asym, (unsigned long long)bad);
    }
}

__global__ void __launch_bounds__(256) check_vec_kernel(const int32_t *b, int64_t n, const double *X0, int64_t nx,
                                                        const double *p0, CheckOut *o) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * 256;
    uint64_t bm = 0, xbad = 0, pbad = 0;
    for (int64_t i = t; i < n; i += stride) {
        const int64_t v = b[i];
        bm = max(bm, (uint64_t)(v < 0 ? -v : v));
        if (p0 && !isfinite(p0[i])) ++pbad;
    }
    if (X0)
        for (int64_t i = t; i < nx; i += stride) {
            const double v = X0[i];
            if (!(v >= 0.0 && v <= 1.0)) ++xbad;
        }
    for (int off = 32; off >= 1; off >>= 1) {
        bm = max(bm, (uint64_t)__shfl_xor((long long)bm, off, 64));
        xbad += (uint64_t)__shfl_xor((long long)xbad, off, 64);
        pbad += (uint64_t)__shfl_xor((long long)pbad, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (bm) atomicMax((unsigned long long *)&o->bmax, (unsigned long long)bm);
        if (xbad) atomicAdd((unsigned long long *)&o->x0_bad, (unsigned long long)xbad);
        if (pbad) atomicAdd((unsigned long long *)&o->p0_bad, (unsigned long long)pbad);
    }
}

__global__ void check_init_kernel(CheckOut *o) {
    if (threadIdx.x == 0) {
        o->qmax = o->offmax = o->bmax = o->x0_bad = o->p0_bad = 0;
        o->first_asym = ~0ull;
    }
}

hipError_t launch_check(const int32_t *Q, const int32_t *b, int64_t n, const double *X0, int64_t nx,
                        const double *p0, CheckOut *o, int32_t *rownnz, hipStream_t st) {
    if (n < 1 || n > 65536) return hipErrorInvalidValue;
    hipLaunchKernelGGL(check_init_kernel, dim3(1), dim3(64), 0, st, o);
    const unsigned t = (unsigned)((n + kCT - 1) / kCT);
    hipLaunchKernelGGL(check_q_kernel, dim3(t, t), dim3(256), 0, st, Q, n, o, rownnz);
    const int64_t work = std::max<int64_t>(n, X0 ? nx : 0);
    const unsigned g = (unsigned)std::min<int64_t>(1024, (work + 255) / 256);
    hipLaunchKernelGGL(check_vec_kernel, dim3(g), dim3(256), 0, st, b, n, X0, nx, p0, o);
    return hipGetLastError();
}

}  // namespace psdp
