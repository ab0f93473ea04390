// Input checks of an instance on the device (the problem statement of
// Section 2 takes Q symmetric and real; the solve entry points reject
// anything else before they start): exact symmetry with the first offending
// entry, the largest |Q_ij| overall and off the diagonal, the largest |b_i|,
// the off-diagonal nonzeros of every row (for the sparse-row products),
// starts X0 in [0,1] and a finite p0. For real (FP64) data also the
// non-finite entries and the off-diagonal entries that an operand type
// could not hold exactly (non-integral or beyond 127 for int8, not a float
// or not a bfloat16). One pass over Q in 32 x 32 tiles: a block compares its
// tile with the transposed tile through LDS. The host reads a few words back
// instead of the whole matrix. Magnitudes of real data are returned as the
// bit patterns of non-negative doubles, whose unsigned order is their
// numeric order.
#include <algorithm>
#include <type_traits>

#include "launch.hpp"

namespace psdp {

constexpr int kCT = 32;  // tile edge; blocks of kCT x 8 threads, 4 rows each

template <typename T> __device__ __forceinline__ uint64_t mag_bits(T v) {
    if constexpr (std::is_same<T, double>::value) return (uint64_t)__double_as_longlong(fabs(v));
    else return (uint64_t)(v < 0 ? -(int64_t)v : (int64_t)v);
}

template <typename T>
__global__ void __launch_bounds__(256) check_q_kernel(const T *Q, int64_t n, CheckOut *o, int32_t *rownnz) {
    constexpr bool kReal = std::is_same<T, double>::value;
    __shared__ T tB[kCT][kCT + 1];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int64_t i0 = (int64_t)blockIdx.y * kCT, j0 = (int64_t)blockIdx.x * kCT;
    // tile B = Q[j0.., i0..], stored so that tB[c][r] = Q[j0 + r][i0 + c]
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int r = ty + 8 * k;
        const int64_t gi = j0 + r, gj = i0 + tx;
        tB[tx][r] = (gi < n && gj < n) ? Q[gi * n + gj] : (T)0;
    }
    __syncthreads();
    uint64_t amax = 0, omax = 0, bad = ~0ull;
    uint64_t nonfin = 0, nonint = 0, non32 = 0, non16 = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int r = ty + 8 * k;
        const int64_t i = i0 + r, j = j0 + tx;
        const bool in = i < n && j < n;
        const T v = in ? Q[i * n + j] : (T)0;
        if (in) {
            bool fin = true;
            if constexpr (kReal) {
                fin = isfinite(v);
                if (!fin) ++nonfin;
                if (fin && i != j) {
                    if (!(rint(v) == v && fabs(v) <= 127.0)) ++nonint;
                    if ((double)__double2float_rn(v) != v) ++non32;
                    if ((double)__bfloat162float(__float2bfloat16(__double2float_rn(v))) != v ||
                        (double)__double2float_rn(v) != v)
                        ++non16;
                }
            }
            // Q[j][i] is tB[r][tx] (= Q[j0 + tx][i0 + r]); a NaN is reported as
            // non-finite, not as an asymmetry
            if (fin && v != tB[r][tx]) bad = min(bad, (uint64_t)(i * n + j));
            if (fin) {
                const uint64_t a = mag_bits(v);
                amax = max(amax, a);
                if (i != j) omax = max(omax, a);
            }
        }
        if (rownnz) {
            // the 32 lanes of this row sit in one half of the wave
            const uint64_t m = __ballot(in && i != j && v != (T)0);
            const int cnt = __popcll((threadIdx.x & 32) ? (m >> 32) : (m & 0xffffffffull));
            if (tx == 0 && i < n && cnt) atomicAdd(&rownnz[i], cnt);
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        amax = max(amax, (uint64_t)__shfl_xor((long long)amax, off, 64));
        omax = max(omax, (uint64_t)__shfl_xor((long long)omax, off, 64));
        bad = min(bad, (uint64_t)__shfl_xor((long long)bad, off, 64));
        if constexpr (kReal) {
            nonfin += (uint64_t)__shfl_xor((long long)nonfin, off, 64);
            nonint += (uint64_t)__shfl_xor((long long)nonint, off, 64);
            non32 += (uint64_t)__shfl_xor((long long)non32, off, 64);
            non16 += (uint64_t)__shfl_xor((long long)non16, off, 64);
        }
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
        if (nonfin) atomicAdd((unsigned long long *)&o->nonfinite, (unsigned long long)nonfin);
        if (nonint) atomicAdd((unsigned long long *)&o->nonint_off, (unsigned long long)nonint);
        if (non32) atomicAdd((unsigned long long *)&o->non32_off, (unsigned long long)non32);
        if (non16) atomicAdd((unsigned long long *)&o->non16_off, (unsigned long long)non16);
    }
}

template <typename T>
__global__ void __launch_bounds__(256) check_vec_kernel(const T *b, int64_t n, const double *X0, int64_t nx,
                                                        const double *p0, CheckOut *o) {
    constexpr bool kReal = std::is_same<T, double>::value;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * 256;
    uint64_t bm = 0, xbad = 0, pbad = 0, bbad = 0;
    for (int64_t i = t; i < n; i += stride) {
        const T v = b[i];
        if constexpr (kReal) {
            if (!isfinite(v)) ++bbad;
            else bm = max(bm, mag_bits(v));
        } else {
            bm = max(bm, mag_bits(v));
        }
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
        bbad += (uint64_t)__shfl_xor((long long)bbad, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (bm) atomicMax((unsigned long long *)&o->bmax, (unsigned long long)bm);
        if (xbad) atomicAdd((unsigned long long *)&o->x0_bad, (unsigned long long)xbad);
        if (pbad) atomicAdd((unsigned long long *)&o->p0_bad, (unsigned long long)pbad);
        if (bbad) atomicAdd((unsigned long long *)&o->nonfinite, (unsigned long long)bbad);
    }
}

__global__ void check_init_kernel(CheckOut *o) {
    if (threadIdx.x == 0) {
        o->qmax = o->offmax = o->bmax = o->x0_bad = o->p0_bad = 0;
        o->nonfinite = o->nonint_off = o->non32_off = o->non16_off = 0;
        o->first_asym = ~0ull;
    }
}

template <typename T>
static hipError_t check_typed(const T *Q, const T *b, int64_t n, const double *X0, int64_t nx, const double *p0,
                              CheckOut *o, int32_t *rownnz, hipStream_t st) {
    if (n < 1 || n > 65536) return hipErrorInvalidValue;
    hipLaunchKernelGGL(check_init_kernel, dim3(1), dim3(64), 0, st, o);
    const unsigned t = (unsigned)((n + kCT - 1) / kCT);
    hipLaunchKernelGGL(check_q_kernel<T>, dim3(t, t), dim3(256), 0, st, Q, n, o, rownnz);
    const int64_t work = std::max<int64_t>(n, X0 ? nx : 0);
    const unsigned g = (unsigned)std::min<int64_t>(1024, (work + 255) / 256);
    hipLaunchKernelGGL(check_vec_kernel<T>, dim3(g), dim3(256), 0, st, b, n, X0, nx, p0, o);
    return hipGetLastError();
}

hipError_t launch_check(const int32_t *Q, const int32_t *b, int64_t n, const double *X0, int64_t nx,
                        const double *p0, CheckOut *o, int32_t *rownnz, hipStream_t st) {
    return check_typed<int32_t>(Q, b, n, X0, nx, p0, o, rownnz, st);
}

hipError_t launch_check(const double *Q, const double *b, int64_t n, const double *X0, int64_t nx,
                        const double *p0, CheckOut *o, int32_t *rownnz, hipStream_t st) {
    return check_typed<double>(Q, b, n, X0, nx, p0, o, rownnz, st);
}

}  // namespace psdp
