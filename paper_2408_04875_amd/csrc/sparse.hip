// Exact integer Q.X products from a compressed sparse row copy of Q_off, for
// the I8 operand path when Q is sparse (Max-Cut graphs, 10%-density
// instances) and few columns are live. They produce the same integers as the
// dense digit products (qx8.hip), so the solver may use either for any sweep
// without changing a result.
//
// Storage: row i's nonzeros Q_ij (j != i) at rowptr[i] .. rowptr[i + 1] - 1,
// in increasing j, each packed in one 32-bit word: j in bits 0-15 (n <= 65536)
// and the int8 value in bits 16-23. Operand: the integer grid values of each
// column as int32 words, T = rint(x 2^27) for a subproblem iterate and the
// two halves T = T_hi 2^28 + T_lo of a lambda_min / CG vector (the split the
// digit planes encode). Every product Q_ij T_j is below 2^34 and a row sum
// below 2^51, so int64 accumulation is exact.
//
// One wave per row: lanes stride over the row's nonzeros, each lane keeps
// int64 partial sums for a group of columns, and the wave adds them with
// lane exchanges; lane 0 stores the result.
#include "launch.hpp"

namespace psdp {

// ---------------------------------------------------------------------------
// Building the rows from the int8 operand copy (row-major, leading dimension
// ldq, zero diagonal); the row starts come from the row nonzero counts of the
// input checks.

__global__ void __launch_bounds__(kBlock) csr_fill_kernel(const int8_t *Q8, int64_t ldq, int64_t n,
                                                          const int32_t *rowptr, uint32_t *pk) {
    const int64_t i = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= n) return;
    const int8_t *row = Q8 + i * ldq;
    const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    int64_t pos = rowptr[i];
    for (int64_t j0 = 0; j0 < n; j0 += 64) {
        const int64_t j = j0 + lane;
        const int8_t v = j < n ? row[j] : (int8_t)0;
        const unsigned long long m = __ballot(v != 0);
        if (v != 0) pk[pos + __popcll(m & below)] = (uint32_t)j | ((uint32_t)(uint8_t)v << 16);
        pos += __popcll(m);
    }
}

hipError_t launch_csr_fill(const int8_t *Q8, int64_t ldq, int64_t n, const int32_t *rowptr, uint32_t *pk,
                           hipStream_t st) {
    const unsigned grid = (unsigned)((n + kBlock / 64 - 1) / (kBlock / 64));
    hipLaunchKernelGGL(csr_fill_kernel, dim3(grid), dim3(kBlock), 0, st, Q8, ldq, n, rowptr, pk);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Products.

struct SparseArgs {
    const int32_t *rowptr;
    const uint32_t *pk;
    int64_t n;
    const int32_t *w0, *w1;  // operand words: T (main), or T_hi and T_lo (aux); column c at c * ldw,
                             // zero_col + 1 columns (an empty list slot names the all-zero column)
    int64_t ldw;
    const int32_t *active;   // live list (zero_col + 1 readable entries) and its count
    const int32_t *nactive;
    int zero_col;
    int64_t *U0, *U1;        // outputs, column c at c * ldu
    int64_t ldu;
};

constexpr int kSparseGroup = 4;  // columns per pass over a row's nonzeros

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// H = 2: the two halves of an 8-digit operand; H = 1: a 4-digit operand.
template <int H>
__device__ __forceinline__ void sparse_row(const SparseArgs &a, int64_t i) {
    const int lane = threadIdx.x & 63;
    const int kb = a.rowptr[i], ke = a.rowptr[i + 1];
    const int nact = *a.nactive;
    for (int c0 = 0; c0 < nact; c0 += kSparseGroup) {  // uniform over the wave
        int64_t col[kSparseGroup];
#pragma unroll
        for (int q = 0; q < kSparseGroup; ++q) {
            // entries past the count are replaced by the all-zero column
            const int slot = c0 + q;
            const int e = a.active[min(slot, a.zero_col)];
            col[q] = slot < nact ? (int64_t)e : (int64_t)a.zero_col;
        }
        const int cnt = min(kSparseGroup, nact - c0);  // live columns in this group (uniform)
        int64_t s0[kSparseGroup] = {}, s1[kSparseGroup] = {};
        for (int k = kb + lane; k < ke; k += 64) {
            const uint32_t wd = a.pk[k];
            const int64_t j = (int64_t)(wd & 0xffffu);
            const int64_t v = (int64_t)(int8_t)(uint8_t)(wd >> 16);
#pragma unroll
            for (int q = 0; q < kSparseGroup; ++q) {
                if (q >= cnt) break;
                s0[q] += v * (int64_t)a.w0[col[q] * a.ldw + j];
                if (H == 2) s1[q] += v * (int64_t)a.w1[col[q] * a.ldw + j];
            }
        }
#pragma unroll
        for (int q = 0; q < kSparseGroup; ++q) {
            s0[q] = wave_sum_i64(s0[q]);
            if (H == 2) s1[q] = wave_sum_i64(s1[q]);
        }
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < kSparseGroup; ++q) {
                if (c0 + q >= nact) break;
                if (col[q] == a.zero_col) continue;  // an empty slot of the list
                a.U0[col[q] * a.ldu + i] = s0[q];
                if (H == 2) a.U1[col[q] * a.ldu + i] = s1[q];
            }
        }
    }
}

// Blocks [0, nb1) take the subproblem columns' rows (4 rows per block), the
// next nb2 blocks the lambda_min / CG columns' rows.
__global__ void __launch_bounds__(kBlock) sparse_kernel(SparseArgs m, SparseArgs x, int nb1) {
    const int bx = blockIdx.x;
    const int w = threadIdx.x >> 6;
    if (bx < nb1) {
        const int64_t i = (int64_t)bx * (kBlock / 64) + w;
        if (i < m.n) sparse_row<1>(m, i);
    } else {
        const int64_t i = (int64_t)(bx - nb1) * (kBlock / 64) + w;
        if (i < x.n) sparse_row<2>(x, i);
    }
}

hipError_t launch_sparse(const SparseJob *main4, const SparseJob *aux8, hipStream_t st) {
    SparseArgs a{}, b{};
    int nb1 = 0, nb2 = 0;
    auto fill = [](const SparseJob &j, SparseArgs &s, int *nb) {
        s.rowptr = j.rowptr;
        s.pk = j.pk;
        s.n = j.n;
        s.w0 = j.w0;
        s.w1 = j.w1;
        s.ldw = j.ldw;
        s.active = j.active;
        s.nactive = j.nactive;
        s.zero_col = j.zero_col;
        s.U0 = j.U0;
        s.U1 = j.U1;
        s.ldu = j.ldu;
        *nb = (int)((j.n + kBlock / 64 - 1) / (kBlock / 64));
    };
    if (main4 && main4->on) fill(*main4, a, &nb1);
    if (aux8 && aux8->on) fill(*aux8, b, &nb2);
    if (nb1 + nb2 == 0) return hipSuccess;
    hipLaunchKernelGGL(sparse_kernel, dim3((unsigned)(nb1 + nb2)), dim3(kBlock), 0, st, a, b, nb1);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Operand words from FP64 columns (stand-alone product): D = 4, T = rint(x
// 2^27) for x in [0,1]; D = 8, the column's exponent e from its largest
// magnitude, T = rint(v 2^(55 - e)) split into halves.

template <int D>
__global__ void __launch_bounds__(kBlock) words_from_vectors_kernel(const double *X, int64_t n, int64_t ldx,
                                                                    int32_t *w0, int32_t *w1, int64_t ldw,
                                                                    int32_t *escale) {
    const int64_t c = blockIdx.x;
    const double *x = X + c * ldx;
    if constexpr (D == 4) {
        for (int64_t i = threadIdx.x; i < n; i += kBlock) w0[c * ldw + i] = (int32_t)__double2ll_rn(x[i] * kMainScale);
    } else {
        __shared__ double red[kWaves];
        double mx[1] = {0.0};
        for (int64_t i = threadIdx.x; i < n; i += kBlock) mx[0] = fmax(mx[0], fabs(x[i]));
        block_max<1>(mx, red);
        const int e = digits8_exponent(mx[0]);
        for (int64_t i = threadIdx.x; i < n; i += kBlock) {
            int32_t hi, lo;
            split8(x[i], e, &hi, &lo);
            w0[c * ldw + i] = hi;
            w1[c * ldw + i] = lo;
        }
        if (threadIdx.x == 0) escale[c] = e;
    }
}

hipError_t launch_words_from_vectors(const double *X, int64_t n, int64_t ldx, int B, int D, int32_t *w0,
                                     int32_t *w1, int64_t ldw, int32_t *escale, hipStream_t st) {
    if (D == 4)
        hipLaunchKernelGGL(words_from_vectors_kernel<4>, dim3(B), dim3(kBlock), 0, st, X, n, ldx, w0, w1, ldw, escale);
    else if (D == 8)
        hipLaunchKernelGGL(words_from_vectors_kernel<8>, dim3(B), dim3(kBlock), 0, st, X, n, ldx, w0, w1, ldw, escale);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace psdp
