// Symmetric Q.x for one instance and one column from the unique half of Q:
// the O(n^2) part of every penalty-gradient evaluation (eq. (kkt1)) and of
// every lambda_min and x^0 matvec (eqs. (alpha), (gamma)) on the
// single-instance path, reading n (n + 1) / 2 entries instead of n^2.
//
// Storage: Q_off (zero diagonal) in T x T tiles (T = 128), only the tiles
// (bi, bj) with bi <= bj, each tile row-major and contiguous, in row-major
// order of the upper triangle; entries past n are zero.
//
// A block (512 threads) reads one tile once and forms both of its
// contributions: the direct one, tile x_bj, to rows bi*T.., and (off the
// diagonal) the transposed one, tile^T x_bi, to rows bj*T... Thread t holds
// 4 consecutive columns (t % 32) * 4 of rows t / 32 + 16 k (k < 8); a row's
// direct sum is completed across its 32 lanes by a fixed butterfly, a
// column's transposed sum across the 16 row groups through LDS in fixed
// order. Every tile writes its two partial vectors to staging buffers, and a
// second kernel adds them per row in a fixed order (symv_reduce_kernel):
// the direct parts of the tiles (bi, bj >= bi), then the transposed parts
// of the tiles (bk < bi, bi). All products and sums are FP64 (Q
// entries widened exactly), the order fixed, so the result is
// reproducible; it differs from the row-by-row GEMV only by summation order.
#include "launch.hpp"

namespace psdp {

constexpr int kSymT = 128;

// Packing: block (tile t, 32-row part) copies its part of tile (bi, bj) of
// the zero-diagonal operand Qop (row-major, leading dimension ld >= n, zero
// padded up to ld); rows or columns at or past ld are zero.
template <typename QT>
__global__ void __launch_bounds__(kBlock) symv_pack_kernel(const QT *Qop, int64_t ld, const int2 *tiles, QT *P) {
    const int t = blockIdx.x;
    const int2 bij = tiles[t];
    QT *tp = P + (int64_t)t * kSymT * kSymT;
    for (int e = blockIdx.y * 32 * kSymT + threadIdx.x; e < (blockIdx.y + 1) * 32 * kSymT; e += kBlock) {
        const int r = e / kSymT, c = e % kSymT;
        const int64_t i = (int64_t)bij.x * kSymT + r, j = (int64_t)bij.y * kSymT + c;
        tp[e] = (i < ld && j < ld) ? Qop[i * ld + j] : from_f64<QT>(0.0);
    }
}

// Raw loads of 4 consecutive entries (kept in their storage type until used,
// so that a thread holds its 8 rows in few registers) and their FP64 values.
template <typename QT> struct Raw4;
template <> struct Raw4<double> {
    double2 a, b;
    __device__ __forceinline__ void load(const double *q) { a = *(const double2 *)q; b = *(const double2 *)(q + 2); }
    __device__ __forceinline__ double operator[](int u) const { return u == 0 ? a.x : u == 1 ? a.y : u == 2 ? b.x : b.y; }
};
template <> struct Raw4<float> {
    float4 a;
    __device__ __forceinline__ void load(const float *q) { a = *(const float4 *)q; }
    __device__ __forceinline__ double operator[](int u) const {
        return (double)(u == 0 ? a.x : u == 1 ? a.y : u == 2 ? a.z : a.w);
    }
};
template <> struct Raw4<__hip_bfloat16> {
    uint2 a;
    __device__ __forceinline__ void load(const __hip_bfloat16 *q) { a = *(const uint2 *)q; }
    __device__ __forceinline__ double operator[](int u) const {
        const uint32_t w = u < 2 ? a.x : a.y;
        return (double)__uint_as_float((u & 1) ? (w & 0xffff0000u) : (w << 16));
    }
};

constexpr int kSymThreads = 512;  // 16 row groups of 32 lanes; 8 rows per thread

// One block per tile (grid = the tile count): two blocks per CU.
template <typename QT>
__global__ void __launch_bounds__(kSymThreads) symv_tile_kernel(const QT *P, const int2 *tiles, int64_t ntiles,
                                                                const double *x, int64_t ld, double *Dp, double *Tp,
                                                                const int32_t *live) {
    __shared__ double part[16][kSymT];
    __shared__ double dpart[kSymT];
    const int64_t t = blockIdx.x;
    if ((live && *live == 0) || t >= ntiles) return;
    const int2 bij = tiles[t];
    const int bi = bij.x, bj = bij.y;
    const int tid = threadIdx.x, l = tid & 31, rg = tid >> 5;
    const int c4 = l * 4;
    const QT *tp = P + t * kSymT * kSymT;
    // the thread's rows rg + 16 k of the tile: every load is issued first
    Raw4<QT> q[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) q[k].load(tp + (rg + 16 * k) * kSymT + c4);
    double xj[4], xi[8];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t j = (int64_t)bj * kSymT + c4 + u;
        xj[u] = j < ld ? x[j] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int64_t i = (int64_t)bi * kSymT + rg + 16 * k;
        xi[k] = i < ld ? x[i] : 0.0;
    }
    double d[8], tc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const double v0 = q[k][0], v1 = q[k][1], v2 = q[k][2], v3 = q[k][3];
        d[k] = fma(v3, xj[3], fma(v2, xj[2], fma(v1, xj[1], v0 * xj[0])));
        tc[0] = fma(v0, xi[k], tc[0]);
        tc[1] = fma(v1, xi[k], tc[1]);
        tc[2] = fma(v2, xi[k], tc[2]);
        tc[3] = fma(v3, xi[k], tc[3]);
    }
    // direct sums: butterfly over the 32 lanes of a row group (offsets 16,
    // 8, 4 halve the rows a lane holds, offsets 2 and 1 add the remaining
    // lanes); lanes with equal bits 4..2 then hold row k = 4 b4 + 2 b3 + b2
#pragma unroll
    for (int s = 0, off = 16; s < 3; ++s, off >>= 1) {
        const int h = 4 >> s;
        const bool up = (l & off) != 0;
#pragma unroll
        for (int k = 0; k < h; ++k) {
            const double send = up ? d[k] : d[k + h];
            const double keep = up ? d[k + h] : d[k];
            d[k] = keep + __shfl_xor(send, off, 64);
        }
    }
    d[0] = d[0] + __shfl_xor(d[0], 2, 64);
    d[0] = d[0] + __shfl_xor(d[0], 1, 64);
    const int k = ((l >> 4) & 1) * 4 + ((l >> 3) & 1) * 2 + ((l >> 2) & 1);
    if ((l & 3) == 0) dpart[rg + 16 * k] = d[0];
    // transposed sums (off the diagonal: a diagonal tile holds both
    // triangles, so its direct part is its whole product): the 16 row
    // groups of each column, in group order
    if (bi != bj) {
#pragma unroll
        for (int u = 0; u < 4; ++u) part[rg][c4 + u] = tc[u];
    }
    __syncthreads();
    if (tid < kSymT) {
        Dp[t * kSymT + tid] = dpart[tid];
    } else if (tid < 2 * kSymT && bi != bj) {
        const int c = tid - kSymT;
        double sm = part[0][c];
#pragma unroll
        for (int g = 1; g < 16; ++g) sm += part[g][c];
        Tp[t * kSymT + c] = sm;
    }
}

// Tile index of (bi, bj), bi <= bj, in row-major order of the upper triangle.
__device__ __forceinline__ int64_t sym_tile(int bi, int bj, int nb) {
    return (int64_t)bi * nb - (int64_t)bi * (bi - 1) / 2 + (bj - bi);
}

// Four blocks per tile row bi, 256 threads each: row r of the block's 32
// is summed by 8 threads, four over quarters of its direct parts (bj = bi ..
// nb - 1) and four over quarters of its transposed parts (bk = 0 .. bi - 1),
// each in increasing tile order; the eight sums are then added in that
// order (direct quarters, then transposed quarters).
constexpr int kSymReduceRows = 32;
__global__ void __launch_bounds__(kBlock) symv_reduce_kernel(const double *Dp, const double *Tp, int nb, int64_t n,
                                                             double *y, const int32_t *live) {
    __shared__ double ps[8][kSymReduceRows];
    if (live && *live == 0) return;
    const int bi = blockIdx.x / (kSymT / kSymReduceRows);
    const int r = (blockIdx.x % (kSymT / kSymReduceRows)) * kSymReduceRows + (threadIdx.x & (kSymReduceRows - 1));
    const int q = threadIdx.x / kSymReduceRows;
    // a quarter's parts in increasing tile order, eight loads in flight at a
    // time (the additions keep that order)
    auto quarter = [&](const double *S, int lo, int hi, bool direct) {
        double s = 0.0;
        for (int b0 = lo; b0 < hi; b0 += 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int b = b0 + u;
                v[u] = b < hi ? S[(direct ? sym_tile(bi, b, nb) : sym_tile(b, bi, nb)) * kSymT + r] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (b0 + u < hi) s += v[u];
        }
        return s;
    };
    double s;
    if (q < 4) {
        const int cnt = nb - bi, per = (cnt + 3) / 4;
        const int lo = bi + q * per;
        s = quarter(Dp, lo, min(nb, lo + per), true);
    } else {
        const int per = (bi + 3) / 4;
        const int lo = (q - 4) * per;
        s = quarter(Tp, lo, min(bi, lo + per), false);
    }
    ps[q][threadIdx.x & (kSymReduceRows - 1)] = s;
    __syncthreads();
    const int64_t i = (int64_t)bi * kSymT + r;
    if (threadIdx.x < kSymReduceRows && i < n) {
        double v = ps[0][threadIdx.x];
#pragma unroll
        for (int g = 1; g < 8; ++g) v += ps[g][threadIdx.x];
        y[i] = v;
    }
}

int symv_blocks(int64_t n) { return (int)((n + kSymT - 1) / kSymT); }

std::vector<int32_t> symv_tile_list(int nb) {
    std::vector<int32_t> v;
    v.reserve((size_t)nb * (nb + 1));
    for (int bi = 0; bi < nb; ++bi)
        for (int bj = bi; bj < nb; ++bj) {
            v.push_back(bi);
            v.push_back(bj);
        }
    return v;
}

int64_t symv_packed_elems(int nb) { return (int64_t)nb * (nb + 1) / 2 * kSymT * kSymT; }

hipError_t launch_symv_pack(int dtype, const void *Qop, int64_t ld, const SymTiles &s, hipStream_t st) {
    const dim3 grid((unsigned)s.ntiles, kSymT / 32);
    if (dtype == PSDP_F64)
        hipLaunchKernelGGL(symv_pack_kernel<double>, grid, dim3(kBlock), 0, st, (const double *)Qop, ld, s.tiles,
                           (double *)s.P);
    else if (dtype == PSDP_F32)
        hipLaunchKernelGGL(symv_pack_kernel<float>, grid, dim3(kBlock), 0, st, (const float *)Qop, ld, s.tiles,
                           (float *)s.P);
    else if (dtype == PSDP_BF16)
        hipLaunchKernelGGL(symv_pack_kernel<__hip_bfloat16>, grid, dim3(kBlock), 0, st, (const __hip_bfloat16 *)Qop,
                           ld, s.tiles, (__hip_bfloat16 *)s.P);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_symv(int dtype, const SymTiles &s, const double *x, int64_t ld, int64_t n, double *y,
                       hipStream_t st) {
    const unsigned grid = (unsigned)s.ntiles;
    if (dtype == PSDP_F64)
        hipLaunchKernelGGL(symv_tile_kernel<double>, dim3(grid), dim3(kSymThreads), 0, st,
                           (const double *)s.P, s.tiles, s.ntiles, x, ld, s.D, s.T, s.live);
    else if (dtype == PSDP_F32)
        hipLaunchKernelGGL(symv_tile_kernel<float>, dim3(grid), dim3(kSymThreads), 0, st,
                           (const float *)s.P, s.tiles, s.ntiles, x, ld, s.D, s.T, s.live);
    else if (dtype == PSDP_BF16)
        hipLaunchKernelGGL(symv_tile_kernel<__hip_bfloat16>, dim3(grid), dim3(kSymThreads), 0, st,
                           (const __hip_bfloat16 *)s.P, s.tiles, s.ntiles, x, ld, s.D, s.T, s.live);
    else
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(symv_reduce_kernel, dim3((unsigned)s.nb * (kSymT / kSymReduceRows)), dim3(kBlock), 0, st, s.D,
                       s.T, s.nb, n, y, s.live);
    return hipGetLastError();
}

}  // namespace psdp
