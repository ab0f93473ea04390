// Symmetric Q.x for one instance and one column from the unique half of Q:
// the O(n^2) part of every penalty-gradient evaluation (eq. (kkt1)) and of
// every lambda_min and x^0 matvec (eqs. (alpha), (gamma)) on the
// single-instance path, reading n (n + 1) / 2 entries instead of n^2.
//
// Storage: Q_off (zero diagonal) in T x T tiles (T = 128), only the tiles
// (bi, bj) with bi <= bj, each tile row-major and contiguous, in row-major
// order of the upper triangle; entries past n are zero.
//
// A block reads one tile once and forms both of its contributions: the
// direct one, tile x_bj, to rows bi*T.., and (off the diagonal) the
// transposed one, tile^T x_bi, to rows bj*T... Each thread holds a few
// consecutive columns of a few rows spaced evenly through the tile (the
// shape per storage type is SymShape below); a row's direct sum is
// completed across the lanes of its row group by a fixed butterfly, a
// column's transposed sum across the row groups through LDS in fixed
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

// Raw loads of CW consecutive entries of one row (kept in their storage
// type until used, so that a thread holds its 8 rows in few registers) and
// their FP64 values.
template <typename QT, int CW> struct RawRow;
template <> struct RawRow<double, 4> {
    double2 a, b;
    __device__ __forceinline__ void load(const double *q) { a = *(const double2 *)q; b = *(const double2 *)(q + 2); }
    __device__ __forceinline__ double operator[](int u) const { return u == 0 ? a.x : u == 1 ? a.y : u == 2 ? b.x : b.y; }
};
__device__ __forceinline__ double sym_f32(const float4 &a, int u) {
    return (double)(u == 0 ? a.x : u == 1 ? a.y : u == 2 ? a.z : a.w);
}
template <> struct RawRow<float, 4> {
    float4 a;
    __device__ __forceinline__ void load(const float *q) { a = *(const float4 *)q; }
    __device__ __forceinline__ double operator[](int u) const { return sym_f32(a, u); }
};
template <> struct RawRow<float, 8> {
    float4 a, b;
    __device__ __forceinline__ void load(const float *q) { a = *(const float4 *)q; b = *(const float4 *)(q + 4); }
    __device__ __forceinline__ double operator[](int u) const { return u < 4 ? sym_f32(a, u) : sym_f32(b, u - 4); }
};
// a BF16 value is the high half of an FP32 word
__device__ __forceinline__ double sym_bf16(uint32_t w, int odd) {
    return (double)__uint_as_float(odd ? (w & 0xffff0000u) : (w << 16));
}
template <> struct RawRow<__hip_bfloat16, 4> {
    uint2 a;
    __device__ __forceinline__ void load(const __hip_bfloat16 *q) { a = *(const uint2 *)q; }
    __device__ __forceinline__ double operator[](int u) const { return sym_bf16(u < 2 ? a.x : a.y, u & 1); }
};
template <> struct RawRow<__hip_bfloat16, 8> {
    uint4 a;
    __device__ __forceinline__ void load(const __hip_bfloat16 *q) { a = *(const uint4 *)q; }
    __device__ __forceinline__ double operator[](int u) const {
        return sym_bf16(u < 2 ? a.x : u < 4 ? a.y : u < 6 ? a.z : a.w, u & 1);
    }
};

// Shape of the tile kernel by storage type: CW columns and R rows per
// thread, in G = T / R row groups of L = T / CW lanes. FP32 and BF16 threads
// hold 8 columns of 4 rows (32 or 16 bytes of a row per load), FP64 threads
// 4 columns of 8 rows (32 bytes), so that the loads of a tile are issued at
// once from few registers (measured at n = 16384: 8 x 4 per thread read 1.3x
// faster than 4 x 8 in both FP32 and BF16). LDS: FP32 and BF16 tiles take
// the tile's x entries from LDS and hand their row sums to LDS at once
// instead of keeping them for a butterfly, which holds them to 80 registers:
// six waves per SIMD, three 512-thread blocks per CU instead of two (BF16
// 1.29x faster at n = 16384).
template <typename QT> struct SymShape {
    static constexpr int CW = sizeof(QT) == 8 ? 4 : 8;
    static constexpr int R = sizeof(QT) == 8 ? 8 : 4;
    static constexpr int L = kSymT / CW, G = kSymT / R, threads = L * G;
    static constexpr bool LDS = sizeof(QT) != 8;
    static constexpr int waves = LDS ? 6 : 4;  // minimum per SIMD
};

// The products of one tile tp = (bi, bj) by one block: lane l of row group g
// holds columns l CW .. l CW + CW - 1 of rows g + G k (k < R); the direct
// part goes to Do, the transposed part (off the diagonal) to To, T entries
// each. x holds ld entries (ld >= the instance's n, zero padded).
template <typename QT>
__device__ __forceinline__ void sym_tile_body(const QT *tp, int bi, int bj, const double *x, int64_t ld, double *Do,
                                              double *To) {
    using S = SymShape<QT>;
    constexpr int CW = S::CW, R = S::R, L = S::L, G = S::G;
    static_assert(R >= 2 && R <= L && (R & (R - 1)) == 0 && L <= 64 && (L & (L - 1)) == 0, "tile kernel shape");
    static_assert(S::threads >= 2 * kSymT, "one thread per output of the tile");
    __shared__ double part[G][kSymT];
    const int tid = threadIdx.x, l = tid % L, rg = tid / L;
    const int c0 = l * CW;
    if constexpr (S::LDS) {
        // x of the tile's rows and columns staged in LDS; the partial row sum
        // of every (row, lane) goes to dl, and a row's direct sum adds its L
        // lanes in lane order
        __shared__ double xs[kSymT], xsj[kSymT];
        __shared__ double dl[R][G][L];
        RawRow<QT, CW> q[R];
#pragma unroll
        for (int k = 0; k < R; ++k) q[k].load(tp + (rg + G * k) * kSymT + c0);
        if (tid < kSymT) {
            const int64_t i = (int64_t)bi * kSymT + tid;
            xs[tid] = i < ld ? x[i] : 0.0;
        } else if (tid < 2 * kSymT) {
            const int64_t j = (int64_t)bj * kSymT + (tid - kSymT);
            xsj[tid - kSymT] = j < ld ? x[j] : 0.0;
        }
        __syncthreads();
        const double *xj = &xsj[c0];
        double tc[CW];
#pragma unroll
        for (int u = 0; u < CW; ++u) tc[u] = 0.0;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const double xi = xs[rg + G * k];
            double s = q[k][0] * xj[0];
#pragma unroll
            for (int u = 1; u < CW; ++u) s = fma(q[k][u], xj[u], s);
            dl[k][rg][l] = s;
#pragma unroll
            for (int u = 0; u < CW; ++u) tc[u] = fma(q[k][u], xi, tc[u]);
        }
        if (bi != bj) {
#pragma unroll
            for (int u = 0; u < CW; ++u) part[rg][c0 + u] = tc[u];
        }
        __syncthreads();
        if (tid < kSymT) {
            // row tid = g + G k
            const int g = tid % G, k = tid / G;
            double sm = dl[k][g][0];
#pragma unroll
            for (int u = 1; u < L; ++u) sm += dl[k][g][u];
            Do[tid] = sm;
        } else if (tid < 2 * kSymT && bi != bj) {
            const int c = tid - kSymT;
            double sm = part[0][c];
#pragma unroll
            for (int g = 1; g < G; ++g) sm += part[g][c];
            To[c] = sm;
        }
        return;
    }
    __shared__ double dpart[kSymT];
    // the thread's rows of the tile: every load is issued first
    RawRow<QT, CW> q[R];
#pragma unroll
    for (int k = 0; k < R; ++k) q[k].load(tp + (rg + G * k) * kSymT + c0);
    double xj[CW], xi[R];
#pragma unroll
    for (int u = 0; u < CW; ++u) {
        const int64_t j = (int64_t)bj * kSymT + c0 + u;
        xj[u] = j < ld ? x[j] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int64_t i = (int64_t)bi * kSymT + rg + G * k;
        xi[k] = i < ld ? x[i] : 0.0;
    }
    double d[R], tc[CW];
#pragma unroll
    for (int u = 0; u < CW; ++u) tc[u] = 0.0;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        double s = q[k][0] * xj[0];
#pragma unroll
        for (int u = 1; u < CW; ++u) s = fma(q[k][u], xj[u], s);
        d[k] = s;
#pragma unroll
        for (int u = 0; u < CW; ++u) tc[u] = fma(q[k][u], xi[k], tc[u]);
    }
    // direct sums: butterfly over the L lanes of a row group. The offsets
    // L/2, L/4, .. (log2 R of them) halve the rows a lane holds: at offset o
    // a lane with bit o set keeps the upper half of its rows, one without
    // the lower half, each adding its partner's copy. The smaller offsets
    // then add the lanes that hold the same row, which is
    // k = sum over those halving steps of bit(l, o) * (rows halved away).
    int k = 0;
#pragma unroll
    for (int h = R / 2, off = L / 2; h >= 1; h >>= 1, off >>= 1) {
        const bool up = (l & off) != 0;
        if (up) k += h;
#pragma unroll
        for (int r = 0; r < h; ++r) {
            const double send = up ? d[r] : d[r + h];
            const double keep = up ? d[r + h] : d[r];
            d[r] = keep + __shfl_xor(send, off, 64);
        }
    }
#pragma unroll
    for (int off = L / (2 * R); off >= 1; off >>= 1) d[0] = d[0] + __shfl_xor(d[0], off, 64);
    if (l % (L / R) == 0) dpart[rg + G * k] = d[0];
    // transposed sums (off the diagonal: a diagonal tile holds both
    // triangles, so its direct part is its whole product): the G row groups
    // of each column, in group order
    if (bi != bj) {
#pragma unroll
        for (int u = 0; u < CW; ++u) part[rg][c0 + u] = tc[u];
    }
    __syncthreads();
    if (tid < kSymT) {
        Do[tid] = dpart[tid];
    } else if (tid < 2 * kSymT && bi != bj) {
        const int c = tid - kSymT;
        double sm = part[0][c];
#pragma unroll
        for (int g = 1; g < G; ++g) sm += part[g][c];
        To[c] = sm;
    }
}

// One block per tile of one instance (grid = the tile count).
template <typename QT>
__global__ void __launch_bounds__(SymShape<QT>::threads, SymShape<QT>::waves)
    symv_tile_kernel(const QT *P, const int2 *tiles, int64_t ntiles, const double *x, int64_t ld, double *Dp,
                     double *Tp, const int32_t *live) {
    const int64_t t = blockIdx.x;
    if ((live && *live == 0) || t >= ntiles) return;
    const int2 bij = tiles[t];
    sym_tile_body<QT>(P + t * kSymT * kSymT, bij.x, bij.y, x, ld, Dp + t * kSymT, Tp + t * kSymT);
}

// Group product: one block per entry of the work list over the live
// instances' tiles; a finished column's entries read nothing (issuing the
// tile's loads beside the load of the column's phase, and storing nothing
// for a finished column, was 13% slower over the uneven batch: up to a
// quarter of the list belongs to finished columns between rebuilds).
template <typename QT>
__global__ void __launch_bounds__(SymShape<QT>::threads, SymShape<QT>::waves)
    symv_group_tile_kernel(const QT *P, const SymGroupTile *list, int64_t nlist, const Col *col, const double *op,
                           double *Dp, double *Tp) {
    const int64_t e = blockIdx.x;
    if (e >= nlist) return;
    const SymGroupTile d = list[e];
    if (col[d.col].phase == PH_DONE) return;
    const int64_t t = d.t;
    sym_tile_body<QT>(P + t * kSymT * kSymT, d.bi, d.bj, op + d.off, d.ld, Dp + t * kSymT, Tp + t * kSymT);
}

__host__ __device__ int symv_blocks(int64_t n) { return (int)((n + kSymT - 1) / kSymT); }

// Tile index of (bi, bj), bi <= bj, in row-major order of the upper triangle.
__device__ __forceinline__ int64_t sym_tile(int bi, int bj, int nb) {
    return (int64_t)bi * nb - (int64_t)bi * (bi - 1) / 2 + (bj - bi);
}

// A block of 256 threads sums 32 RPT rows of tile row bi: row r is summed
// by 8 threads, four over quarters of its direct parts (bj = bi .. nb - 1)
// and four over quarters of its transposed parts (bk = 0 .. bi - 1), each in
// increasing tile order, and the eight sums are then added in that order
// (direct quarters, then transposed quarters), whatever RPT is and however
// many loads (UB per row) are in flight. part: which block of 32 RPT rows of
// the tile row; tile indices start at base.
constexpr int kSymReduceRows = 32;
static_assert(kBlock == 8 * kSymReduceRows, "eight summing threads per row");
template <int RPT, int UB>
__device__ __forceinline__ void sym_reduce_body(const double *Dp, const double *Tp, int64_t base, int bi, int part,
                                                int nb, int64_t n, double *y) {
    constexpr int RB = kSymReduceRows * RPT;
    __shared__ double ps[8][RB];
    const int rl = threadIdx.x & (kSymReduceRows - 1);
    const int q = threadIdx.x / kSymReduceRows;
    // a quarter's parts in increasing tile order, for each of the thread's
    // rows (rows (part RPT + m) 32 + rl; the additions keep that order)
    auto quarter = [&](const double *S, int lo, int hi, bool direct, double (&s)[RPT]) {
#pragma unroll
        for (int m = 0; m < RPT; ++m) s[m] = 0.0;
        for (int b0 = lo; b0 < hi; b0 += UB) {
            double v[UB][RPT];
#pragma unroll
            for (int u = 0; u < UB; ++u) {
                const int b = b0 + u;
                const int64_t t = b < hi ? base + (direct ? sym_tile(bi, b, nb) : sym_tile(b, bi, nb)) : 0;
#pragma unroll
                for (int m = 0; m < RPT; ++m)
                    v[u][m] = b < hi ? S[t * kSymT + (part * RPT + m) * kSymReduceRows + rl] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < UB; ++u)
#pragma unroll
                for (int m = 0; m < RPT; ++m)
                    if (b0 + u < hi) s[m] += v[u][m];
        }
    };
    double s[RPT];
    if (q < 4) {
        const int cnt = nb - bi, per = (cnt + 3) / 4;
        const int lo = bi + q * per;
        quarter(Dp, lo, min(nb, lo + per), true, s);
    } else {
        const int per = (bi + 3) / 4;
        const int lo = (q - 4) * per;
        quarter(Tp, lo, min(bi, lo + per), false, s);
    }
#pragma unroll
    for (int m = 0; m < RPT; ++m) ps[q][m * kSymReduceRows + rl] = s[m];
    __syncthreads();
    if (threadIdx.x < RB) {
        const int64_t i = (int64_t)bi * kSymT + part * RB + threadIdx.x;
        if (i < n) {
            double v = ps[0][threadIdx.x];
#pragma unroll
            for (int g = 1; g < 8; ++g) v += ps[g][threadIdx.x];
            y[i] = v;
        }
    }
}

__global__ void __launch_bounds__(kBlock) symv_reduce_kernel(const double *Dp, const double *Tp, int nb, int64_t n,
                                                             double *y, const int32_t *live) {
    if (live && *live == 0) return;
    constexpr int kParts = kSymT / kSymReduceRows;
    sym_reduce_body<1, 32>(Dp, Tp, 0, blockIdx.x / kParts, blockIdx.x % kParts, nb, n, y);
}

// Group reduction: one block per entry of the list of the live instances'
// tile rows (column, bi, vector offset, n, first tile index), each thread
// taking its quarter of the parts for four rows 32 apart (the instances are
// small: a quarter holds a few parts), with the single-instance order.
__global__ void __launch_bounds__(kBlock) symv_group_reduce_kernel(const double *Dp, const double *Tp,
                                                                   const SymGroupRow *rows, int64_t nrows,
                                                                   const Col *col, double *U) {
    const int64_t e = blockIdx.x;
    if (e >= nrows) return;
    const SymGroupRow d = rows[e];
    if (col[d.col].phase == PH_DONE) return;
    sym_reduce_body<kSymT / kSymReduceRows, 8>(Dp, Tp, d.base, d.bi, 0, symv_blocks(d.n), d.n, U + d.off);
}

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
        hipLaunchKernelGGL(symv_tile_kernel<double>, dim3(grid), dim3(SymShape<double>::threads), 0, st,
                           (const double *)s.P, s.tiles, s.ntiles, x, ld, s.D, s.T, s.live);
    else if (dtype == PSDP_F32)
        hipLaunchKernelGGL(symv_tile_kernel<float>, dim3(grid), dim3(SymShape<float>::threads), 0, st,
                           (const float *)s.P, s.tiles, s.ntiles, x, ld, s.D, s.T, s.live);
    else if (dtype == PSDP_BF16)
        hipLaunchKernelGGL(symv_tile_kernel<__hip_bfloat16>, dim3(grid), dim3(SymShape<__hip_bfloat16>::threads), 0, st,
                           (const __hip_bfloat16 *)s.P, s.tiles, s.ntiles, x, ld, s.D, s.T, s.live);
    else
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(symv_reduce_kernel, dim3((unsigned)s.nb * (kSymT / kSymReduceRows)), dim3(kBlock), 0, st, s.D,
                       s.T, s.nb, n, y, s.live);
    return hipGetLastError();
}

hipError_t launch_symv_group(int dtype, const SymGroup &g, const Work &w, hipStream_t st) {
    if (g.nlist < 1 || g.nrows < 1) return hipSuccess;
    const dim3 grid((unsigned)g.nlist);
    const double *op = (const double *)w.op;
    if (dtype == PSDP_F64)
        hipLaunchKernelGGL(symv_group_tile_kernel<double>, grid, dim3(SymShape<double>::threads), 0, st,
                           (const double *)g.P, g.list, g.nlist, w.col, op, g.D, g.T);
    else if (dtype == PSDP_F32)
        hipLaunchKernelGGL(symv_group_tile_kernel<float>, grid, dim3(SymShape<float>::threads), 0, st,
                           (const float *)g.P, g.list, g.nlist, w.col, op, g.D, g.T);
    else if (dtype == PSDP_BF16)
        hipLaunchKernelGGL(symv_group_tile_kernel<__hip_bfloat16>, grid, dim3(SymShape<__hip_bfloat16>::threads), 0,
                           st, (const __hip_bfloat16 *)g.P, g.list, g.nlist, w.col, op, g.D, g.T);
    else
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(symv_group_reduce_kernel, dim3((unsigned)g.nrows), dim3(kBlock), 0, st, g.D, g.T, g.rows,
                       g.nrows, w.col, (double *)w.U);
    return hipGetLastError();
}

}  // namespace psdp
