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
// Each product launch first stages the live columns' operand words so that
// the 16 halves of a pass sit together for every row index, then runs one
// wave per row of Q over the row's nonzeros (sparse_row below).
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
    int32_t *stage;          // staging of the live operands, pass-interleaved (below)
    int64_t passes;          // passes the staging holds
};

typedef int intx4 __attribute__((ext_vector_type(4)));

// Operand halves per pass: 16 subproblem columns, or 8 lambda_min / CG
// columns (two halves each); NC = 16 / H columns per pass.
constexpr int kSparseHalves = 16;

int64_t sparse_stage_passes(int cols, int H) {
    const int nc = kSparseHalves / H;
    return std::max<int64_t>(1, (cols + nc - 1) / nc);
}

template <int H> __device__ __forceinline__ int64_t sparse_pass_count(const SparseArgs &a, int nact) {
    constexpr int NC = kSparseHalves / H;
    return min((int64_t)((nact + NC - 1) / NC), a.passes);
}

// Staging: pass p covers the live-list slots p NC .. p NC + NC - 1; word
// v = h NC + q of operand row j is half h of slot p NC + q's operand at j,
// stored at stage[(p ldw + j) 16 + v]. The product kernel then finds a
// nonzero's 16 operand halves of a pass in one 64-byte segment: a wave's
// gathers touch one segment per nonzero instead of one per column half.
// Slots past the count take the all-zero column.
template <int H>
__device__ __forceinline__ void stage_quarter(const SparseArgs &a, int64_t j, int u) {
    constexpr int NC = kSparseHalves / H;
    const int nact = *a.nactive;
    const int64_t np = sparse_pass_count<H>(a, nact);
    for (int64_t p = 0; p < np; ++p) {  // uniform
        int wv[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int v = 4 * u + e, q = v % NC;
            const int slot = (int)p * NC + q;
            const int ent = a.active[min(slot, a.zero_col)];
            const int64_t c = slot < nact ? (int64_t)ent : (int64_t)a.zero_col;
            const int32_t *w = a.w0;
            if constexpr (H == 2) w = v < NC ? a.w0 : a.w1;
            wv[e] = w[c * a.ldw + j];
        }
        *(intx4 *)(a.stage + (p * a.ldw + j) * kSparseHalves + 4 * u) = intx4{wv[0], wv[1], wv[2], wv[3]};
    }
}

// One wave per row. Lane l takes quarter u = l % 4 (staged words 4u .. 4u + 3)
// of 16 nonzeros at a time, k = k0 + l / 4 + 16 t for t < 4, and keeps 4
// int64 sums. The 16 lanes of a quarter are then added in a butterfly that
// first halves the values each lane carries (lane offsets 32 and 16: a lane
// keeps the lower or upper half by its bit of the offset and adds its
// partner's copy of that half), then adds over offsets 8 and 4: lane l ends
// with the total of value 4u + 2 bit5(l) + bit4(l), and the lanes with bits 2
// and 3 clear store the 16 totals. Integer sums: exact in any order.
// H = 2: the two halves of an 8-digit operand; H = 1: a 4-digit operand.
template <int H>
__device__ __forceinline__ void sparse_row(const SparseArgs &a, int64_t i) {
    constexpr int NC = kSparseHalves / H;
    const int lane = threadIdx.x & 63, u = lane & 3;
    const int kb = a.rowptr[i], ke = a.rowptr[i + 1];
    const int nact = *a.nactive;
    const int64_t np = sparse_pass_count<H>(a, nact);
    for (int64_t p = 0; p < np; ++p) {  // uniform
        const int32_t *G = a.stage + p * a.ldw * kSparseHalves + 4 * u;
        // the value this lane stores if any, and its list entry, read ahead
        const int vix = 4 * u + ((lane & 32) ? 2 : 0) + ((lane & 16) ? 1 : 0);
        const int q = vix % NC, h = vix / NC;
        const int slot = (int)p * NC + q;
        const int ent = a.active[min(slot, a.zero_col)];
        int64_t s[4] = {0, 0, 0, 0};
        for (int k0 = kb; k0 < ke; k0 += 64) {  // uniform
            uint32_t wd[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int k = k0 + (lane >> 2) + 16 * t;
                wd[t] = k < ke ? a.pk[k] : 0u;  // past the row: column 0, value 0
            }
            intx4 g[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) g[t] = *(const intx4 *)(G + (int64_t)(wd[t] & 0xffffu) * kSparseHalves);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int64_t v = (int64_t)(int8_t)(uint8_t)(wd[t] >> 16);
#pragma unroll
                for (int e = 0; e < 4; ++e) s[e] += v * (int64_t)g[t][e];
            }
        }
        {
            const bool up = (lane & 32) != 0;
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int64_t keep = up ? s[r + 2] : s[r], send = up ? s[r] : s[r + 2];
                s[r] = keep + __shfl_xor(send, 32, 64);
            }
        }
        {
            const bool up = (lane & 16) != 0;
            const int64_t keep = up ? s[1] : s[0], send = up ? s[0] : s[1];
            s[0] = keep + __shfl_xor(send, 16, 64);
        }
        s[0] += __shfl_xor(s[0], 8, 64);
        s[0] += __shfl_xor(s[0], 4, 64);
        // no store for slots past the count or empty slots
        if ((lane & 12) == 0 && slot < nact && ent != a.zero_col) (h ? a.U1 : a.U0)[(int64_t)ent * a.ldu + i] = s[0];
    }
}

// Blocks [0, nb1) serve the subproblem columns, the next ones the
// lambda_min / CG columns: 64 operand rows per block for the staging,
// kBlock / 64 rows of Q per block for the product.
static_assert(kBlock / 64 == kSparseHalves / 4, "one staging wave per four words");
__global__ void __launch_bounds__(kBlock) sparse_stage_kernel(SparseArgs m, SparseArgs x, int nb1) {
    // wave u writes words 4u .. 4u + 3 of 64 consecutive operand rows
    const int bx = blockIdx.x;
    const int u = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (bx < nb1) {
        const int64_t j = (int64_t)bx * 64 + lane;
        if (j < m.n) stage_quarter<1>(m, j, u);
    } else {
        const int64_t j = (int64_t)(bx - nb1) * 64 + lane;
        if (j < x.n) stage_quarter<2>(x, j, u);
    }
}

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
    int nb1 = 0, nb2 = 0, ns1 = 0, ns2 = 0;
    bool ok = true;
    auto fill = [&ok](const SparseJob &j, int H, SparseArgs &s, int *nb, int *ns) {
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
        s.stage = j.stage;
        s.passes = j.passes;
        // the staging must hold every pass of the largest live count
        ok = ok && j.stage && j.n <= j.ldw && j.max_live <= j.zero_col &&
             j.passes >= sparse_stage_passes(j.max_live, H);
        *nb = (int)((j.n + kBlock / 64 - 1) / (kBlock / 64));
        *ns = (int)((j.n + 63) / 64);
    };
    if (main4 && main4->on) fill(*main4, 1, a, &nb1, &ns1);
    if (aux8 && aux8->on) fill(*aux8, 2, b, &nb2, &ns2);
    if (!ok) return hipErrorInvalidValue;
    if (nb1 + nb2 == 0) return hipSuccess;
    hipLaunchKernelGGL(sparse_stage_kernel, dim3((unsigned)(ns1 + ns2)), dim3(kBlock), 0, st, a, b, ns1);
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
