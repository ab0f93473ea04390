// Exact integer Q.X products of the I8 operand path on gfx950 int8 MFMA:
// the O(n^2) part of every penalty-gradient evaluation (eq. (kkt1)), of every
// lambda_min matvec (eq. (alpha)) and of every x^0 CG matvec (eq. (gamma)).
//
// Q (integer, |Q_ij| <= 127 off the diagonal) is stored once as int8 with a
// zero diagonal, ldq x ldq row-major (ldq a multiple of 64; rows allocated up
// to a multiple of kDigitRowsAlign, the extra rows zero). A vector operand is
// an integer column T in signed base-128 digits (put_digits4 / put_digits8):
// 4 digits for an iterate on the grid 2^-27, 8 digits (two 4-digit halves)
// for a lambda_min / CG vector scaled by a power of two. Digit plane t of
// column c starts at dig + (c D + t) ldq.
//
// v_mfma_i32_16x16x64_i8 forms every digit product exactly in int32
// (|sum| <= 64 * 127 * n < 2^31 for n <= 65536) and the epilogue combines
// four digits in int64, U = ((Y0 128 + Y1) 128 + Y2) 128 + Y3 = Q T exactly.
// The kernel computes D^T Q (Q is symmetric, so its row i is column i): the
// A operand is the digit matrix (row r = (column, digit), K = n), the B
// operand is Q. Register q of lane l of the accumulator holds row
// 4 (l / 16) + q, column l % 16 (measured on gfx950), so the four digit rows
// of one column land in one lane and combine without lane exchange; with 8
// digits, the lane groups alternate between the high and the low half. Lane
// l feeds A row l % 16 and B column l % 16 with the 16-byte K run
// 16 (l / 16) .. + 15 of that row; A and B use the same run, so the sum
// covers the same products whatever K order the unit applies.
//
// Work split: a block of 4 waves owns one group of MT digit tiles (16 MT / D
// columns), one block of rows of Q and one K slice (DigitShape below); the
// waves read the same digit rows (L1 hits).
// Blocks are ordered so that the column groups sharing one Q block run on
// one XCD (one L2). Partial sums are integers, so K slices add exactly, in
// any order, into the one product buffer (atomically when there are several
// slices; the buffer is then zero beforehand). The grid
// is sized for an estimate of the live count; blocks loop over further
// column groups, so the estimate changes only the speed.
#include <algorithm>

#include "launch.hpp"

namespace psdp {

typedef int intx4 __attribute__((ext_vector_type(4)));

struct DigitArgs {
    const int8_t *Q;
    int64_t ldq;
    const int8_t *dig;
    const int32_t *active;
    const int32_t *nactive;
    int64_t *U0, *U1;
    int64_t ldu, nrow, kchunk;
    int AG, IB, KS, zero_col;
};

// Block layouts, all 4 waves (chosen by timing sweeps on gfx950 at n = 2500):
//  up to 8 columns (DigitShape MT = 1, NT = 2, WK = 4): the waves split the K
//    slice of one 32-row block into 4 parts and wave 0 adds the parts from
//    LDS, so that even one column keeps many blocks busy without many output
//    slices;
//  more columns (DigitLdsShape, below): the digit tile is shared through
//    LDS; MT = 4, NT = 1 (64-row blocks) up to about 48 live columns, then
//    MT = 8, NT = 2 (128-row blocks); 1.2-1.7x faster than register-only
//    layouts from 8 to 256 live columns.
// UNR K steps of 64 per register stage; two stages alternate so that the
// loads of the next stage are in flight while the current one multiplies.
template <int MT, int NT, int WK, int UNR> struct DigitShape {
    static constexpr int kMT = MT, kNT = NT, kWK = WK, kWR = 4 / WK, kUNR = UNR;
    static constexpr int kRows = kWR * 16 * NT;  // Q rows per block
};
typedef DigitShape<1, 2, 4, 2> DigitFew;

__device__ __forceinline__ int64_t combine4(const intx4 &a) {
    return (((int64_t)a[0] * 128 + (int64_t)a[1]) * 128 + (int64_t)a[2]) * 128 + (int64_t)a[3];
}

__device__ __forceinline__ intx4 ld16(const int8_t *p) { return *(const intx4 *)p; }

// A K slice's part of one product element. With one slice it is the
// product and overwrites the element; with several, every slice adds its
// part with a 64-bit atomic add (integers: exact and independent of the
// order), onto an element the consumer has left at zero.
__device__ __forceinline__ void put_partial(const DigitArgs &da, int64_t *u, int64_t v) {
    if (da.KS > 1) atomicAdd((unsigned long long *)u, (unsigned long long)v);
    else *u = v;
}

template <int D, typename S>
__device__ __forceinline__ void digit_body(const DigitArgs &da, int L) {
    constexpr int MT = S::kMT, NT = S::kNT, WK = S::kWK, WR = S::kWR, UNR = S::kUNR;
    constexpr int RA = 16 * MT;  // digit rows per column group
    constexpr int CA = RA / D;   // columns per column group
    __shared__ intx4 part[WK > 1 ? WK - 1 : 1][MT * NT][64];
    if (L >= da.AG * da.IB * da.KS) return;
    // the wave index through readfirstlane: the K bounds and the loop
    // control below are then scalar, and the loads need no exec masking
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wr = wv % WR, wk = wv / WR;
    const int m = lane & 15, g = lane >> 4;
    const int nact = *da.nactive;
    const int ag0 = L % da.AG;
    const int rest = L / da.AG;
    const int ib = rest % da.IB, kz = rest / da.IB;
    const int64_t ldq = da.ldq;
    const int64_t i0 = ((int64_t)ib * WR + wr) * (16 * NT);
    // the block's K slice, split into WK parts of whole stages (UNR steps of
    // 64); the last part may end with a few single steps
    const int64_t kb0 = (int64_t)kz * da.kchunk;
    const int64_t ke0 = min(ldq, kb0 + da.kchunk);
    const int64_t nch = ke0 > kb0 ? (ke0 - kb0) / 64 : 0;
    const int64_t per = ((nch + WK - 1) / WK + UNR - 1) / UNR * UNR;
    const int64_t kb = kb0 + 64 * min(nch, per * wk);
    const int64_t ke = kb0 + 64 * min(nch, per * (wk + 1));
    const int64_t nstage = (ke - kb) / (64 * UNR);
    const int8_t *bq[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) bq[t] = da.Q + (i0 + 16 * t + m) * ldq + 16 * g;
    // two register stages: the next stage's loads are issued before the
    // current stage multiplies. Every load is unconditional and in bounds (a
    // prefetch past the last stage reloads the current one), so the code is
    // straight-line and the waits count loads exactly.
    intx4 a0[UNR][MT], b0[UNR][NT], a1[UNR][MT], b1[UNR][NT];
    const int8_t *ap[MT];
    auto load_b = [&](intx4 (&b)[UNR][NT], int64_t k) {
#pragma unroll
        for (int u = 0; u < UNR; ++u)
#pragma unroll
            for (int t = 0; t < NT; ++t) b[u][t] = ld16(bq[t] + k + 64 * u);
    };
    auto load = [&](intx4 (&a)[UNR][MT], intx4 (&b)[UNR][NT], int64_t k) {
#pragma unroll
        for (int u = 0; u < UNR; ++u)
#pragma unroll
            for (int s = 0; s < MT; ++s) a[u][s] = ld16(ap[s] + k + 64 * u);
        load_b(b, k);
    };
    // The first stage's Q rows do not depend on the live list: they load
    // while the live count and the list entries are in flight.
    if (nstage > 0) load_b(b0, kb);
    for (int ag = ag0;; ag += da.AG) {  // uniform over the block
        // list entries read in the same round as the count (slots clamped
        // to the list, which holds zero_col + 1 entries; entries past the
        // count are replaced below)
        int cr[MT], ce[MT];  // entries of the loaded rows and of the stored rows
#pragma unroll
        for (int s = 0; s < MT; ++s) {
            cr[s] = da.active[min((ag * RA + s * 16 + m) / D, da.zero_col)];
            ce[s] = da.active[min((ag * RA + s * 16 + 4 * g) / D, da.zero_col)];
        }
        if (ag * CA >= nact) break;
#pragma unroll
        for (int s = 0; s < MT; ++s) {
            const int r = ag * RA + s * 16 + m;
            const int64_t c = r / D < nact ? (int64_t)cr[s] : (int64_t)da.zero_col;
            ap[s] = da.dig + (c * D + (r % D)) * ldq + 16 * g;
        }
        intx4 acc[MT][NT];
#pragma unroll
        for (int s = 0; s < MT; ++s)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[s][t] = intx4{0, 0, 0, 0};
        auto mult = [&](const intx4 (&a)[UNR][MT], const intx4 (&b)[UNR][NT]) {
#pragma unroll
            for (int u = 0; u < UNR; ++u)
#pragma unroll
                for (int s = 0; s < MT; ++s)
#pragma unroll
                    for (int t = 0; t < NT; ++t)
                        acc[s][t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[u][s], b[u][t], acc[s][t], 0, 0, 0);
        };
        int64_t k = kb;
        if (nstage > 0) {
            if (ag == ag0) {  // Q rows already loaded
#pragma unroll
                for (int u = 0; u < UNR; ++u)
#pragma unroll
                    for (int s = 0; s < MT; ++s) a0[u][s] = ld16(ap[s] + k + 64 * u);
            } else {
                load(a0, b0, k);
            }
            for (int64_t st = 0; st < nstage; st += 2) {
                const bool m1 = st + 1 < nstage;
                load(a1, b1, m1 ? k + 64 * UNR : k);
                mult(a0, b0);
                if (!m1) {
                    k += 64 * UNR;
                    break;
                }
                const bool m2 = st + 2 < nstage;
                load(a0, b0, m2 ? k + 128 * UNR : k);
                mult(a1, b1);
                k += 128 * UNR;
            }
        }
        for (; k < ke; k += 64) {  // fewer than UNR single steps
            intx4 a[MT], b[NT];
#pragma unroll
            for (int s = 0; s < MT; ++s) a[s] = ld16(ap[s] + k);
#pragma unroll
            for (int t = 0; t < NT; ++t) b[t] = ld16(bq[t] + k);
#pragma unroll
            for (int s = 0; s < MT; ++s)
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    acc[s][t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[s], b[t], acc[s][t], 0, 0, 0);
        }
        if constexpr (WK > 1) {
            // integer partial sums: wave 0 adds the other K parts (exact in any order)
            __syncthreads();  // the previous group's parts have been read
            if (wk > 0) {
#pragma unroll
                for (int s = 0; s < MT; ++s)
#pragma unroll
                    for (int t = 0; t < NT; ++t) part[wk - 1][s * NT + t][lane] = acc[s][t];
            }
            __syncthreads();
            if (wk == 0) {
#pragma unroll
                for (int q = 0; q < WK - 1; ++q)
#pragma unroll
                    for (int s = 0; s < MT; ++s)
#pragma unroll
                        for (int t = 0; t < NT; ++t) acc[s][t] += part[q][s * NT + t][lane];
            }
        }
        if (wk == 0) {
            // lane group g holds digit rows 4 g .. 4 g + 3 of each tile: one
            // column's 4 digits, or (D = 8) one half of one column's 8 digits
#pragma unroll
            for (int s = 0; s < MT; ++s) {
                const int row0 = ag * RA + s * 16 + 4 * g;
                if (row0 / D >= nact || ce[s] == da.zero_col) continue;  // no store for an empty slot
                int64_t *Uo = (D == 8 && ((row0 >> 2) & 1)) ? da.U1 : da.U0;
                Uo += (int64_t)ce[s] * da.ldu;
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const int64_t i = i0 + 16 * t + m;
                    if (i < da.nrow) put_partial(da, Uo + i, combine4(acc[s][t]));
                }
            }
        }
    }
}

// Many-column layout with the digit tile in LDS: the block's 4 waves own 4
// consecutive 16 NT-row blocks of Q and share MT digit tiles, which the whole
// block copies into LDS once per K step of 64 (double-buffered, in the
// swizzled layout of digit_lds_off so that neither the copies nor the
// 16-byte fragment reads collide in banks).
// Each wave then loads only its own Q rows from global memory. The digit
// pieces and Q rows of the next four K steps are in flight in registers
// while the current step multiplies. MT must be a multiple of 4 (each thread
// copies MT / 4 pieces of 16 bytes per step).
template <int MT, int NT, int PF = 4> struct DigitLdsShape {
    static constexpr int kMT = MT, kNT = NT, kWR = 4, kPF = PF;
    static constexpr int kRows = 4 * 16 * NT;
};

// Byte offset of 16-byte chunk c of digit row r in an LDS stage: rows of 64
// bytes, chunk c stored at slot c ^ ((r >> 1) & 3). Of the layouts measured
// on gfx950 with the LDS bank-conflict counter (row strides 64 to 256 bytes,
// several XOR swizzles) this is the one whose fragment reads (lane: row
// l % 16, chunk l / 16) and tile writes (lane: row l / 4, chunk l % 4) both
// count no conflict cycles; the former 80-byte padded rows counted 3.8 per
// read and 8.0 per write instruction.
__device__ __forceinline__ int digit_lds_off(int r, int c) { return r * 64 + 16 * (c ^ ((r >> 1) & 3)); }
constexpr int kDigitLdsRow = 64;

template <int D, typename S>
__device__ __forceinline__ void digit_body_lds(const DigitArgs &da, int L) {
    constexpr int MT = S::kMT, NT = S::kNT, PC = MT / 4;
    constexpr int RA = 16 * MT, CA = RA / D;
    constexpr int ROWB = kDigitLdsRow;
    static_assert(MT % 4 == 0, "MT must be a multiple of 4");
    __shared__ __attribute__((aligned(16))) int8_t As[2][RA * ROWB];
    if (L >= da.AG * da.IB * da.KS) return;
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int m = lane & 15, g = lane >> 4;
    const int nact = *da.nactive;
    const int ag0 = L % da.AG;
    const int rest = L / da.AG;
    const int ib = rest % da.IB, kz = rest / da.IB;
    const int64_t ldq = da.ldq;
    const int64_t i0 = ((int64_t)ib * 4 + wv) * (16 * NT);
    const int64_t kb = (int64_t)kz * da.kchunk;
    const int64_t ke = min(ldq, kb + da.kchunk);
    const int8_t *bq[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) bq[t] = da.Q + (i0 + 16 * t + m) * ldq + 16 * g;
    // the first K step's Q rows do not depend on the live list: they load
    // while the live count and the list entries are in flight
    intx4 bpre[NT];
    if (kb < ke) {
#pragma unroll
        for (int t = 0; t < NT; ++t) bpre[t] = ld16(bq[t] + kb);
    }
    for (int ag = ag0;; ag += da.AG) {  // uniform over the block
        // this thread's pieces of the digit tile: piece p = threadIdx.x + 256 q
        // is row p / 4, bytes 16 (p % 4) .. + 15 of the K step. The list
        // entries of its rows and of the stored rows are read in the same
        // round as the count (slots clamped to the list, which holds
        // zero_col + 1 entries; entries past the count are replaced below).
        int cr[PC], ce[MT];
#pragma unroll
        for (int q = 0; q < PC; ++q)
            cr[q] = da.active[min((ag * RA + ((int)threadIdx.x + 256 * q) / 4) / D, da.zero_col)];
#pragma unroll
        for (int s = 0; s < MT; ++s) ce[s] = da.active[min((ag * RA + s * 16 + 4 * g) / D, da.zero_col)];
        if (ag * CA >= nact) break;
        const int8_t *af[PC];
        int ao[PC];
#pragma unroll
        for (int q = 0; q < PC; ++q) {
            const int pce = threadIdx.x + 256 * q;
            const int r = pce >> 2, cb = pce & 3;
            const int64_t c = (ag * RA + r) / D < nact ? (int64_t)cr[q] : (int64_t)da.zero_col;
            af[q] = da.dig + (c * D + ((ag * RA + r) % D)) * ldq + 16 * cb;
            ao[q] = digit_lds_off(r, cb);
        }
        intx4 acc[MT][NT];
#pragma unroll
        for (int s = 0; s < MT; ++s)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[s][t] = intx4{0, 0, 0, 0};
        if (kb < ke) {
            // A ring of PF register stages: the loads of K step s + PF are
            // issued while step s multiplies, and a step's digit pieces go to
            // LDS (double buffer, one barrier per step) only when the step
            // comes up. Loads past the last step reread it (in bounds).
            constexpr int PF = S::kPF;
            const int nst = (int)((ke - kb) / 64);
            intx4 ra[PF][PC], rb[PF][NT];
            auto issue = [&](intx4 (&xa)[PC], intx4 (&xb)[NT], int s) {
                const int64_t k = kb + 64 * (int64_t)min(s, nst - 1);
#pragma unroll
                for (int q = 0; q < PC; ++q) xa[q] = ld16(af[q] + k);
#pragma unroll
                for (int t = 0; t < NT; ++t) xb[t] = ld16(bq[t] + k);
            };
#pragma unroll
            for (int u = 0; u < PF; ++u) {
                if (u == 0 && ag == ag0) {  // the first step's Q rows are already loaded
#pragma unroll
                    for (int q = 0; q < PC; ++q) ra[0][q] = ld16(af[q] + kb);
#pragma unroll
                    for (int t = 0; t < NT; ++t) rb[0][t] = bpre[t];
                } else {
                    issue(ra[u], rb[u], u);
                }
            }
            // step s uses ring stage s % PF and LDS buffer s & 1 (PF is even)
            auto step = [&](int u, bool refill, int snext) {
#pragma unroll
                for (int q = 0; q < PC; ++q) *(intx4 *)&As[u & 1][ao[q]] = ra[u][q];
                __syncthreads();
                intx4 b[NT];
#pragma unroll
                for (int t = 0; t < NT; ++t) b[t] = rb[u][t];
                if (refill) issue(ra[u], rb[u], snext);
                intx4 a[MT];
#pragma unroll
                for (int s = 0; s < MT; ++s) a[s] = *(const intx4 *)&As[u & 1][digit_lds_off(s * 16 + m, g)];
#pragma unroll
                for (int s = 0; s < MT; ++s)
#pragma unroll
                    for (int t = 0; t < NT; ++t)
                        acc[s][t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[s], b[t], acc[s][t], 0, 0, 0);
            };
            // whole groups of PF steps in a loop with a single path through
            // its body (an early exit inside it made the compiler copy the
            // ring registers at the back edge and wait for every load in
            // flight), then the last nst % PF steps from the filled ring
            const int nfull = nst / PF * PF;
            for (int s0 = 0; s0 < nfull; s0 += PF) {
#pragma unroll
                for (int u = 0; u < PF; ++u) step(u, true, s0 + u + PF);
            }
            const int rest = nst - nfull;  // uniform
#pragma unroll
            for (int u = 0; u < PF - 1; ++u)
                if (u < rest) step(u, false, 0);
        }
#pragma unroll
        for (int s = 0; s < MT; ++s) {
            const int row0 = ag * RA + s * 16 + 4 * g;
            if (row0 / D >= nact || ce[s] == da.zero_col) continue;  // no store for an empty slot
            int64_t *Uo = (D == 8 && ((row0 >> 2) & 1)) ? da.U1 : da.U0;
            Uo += (int64_t)ce[s] * da.ldu;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int64_t i = i0 + 16 * t + m;
                if (i < da.nrow) put_partial(da, Uo + i, combine4(acc[s][t]));
            }
        }
        __syncthreads();  // LDS is refilled by the next column group
    }
}

typedef DigitLdsShape<4, 1> DigitMid;
typedef DigitLdsShape<8, 2> DigitMany;
// Wider tiles for the widest products: 256 rows of Q per block (64 per
// wave, twice the operand reuse of each digit fragment read from LDS), or
// 256 digit rows per block (twice the reuse of each Q row). Their
// accumulators and register rings leave room for one block per CU.
typedef DigitLdsShape<8, 4> DigitWide;
typedef DigitLdsShape<16, 2> DigitTall;

// DigitJob.mt codes of the layouts
constexpr int kLayoutFew = 1, kLayoutMid = 2, kLayoutMany = 4, kLayoutWide = 8, kLayoutTall = 16;

bool digit_layout_valid(int mt) {
    return mt == kLayoutFew || mt == kLayoutMid || mt == kLayoutMany || mt == kLayoutWide || mt == kLayoutTall;
}

// Calls f with a value of the shape type of layout code mt.
template <typename F> static void with_layout(int mt, F &&f) {
    switch (mt) {
        case kLayoutMid: f(DigitMid{}); break;
        case kLayoutMany: f(DigitMany{}); break;
        case kLayoutWide: f(DigitWide{}); break;
        case kLayoutTall: f(DigitTall{}); break;
        default: f(DigitFew{}); break;
    }
}
static int layout_ca(int mt, int D) {
    int ca = 0;
    with_layout(mt, [&](auto s) { ca = 16 * decltype(s)::kMT / D; });
    return ca;
}
static int layout_rows(int mt) {
    int rows = 0;
    with_layout(mt, [&](auto s) { rows = decltype(s)::kRows; });
    return rows;
}

template <int D, typename S> struct DigitBody {
    static __device__ __forceinline__ void run(const DigitArgs &da, int L) { digit_body<D, S>(da, L); }
};
template <int D, int MT, int NT, int PF> struct DigitBody<D, DigitLdsShape<MT, NT, PF>> {
    static __device__ __forceinline__ void run(const DigitArgs &da, int L) {
        digit_body_lds<D, DigitLdsShape<MT, NT, PF>>(da, L);
    }
};

// Blocks b and b + 8 run on the same XCD; consecutive tile ids go to one XCD.
// nb is a multiple of 8, so this is a bijection of [0, nb).
__device__ __forceinline__ int xcd_order(int b, int nb) { return (b & 7) * (nb >> 3) + (b >> 3); }

// Blocks per CU the register budget is set for: two for the smaller tiles
// (at most 256 registers per lane; the many-column layout otherwise takes
// 312 with its accumulators and runs one wave per SIMD, and whole n = 2500
// solves are 3% faster with two), one for the widest tiles.
template <typename S> struct DigitMinBlocks { static constexpr int value = 2; };
template <> struct DigitMinBlocks<DigitWide> { static constexpr int value = 1; };
template <> struct DigitMinBlocks<DigitTall> { static constexpr int value = 1; };
template <typename S1, typename S2> constexpr int kDigitMinBlocks =
    DigitMinBlocks<S1>::value < DigitMinBlocks<S2>::value ? DigitMinBlocks<S1>::value : DigitMinBlocks<S2>::value;

// The 4-digit product (subproblem columns) in the first nb1 blocks, the
// 8-digit product (lambda_min / CG columns) in the next nb2.
template <typename S1, typename S2>
__global__ void __launch_bounds__(kBlock, (kDigitMinBlocks<S1, S2>)) digit_kernel(DigitArgs a, DigitArgs b, int nb1,
                                                                                  int nb2) {
    const int bx = blockIdx.x;
    if (bx < nb1) DigitBody<4, S1>::run(a, xcd_order(bx, nb1));
    else DigitBody<8, S2>::run(b, xcd_order(bx - nb1, nb2));
}

// j.mt selects the layout (kLayoutFew, kLayoutMid, kLayoutMany).
static DigitArgs digit_args(const int8_t *Q8, int64_t ldq, int64_t nrow, int64_t ldu, const DigitJob &j, int D,
                            int *nb) {
    DigitArgs a{};
    const int CA = layout_ca(j.mt, D);
    const int rows = layout_rows(j.mt);
    const int ks = std::max(1, std::min(8, j.ks));
    int64_t kc = (ldq + ks - 1) / ks;
    kc = (kc + 63) / 64 * 64;
    a.Q = Q8;
    a.ldq = ldq;
    a.dig = j.dig;
    a.active = j.active;
    a.nactive = j.nactive;
    a.U0 = j.U0;
    a.U1 = j.U1;
    a.ldu = ldu;
    a.nrow = nrow;
    a.kchunk = kc;
    a.AG = std::max(1, (j.est + CA - 1) / CA);
    a.IB = (int)((ldq + rows - 1) / rows);
    a.KS = ks;  // a slice with an empty K range adds zeros
    a.zero_col = j.zero_col;
    const int total = a.AG * a.IB * a.KS;
    *nb = (total + 7) / 8 * 8;
    return a;
}

// The estimate is the smaller of this product's last polled column count
// plus 16 (columns move between the two products) and the last polled total
// live count (which only falls). The few-column layout serves up to 8: at
// n = 2500 whole solves ran 2% faster than with a bound of 20, whose
// few-column launches for 10-20 columns took 11-16 us.
void digit_layout(int est, int D, int64_t ldq, int *mt, int *blocks) {
    *mt = est <= 8 ? kLayoutFew : est <= 64 ? kLayoutMid : kLayoutMany;
    *blocks = digit_blocks(*mt, est, D, ldq);
}

int digit_blocks(int mt, int est, int D, int64_t ldq) {
    const int CA = layout_ca(mt, D);
    const int rows = layout_rows(mt);
    return std::max(1, (est + CA - 1) / CA) * (int)((ldq + rows - 1) / rows);
}

// Measured on gfx950 over whole n = 2500 solves: the many-column layout does
// best with about 512 blocks in the launch and at most 2 slices (3 or 4 were
// slower), the mid layout with about 1024 blocks and at most 4 slices (1.7%
// faster solves than 2; 6 or 8 were slower), the few-column layout with 2
// slices unless the launch is already large.
int digit_slices(int mt, int blocks_total) {
    blocks_total = std::max(1, blocks_total);
    if (mt <= kLayoutFew) return std::max(1, std::min(2, (1024 + blocks_total / 2) / blocks_total));
    if (mt == kLayoutMid) return std::max(1, std::min(4, (1024 + blocks_total / 2) / blocks_total));
    return std::max(1, std::min(2, (512 + blocks_total / 2) / blocks_total));
}

template <typename S1, typename S2>
static void digit_go(const DigitArgs &a, const DigitArgs &b, int nb1, int nb2, hipStream_t st) {
    hipLaunchKernelGGL((digit_kernel<S1, S2>), dim3((unsigned)(nb1 + nb2)), dim3(kBlock), 0, st, a, b, nb1, nb2);
}

// Either job may be null or have est = 0 (then it is not launched). Rows of
// Q8 up to a multiple of kDigitRowsAlign must exist (zero past ldq).
hipError_t launch_digit(const int8_t *Q8, int64_t ldq, int64_t nrow, int64_t ldu, const DigitJob *main4,
                        const DigitJob *aux8, hipStream_t st) {
    if (ldq % 64 != 0 || nrow > ldu || nrow > ldq) return hipErrorInvalidValue;
    DigitArgs a{}, b{};
    int nb1 = 0, nb2 = 0, l1 = kLayoutFew, l2 = kLayoutFew;
    if (main4 && main4->est > 0) {
        if (!digit_layout_valid(main4->mt)) return hipErrorInvalidValue;
        a = digit_args(Q8, ldq, nrow, ldu, *main4, 4, &nb1);
        l1 = main4->mt;
    }
    if (aux8 && aux8->est > 0) {
        if (!digit_layout_valid(aux8->mt)) return hipErrorInvalidValue;
        b = digit_args(Q8, ldq, nrow, ldu, *aux8, 8, &nb2);
        l2 = aux8->mt;
    }
    if (nb1 + nb2 == 0) return hipSuccess;
    with_layout(l1, [&](auto s1) {
        with_layout(l2, [&](auto s2) { digit_go<decltype(s1), decltype(s2)>(a, b, nb1, nb2, st); });
    });
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Stand-alone product on user vectors (psdp_qx_digits): digits from the FP64
// columns, then the summed slices back to FP64.

// One block per column. D = 4: entries in [0,1] on the grid 2^-27. D = 8:
// the column's scale exponent from its largest magnitude, then 8 digits.
template <int D>
__global__ void __launch_bounds__(kBlock) digits_from_vectors_kernel(const double *X, int64_t n, int64_t ldx,
                                                                     int8_t *dig, int64_t ldq, int32_t *escale) {
    const int64_t c = blockIdx.x;
    const double *x = X + c * ldx;
    int8_t *p = dig + c * D * ldq;
    if constexpr (D == 4) {
        for (int64_t i = threadIdx.x; i < n; i += kBlock) put_digits4(p, ldq, (uint32_t)i, (int32_t)__double2ll_rn(x[i] * kMainScale));
    } else {
        __shared__ double red[kWaves];
        double mx[1] = {0.0};
        for (int64_t i = threadIdx.x; i < n; i += kBlock) mx[0] = fmax(mx[0], fabs(x[i]));
        block_max<1>(mx, red);
        const int e = digits8_exponent(mx[0]);
        for (int64_t i = threadIdx.x; i < n; i += kBlock) put_digits8(p, ldq, (uint32_t)i, x[i], e);
        if (threadIdx.x == 0) escale[c] = e;
    }
}

hipError_t launch_digits_from_vectors(const double *X, int64_t n, int64_t ldx, int B, int D, int8_t *dig,
                                      int64_t ldq, int32_t *escale, hipStream_t st) {
    if (D == 4)
        hipLaunchKernelGGL(digits_from_vectors_kernel<4>, dim3(B), dim3(kBlock), 0, st, X, n, ldx, dig, ldq, escale);
    else if (D == 8)
        hipLaunchKernelGGL(digits_from_vectors_kernel<8>, dim3(B), dim3(kBlock), 0, st, X, n, ldx, dig, ldq, escale);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

__global__ void __launch_bounds__(kBlock) digit_combine_kernel(const int64_t *U0, const int64_t *U1, int64_t n,
                                                               int64_t ldu, int D, const int32_t *escale,
                                                               double *Y) {
    const int64_t c = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t idx = c * ldu + i;
    Y[c * n + i] = D == 4 ? (double)U0[idx] / kMainScale : digits8_value(U0[idx], U1[idx], escale[c]);
}

hipError_t launch_digit_combine(const int64_t *U0, const int64_t *U1, int64_t n, int64_t ldu, int B, int D,
                                const int32_t *escale, double *Y, hipStream_t st) {
    const dim3 grid((unsigned)((n + kBlock - 1) / kBlock), (unsigned)B);
    hipLaunchKernelGGL(digit_combine_kernel, grid, dim3(kBlock), 0, st, U0, U1, n, ldu, D, escale, Y);
    return hipGetLastError();
}

}  // namespace psdp
