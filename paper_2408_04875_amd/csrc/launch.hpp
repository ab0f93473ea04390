// Host-side launchers of the gfx950 vectorized-PSDP library, implemented in
// the kernel translation units and called by the entry points (api.hip).
#pragma once

#include <vector>

#include "common.hpp"

namespace psdp {

// ---------------------------------------------------------------------------
// Host-side launchers implemented in the kernel translation units.

// Device-side input checks (check.hip): the first asymmetric entry as
// i n + j (all ones when Q is symmetric), the largest |Q_ij|, off-diagonal
// |Q_ij| and |b_i|, and the counts of X0 entries outside [0,1] and of
// non-finite p0 entries. rownnz (nullable, zeroed beforehand) gets the
// off-diagonal nonzeros of every row.
// Real (FP64) data: the magnitudes are bit patterns of non-negative doubles;
// nonfinite counts NaN/Inf entries of Q and b; nonint_off, non32_off and
// non16_off count the off-diagonal entries of Q that are not integers in
// [-127, 127], not floats, not bfloat16 values (zero for integer data).
struct CheckOut {
    uint64_t qmax, offmax, bmax, x0_bad, p0_bad, first_asym;
    uint64_t nonfinite, nonint_off, non32_off, non16_off;
};
hipError_t launch_check(const int32_t *Q, const int32_t *b, int64_t n, const double *X0, int64_t nx,
                        const double *p0, CheckOut *o, int32_t *rownnz, hipStream_t st);
hipError_t launch_check(const double *Q, const double *b, int64_t n, const double *X0, int64_t nx,
                        const double *p0, CheckOut *o, int32_t *rownnz, hipStream_t st);
hipError_t launch_prep_q(int dtype, const int32_t *Q, int64_t n, int64_t ld, int perturb,
                         double sigma, uint64_t seed, void *Qop, double *R, double *dq,
                         hipStream_t st);
hipError_t launch_prep_q(int dtype, const double *Q, int64_t n, int64_t ld, int perturb,
                         double sigma, uint64_t seed, void *Qop, double *R, double *dq,
                         hipStream_t st);
hipError_t launch_gamma(const int32_t *b, const double *R, const double *dq, int64_t n, int64_t ld,
                        double *bd, double *gam, double *dgi, double *lni, hipStream_t st);
hipError_t launch_gamma(const double *b, const double *R, const double *dq, int64_t n, int64_t ld,
                        double *bd, double *gam, double *dgi, double *lni, hipStream_t st);
hipError_t launch_perturbation(int64_t n, double sigma, uint64_t seed, int mode, double *mu,
                               hipStream_t st);
hipError_t launch_round_objective(const int32_t *Q, const int32_t *b, int64_t n,
                                  const double *X, int64_t ldx, int64_t B, uint8_t *xhat,
                                  int64_t ldh, int64_t *obj, int64_t *partial, hipStream_t st);
// Real data: obj_c is the exact sum of the selected Q_ij and b_i rounded once
// to FP64 (nearest, ties to even). acc: B * kObjAccWords int64 words of
// scratch, zero on entry (left zero on return).
constexpr int64_t kObjAccWords = 2 * 2048;
hipError_t launch_round_objective(const double *Q, const double *b, int64_t n,
                                  const double *X, int64_t ldx, int64_t B, uint8_t *xhat,
                                  int64_t ldh, double *obj, int64_t *acc, hipStream_t st);

// GEMM operand mode: FP32-stored Q (exact) widened to FP64, FP64 operands.
constexpr int kGemmF32QF64 = 16;

// Q.X products. U receives sum_j Qop[i][j] * op[j] for every live column.
hipError_t launch_gemv(int dtype, const Inst *inst_host, int ninst_same, const Work &w,
                       int ncol_max, hipStream_t st);
hipError_t launch_gemv_group(int dtype, const Work &w, const int64_t *rowstart, const int32_t *unitcol,
                             int64_t total_rows, hipStream_t st);
hipError_t launch_stream(int dtype, const void *Qop, int64_t ld, const void *op, void *U,
                         const int32_t *active, const int32_t *nactive, int64_t slice, int ksplit,
                         int ncol, int nt, hipStream_t st);
hipError_t launch_stream2(const void *Qop, int64_t ld, const void *op1, void *U1, const int32_t *active1,
                          const int32_t *nactive1, int64_t slice1, int ks1, int nt1, const void *op2,
                          void *U2, const int32_t *active2, const int32_t *nactive2, int64_t slice2,
                          int ks2, int nt2, int ncol1, int ncol2, hipStream_t st);
hipError_t launch_gemm(int dtype, const void *Qop, int64_t ld, const void *op, void *U,
                       const int32_t *active, const int32_t *nactive, int64_t slice, int ksplit,
                       int ncol_max, hipStream_t st);

// Exact integer products: U[c][i] = sum_k Q8[i][k] T[c][k], where T is a
// column's value in base-128 digits (4 digits, or 8 digits whose two 4-digit
// halves go to U0 and U1). With ks > 1 the K slices add their parts with
// atomic adds, so the live columns' outputs must be zero beforehand; with
// ks = 1 they are overwritten.
struct DigitJob {
    const int8_t *dig;       // digit planes [ncol + 1][D][ldq]; column ncol is zero
    const int32_t *active;   // live column list and its device count
    const int32_t *nactive;
    int64_t *U0, *U1;        // outputs: column stride ldu
    int zero_col;            // index of the all-zero column
    int ks;                  // K slices (1..8)
    int mt;                  // block layout: 1 few columns, 2 middle, 4 many, 8 wide, 16 tall
    int est;                 // live count the grid is sized for (0: no launch)
};
constexpr int kDigitRowsAlign = 256;  // Q8 rows are allocated up to a multiple of this
// Layout (DigitJob.mt) and base block count (one K slice) of a product sized
// for est columns of D digits; digit_slices then spreads the K range of both
// products of a sweep over enough blocks in total.
void digit_layout(int est, int D, int64_t ldq, int *mt, int *blocks);
int digit_slices(int mt, int blocks_total);
bool digit_layout_valid(int mt);
int digit_blocks(int mt, int est, int D, int64_t ldq);  // blocks of one K slice
hipError_t launch_digit(const int8_t *Q8, int64_t ldq, int64_t nrow, int64_t ldu, const DigitJob *main4,
                        const DigitJob *aux8, hipStream_t st);
hipError_t launch_digits_from_vectors(const double *X, int64_t n, int64_t ldx, int B, int D, int8_t *dig,
                                      int64_t ldq, int32_t *escale, hipStream_t st);
hipError_t launch_digit_combine(const int64_t *U0, const int64_t *U1, int64_t n, int64_t ldu, int B, int D,
                                const int32_t *escale, double *Y, hipStream_t st);

// Exact integer products from the compressed sparse rows of Q_off (sparse.hip):
// the same integers as the digit products, read from int32 operand words.
struct SparseJob {
    int on;                  // 0: not launched
    const int32_t *rowptr;   // n + 1 row starts
    const uint32_t *pk;      // packed nonzeros: column in bits 0-15, int8 value in bits 16-23
    int64_t n;
    const int32_t *w0, *w1;  // operand words: T, or T_hi and T_lo; column c at c * ldw, zero_col + 1 columns
    int64_t ldw;
    const int32_t *active;   // live list (zero_col + 1 readable entries) and its device count
    const int32_t *nactive;
    int zero_col;            // an all-zero operand column
    int64_t *U0, *U1;        // outputs (U1 for the low half), column c at c * ldu
    int64_t ldu;
    int32_t *stage;          // staging of the live operands: passes x ldw x 16 words, no initial contents
    int64_t passes;          // at least sparse_stage_passes(max_live, H), H = 1 (main) or 2 (aux)
    int max_live;            // largest live count the list may hold (at most zero_col)
};
// Passes of 16 operand halves that cols live columns of H halves need.
int64_t sparse_stage_passes(int cols, int H);
hipError_t launch_csr_fill(const int8_t *Q8, int64_t ldq, int64_t n, const int32_t *rowptr, uint32_t *pk,
                           hipStream_t st);
hipError_t launch_sparse(const SparseJob *main4, const SparseJob *aux8, hipStream_t st);
hipError_t launch_words_from_vectors(const double *X, int64_t n, int64_t ldx, int B, int D, int32_t *w0,
                                     int32_t *w1, int64_t ldw, int32_t *escale, hipStream_t st);

// Symmetric single-instance product from the unique half of Q (symv.hip):
// packed upper tiles of 128 x 128, one block per tile, partial vectors
// summed per row in a fixed order.
struct SymTiles {
    const void *P;        // packed tiles (Q's storage type)
    const int2 *tiles;    // (bi, bj) of every tile, row-major upper-triangle order
    int nb;               // tile rows: ceil(n / 128)
    int64_t ntiles;       // nb (nb + 1) / 2
    double *D, *T;        // staging: the direct and transposed partial vectors, ntiles x 128 each
    const int32_t *live;  // nullable: the live count; nothing runs when it is 0
};
__host__ __device__ int symv_blocks(int64_t n);
std::vector<int32_t> symv_tile_list(int nb);
int64_t symv_packed_elems(int nb);
hipError_t launch_symv_pack(int dtype, const void *Qop, int64_t ld, const SymTiles &s, hipStream_t st);
hipError_t launch_symv(int dtype, const SymTiles &s, const double *x, int64_t ld, int64_t n, double *y,
                       hipStream_t st);
// Group product from the unique halves: the packed tiles of every instance
// (each instance's tiles from its first tile index on, in the order of
// symv_tile_list), a work list over the live instances' tiles and one over
// their tile rows; staging indexed by the global tile. Finished columns'
// entries store nothing.
struct SymGroupTile {
    int32_t t, col, bi, bj;  // global tile index, column, tile position
    int64_t off, ld;         // the column's vector offset and leading dimension
};
struct SymGroupRow {
    int32_t col, bi;         // column, tile row
    int64_t off, n, base;    // vector offset, size, first tile index of the column
};
struct SymGroup {
    const void *P;
    const SymGroupTile *list;
    int64_t nlist;
    const SymGroupRow *rows;
    int64_t nrows;
    double *D, *T;
};
hipError_t launch_symv_group(int dtype, const SymGroup &g, const Work &w, hipStream_t st);

// Solver kernels.
hipError_t launch_solver_init(int optype, const Work &w, const double *X0, int use_cg,
                              hipStream_t st);
hipError_t launch_solver_step(int optype, int utype, const Work &w, int64_t nmax, hipStream_t st);
hipError_t launch_compact(const Work &w, hipStream_t st);

// Evaluation and adjoint.
hipError_t launch_eval(int dtype, int vtype, const void *Q, int64_t ldq, const void *b,
                       const void *p, const void *X, int64_t n, int64_t B, void *h, void *G,
                       double *ws, hipStream_t st);
hipError_t launch_adjoint(int dtype, int vtype, const void *X, const void *G, const void *w,
                          int64_t n, int64_t B, void *dX, void *dQ, void *db, void *dp,
                          hipStream_t st);

}  // namespace psdp
