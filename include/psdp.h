/*
 * psdp.h - C ABI of the MI355X (gfx950) vectorized-PSDP library.
 *
 * Problem (Huo and Gu, "A Vectorized Positive Semidefinite Penalty Method for
 * Unconstrained Binary Quadratic Programming", Section 2, eq. (bqp)):
 *     minimize f(x) = x^T Q x + b^T x  over x in {0,1}^n,  Q real symmetric.
 * The method replaces the binary constraint by the box 0 <= x <= 1 and the
 * penalty h(x, p) = f(x) + sum_i p_i (x_i - x_i^2) (eq. (p1)), solves the
 * box-constrained subproblem with projected alternating Barzilai-Borwein
 * steps (Algorithm 2) or a diagonal proximal-point step (Algorithm 1), and
 * raises p by alpha * z with alpha = eta * lambda_min(Z^-1/2 Qbar_II Z^-1/2)
 * (eqs. (pp1), (alpha1)) until x is binary (Algorithm 3).
 *
 * Conventions shared by every entry point:
 *  - Every function returns psdp_status; 0 is success, negatives are errors.
 *    psdp_last_error() returns a thread-local message for the last failure.
 *  - Pointers marked "device" are device memory owned by the caller; the
 *    library never frees or retains them after the call returns. Pointers
 *    marked "host" are host memory.
 *  - Matrices are dense. Q is row-major n x n with leading dimension ldq (for
 *    a symmetric Q row- and column-major coincide). Batches of vectors
 *    ("X", n x B) are column-major with leading dimension n: column c is the
 *    contiguous vector x_c (a torch tensor of shape (B, n)).
 *  - Work is enqueued on `stream` (0 = the null stream). The solve entry
 *    points block until their result is on the host side of their outputs'
 *    stream order (they synchronize `stream` before returning); the
 *    evaluation, adjoint and objective entry points are stream-ordered and
 *    return without synchronizing.
 *  - No C++ exception crosses this boundary and nothing aborts. Argument
 *    validation happens before any solve work (the checks of the data run
 *    as kernels on the caller's stream). Reaching an iteration cap is
 *    not an error: the status is PSDP_OK and psdp_stats.exit_reason says why
 *    the solve stopped.
 *  - Calls are serialized per process by an internal lock (the solve
 *    workspace is cached per device and reused across calls).
 */
#ifndef PSDP_H
#define PSDP_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PSDP_OK = 0,
    PSDP_E_INVALID = -1,        /* bad size, null pointer, bad enum, bad params */
    PSDP_E_NOT_SYMMETRIC = -2,  /* Q is not exactly symmetric */
    PSDP_E_NONFINITE = -3,      /* NaN/Inf in an input, or x0 outside [0,1] */
    PSDP_E_OVERFLOW = -4,       /* exact int64 objective bound would overflow */
    PSDP_E_DEVICE = -5,         /* HIP runtime error (detail in psdp_last_error) */
    PSDP_E_NOMEM = -6,          /* device allocation failed */
    PSDP_E_UNSUPPORTED = -7,    /* valid but unsupported combination */
    PSDP_E_INTERNAL = -8        /* a bookkeeping check of the library failed (a library bug) */
} psdp_status;

/* Subproblem solver: Algorithm 2 (projected alternating BB) or Algorithm 1
 * (proximal point with the diagonal H_p of Section 3.1). */
typedef enum { PSDP_INNER_PABB = 0, PSDP_INNER_PPA = 1 } psdp_inner;

/* Storage/arithmetic type of the Q.X product operands. F64 runs FP64 MFMA /
 * FP64 FMA; F32 runs FP32 MFMA with FP32 accumulation (batched) or FP32
 * storage with FP64 accumulation (single instance); BF16 stores Q in bfloat16
 * and accumulates in FP32/FP64. All other solver state is FP64.
 *
 * I8 (solver operands only) makes every product exact integer arithmetic:
 * Q off the diagonal is stored as int8 (so |Q_ij| <= 127 for i != j is
 * required, and FULL perturbation is not available), and the vector operand
 * is split into signed base-128 digits that int8 MFMA multiplies with int32
 * accumulation; the digit products combine in int64. A subproblem iterate
 * x in [0,1]^n is first rounded to the grid 2^-27 (4 digits) and its product
 * is exactly Q_off x_q; a lambda_min or CG vector v is scaled by the power of
 * two 2^e > max|v| and rounded to the grid 2^(e-55) (8 digits), and its
 * product is Q_off v_q rounded once to FP64. psdp_qx_digits exposes this
 * product on its own.
 *
 * With I8 operands the same integers can also come from a compressed sparse
 * row copy of Q_off (int8 values, int64 accumulation): see
 * psdp_params.sparse and psdp_qx_sparse. Either product gives identical
 * results, so the choice changes the speed only. */
typedef enum { PSDP_F64 = 0, PSDP_F32 = 1, PSDP_BF16 = 2, PSDP_I8 = 3 } psdp_dtype;

/* Random symmetric perturbation of Q before the reformation (Section 3.5,
 * "Random Perturbation"): none, every entry (i <= j, mirrored), or the
 * diagonal only. */
typedef enum { PSDP_PERTURB_NONE = 0, PSDP_PERTURB_FULL = 1, PSDP_PERTURB_DIAG = 2 } psdp_perturb;

/* Why a solve stopped. */
typedef enum {
    PSDP_EXIT_CONVERGED = 0,   /* max_i min(x_i, 1 - x_i) <= tol_binary (Algorithm 3) */
    PSDP_EXIT_OUTER_CAP = 1,   /* max_outer penalty updates reached */
    PSDP_EXIT_STALL = 2        /* stall_outer consecutive subproblems did not move x,
                                  or the cap was hit with a component at 1/2 */
} psdp_exit;

typedef struct {
    uint32_t struct_size;      /* sizeof(psdp_params); set by psdp_params_default */
    int32_t inner;             /* psdp_inner */
    int32_t qx_dtype;          /* psdp_dtype of the Q.X operands */
    int32_t perturb;           /* psdp_perturb */
    int32_t max_inner;         /* subproblem iteration cap (10000, Section 5) */
    int32_t max_outer;         /* penalty update cap (1000, Section 5) */
    int32_t stall_outer;       /* no-progress exit after this many non-moving subproblems (2) */
    int32_t eig_maxit;         /* lambda_min iteration cap (LOBPCG) (500) */
    int32_t cg_maxit;          /* x^0 linear solve iteration cap (500) */
    int32_t timing;            /* 1: time every Q.X launch with HIP events (psdp_stats.qx_*) */
    int32_t poll_sweeps;       /* sweeps enqueued between host polls of the live count (64) */
    int32_t gemm_variant;      /* batched Q.X kernel choice; -1 = chosen per live count */
    int32_t graph;             /* 1: replay batches of sweeps as HIP graphs (1); timing = 1
                                  launches eagerly */
    int32_t sparse;            /* I8 only: -1 (default) builds a sparse copy of Q_off when
                                  n >= 4096 and at most 1/64 of it is nonzero, and uses it for
                                  the sweeps with nonzeros x 2 x live columns <= n^2 / 4 (the
                                  range where it was measured faster on gfx950); 1 builds it
                                  whatever the size and uses it for every sweep; 0 never */
    int32_t lambda_reuse;      /* 1 (default): after a subproblem that left x unchanged,
                                  lambda_min is the previous value minus the previous alpha (I and
                                  z are unchanged, so eq. (alpha) shifted the scaled matrix by
                                  exactly -alpha) and no LOBPCG runs; 0: every update runs LOBPCG */
    int32_t slots;             /* batched solves: columns advanced together; 0 (default) or >= B
                                  gives every start its own column; 0 < slots < B keeps that many
                                  columns and queues the other starts in index order, a column
                                  taking the next start when its own ends (each start performs the
                                  same arithmetic either way; outputs stay per start) */
    int32_t lanes;             /* batched solves with integer products: L = 2 to 4 runs the
                                  columns as L lanes, concurrent launch sequences on L streams,
                                  each over 1/L of the columns and of the starts (each start
                                  performs the same arithmetic either way); 1 one sequence; 0
                                  (default) two from 512 columns on. Values outside 0..4 are
                                  rejected (PSDP_E_INVALID) */
    int32_t gemv_sym;          /* single-instance and group solves (one column per instance,
                                  floating-point operands): 1 reads Q from its unique half, stored
                                  as 128 x 128 upper tiles (each tile read once for its row and
                                  column contributions, partial sums added in a fixed order, the
                                  same in both); 0 reads full rows; -1 (default) takes the tiles
                                  from n = 4096 on, and in a group also once the stored matrices
                                  reach 256 MiB. Both are FP64 sums of exact products; they differ
                                  in summation order only */
    double tol_kkt;            /* delta of eq. (cret) (1e-5) */
    double tol_binary;         /* Algorithm 3 loop tolerance (1e-5) */
    double eta;                /* eq. (alpha1) scaling, 0 < eta < 1 (0.999) */
    double eps_hp;             /* epsilon in H_p (1e-8) */
    double lambda_floor_rel;   /* alpha uses max(lambda, lambda_floor_rel * rho) (1e-8) */
    double alpha_min, alpha_max; /* BB step clamp (1e-30, 1e30) */
    double sigma;              /* perturbation standard deviation (absolute) (0) */
    double eig_tol;            /* LOBPCG relative residual tolerance (1e-7) */
    double cg_tol;             /* x^0 relative residual tolerance (1e-12) */
    uint64_t seed;             /* perturbation seed */
} psdp_params;

typedef struct {
    int32_t exit_reason;       /* psdp_exit */
    int32_t outer_iters;       /* penalty updates performed */
    int64_t inner_iters;       /* penalty-gradient evaluations in subproblems */
    int64_t aux_matvecs;       /* Q products spent on lambda_min and x^0 */
    double final_cret_rel;     /* cret/rho at the last evaluation */
    double final_binary_gap;   /* max_i min(x_i, 1 - x_i) of the final iterate */
    int64_t sweeps;            /* Q.X sweeps of the whole launch (same for every column) */
    double qx_seconds;         /* summed Q.X kernel time (timing = 1), whole launch */
    double qx_flops;           /* algorithmic flops of those Q.X launches (2 n^2 per column) */
    int64_t qx_launches;       /* number of Q.X launches timed */
    double aux_seconds;        /* split precision (batched F32, I8): summed time of the
                                  lambda_min / CG products (timing = 1) */
    double aux_flops;          /* algorithmic flops of those products */
    double step_seconds;       /* summed time of the per-column step kernel (timing = 1) */
    int64_t step_launches;     /* number of step launches timed */
    int64_t column_steps;      /* column updates performed by those launches (all columns) */
    int64_t sparse_sweeps;     /* sweeps whose products used the sparse copy of Q (I8) */
} psdp_stats;

/* Fills *p with the defaults listed above. */
void psdp_params_default(psdp_params *p);

/* Static description of a status code. */
const char *psdp_status_string(psdp_status s);

/* Thread-local detail of the last error (empty string if none). */
const char *psdp_last_error(void);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int32_t psdp_version(void);

/*
 * psdp_solve_i32 - Algorithm 3 on B independent starts of one integer instance.
 *
 * Q       device, int32, n x n row-major (ldq = n), exactly symmetric.
 * b       device, int32, length n.
 * X0      device, double, n x B column-major, entries in [0,1]; NULL means
 *         every column starts from x^0 of eq. (gamma) (then B must be 1).
 * p0      device, double, length n, initial penalty of the reformulated
 *         problem (Algorithm 3 starts from 0); NULL means 0.
 * B       number of starts (>= 1). B = 1 runs the single-instance path
 *         (GEMV Q.x, FP64 accumulation, Q stored in qx_dtype); B > 1 runs
 *         all starts together (MFMA Q.X per sweep). With B > 1 and F32
 *         operands the subproblem products run on FP32 MFMA while the
 *         lambda_min and x^0 products keep FP64 operands (FP64 MFMA).
 *         With I8 operands every B (including 1) runs the exact integer
 *         digit products described at psdp_dtype.
 * prm     host, parameters (psdp_params_default then edit; NULL = defaults).
 * xhat    device, uint8, n x B: rounded solutions, x_i = 1 iff x_i > 1/2.
 * obj     device, int64, length B: f(xhat) on the original Q and b, exact.
 * X_out   device, double, n x B, nullable: final continuous iterates.
 * best    host, nullable: index of the smallest objective (lowest index on ties).
 * stats   host, nullable: array of B psdp_stats.
 * Errors: PSDP_E_INVALID (n < 1, B < 1, null required pointer, bad params),
 *         PSDP_E_NOT_SYMMETRIC, PSDP_E_NONFINITE (X0 outside [0,1]),
 *         PSDP_E_OVERFLOW (n^2 max|Q| + n max|b| >= 2^62),
 *         PSDP_E_UNSUPPORTED (FULL perturbation with BF16 operands; I8
 *         operands with |Q_ij| > 127 off the diagonal or a FULL
 *         perturbation; BF16 with B > 1), PSDP_E_DEVICE / PSDP_E_NOMEM.
 * Validation runs on the device (symmetry with the first offending entry,
 * magnitudes, X0 in [0,1], p0 finite); a few words come back to the host.
 */
psdp_status psdp_solve_i32(const int32_t *Q, const int32_t *b, int64_t n,
                           const double *X0, const double *p0, int32_t B,
                           const psdp_params *prm, uint8_t *xhat, int64_t *obj,
                           double *X_out, int32_t *best, psdp_stats *stats,
                           hipStream_t stream);

/*
 * psdp_solve_i32_ex - psdp_solve_i32 plus a per-penalty-update trace and a
 * replay of given penalty steps.
 * trace     host, nullable: B x trace_cap records of 6 doubles
 *           {s, |I|, lambda_min, alpha, subproblem evaluations, final cret/rho},
 *           one record per completed subproblem (unused records untouched).
 * trace_cap records per column (>= 1 when trace is given).
 * alpha_in  host, nullable: B x alpha_cap penalty steps, row c for start c.
 *           Penalty update s < alpha_cap of start c takes
 *           alpha = alpha_in[c * alpha_cap + s] in place of
 *           eta * max(lambda_min, lambda_floor_rel * rho) (eqs. (alpha),
 *           (alpha1)); lambda_min is still computed and traced. Later updates
 *           compute alpha. A parity hook: with another implementation's
 *           steps, the rest of every update (the penalty update eq. (pp1),
 *           the subproblem, the exit tests) can be compared step by step.
 *           Entries must be finite and > 0 (else PSDP_E_INVALID).
 * alpha_cap steps per start (>= 1 when alpha_in is given).
 */
psdp_status psdp_solve_i32_ex(const int32_t *Q, const int32_t *b, int64_t n,
                              const double *X0, const double *p0, int32_t B,
                              const psdp_params *prm, uint8_t *xhat, int64_t *obj,
                              double *X_out, int32_t *best, psdp_stats *stats,
                              double *trace, int32_t trace_cap,
                              const double *alpha_in, int32_t alpha_cap, hipStream_t stream);

/*
 * psdp_solve_f64 - Algorithm 3 on B starts of one instance with real data:
 * Q real symmetric and b real (Section 2, eq. (bqp)), both FP64.
 *
 * Arguments as psdp_solve_i32, except:
 * Q, b    device, double; Q n x n row-major, exactly symmetric, finite.
 * obj     device, double, length B: f(xhat) on the original Q and b, the
 *         exact value of the sum of the selected entries rounded once to
 *         FP64 (nearest, ties to even), so it does not depend on any
 *         summation order.
 * Operand types: F64 for any data; F32 and BF16 when every off-diagonal
 * entry of Q is exactly a float / a bfloat16 value (BF16 also without a
 * FULL perturbation); I8 when every off-diagonal entry is an integer in
 * [-127, 127] (and no FULL perturbation). Otherwise PSDP_E_UNSUPPORTED.
 * The perturbed entry Q_ij + mu_ij (Section 3.5) is rounded once to FP64.
 * Errors as psdp_solve_i32, with PSDP_E_NONFINITE also for NaN/Inf in Q or
 * b and PSDP_E_OVERFLOW when n^2 max|Q| + n max|b| >= 1e300.
 */
psdp_status psdp_solve_f64(const double *Q, const double *b, int64_t n,
                           const double *X0, const double *p0, int32_t B,
                           const psdp_params *prm, uint8_t *xhat, double *obj,
                           double *X_out, int32_t *best, psdp_stats *stats,
                           hipStream_t stream);

/* psdp_solve_f64 plus the trace and the replayed steps of psdp_solve_i32_ex. */
psdp_status psdp_solve_f64_ex(const double *Q, const double *b, int64_t n,
                              const double *X0, const double *p0, int32_t B,
                              const psdp_params *prm, uint8_t *xhat, double *obj,
                              double *X_out, int32_t *best, psdp_stats *stats,
                              double *trace, int32_t trace_cap,
                              const double *alpha_in, int32_t alpha_cap, hipStream_t stream);

/*
 * psdp_solve_host_i32, psdp_solve_host_f64 - the same solves with every
 * pointer in host memory (Q row-major n x n, b length n, X0 n x B
 * column-major or NULL, p0 length n or NULL, xhat n x B, obj length B,
 * X_out n x B or NULL, best and stats as above). The library copies the
 * inputs to the current device, solves, copies the outputs back and frees
 * its copies before returning. Errors as the device-pointer entries.
 */
psdp_status psdp_solve_host_i32(const int32_t *Q, const int32_t *b, int64_t n,
                                const double *X0, const double *p0, int32_t B,
                                const psdp_params *prm, uint8_t *xhat, int64_t *obj,
                                double *X_out, int32_t *best, psdp_stats *stats);
psdp_status psdp_solve_host_f64(const double *Q, const double *b, int64_t n,
                                const double *X0, const double *p0, int32_t B,
                                const psdp_params *prm, uint8_t *xhat, double *obj,
                                double *X_out, int32_t *best, psdp_stats *stats);

/*
 * psdp_solve_group_i32 - Algorithm 3 on `count` independent instances of
 * different sizes, all advanced together (one column per instance).
 *
 * n       host, int64[count], sizes (>= 1).
 * Q       host array of `count` device pointers, int32 n_i x n_i row-major.
 * b       host array of `count` device pointers, int32 length n_i.
 * seeds   host, uint64[count], nullable: per-instance perturbation seeds
 *         (NULL uses prm->seed for every instance).
 * sigmas  host, double[count], nullable: per-instance perturbation standard
 *         deviations (NULL uses prm->sigma for every instance); each finite
 *         and >= 0.
 * xhat    host array of `count` device pointers, uint8 length n_i.
 * obj     device, int64[count].
 * stats   host, nullable: array of `count` psdp_stats.
 * Every instance starts from its own x^0 (eq. (gamma)) with p^0 = 0.
 * Errors as psdp_solve_i32.
 */
psdp_status psdp_solve_group_i32(int32_t count, const int64_t *n,
                                 const int32_t *const *Q, const int32_t *const *b,
                                 const uint64_t *seeds, const double *sigmas, const psdp_params *prm,
                                 uint8_t *const *xhat, int64_t *obj,
                                 psdp_stats *stats, hipStream_t stream);

/*
 * psdp_eval_penalty_grad - h(x_c, p) and grad h(x_c, p) for B points (eq. (p1)
 * and the gradient 2 (Q - Diag p) x + (b + p) of eq. (kkt1)), exactly as
 * written, with the given p (no reformation, no perturbation).
 *
 * dtype   psdp_dtype of Q and X (F64, F32 or BF16).
 * vtype   psdp_dtype of b, p, h and G (F64 or F32).
 * Q       device, n x n, leading dimension ldq >= n, symmetric (not checked).
 * b, p    device, length n.
 * X       device, n x B column-major.
 * h       device, length B.
 * G       device, n x B column-major, nullable.
 * Stream-ordered; no host synchronization. Errors: PSDP_E_INVALID.
 */
psdp_status psdp_eval_penalty_grad(int32_t dtype, int32_t vtype, const void *Q, int64_t ldq,
                                   const void *b, const void *p, const void *X,
                                   int64_t n, int64_t B, void *h, void *G,
                                   hipStream_t stream);

/*
 * psdp_eval_penalty_grad_noalloc - psdp_eval_penalty_grad (same arguments,
 * same kernels, bit-identical h and G) for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation. The product workspace (8 n B + 4 B +
 * 320 bytes) lives in a fixed 32 MiB device array of the library, one per
 * device, held until the process ends; no hipMalloc or other allocation
 * happens in the call. Calls that overlap on one device share that array
 * and race: serialize them (one stream, or events). Every word the
 * evaluation reads from the array is written by the same call first.
 * Errors: as psdp_eval_penalty_grad, and PSDP_E_UNSUPPORTED when
 * 8 n B + 4 B + 320 exceeds 32 MiB.
 */
psdp_status psdp_eval_penalty_grad_noalloc(int32_t dtype, int32_t vtype, const void *Q, int64_t ldq,
                                           const void *b, const void *p, const void *X,
                                           int64_t n, int64_t B, void *h, void *G,
                                           hipStream_t stream);

/*
 * psdp_penalty_adjoint - gradients of L = sum_c w_c h(x_c, p) (h of eq. (p1),
 * linear in Q, b and p):
 *   dX[:, c] = w_c G[:, c]             (G = grad h from psdp_eval_penalty_grad)
 *   dQ       = X Diag(w) X^T           (n x n, entries of Q taken as independent)
 *   db       = X w,   dp = (X - X o X) w.
 * dtype   psdp_dtype of X and dQ (F32 or F64); vtype of G, w, dX, db, dp.
 * X, G    device, n x B column-major. w: device, length B.
 * dX, dQ (ld n), db, dp: device outputs, each nullable (skipped when NULL).
 * Stream-ordered. Errors: PSDP_E_INVALID, PSDP_E_UNSUPPORTED (BF16).
 */
psdp_status psdp_penalty_adjoint(int32_t dtype, int32_t vtype, const void *X, const void *G,
                                 const void *w, int64_t n, int64_t B,
                                 void *dX, void *dQ, void *db, void *dp,
                                 hipStream_t stream);

/*
 * psdp_round_objective_i32 - the final step of the solve on given iterates:
 * xhat_ic = 1 iff X_ic > 1/2 and obj_c = xhat_c^T Q xhat_c + b^T xhat_c
 * (the objective of Section 2, eq. (bqp)), in exact int64 arithmetic on the
 * original integer data. The paper never states how the final continuous
 * point becomes binary; rounding at 1/2 with ties to 0 is this library's
 * reading.
 * Q device int32 n x n; b device int32; X device double n x B;
 * xhat device uint8 n x B; obj device int64[B]. Stream-ordered.
 * Errors: PSDP_E_INVALID.
 */
psdp_status psdp_round_objective_i32(const int32_t *Q, const int32_t *b, int64_t n,
                                     const double *X, int64_t B, uint8_t *xhat,
                                     int64_t *obj, hipStream_t stream);

/*
 * psdp_round_objective_f64 - the same for real data: Q device double n x n,
 * b device double; obj device double[B] is the exact sum of the selected
 * Q_ij and b_i rounded once to FP64 (nearest, ties to even). The call
 * allocates B * 32 KiB of stream-ordered scratch. Stream-ordered.
 * Errors: PSDP_E_INVALID (n > 65536, B > 65535, null pointer).
 */
psdp_status psdp_round_objective_f64(const double *Q, const double *b, int64_t n,
                                     const double *X, int64_t B, uint8_t *xhat,
                                     double *obj, hipStream_t stream);

/*
 * psdp_perturbation - the symmetric perturbation mu of Section 3.5 as this
 * library draws it: for i <= j and t = 0..3, c = (i n + j) 4 + t,
 * key = SplitMix64(seed), u_t = SplitMix64(key XOR c) >> 11;
 * S = sum u_t (exact integer);
 * N = (double(S) 2^-53 - 2) sqrt(3); mu_ij = mu_ji = rint(N sigma 2^16) 2^-16.
 * mode FULL fills all entries, DIAG only the diagonal, NONE writes zeros.
 * mu: device, double, n x n. Stream-ordered. Errors: PSDP_E_INVALID.
 */
psdp_status psdp_perturbation(int64_t n, double sigma, uint64_t seed, int32_t mode,
                              double *mu, hipStream_t stream);

/*
 * psdp_qx_digits - the exact integer Q.X product of the I8 solver path
 * (the O(n^2) part of every gradient evaluation, eq. (kkt1), and of every
 * lambda_min and x^0 matvec, eqs. (alpha) and (gamma)) on given vectors:
 * Y[:, c] = Q_off X_q[:, c], Q_off = Q with a zero diagonal.
 *
 * digits 4: entries of X must lie in [0,1]; X_q = rint(X 2^27) 2^-27 (ties
 *           to even) and Y is exact.
 * digits 8: for each column, e_c is the least integer with
 *           max_i |X_ic| < 2^e_c (e_c = 0 for a zero column);
 *           X_q = rint(X 2^(55 - e_c)) 2^(e_c - 55) and Y is X_q's exact
 *           product rounded once to double (ties to even).
 * Q       device, int32, n x n row-major, |Q_ij| <= 127 for i != j (the
 *         diagonal is ignored; symmetry is not checked, the product uses row
 *         i of Q for Y_ic).
 * X       device, double, n x B column-major (leading dimension n).
 * Y       device, double, n x B column-major (leading dimension n), output.
 * The call allocates its own device workspace, reads Q back to the host once
 * for the range check, and synchronizes `stream` before returning.
 * Errors: PSDP_E_INVALID (n < 1 or n > 65536, B < 1, digits not 4 or 8, null
 *         pointer), PSDP_E_NONFINITE (non-finite X, or digits 4 with X
 *         outside [0,1]), PSDP_E_UNSUPPORTED (|Q_ij| > 127 off the diagonal),
 *         PSDP_E_DEVICE / PSDP_E_NOMEM.
 */
psdp_status psdp_qx_digits(const int32_t *Q, int64_t n, const double *X, int32_t B,
                           int32_t digits, double *Y, hipStream_t stream);

/*
 * psdp_qx_digits_ex - psdp_qx_digits with the product's kernel settings
 * given, and optionally timed (the same product as above: every setting
 * yields the same integers, so Y does not depend on them).
 * layout  block layout of the int8 MFMA kernel: 1 (few columns: the K range
 *         of one 32-row block split over the four waves), 2 (64-row blocks,
 *         the digit tile shared through LDS), 4 (128-row blocks), 8 (256-row
 *         blocks), 16 (128-row blocks with 256 digit rows); 0 = the
 *         library's choice for B columns (its table for n, see
 *         psdp_set_digit_table, else its built-in rule).
 * slices  K slices, 1..8 (0 = the library's choice).
 * reps    > 0: after Y is formed, the product is launched reps more times
 *         between two HIP events on `stream`, and *us receives the average
 *         microseconds per launch (host pointer; unused when reps = 0).
 * Errors: as psdp_qx_digits, and PSDP_E_INVALID for a layout, slices or reps
 *         out of range.
 */
psdp_status psdp_qx_digits_ex(const int32_t *Q, int64_t n, const double *X, int32_t B,
                              int32_t digits, int32_t layout, int32_t slices, int32_t reps,
                              double *us, double *Y, hipStream_t stream);

/*
 * psdp_set_digit_table - the exact integer product's settings for problems
 * with n variables (no paper passage: a speed setting, for the package's
 * autotuner). For products of `digits` digits (4: subproblem iterates,
 * 8: lambda_min and CG vectors), entry q holds the layout and K slices
 * (as in psdp_qx_digits_ex, nonzero) used when the product's live-column
 * estimate is at most max_cols[q]; max_cols increases with q, and the last
 * entry also covers every larger estimate. Used by the solves, by
 * psdp_qx_digits and by psdp_digit_choice from the next call on; count = 0
 * removes the table for (n, digits). The arrays are host memory, copied.
 * Errors: PSDP_E_INVALID (n, digits, count, a null array, max_cols not
 *         positive and increasing, a layout or slice count out of range).
 */
psdp_status psdp_set_digit_table(int64_t n, int32_t digits, int32_t count, const int32_t *max_cols,
                                 const int32_t *layout, const int32_t *slices);

/*
 * psdp_digit_choice - the settings the solves use for one launch holding a
 * 4-digit product of est4 columns and an 8-digit product of est8 columns
 * (0 = no such product) at n variables: choice[0..3] (host) = layout and K
 * slices of the 4-digit product, then of the 8-digit product.
 * Errors: PSDP_E_INVALID (n out of range, a negative estimate, null choice).
 */
psdp_status psdp_digit_choice(int64_t n, int32_t est4, int32_t est8, int32_t *choice);

/*
 * psdp_qx_dense - the floating-point Q.X product of the batched solver path
 * (the O(n^2) part of every gradient evaluation, eq. (kkt1)) on given
 * vectors: Y[:, c] = Q_off X[:, c], Q_off = Q with a zero diagonal, through
 * the kernel and split-K the solver picks for B live columns (the streaming
 * MFMA kernel up to 64 columns, the LDS-tiled MFMA GEMM above), with the
 * K slices summed in FP64 in slice order as the solver's column kernel
 * reads them.
 * dtype   F32: FP32 operands, FP32 MFMA accumulation within a slice (X is
 *         rounded to float); F64: FP64 operands and FP64 MFMA (Q read from
 *         its exact FP32 copy).
 * Q       device, int32, n x n row-major, |Q_ij| <= 2^24 (the diagonal is
 *         ignored; symmetry is checked).
 * X, Y    device, double, n x B column-major (leading dimension n).
 * The call allocates its own workspace and synchronizes `stream`.
 * Errors: PSDP_E_INVALID (dtype, sizes, null pointer), PSDP_E_NOT_SYMMETRIC,
 *         PSDP_E_UNSUPPORTED (|Q_ij| > 2^24), PSDP_E_DEVICE / PSDP_E_NOMEM.
 */
psdp_status psdp_qx_dense(int32_t dtype, const int32_t *Q, int64_t n, const double *X, int32_t B,
                          double *Y, hipStream_t stream);

/*
 * psdp_qx_single - the single-instance solver's product on one vector
 * (the O(n^2) part of eq. (kkt1) and of the lambda_min and x^0 matvecs,
 * eqs. (alpha) and (gamma)): y = Q_off x, Q_off = Q with a zero diagonal,
 * stored as `dtype` (F64, F32 or BF16; exact for integer Q within the
 * type's integer range) and multiplied and summed in FP64, through the
 * row-by-row GEMV (sym = 0) or the product from the unique half of Q in
 * packed 128 x 128 upper tiles (sym = 1; see psdp_params.gemv_sym).
 * Q       device, int32, n x n row-major, symmetric (checked).
 * x, y    device, double, n entries; y is the output.
 * The call allocates its own workspace and synchronizes `stream`.
 * Errors: PSDP_E_INVALID (dtype, sym, n, null pointer), PSDP_E_NOT_SYMMETRIC,
 *         PSDP_E_DEVICE / PSDP_E_NOMEM.
 */
psdp_status psdp_qx_single(int32_t dtype, const int32_t *Q, int64_t n, const double *x, int32_t sym,
                           double *y, hipStream_t stream);

/*
 * psdp_qx_sparse - the same product as psdp_qx_digits (same arguments, same
 * rounding, bit-identical Y), computed from a compressed sparse row copy of
 * Q_off built on the device: one int32 word per operand entry (T, or T_hi
 * and T_lo with T = T_hi 2^28 + T_lo for 8 digits) times the int8 nonzeros,
 * accumulated exactly in int64. Work and time grow with the nonzeros; the
 * solver uses this form for sparse Q (psdp_params.sparse).
 * Errors: as psdp_qx_digits, and PSDP_E_UNSUPPORTED when Q_off has 2^31 or
 * more nonzeros.
 */
psdp_status psdp_qx_sparse(const int32_t *Q, int64_t n, const double *X, int32_t B,
                           int32_t digits, double *Y, hipStream_t stream);

/* Releases the cached device workspace of every device (optional). */
void psdp_release(void);

/* Column bookkeeping of a batched solve's workspace (no paper passage: the
 * layout of the library's own buffers, for callers that size device memory
 * and for host-side tests of the layout). The product kernels read the
 * live-column lists and, through them, the per-column operand buffers; a
 * list slot left empty (its column ended or changed product) names column
 * zero_col, whose operand data stay zero, and the kernels read list entries
 * up to index zero_col. So every list and every operand buffer read through
 * a list holds zero_col + 1 columns; the solve entry points check this when
 * they allocate and fail with PSDP_E_INTERNAL if it does not hold. */
typedef struct {
    int64_t ld;            /* leading dimension of the per-column vectors (elements) */
    int32_t ncol;          /* columns advanced together: B, or params.slots when 0 < slots < B */
    int32_t zero_col;      /* the all-zero column that empty list slots name */
    int32_t list_len;      /* entries of each live-column list */
    int32_t digit_cols;    /* columns of the digit planes (I8 operands), 0 otherwise */
    int32_t word_cols;     /* columns of the sparse products' operand words (I8 with a
                              sparse copy of Q), 0 otherwise */
    int32_t ok;            /* 1 when every list-indexed buffer holds zero_col + 1 columns */
} psdp_column_plan;

/* Fills *out with the plan that psdp_solve_i32 / psdp_solve_f64 would use for
 * n, B starts and *prm (NULL = defaults); sparse_copy = 1 when the sparse copy
 * of Q is built (params.sparse = 1, or the automatic rule for the data).
 * Host only: no device work, callable without a GPU. PSDP_E_INVALID for
 * n outside [1, 65536], B < 1 or bad params. */
psdp_status psdp_plan_columns(int64_t n, int32_t B, const psdp_params *prm, int32_t sparse_copy,
                              psdp_column_plan *out);

#ifdef __cplusplus
}
#endif

#endif /* PSDP_H */
