// Per-column solver state machine of the vectorized PSDP method.
//
// One workgroup (512 threads) owns one column (one start of one instance).
// Every sweep the Q.X kernels apply the off-diagonal part of the (perturbed)
// Q to one vector per live column; this kernel consumes that product
// according to the column's phase and prepares the next operand:
//   PH_INNER  subproblem step of Algorithm 2 (projected alternating BB,
//             eqs. (bb1), (x2)) or Algorithm 1 (diagonal proximal step,
//             eqs. (d2), (x1)), stopping rule eq. (cret) (Section 3.3);
//   PH_EIG0/  lambda_min of Z_II^-1/2 Qbar_II Z_II^-1/2 (eq. (alpha)) by
//   PH_EIG    LOBPCG on the pencil (Qbar_II, Z_II) with a Jacobi
//             preconditioner, then the penalty update eq. (pp1), (alpha1);
//   PH_CG     x^0 from 2 (Q + Diag gamma) x = gamma - b (eq. (gamma)) by
//             Jacobi-preconditioned conjugate gradients.
// The reformulated matrix Q_r - Diag p = Q_off + Diag((Q_ii + gamma_i) - p_i)
// is never formed: the product covers Q_off and the FP64 diagonal
// (dq + gamma) - p is applied here, so the gradient is exactly the paper's
// 2 (Q_r - Diag p) x + (b_r + p) with b_r = b - gamma.
//
// Element loops are unrolled EPT times per thread so that every load of a
// pass is in flight at once; every live column appends itself to the
// live-column lists of the next sweep.
#include <type_traits>

#include "launch.hpp"

namespace psdp {

// Uniform operands. A column's sizes and offsets are read from its LDS
// record; passing them through readfirstlane tells the compiler that every
// lane holds the same value, so the vector base pointers stay in scalar
// registers and each element costs one 32-bit offset register for all the
// arrays it touches, instead of a 64-bit address per array.
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni(int64_t v) {
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// A column or instance vector: uniform base, elements addressed by a 32-bit
// byte offset (n <= 65536, so i * 8 never wraps).
template <typename T>
struct UVec {
    T *p;
    __device__ __forceinline__ T &operator[](uint32_t i) const {
        return *reinterpret_cast<T *>(reinterpret_cast<char *>(const_cast<typename std::remove_const<T>::type *>(p)) +
                                      i * (uint32_t)sizeof(T));
    }
    // entries i and i + 1 as one V (i even: the vectors' bases are aligned
    // to 256 bytes, so a pair of 8-byte entries is one 16-byte access)
    template <typename V> __device__ __forceinline__ V &pair(uint32_t i) const {
        return *reinterpret_cast<V *>(reinterpret_cast<char *>(const_cast<typename std::remove_const<T>::type *>(p)) +
                                      i * (uint32_t)sizeof(T));
    }
};
template <typename T> __device__ __forceinline__ UVec<T> uvec(T *base, int64_t off) { return UVec<T>{base + off}; }

// The uniform facts of a column every pass needs.
struct ColView {
    uint32_t n;   // length
    int64_t off;  // column vector offset
    int64_t io;   // instance vector offset
};
__device__ __forceinline__ ColView view(const Col &c) {
    return ColView{(uint32_t)uni((int32_t)c.n), uni(c.off), uni(c.ioff)};
}

// Visits i = threadIdx.x + j * kSB (+ multiples of EPT * kSB) for i < n
// (set-up code; the per-sweep passes use the chunked form below).
#define FOR_I(n)                                                       \
    for (uint32_t _b = 0; _b < (n); _b += (uint32_t)(EPT * kSB))       \
        _Pragma("unroll") for (int _j = 0; _j < EPT; ++_j)             \
            if (const uint32_t i = _b + threadIdx.x + (uint32_t)(_j * kSB); i < (n))

// Per-sweep passes work on chunks of EPT elements per thread: element j of
// chunk _b is i = _b + threadIdx.x + j kSB. CHUNK_INDEX clamps it to n - 1
// (ix[j]) and records whether it is real (ok[j]), so every load of a chunk is
// unconditional and in bounds and all of them issue before the first wait; a
// branch per element would make the loads wait element by element. Results
// of clamped elements are discarded (selects, guarded stores), in the same
// per-thread order as before, so the arithmetic is unchanged. Within a pass
// (and between the passes of one step, which keep values in registers or
// LDS) every element is read and written by the same thread; a later phase
// of the same launch may map elements to threads differently (the subproblem
// passes use the pairs below) and reads them only after a block barrier.
#define CHUNKS(n) for (uint32_t _b = 0; _b < (n); _b += (uint32_t)(EPT * kSB))
#define CHUNK_INDEX(n)                                                 \
    uint32_t ix[EPT];                                                  \
    bool ok[EPT];                                                      \
    _Pragma("unroll") for (int _j = 0; _j < EPT; ++_j) {               \
        const uint32_t _i = _b + threadIdx.x + (uint32_t)(_j * kSB);   \
        ok[_j] = _i < (n);                                             \
        ix[_j] = ok[_j] ? _i : (n) - 1;                                \
    }
#define FOR_J _Pragma("unroll") for (int _j = 0; _j < EPT; ++_j)

// The subproblem passes (PAIR: an even EPT) map a chunk in pairs instead:
// thread t holds elements 2 (t + k kSB) and 2 (t + k kSB) + 1 (k < EPT / 2),
// so that each access of the thread to a column vector moves two entries at
// once (16 bytes for 8-byte entries). The passes issue one memory instruction
// per entry and vector, and a CU's memory pipeline takes a 16-byte access per
// lane about as fast as an 8-byte one, so pairs halve the time the pipeline
// is busy with a column. A pair past n repeats the last pair of the column
// (in bounds: when n is odd its second entry is padding, since ld > n), and
// entries past n are discarded as above; a stored pair whose second entry is
// past n stores zero there (padding entries stay zero).
template <int EPT> constexpr bool kPair = EPT % 2 == 0;
template <int EPT>
__device__ __forceinline__ void chunk_map(uint32_t b, uint32_t n, uint32_t (&ix)[EPT], bool (&ok)[EPT]) {
    if constexpr (kPair<EPT>) {
#pragma unroll
        for (int k = 0; k < EPT / 2; ++k) {
            const uint32_t i = b + 2u * (threadIdx.x + (uint32_t)(k * kSB));
            const uint32_t c = i < n ? i : ((n - 1u) & ~1u);
            ix[2 * k] = c;
            ix[2 * k + 1] = c + 1u;
            ok[2 * k] = i < n;
            ok[2 * k + 1] = i + 1u < n;
        }
    } else {
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const uint32_t i = b + threadIdx.x + (uint32_t)(j * kSB);
            ok[j] = i < n;
            ix[j] = ok[j] ? i : n - 1u;
        }
    }
}
#define CHUNK_PAIRS(n)                                                 \
    uint32_t ix[EPT];                                                  \
    bool ok[EPT];                                                      \
    chunk_map<EPT>(_b, (n), ix, ok);

template <typename T> struct PairOf;
template <> struct PairOf<double> { using type = double2; };
template <> struct PairOf<int64_t> { using type = longlong2; };
template <> struct PairOf<float> { using type = float2; };
template <> struct PairOf<int32_t> { using type = int2; };

// Loads of one chunk's entries of a vector, as pairs when PAIR.
template <bool PAIR, int EPT, typename T>
__device__ __forceinline__ void ld_chunk(const UVec<T> &v, const uint32_t (&ix)[EPT],
                                         typename std::remove_const<T>::type (&o)[EPT]) {
    using E = typename std::remove_const<T>::type;
    if constexpr (PAIR && kPair<EPT> && (sizeof(E) == 8 || sizeof(E) == 4)) {
        using V = typename PairOf<E>::type;
#pragma unroll
        for (int k = 0; k < EPT / 2; ++k) {
            const V a = v.template pair<const V>(ix[2 * k]);
            o[2 * k] = a.x;
            o[2 * k + 1] = a.y;
        }
    } else {
        FOR_J o[_j] = v[ix[_j]];
    }
}
// Stores of one chunk's real entries, as pairs when PAIR.
template <bool PAIR, int EPT, typename T>
__device__ __forceinline__ void st_chunk(const UVec<T> &v, const uint32_t (&ix)[EPT], const bool (&ok)[EPT],
                                         const T (&val)[EPT]) {
    if constexpr (PAIR && kPair<EPT> && (sizeof(T) == 8 || sizeof(T) == 4)) {
        using V = typename PairOf<T>::type;
#pragma unroll
        for (int k = 0; k < EPT / 2; ++k)
            if (ok[2 * k]) {
                V a;
                a.x = val[2 * k];
                a.y = ok[2 * k + 1] ? val[2 * k + 1] : T(0);
                v.template pair<V>(ix[2 * k]) = a;
            }
    } else {
        FOR_J if (ok[_j]) v[ix[_j]] = val[_j];
    }
}

template <typename OpT> constexpr bool kDigits = std::is_same<OpT, int8_t>::value;

// The products of one chunk (elements ix[j]) for a subproblem column: every
// slice's loads for all elements issue together. Integer path: Q x_q on the
// grid 2^-27, exact, in one buffer that the product's K slices add into;
// each real element is cleared once read when the next product adds into
// it (w.clear_main).
template <typename UT, int EPT, bool PAIR = false>
__device__ __forceinline__ void uval_chunk(const Work &w, const ColView &cv, const uint32_t (&ix)[EPT],
                                           const bool (&ok)[EPT], double (&u)[EPT]) {
    if constexpr (std::is_same<UT, int64_t>::value) {
        const UVec<int64_t> U = uvec((int64_t *)w.U, cv.off);
        int64_t s[EPT];
        ld_chunk<PAIR>(U, ix, s);
        if (w.clear_main) {
            int64_t z[EPT];
            FOR_J z[_j] = 0;
            st_chunk<PAIR>(U, ix, ok, z);
        }
        FOR_J u[_j] = (double)s[_j] / kMainScale;
    } else {
        const UVec<const UT> U = uvec((const UT *)w.U, cv.off);
        FOR_J u[_j] = to_f64<UT>(U[ix[_j]]);
        for (int t = 1; t < w.ksplit; ++t) {
            const UVec<const UT> Ut = uvec(U.p, (int64_t)t * w.slice);
            FOR_J u[_j] += to_f64<UT>(Ut[ix[_j]]);
        }
    }
}

// The same for a lambda_min / CG column (FP64 buffers when precision is
// split; on the integer path the two int64 halves of the 8-digit product,
// scaled by 2^escale, cleared once read when w.clear_aux is set).
template <typename UT, int EPT>
__device__ __forceinline__ void uaux_chunk(const Work &w, const Col &c, const ColView &cv,
                                           const uint32_t (&ix)[EPT], const bool (&ok)[EPT], double (&u)[EPT]) {
    if constexpr (std::is_same<UT, int64_t>::value) {
        const UVec<int64_t> H = uvec((int64_t *)w.U_aux, cv.off), L = uvec(w.U_lo, cv.off);
        int64_t hi[EPT], lo[EPT];
        FOR_J {
            hi[_j] = H[ix[_j]];
            lo[_j] = L[ix[_j]];
        }
        if (w.clear_aux) {
            FOR_J if (ok[_j]) {
                H[ix[_j]] = 0;
                L[ix[_j]] = 0;
            }
        }
        const int e = uni(c.escale);
        FOR_J u[_j] = digits8_value(hi[_j], lo[_j], e);
    } else {
        if (!w.split) {
            uval_chunk<UT, EPT>(w, cv, ix, ok, u);
            return;
        }
        const UVec<const double> U = uvec((const double *)w.U_aux, cv.off);
        FOR_J u[_j] = U[ix[_j]];
        for (int t = 1; t < w.ksplit_aux; ++t) {
            const UVec<const double> Ut = uvec(U.p, (int64_t)t * w.slice_aux);
            FOR_J u[_j] += Ut[ix[_j]];
        }
    }
}

// Next operand of a lambda_min / CG column. The integer path keeps the FP64
// value; its digits follow in aux_digits once the column's largest
// magnitude is known.
template <typename OpT>
__device__ __forceinline__ void put_aux(const Work &w, const ColView &cv, uint32_t i, double v) {
    if (kDigits<OpT> || w.split) uvec(w.op_aux, cv.off)[i] = v;
    else uvec((OpT *)w.op, cv.off)[i] = from_f64<OpT>(v);
}

// Digit planes of a column: [4][ld] int8 for the subproblem operand, [8][ld]
// for the lambda_min / CG operand.
__device__ __forceinline__ int8_t *main_planes(const Work &w, const Col &c) {
    return w.dig + (int64_t)uni(c.id) * 4 * uni(c.ld);
}
__device__ __forceinline__ int8_t *aux_planes(const Work &w, const Col &c) {
    return w.dig_aux + (int64_t)uni(c.id) * 8 * uni(c.ld);
}

// Next operand of a subproblem column (x in [0,1]; the integer path rounds
// it to the grid 2^-27 and writes its 4 digits).
template <typename OpT>
__device__ __forceinline__ void put_main(const Work &w, const Col &c, const ColView &cv, uint32_t i, double v) {
    if constexpr (kDigits<OpT>) {
        const int64_t T = __double2ll_rn(v * kMainScale);
        put_digits4(main_planes(w, c), uni(c.ld), i, (int32_t)T);
        if (w.tw) uvec(w.tw, cv.off)[i] = (int32_t)T;
    } else {
        uvec((OpT *)w.op, cv.off)[i] = from_f64<OpT>(v);
    }
}

// The four base-128 digits of T, as put_digits4 splits it.
__device__ __forceinline__ void digits4_of(int32_t T, int32_t (&d)[4]) {
    d[0] = (T + (1 << 20)) >> 21;
    T -= d[0] << 21;
    d[1] = (T + (1 << 13)) >> 14;
    T -= d[1] << 14;
    d[2] = (T + (1 << 6)) >> 7;
    T -= d[2] << 7;
    d[3] = T;
}

// put_main for one chunk's real entries; in pairs (PAIR and an even EPT) on
// the integer path: two entries' digits per plane as one 2-byte store (a
// second entry past n gets the digits of 0).
template <typename OpT, int EPT, bool PAIR>
__device__ __forceinline__ void put_main_chunk(const Work &w, const Col &c, const ColView &cv,
                                               const uint32_t (&ix)[EPT], const bool (&ok)[EPT],
                                               const double (&v)[EPT]) {
    if constexpr (kDigits<OpT> && PAIR && kPair<EPT>) {
        int8_t *pl = main_planes(w, c);
        const int64_t ld = uni(c.ld);
        const UVec<int32_t> tw{w.tw ? w.tw + cv.off : nullptr};
#pragma unroll
        for (int k = 0; k < EPT / 2; ++k) {
            if (!ok[2 * k]) continue;
            const uint32_t i = ix[2 * k];
            const int32_t T0 = (int32_t)__double2ll_rn(v[2 * k] * kMainScale);
            const int32_t T1 = ok[2 * k + 1] ? (int32_t)__double2ll_rn(v[2 * k + 1] * kMainScale) : 0;
            int32_t a[4], b[4];
            digits4_of(T0, a);
            digits4_of(T1, b);
#pragma unroll
            for (int t = 0; t < 4; ++t)
                *reinterpret_cast<uint16_t *>(pl + t * ld + i) = (uint16_t)((a[t] & 0xff) | ((b[t] & 0xff) << 8));
            if (w.tw) tw.template pair<int2>(i) = make_int2(T0, T1);
        }
    } else {
        FOR_J if (ok[_j]) put_main<OpT>(w, c, cv, ix[_j], v[_j]);
    }
}

// Integer path: 8 digits of the lambda_min / CG operand just written by
// put_aux (every thread rereads its own elements), scaled by 2^-e with e the
// least integer above log2(maxabs). No-op on the floating-point paths.
// regs: the operand's values when the column is one chunk and use_regs is set.
template <typename OpT, int EPT>
__device__ __forceinline__ void aux_digits(const Work &w, Col &c, const ColView &cv, double maxabs,
                                           const double (&regs)[EPT], bool use_regs) {
    if constexpr (kDigits<OpT>) {
        const int e = digits8_exponent(maxabs);
        const uint32_t n = cv.n;
        const UVec<const double> src = uvec((const double *)w.op_aux, cv.off);
        int8_t *dst = aux_planes(w, c);
        const int64_t ld = uni(c.ld);
        const bool words = w.tw_hi != nullptr;
        const UVec<int32_t> wh{words ? w.tw_hi + cv.off : nullptr}, wl{words ? w.tw_lo + cv.off : nullptr};
        CHUNKS(n) {
            CHUNK_INDEX(n)
            double v[EPT];
            if (use_regs) {
                FOR_J v[_j] = regs[_j];
            } else {
                FOR_J v[_j] = src[ix[_j]];
            }
            FOR_J if (ok[_j]) {
                int32_t hi, lo;
                split8(v[_j], e, &hi, &lo);
                put_digits4(dst, ld, ix[_j], hi);
                put_digits4(dst + 4 * ld, ld, ix[_j], lo);
                if (words) {
                    wh[ix[_j]] = hi;
                    wl[ix[_j]] = lo;
                }
            }
        }
        // every read of c.escale this sweep (the first pass) precedes the
        // block reductions that the callers ran since
        if (threadIdx.x == 0) c.escale = e;
    }
}

template <typename OpT, int EPT>
__device__ __forceinline__ void aux_digits(const Work &w, Col &c, const ColView &cv, double maxabs) {
    const double none[EPT] = {};
    aux_digits<OpT, EPT>(w, c, cv, maxabs, none, false);
}

__device__ __forceinline__ bool interior(double x) { return x > 0.0 && x < 1.0; }

// The diagonal of Q_r - Diag p for one column, (Q_ii + gamma_i) - p_i, read
// as dg[i] from the instance vector dgi and the column's penalty.
struct DiagView {
    UVec<const double> dgi, p;
    __device__ __forceinline__ double operator[](uint32_t i) const { return dgi[i] - p[i]; }
};

template <int N> __device__ __forceinline__ void bsum(double (&v)[N], double *red) {
    block_sum<N, kSB>(v, red);
}
template <int N> __device__ __forceinline__ void bmax(double (&v)[N], double *red) {
    block_max<N, kSB>(v, red);
}

template <typename OpT, int EPT>
__device__ void eig_finish(const Work &w, Col &c, const ColView &cv, double *red, double lam);

// ---------------------------------------------------------------------------
// Outer loop head (Algorithm 3): exit tests, then start lambda_min.

template <typename OpT, int EPT>
__device__ void outer_begin(const Work &w, Col &c, const ColView &cv, double *red) {
    const uint32_t n = cv.n;
    const UVec<const double> x = uvec((const double *)w.x, cv.off), pp = uvec((const double *)w.p, cv.off);
    const UVec<const double> dgi = uvec((const double *)w.dgi, cv.io), lni = uvec((const double *)w.lni, cv.io);
    const UVec<const double> R = uvec((const double *)w.R, cv.io);
    double mx[4] = {0.0, 0.0, 0.0, 0.0};  // binary gap, pinned-at-half flag, row term, |b_r + p|
    double sm[2] = {0.0, 0.0};            // sum of z over I, |I|
    CHUNKS(n) {
        CHUNK_INDEX(n)
        double xv[EPT], pv[EPT], Av[EPT], Rv[EPT], bv[EPT];
        FOR_J {
            const uint32_t i = ix[_j];
            xv[_j] = x[i];
            pv[_j] = pp[i];
            Av[_j] = dgi[i];
            Rv[_j] = R[i];
            bv[_j] = lni[i];
        }
        FOR_J {
            Av[_j] = Av[_j] - pv[_j];
            bv[_j] = bv[_j] + pv[_j];
        }
        FOR_J {
            if (!ok[_j]) continue;
            const double xi = xv[_j];
            mx[0] = fmax(mx[0], fmin(xi, 1.0 - xi));
            if (fabs(xi - 0.5) < 1e-9) mx[1] = 1.0;
            if (interior(xi)) {
                sm[0] += xi - xi * xi;
                sm[1] += 1.0;
            }
            mx[2] = fmax(mx[2], 2.0 * (Rv[_j] + fabs(Av[_j])));
            mx[3] = fmax(mx[3], fabs(bv[_j]));
        }
    }
    block_maxsum<4, 2, kSB>(mx, sm, red);
    const double rho = fmax(1.0, fmax(mx[2], mx[3]));
    int32_t exitr = -1;
    if (mx[0] <= w.tol_binary) exitr = PSDP_EXIT_CONVERGED;
    else if (c.stall >= w.stall_outer) exitr = PSDP_EXIT_STALL;
    else if (c.s >= w.max_outer) exitr = mx[1] != 0.0 ? PSDP_EXIT_STALL : PSDP_EXIT_OUTER_CAP;
    if (threadIdx.x == 0) {
        c.rho_outer = rho;
        c.final_bg = mx[0];
        c.nI = (int32_t)sm[1];
        if (exitr >= 0) {
            c.phase = PH_DONE;
            c.exit_reason = exitr;
        } else {
            c.phase = PH_EIG0;
            c.it = 0;
            c.hasP = 0;
        }
    }
    __syncthreads();
    if (exitr >= 0) return;
    if (w.lambda_reuse && c.stall > 0) {
        // the last subproblem left x as it was: I and z are unchanged and the
        // penalty update shifted the scaled matrix of eq. (alpha) by -alpha, so
        // its smallest eigenvalue moved by exactly -alpha; no LOBPCG is needed
        eig_finish<OpT, EPT>(w, c, cv, red, c.lam - c.alpha);
        return;
    }
    // first LOBPCG vector: constant on I, normalized in the Z inner product
    // z = x - x^2 for lambda_min (positive exactly on I: for 0 < x < 1 it
    // rounds to a positive double)
    const double v0 = 1.0 / sqrt(sm[0]);
    const UVec<double> v = uvec(w.v, cv.off), zx = uvec(w.zx, cv.off);
    CHUNKS(n) {
        CHUNK_INDEX(n)
        double xv[EPT];
        FOR_J xv[_j] = x[ix[_j]];
        FOR_J {
            if (!ok[_j]) continue;
            const double xi = xv[_j];
            const double vi = interior(xi) ? v0 : 0.0;
            v[ix[_j]] = vi;
            zx[ix[_j]] = xi - xi * xi;
            put_aux<OpT>(w, cv, ix[_j], vi);
        }
    }
    aux_digits<OpT, EPT>(w, c, cv, v0);
}

// ---------------------------------------------------------------------------
// Penalty update: alpha = eta * max(lambda, floor * rho), p_I += alpha z_I
// (eqs. (pp1), (alpha1)); then the next subproblem starts from the same x.

template <typename OpT, int EPT>
__device__ void eig_finish(const Work &w, Col &c, const ColView &cv, double *red, double lam) {
    const uint32_t n = cv.n;
    const UVec<const double> x = uvec((const double *)w.x, cv.off);
    const UVec<double> p = uvec(w.p, cv.off);
    const UVec<const double> dgi = uvec((const double *)w.dgi, cv.io), lni = uvec((const double *)w.lni, cv.io);
    const UVec<const double> R = uvec((const double *)w.R, cv.io);
    double alpha = w.eta * fmax(lam, w.lambda_floor_rel * c.rho_outer);
    if (w.alpha_in && c.s < w.alpha_cap) alpha = w.alpha_in[(int64_t)uni(c.start) * w.alpha_cap + uni(c.s)];
    double mx[2] = {0.0, 0.0};
    CHUNKS(n) {
        CHUNK_INDEX(n)
        double xv[EPT], pv[EPT], dg[EPT], Rv[EPT], bg[EPT];
        FOR_J {
            const uint32_t i = ix[_j];
            xv[_j] = x[i];
            pv[_j] = p[i];
            dg[_j] = dgi[i];
            Rv[_j] = R[i];
            bg[_j] = lni[i];
        }
        FOR_J {
            if (!ok[_j]) continue;
            const uint32_t i = ix[_j];
            const double xi = xv[_j];
            double pi = pv[_j];
            if (interior(xi)) {
                pi = pi + alpha * (xi - xi * xi);
                p[i] = pi;
            }
            const double A = dg[_j] - pi, lb = bg[_j] + pi;
            mx[0] = fmax(mx[0], 2.0 * (Rv[_j] + fabs(A)));
            mx[1] = fmax(mx[1], fabs(lb));
            put_main<OpT>(w, c, cv, i, xi);
        }
    }
    bmax<2>(mx, red);
    if (threadIdx.x == 0) {
        c.rho = fmax(1.0, fmax(mx[0], mx[1]));
        c.lam = lam;
        c.phase = PH_INNER;
        c.k = 0;
        c.inner_start = c.evals;
        c.alpha = alpha;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// End of a subproblem (Algorithm 3, after the subproblem solve); the loop
// head (outer_begin) follows in the step kernel.

template <typename OpT, int EPT>
__device__ void end_subproblem(const Work &w, Col &c, bool moved, double rel) {
    if (threadIdx.x == 0) {
        c.stall = moved ? 0 : c.stall + 1;
        if (w.trace && c.ntrace < w.trace_cap) {
            double *t = w.trace + ((int64_t)c.start * w.trace_cap + c.ntrace) * 6;
            t[0] = (double)c.s;
            t[1] = (double)c.nI;
            t[2] = c.lam;
            t[3] = c.alpha;
            t[4] = (double)(c.evals - c.inner_start);
            t[5] = rel;
            c.ntrace += 1;
        }
        c.s += 1;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Subproblem iteration (Algorithms 1 and 2). Returns true when the
// subproblem ended (the loop head runs next).

template <typename OpT, typename UT, int EPT, bool CACHE>
__device__ bool inner_step(const Work &w, Col &c, const ColView &cv, double *red) {
    const uint32_t n = cv.n;
    const UVec<double> x = uvec(w.x, cv.off), xp = uvec(w.xp, cv.off), g = uvec(w.g, cv.off), gp = uvec(w.gp, cv.off);
    const UVec<const double> p = uvec((const double *)w.p, cv.off), gam = uvec((const double *)w.gam, cv.io);
    const UVec<const double> R = uvec((const double *)w.R, cv.io), dq = uvec((const double *)w.dq, cv.io);
    const UVec<const double> dgi = uvec((const double *)w.dgi, cv.io), lni = uvec((const double *)w.lni, cv.io);
    const int k = c.k;
    double mx[2] = {0.0, 0.0};       // cret, any nonzero step component
    // s's, s'y, y'y of eq. (bb1) as double-double sums (high parts sm, low
    // parts sl): the BB steps take their exact values rounded once
    double sm[3] = {0.0, 0.0, 0.0};
    double sl[3] = {0.0, 0.0, 0.0};
    double xr[EPT], gr[EPT];         // register copies when one pass covers the column
    CHUNKS(n) {
        CHUNK_PAIRS(n)
        double xv[EPT], pv[EPT], Av[EPT], bv[EPT], xpv[EPT], gpv[EPT], u[EPT];
        ld_chunk<true>(x, ix, xv);
        ld_chunk<true>(p, ix, pv);
        ld_chunk<true>(dgi, ix, Av);
        ld_chunk<true>(lni, ix, bv);
        ld_chunk<true>(xp, ix, xpv);  // stale but unused when k == 0
        ld_chunk<true>(gp, ix, gpv);
        uval_chunk<UT, EPT, true>(w, cv, ix, ok, u);
        FOR_J {
            Av[_j] = Av[_j] - pv[_j];  // diagonal of Q_r - Diag p
            bv[_j] = bv[_j] + pv[_j];  // b_r + p
        }
        FOR_J {
            const double xi = xv[_j];
            const double gi = 2.0 * (u[_j] + Av[_j] * xi) + bv[_j];
            if (CACHE) {
                xr[_j] = xi;
                gr[_j] = gi;
            } else if (ok[_j]) {
                g[ix[_j]] = gi;
            }
            if (!ok[_j]) continue;
            double viol;
            if (interior(xi)) viol = fabs(gi);
            else if (xi == 0.0) viol = fmax(-gi, 0.0);
            else viol = fmax(gi, 0.0);
            mx[0] = fmax(mx[0], viol);
            if (k > 0) {
                const double s = xi - xpv[_j];
                const double y = gi - gpv[_j];
                dd_add_prod(sm[0], sl[0], s, s);
                dd_add_prod(sm[1], sl[1], s, y);
                dd_add_prod(sm[2], sl[2], y, y);
                if (s != 0.0) mx[1] = 1.0;
            }
        }
    }
    block_maxsum_dd<2, 3, kSB>(mx, sm, sl, red);  // sm is zero when k == 0
    const double rel = mx[0] / c.rho;
    if (threadIdx.x == 0) {
        c.evals += 1;
        c.final_rel = rel;
    }
    __syncthreads();
    if (rel < w.tol_kkt) {
        end_subproblem<OpT, EPT>(w, c, k > 0, rel);
        return true;
    }
    if (k > 0 && mx[1] == 0.0) {
        end_subproblem<OpT, EPT>(w, c, true, rel);
        return true;
    }
    double alpha = 0.0;
    if (w.inner == PSDP_INNER_PABB) {
        if (k == 0) {
            alpha = 1.0 / c.rho;
        } else {
            double a;
            if (sm[1] <= 0.0) a = w.alpha_max;
            else if (k % 2 == 1) a = sm[0] / sm[1];
            else a = sm[1] / sm[2];
            alpha = fmin(fmax(a, w.alpha_min), w.alpha_max);
        }
    }
    const bool pabb = w.inner == PSDP_INNER_PABB;
    CHUNKS(n) {
        CHUNK_PAIRS(n)
        double xv[EPT], gv[EPT], hp[EPT], xn[EPT];
        if (CACHE) {
            FOR_J {
                xv[_j] = xr[_j];
                gv[_j] = gr[_j];
            }
        } else {
            ld_chunk<true>(x, ix, xv);
            ld_chunk<true>(g, ix, gv);
        }
        if (!pabb) {
            FOR_J {
                const uint32_t i = ix[_j];
                hp[_j] = fmax((R[i] + fabs(dq[i] + gam[i])) - p[i], w.eps_hp);
            }
        }
        FOR_J {
            const double xi = xv[_j], gi = gv[_j];
            if (pabb) xn[_j] = fmin(fmax(xi - alpha * gi, 0.0), 1.0);
            else xn[_j] = fmin(fmax(xi + (-gi / (2.0 * hp[_j])), 0.0), 1.0);
        }
        st_chunk<true>(xp, ix, ok, xv);
        st_chunk<true>(gp, ix, ok, gv);
        st_chunk<true>(x, ix, ok, xn);
        put_main_chunk<OpT, EPT, true>(w, c, cv, ix, ok, xn);
    }
    if (k + 1 >= w.max_inner) {
        __syncthreads();
        end_subproblem<OpT, EPT>(w, c, true, rel);
        return true;
    }
    if (threadIdx.x == 0) c.k = k + 1;
    __syncthreads();
    return false;
}

// ---------------------------------------------------------------------------
// Rayleigh-Ritz for LOBPCG on span{v, w, P}, fully unrolled 3 x 3 code
// (static indexing keeps every array in registers). Without P, the third
// direction is decoupled: unit Gram diagonal, no coupling, and a Ritz value
// far above the others, so it never becomes the minimum and its
// coefficient is exactly zero.

// 1/x and 1/sqrt(x) from the hardware estimates (v_rcp_f64, v_rsq_f64,
// relative error near 2^-24) and one Newton step each, r (2 - x r) and
// r (3 - x r^2) / 2, written as fused corrections: relative error near
// 2^-48 (measured on gfx950 over 2^20 inputs of exponents -200..200: at most
// 11 and 20 ulps), far below what the 3 x 3 Rayleigh-Ritz solve of a LOBPCG
// step needs, and a shorter dependent chain than the correctly rounded
// division and square root (that solve, on one lane, went from 4.1 to
// 2.9 us per step).
__device__ __forceinline__ double rcp_nr(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double rsq_nr(double x) {
    const double r = __builtin_amdgcn_rsq(x);
    return fma(r, fma(-0.5 * x * r, r, 0.5), r);
}

// Cholesky G = L L^T of a 3 x 3 matrix with unit diagonal (L00 = 1); false
// when the basis is numerically dependent.
__device__ __forceinline__ bool chol3(const double (&G)[3][3], double (&L)[3][3]) {
    const double l10 = G[1][0], l20 = G[2][0];
    const double d1 = 1.0 - l10 * l10;
    const double e1 = fmax(d1, 1e-300), r1 = rsq_nr(e1);
    const double l11 = e1 * r1;
    const double l21 = (G[2][1] - l20 * l10) * r1;
    const double d2 = 1.0 - l20 * l20 - l21 * l21;
    const double e2 = fmax(d2, 1e-300);
    const double l22 = e2 * rsq_nr(e2);
    L[0][0] = 1.0; L[0][1] = 0.0; L[0][2] = 0.0;
    L[1][0] = l10; L[1][1] = l11; L[1][2] = 0.0;
    L[2][0] = l20; L[2][1] = l21; L[2][2] = l22;
    return d1 > 1e-12 && d2 > 1e-12;
}

// One Jacobi rotation annihilating C[p][q] (p < q) of a symmetric 3 x 3 C,
// accumulated into V: t = tan of the angle from the stable quadratic root,
// c = 1/sqrt(1 + t^2), s = t c.
template <int PP, int QQ>
__device__ __forceinline__ void jacobi_rot(double (&C)[3][3], double (&V)[3][3]) {
    const double apq = C[PP][QQ];
    if (apq == 0.0) return;
    const double diff = C[QQ][QQ] - C[PP][PP];
    const double y = diff * diff + 4.0 * apq * apq;
    const double t = (diff >= 0.0 ? 2.0 * apq : -2.0 * apq) * rcp_nr(fabs(diff) + y * rsq_nr(y));
    const double cs = rsq_nr(1.0 + t * t), sn = t * cs;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const double a = C[r][PP], b = C[r][QQ];
        C[r][PP] = cs * a - sn * b;
        C[r][QQ] = sn * a + cs * b;
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const double a = C[PP][r], b = C[QQ][r];
        C[PP][r] = cs * a - sn * b;
        C[QQ][r] = sn * a + cs * b;
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const double a = V[r][PP], b = V[r][QQ];
        V[r][PP] = cs * a - sn * b;
        V[r][QQ] = sn * a + cs * b;
    }
}

// sm = {v'Zv, v'Zw, w'Zw, v'ZP, w'ZP, P'ZP, v'Av, v'Aw, w'Aw, v'AP, w'AP, P'AP};
// out = {a_v, a_w, a_P, theta, ok}: the new v = a_v v + a_w w + a_P P.
__device__ __forceinline__ void rayleigh_ritz(const double *sm, bool hasP, double *out) {
    const double d0 = rsq_nr(sm[0]), d1 = rsq_nr(sm[2]);
    const double d2 = hasP ? rsq_nr(sm[5]) : 1.0;
    const double d[3] = {d0, d1, d2};
    double G[3][3], H[3][3];
    G[0][0] = sm[0] * d0 * d0; G[0][1] = sm[1] * d0 * d1; G[1][1] = sm[2] * d1 * d1;
    H[0][0] = sm[6] * d0 * d0; H[0][1] = sm[7] * d0 * d1; H[1][1] = sm[8] * d1 * d1;
    if (hasP) {
        G[0][2] = sm[3] * d0 * d2; G[1][2] = sm[4] * d1 * d2; G[2][2] = sm[5] * d2 * d2;
        H[0][2] = sm[9] * d0 * d2; H[1][2] = sm[10] * d1 * d2; H[2][2] = sm[11] * d2 * d2;
    } else {
        G[0][2] = 0.0; G[1][2] = 0.0; G[2][2] = 1.0;
        H[0][2] = 0.0; H[1][2] = 0.0; H[2][2] = 0.0;  // replaced below
    }
    G[1][0] = G[0][1]; G[2][0] = G[0][2]; G[2][1] = G[1][2];
    H[1][0] = H[0][1]; H[2][0] = H[0][2]; H[2][1] = H[1][2];
    double L[3][3];
    bool ok = chol3(G, L);
    bool useP = hasP;
    if (!ok && hasP) {  // drop P: decouple the third direction
        useP = false;
        G[0][2] = G[1][2] = G[2][0] = G[2][1] = 0.0;
        G[2][2] = 1.0;
        H[0][2] = H[1][2] = H[2][0] = H[2][1] = 0.0;
        ok = chol3(G, L);
    }
    if (!ok || !(sm[2] > 0.0) || !isfinite(d1)) {
        out[0] = out[1] = out[2] = out[3] = out[4] = 0.0;
        return;
    }
    // L^-1 (lower triangular, unit first diagonal entry)
    double Li[3][3];
    const double i11 = rcp_nr(L[1][1]), i22 = rcp_nr(L[2][2]);
    Li[0][0] = 1.0; Li[1][1] = i11; Li[2][2] = i22;
    Li[0][1] = Li[0][2] = Li[1][2] = 0.0;
    Li[1][0] = -L[1][0] * i11;
    Li[2][1] = -L[2][1] * i11 * i22;
    Li[2][0] = -(L[2][0] + L[2][1] * Li[1][0]) * i22;
    // C = L^-1 H L^-T
    double T[3][3], C[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) T[i][j] = Li[i][0] * H[0][j] + Li[i][1] * H[1][j] + Li[i][2] * H[2][j];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) C[i][j] = T[i][0] * Li[j][0] + T[i][1] * Li[j][1] + T[i][2] * Li[j][2];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i + 1; j < 3; ++j) {
            const double sym = 0.5 * (C[i][j] + C[j][i]);
            C[i][j] = sym;
            C[j][i] = sym;
        }
    if (!useP) {  // third Ritz value far above the others
        const double big = 1e3 * (fabs(C[0][0]) + fabs(C[1][1]) + fabs(C[0][1]) + 1.0);
        C[0][2] = C[1][2] = C[2][0] = C[2][1] = 0.0;
        C[2][2] = big;
    }
    double V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int sweep = 0; sweep < 12; ++sweep) {
        const double off = C[0][1] * C[0][1] + C[0][2] * C[0][2] + C[1][2] * C[1][2];
        const double dia = C[0][0] * C[0][0] + C[1][1] * C[1][1] + C[2][2] * C[2][2];
        if (off <= 1e-32 * (dia + 2.0 * off)) break;
        jacobi_rot<0, 1>(C, V);
        jacobi_rot<0, 2>(C, V);
        jacobi_rot<1, 2>(C, V);
    }
    // smallest eigenpair (lowest index on ties), chosen with selects on
    // scalars (an indexed choice would put V on the stack)
    const double c0 = C[0][0], c1 = C[1][1], c2 = C[2][2];
    const bool s1 = c1 < c0;
    double theta = s1 ? c1 : c0;
    double y0 = s1 ? V[0][1] : V[0][0], y1 = s1 ? V[1][1] : V[1][0], y2 = s1 ? V[2][1] : V[2][0];
    const bool s2 = c2 < theta;
    theta = s2 ? c2 : theta;
    y0 = s2 ? V[0][2] : y0;
    y1 = s2 ? V[1][2] : y1;
    y2 = s2 ? V[2][2] : y2;
    // a = D L^-T y
    out[0] = (Li[0][0] * y0 + Li[1][0] * y1 + Li[2][0] * y2) * d[0];
    out[1] = (Li[1][1] * y1 + Li[2][1] * y2) * d[1];
    out[2] = useP ? (Li[2][2] * y2) * d[2] : 0.0;
    out[3] = theta;
    out[4] = 1.0;
}

// ---------------------------------------------------------------------------
// lambda_min: first LOBPCG vector applied.

template <typename OpT, typename UT, int EPT>
__device__ void eig0_step(const Work &w, Col &c, const ColView &cv, double *red) {
    const uint32_t n = cv.n;
    const UVec<const double> zx = uvec((const double *)w.zx, cv.off);
    const DiagView dg{uvec((const double *)w.dgi, cv.io), uvec((const double *)w.p, cv.off)};
    const UVec<double> v = uvec(w.v, cv.off), Av = uvec(w.Av, cv.off), wv = uvec(w.w, cv.off);
    double sm[2] = {0.0, 0.0};  // v'Av, v'Zv
    CHUNKS(n) {
        CHUNK_INDEX(n)
        double zv[EPT], Ad[EPT], vv[EPT], u[EPT];
        FOR_J {
            const uint32_t i = ix[_j];
            zv[_j] = zx[i];
            Ad[_j] = dg[i];
            vv[_j] = v[i];
        }
        uaux_chunk<UT, EPT>(w, c, cv, ix, ok, u);
        FOR_J {
            if (!ok[_j]) continue;
            const double z = zv[_j], vi = vv[_j];
            double av = 0.0;
            if (z > 0.0) {  // i in I
                av = u[_j] + Ad[_j] * vi;
                sm[0] += vi * av;
                sm[1] += z * vi * vi;
            }
            Av[ix[_j]] = av;
        }
    }
    bsum<2>(sm, red);
    const double lam = sm[0] / sm[1];
    double rn[1] = {0.0}, mw[1] = {0.0};
    CHUNKS(n) {
        CHUNK_INDEX(n)
        double zv[EPT], Ad[EPT], vv[EPT], av[EPT];
        FOR_J {
            const uint32_t i = ix[_j];
            zv[_j] = zx[i];
            Ad[_j] = dg[i];
            vv[_j] = v[i];
            av[_j] = Av[i];
        }
        FOR_J {
            if (!ok[_j]) continue;
            const uint32_t i = ix[_j];
            const double z = zv[_j];
            double wi = 0.0;
            if (z > 0.0) {
                const double A = Ad[_j];
                const double r = av[_j] - lam * z * vv[_j];
                rn[0] += r * r / z;
                wi = r / (A != 0.0 ? fabs(A) : 1.0);
            }
            wv[i] = wi;
            mw[0] = fmax(mw[0], fabs(wi));
            put_aux<OpT>(w, cv, i, wi);
        }
    }
    block_maxsum<1, 1, kSB>(mw, rn, red);
    if (threadIdx.x == 0) {
        c.aux += 1;
        c.it = 1;
        c.lam = lam;
        c.hasP = 0;
    }
    __syncthreads();
    // a Ritz value is an upper bound of lambda_min: below the floor of
    // eq. (alpha1)'s maximum it already fixes alpha (the floor), whatever
    // lambda_min is
    const double floor_lam = w.lambda_floor_rel * c.rho_outer;
    if (sqrt(rn[0] / sm[1]) <= w.eig_tol * fabs(lam) || lam < floor_lam || w.eig_maxit <= 1) {
        eig_finish<OpT, EPT>(w, c, cv, red, lam);
        return;
    }
    aux_digits<OpT, EPT>(w, c, cv, mw[0]);
    if (threadIdx.x == 0) c.phase = PH_EIG;
    __syncthreads();
}

// ---------------------------------------------------------------------------
// lambda_min: one LOBPCG iteration (Rayleigh-Ritz on span{v, w, P}).
// CM says where the second pass finds the first pass's values: 0 reloads
// them, 1 keeps all eight in registers (short columns), 2 keeps z and the
// diagonal in registers and the other six in LDS (one chunk of up to 3072
// elements: 144 KB of the 160 KB a workgroup may use).

template <int EPT, int CM> struct EigCache {
    static constexpr int kSlots = CM == 2 ? EPT * kSB : 1;
};

template <typename OpT, typename UT, int EPT, int CM>
__device__ void eig_step(const Work &w, Col &c, const ColView &cv, double *red) {
    constexpr bool CACHE = CM != 0;
    constexpr int NS = EigCache<EPT, CM>::kSlots;
    __shared__ double lc[CM == 2 ? 6 : 1][NS];  // v, w, Aw, Av, P, AP
    const uint32_t n = cv.n;
    const UVec<const double> zx = uvec((const double *)w.zx, cv.off);
    const DiagView dg{uvec((const double *)w.dgi, cv.io), uvec((const double *)w.p, cv.off)};
    const UVec<double> v = uvec(w.v, cv.off), Av = uvec(w.Av, cv.off), P = uvec(w.P, cv.off), AP = uvec(w.AP, cv.off);
    const UVec<double> wv = uvec(w.w, cv.off), Aw = uvec(w.g, cv.off);  // g is free during lambda_min
    const bool hasP = c.hasP != 0;
    // Gram matrices: B = Z-inner products, A = Qbar-inner products
    double sm[12];
#pragma unroll
    for (int j = 0; j < 12; ++j) sm[j] = 0.0;
    // register copies when one pass covers the column (z = 0 marks i outside I)
    double zr[EPT], Ar[EPT], vr[EPT], wr[EPT], awr[EPT], avr[EPT], pr[EPT], apr[EPT];
    CHUNKS(n) {
        CHUNK_INDEX(n)
        double zv[EPT], Ad[EPT], vv[EPT], wvv[EPT], avv[EPT], pv[EPT], apv[EPT], u[EPT];
        FOR_J {
            const uint32_t i = ix[_j];
            zv[_j] = zx[i];
            Ad[_j] = dg[i];
            vv[_j] = v[i];
            wvv[_j] = wv[i];
            avv[_j] = Av[i];
            pv[_j] = hasP ? P[i] : 0.0;
            apv[_j] = hasP ? AP[i] : 0.0;
        }
        uaux_chunk<UT, EPT>(w, c, cv, ix, ok, u);
        FOR_J {
            const double z = zv[_j];
            const bool in_I = ok[_j] && z > 0.0;
            double aw = 0.0;
            if (CACHE) zr[_j] = 0.0;
            if (in_I) {
                const double A = Ad[_j];
                const double wi = wvv[_j], vi = vv[_j];
                aw = u[_j] + A * wi;
                if (CM == 1) {
                    zr[_j] = z;
                    Ar[_j] = A;
                    vr[_j] = vi;
                    wr[_j] = wi;
                    awr[_j] = aw;
                    avr[_j] = avv[_j];
                    pr[_j] = pv[_j];
                    apr[_j] = apv[_j];
                } else if (CM == 2) {
                    const int s = _j * kSB + threadIdx.x;
                    zr[_j] = z;
                    Ar[_j] = A;
                    lc[0][s] = vi;
                    lc[1][s] = wi;
                    lc[2][s] = aw;
                    lc[3][s] = avv[_j];
                    lc[4][s] = pv[_j];
                    lc[5][s] = apv[_j];
                }
                sm[0] += z * vi * vi;
                sm[1] += z * vi * wi;
                sm[2] += z * wi * wi;
                sm[6] += vi * avv[_j];
                sm[7] += vi * aw;
                sm[8] += wi * aw;
                if (hasP) {
                    const double pi = pv[_j];
                    sm[3] += z * vi * pi;
                    sm[4] += z * wi * pi;
                    sm[5] += z * pi * pi;
                    sm[9] += vi * apv[_j];
                    sm[10] += wi * apv[_j];
                    sm[11] += pi * apv[_j];
                }
            }
            if (!CACHE && ok[_j]) Aw[ix[_j]] = aw;
        }
    }
    bsum<12>(sm, red);
    // Rayleigh-Ritz on thread 0; the coefficients go through shared memory
    const bool one = n <= (uint32_t)(EPT * kSB);
    __shared__ double rr[5];  // a0, a1, a2, theta, ok
    if (threadIdx.x == 0) rayleigh_ritz(sm, hasP, rr);
    __syncthreads();
    const bool ok = rr[4] != 0.0;
    const double a[3] = {rr[0], rr[1], rr[2]};
    const double theta = rr[3];
    if (!ok) {
        // the residual direction is numerically inside span{v}: converged
        if (threadIdx.x == 0) c.aux += 1;
        __syncthreads();
        eig_finish<OpT, EPT>(w, c, cv, red, c.lam);
        return;
    }
    double rn[2] = {0.0, 0.0};  // ||r||^2_{Z^-1}, v'Zv
    double mw[1] = {0.0};       // max |w| (scale of the integer operand)
    double wnr[EPT];            // the new operand (one chunk: kept for its digits)
    CHUNKS(n) {
        CHUNK_INDEX(n)
        double zv[EPT], Ad[EPT], vv[EPT], wvv[EPT], awv[EPT], avv[EPT], pv[EPT], apv[EPT];
        if (!CACHE) {
            FOR_J {
                const uint32_t i = ix[_j];
                zv[_j] = zx[i];
                Ad[_j] = dg[i];
                vv[_j] = v[i];
                wvv[_j] = wv[i];
                awv[_j] = Aw[i];
                avv[_j] = Av[i];
                pv[_j] = hasP ? P[i] : 0.0;
                apv[_j] = hasP ? AP[i] : 0.0;
            }
        }
      FOR_J {
        if (!ok[_j]) continue;
        const uint32_t i = ix[_j];
        double z, A, vi, wi, awi, avi, pi, api;
        bool in_I;
        if (CM == 1) {
            z = zr[_j];
            in_I = z > 0.0;
            A = Ar[_j]; vi = vr[_j]; wi = wr[_j]; awi = awr[_j]; avi = avr[_j]; pi = pr[_j]; api = apr[_j];
        } else if (CM == 2) {
            const int s = _j * kSB + threadIdx.x;
            z = zr[_j];
            in_I = z > 0.0;
            A = Ar[_j];
            vi = lc[0][s]; wi = lc[1][s]; awi = lc[2][s]; avi = lc[3][s]; pi = lc[4][s]; api = lc[5][s];
        } else {
            z = zv[_j];
            in_I = z > 0.0;
            A = Ad[_j];
            vi = vv[_j]; wi = wvv[_j]; awi = awv[_j]; avi = avv[_j];
            pi = pv[_j];
            api = apv[_j];
        }
        double wn = 0.0;
        if (in_I) {
            const double vn = a[0] * vi + a[1] * wi + a[2] * pi;
            const double avn = a[0] * avi + a[1] * awi + a[2] * api;
            const double pn = a[1] * wi + a[2] * pi;
            const double apn = a[1] * awi + a[2] * api;
            v[i] = vn;
            Av[i] = avn;
            P[i] = pn;
            AP[i] = apn;
            const double r = avn - theta * z * vn;
            rn[0] += r * r / z;
            rn[1] += z * vn * vn;
            wn = r / (A != 0.0 ? fabs(A) : 1.0);
        }
        wv[i] = wn;
        wnr[_j] = wn;
        mw[0] = fmax(mw[0], fabs(wn));
        put_aux<OpT>(w, cv, i, wn);
      }
    }
    block_maxsum<1, 2, kSB>(mw, rn, red);
    const int it = c.it + 1;
    if (threadIdx.x == 0) {
        c.aux += 1;
        c.it = it;
        c.lam = theta;
        c.hasP = 1;
    }
    __syncthreads();
    // below the floor of alpha's maximum the Ritz value (an upper bound of
    // lambda_min) already fixes alpha: stop (see eig0_step)
    if (sqrt(rn[0] / rn[1]) <= w.eig_tol * fabs(theta) || theta < w.lambda_floor_rel * c.rho_outer ||
        it >= w.eig_maxit) {
        eig_finish<OpT, EPT>(w, c, cv, red, theta);
    } else {
        aux_digits<OpT, EPT>(w, c, cv, mw[0], wnr, one);
    }
}

// ---------------------------------------------------------------------------
// x^0 by Jacobi-preconditioned CG on K = 2 (Q + Diag gamma). Returns true
// when x^0 is done (the loop head runs next).

template <typename OpT, typename UT, int EPT>
__device__ bool cg_step(const Work &w, Col &c, const ColView &cv, double *red) {
    const uint32_t n = cv.n;
    const UVec<double> x = uvec(w.x, cv.off);
    const UVec<double> r = uvec(w.v, cv.off), d = uvec(w.w, cv.off), Kd = uvec(w.Av, cv.off);
    const UVec<const double> gam = uvec((const double *)w.gam, cv.io), dq = uvec((const double *)w.dq, cv.io);
    double s1[1] = {0.0};
    CHUNKS(n) {
        CHUNK_INDEX(n)
        double dg[EPT], dv[EPT], u[EPT];
        FOR_J {
            const uint32_t i = ix[_j];
            dg[_j] = dq[i] + gam[i];
            dv[_j] = d[i];
        }
        uaux_chunk<UT, EPT>(w, c, cv, ix, ok, u);
        FOR_J {
            if (!ok[_j]) continue;
            const double kd = 2.0 * (u[_j] + dg[_j] * dv[_j]);
            Kd[ix[_j]] = kd;
            s1[0] += dv[_j] * kd;
        }
    }
    bsum<1>(s1, red);
    const double a = c.rz / s1[0];
    double s2[2] = {0.0, 0.0};  // r'M^-1 r, r'r
    CHUNKS(n) {
        CHUNK_INDEX(n)
        double xv[EPT], dv[EPT], rv[EPT], kv[EPT], dg[EPT];
        FOR_J {
            const uint32_t i = ix[_j];
            xv[_j] = x[i];
            dv[_j] = d[i];
            rv[_j] = r[i];
            kv[_j] = Kd[i];
            dg[_j] = dq[i] + gam[i];
        }
        FOR_J {
            if (!ok[_j]) continue;
            const uint32_t i = ix[_j];
            x[i] = xv[_j] + a * dv[_j];
            const double ri = rv[_j] - a * kv[_j];
            r[i] = ri;
            const double zz = ri / (2.0 * dg[_j]);
            s2[0] += ri * zz;
            s2[1] += ri * ri;
        }
    }
    bsum<2>(s2, red);
    const int it = c.it + 1;
    if (threadIdx.x == 0) {
        c.aux += 1;
        c.it = it;
    }
    __syncthreads();
    if (sqrt(s2[1]) <= w.cg_tol * c.r0 || it >= w.cg_maxit) return true;
    const double beta = s2[0] / c.rz;
    double md[1] = {0.0};
    CHUNKS(n) {
        CHUNK_INDEX(n)
        double rv[EPT], dv[EPT], dg[EPT];
        FOR_J {
            const uint32_t i = ix[_j];
            rv[_j] = r[i];
            dv[_j] = d[i];
            dg[_j] = dq[i] + gam[i];
        }
        FOR_J {
            if (!ok[_j]) continue;
            const uint32_t i = ix[_j];
            const double zz = rv[_j] / (2.0 * dg[_j]);
            const double dn = zz + beta * dv[_j];
            d[i] = dn;
            md[0] = fmax(md[0], fabs(dn));
            put_aux<OpT>(w, cv, i, dn);
        }
    }
    if constexpr (kDigits<OpT>) {
        bmax<1>(md, red);
        aux_digits<OpT, EPT>(w, c, cv, md[0]);
    }
    if (threadIdx.x == 0) c.rz = s2[0];
    __syncthreads();
    return false;
}

// ---------------------------------------------------------------------------
// Live-column lists for the first sweep, in column order (the column kernel
// builds the later ones). Split precision: `active` gets the subproblem
// columns and `active_aux` the lambda_min / CG columns; otherwise `active`
// gets every live column. Run by one block.

template <int NT>
__device__ void compact_lists(const Work &w) {
    __shared__ int32_t cnt[2][NT];
    const int ncol = w.col_count;
    const int chunk = (ncol + NT - 1) / NT;
    const int lo = w.col_base + threadIdx.x * chunk;
    const int hi = min(w.col_base + ncol, lo + chunk);
    int my0 = 0, my1 = 0;
    for (int ci = lo; ci < hi; ++ci) {
        const int ph = __atomic_load_n(&w.col[ci].phase, __ATOMIC_RELAXED);
        if (ph == PH_DONE) continue;
        if (w.split && ph != PH_INNER) ++my1;
        else ++my0;
    }
    cnt[0][threadIdx.x] = my0;
    cnt[1][threadIdx.x] = my1;
    __syncthreads();
    if (threadIdx.x < 64) {  // exclusive prefix sums by wave 0, NT / 64 entries per lane
        constexpr int E = NT / 64;
        const int lane = threadIdx.x;
        int s0 = 0, s1 = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            s0 += cnt[0][lane * E + e];
            s1 += cnt[1][lane * E + e];
        }
        int i0 = s0, i1 = s1;  // inclusive scan over lanes
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int u0 = __shfl_up(i0, o, 64), u1 = __shfl_up(i1, o, 64);
            if (lane >= o) {
                i0 += u0;
                i1 += u1;
            }
        }
        int a0 = i0 - s0, a1 = i1 - s1;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int v0 = cnt[0][lane * E + e], v1 = cnt[1][lane * E + e];
            cnt[0][lane * E + e] = a0;
            cnt[1][lane * E + e] = a1;
            a0 += v0;
            a1 += v1;
        }
        if (lane == 63) {
            *w.nactive = i0;
            *w.nactive_aux = w.split ? i1 : 0;
            if (w.sweeps) *w.sweeps += 1;
        }
    }
    __syncthreads();
    int p0 = cnt[0][threadIdx.x], p1 = cnt[1][threadIdx.x];
    for (int ci = lo; ci < hi; ++ci) {
        const int ph = __atomic_load_n(&w.col[ci].phase, __ATOMIC_RELAXED);
        if (ph == PH_DONE) continue;
        if (w.split && ph != PH_INNER) w.active_aux[p1++] = ci;
        else w.active[p0++] = ci;
    }
}

// ---------------------------------------------------------------------------
// Queued starts: a column whose start has just ended saves it (final iterate
// and record) and takes the next start from the queue, set up as the first
// starts are (x from X0, the penalty terms of p0); the caller then runs the
// loop head for it. So every start performs the same arithmetic whichever
// column holds it and when. Returns false when the queue is empty.

template <int EPT>
__device__ bool next_start(const Work &w, Col &c, const ColView &cv) {
    __shared__ int32_t nxt;
    const uint32_t n = cv.n;
    const UVec<double> x = uvec(w.x, cv.off), p = uvec(w.p, cv.off);
    double *xf = w.xfin + (int64_t)uni(c.start) * n;
    FOR_I(n) xf[i] = x[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        w.fin[c.start] = c;
        nxt = atomicAdd(w.queue, 1);
    }
    __syncthreads();
    const int32_t s2 = nxt;
    if (s2 >= w.nstart) return false;
    const double *x0 = w.X0 + (int64_t)s2 * n;
    FOR_I(n) {
        x[i] = x0[i];
        p[i] = w.p0 ? w.p0[i] : 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        c.start = s2;
        c.k = c.s = c.stall = c.it = c.hasP = c.exit_reason = c.ntrace = c.nI = 0;
        c.rho = c.rho_outer = c.lam = c.rz = c.r0 = c.final_rel = c.final_bg = c.alpha = 0.0;
        c.evals = c.aux = c.inner_start = 0;
    }
    __syncthreads();
    return true;
}

// ---------------------------------------------------------------------------
// Kernels.

template <typename OpT, typename UT, int EPT, bool CI, int CE>
__global__ void __launch_bounds__(kSB) solver_step_kernel(Work w) {
    const int ci = w.col_base + (int)blockIdx.x;
    __shared__ Col c;
    __shared__ double red[12 * kSWaves];
    if (threadIdx.x == 0) c = w.col[ci];
    __syncthreads();
    const int ph0 = uni(c.phase);
    // Integer path: the column claims its slot in the next sweep's list for
    // its current product now, so that the atomic's round trip overlaps the
    // step; if the step ends the column or moves it to the other product,
    // the slot is filled with the all-zero column (its product is skipped
    // on store) and, when still live, a slot of the other list is claimed.
    const int aux0 = (w.split && ph0 != PH_INNER) ? 1 : 0;
    int slot0 = 0;
    if (kDigits<OpT> && ph0 != PH_DONE && threadIdx.x == 0) slot0 = atomicAdd(&w.next_cnt[aux0], 1);
    if (ph0 != PH_DONE) {
        const ColView cv = view(c);
        const unsigned long long t0 = w.phase_prof ? wall_clock64() : 0ull;
        bool head = false;
        switch (ph0) {
            case PH_INNER: head = inner_step<OpT, UT, EPT, CI>(w, c, cv, red); break;
            case PH_EIG0: eig0_step<OpT, UT, EPT>(w, c, cv, red); break;
            case PH_EIG: eig_step<OpT, UT, EPT, CE>(w, c, cv, red); break;
            case PH_CG: head = cg_step<OpT, UT, EPT>(w, c, cv, red); break;
            default: break;
        }
        // Algorithm 3's loop head after a subproblem or the x^0 solve; with
        // queued starts a column whose start has ended takes the next one and
        // runs the head for it (one call site of the head keeps the kernel's
        // register use down)
        while (head) {
            outer_begin<OpT, EPT>(w, c, cv, red);
            __syncthreads();
            head = w.queue != nullptr && c.phase == PH_DONE && next_start<EPT>(w, c, cv);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            w.col[ci] = c;
            // a live column takes a slot in the next sweep's list; the
            // products read the lists after this kernel has ended, so the
            // slots need no ordering with anything else written here
            const bool live = c.phase != PH_DONE;
            const int aux = (w.split && c.phase != PH_INNER) ? 1 : 0;
            if (kDigits<OpT>) {
                (aux0 ? w.next_active_aux : w.next_active)[slot0] = (live && aux == aux0) ? ci : w.ncol;
                if (live && aux != aux0) {
                    const int slot = atomicAdd(&w.next_cnt[aux], 1);
                    (aux ? w.next_active_aux : w.next_active)[slot] = ci;
                }
            } else if (live) {
                const int slot = atomicAdd(&w.next_cnt[aux], 1);
                (aux ? w.next_active_aux : w.next_active)[slot] = ci;
            }
            if (w.phase_prof) {
                const unsigned long long dt = wall_clock64() - t0;
                atomicAdd(&w.phase_prof[3 * ph0], dt);
                atomicAdd(&w.phase_prof[3 * ph0 + 1], 1ull);
                atomicMax(&w.phase_prof[3 * ph0 + 2], dt);
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        w.clear_cnt[0] = 0;
        w.clear_cnt[1] = 0;
        if (w.sweeps) *w.sweeps += 1;
    }
}

// Column set-up: x from X0 (column ci of an n x B matrix with leading
// dimension n) and the first outer step, or the CG start x = 0, r = gamma - b.
template <typename OpT, int EPT>
__global__ void __launch_bounds__(kSB) solver_init_kernel(Work w, const double *X0, int use_cg) {
    const int ci = w.col_base + (int)blockIdx.x;
    __shared__ Col c;
    __shared__ double red[12 * kSWaves];
    if (threadIdx.x == 0) c = w.col[ci];
    __syncthreads();
    const ColView cv = view(c);
    const uint32_t n = cv.n;
    const UVec<double> x = uvec(w.x, cv.off);
    const UVec<const double> b = uvec((const double *)w.b, cv.io), gam = uvec((const double *)w.gam, cv.io);
    const UVec<const double> dq = uvec((const double *)w.dq, cv.io);
    if (!use_cg) {
        FOR_I(n) x[i] = X0[(int64_t)c.start * n + i];
        __syncthreads();
        outer_begin<OpT, EPT>(w, c, cv, red);
    } else {
        const UVec<double> r = uvec(w.v, cv.off), d = uvec(w.w, cv.off);
        double s[2] = {0.0, 0.0}, mz[1] = {0.0};
        FOR_I(n) {
            x[i] = 0.0;
            const double ri = gam[i] - b[i];
            const double zz = ri / (2.0 * (dq[i] + gam[i]));
            r[i] = ri;
            d[i] = zz;
            mz[0] = fmax(mz[0], fabs(zz));
            put_aux<OpT>(w, cv, i, zz);
            s[0] += ri * zz;
            s[1] += ri * ri;
        }
        block_maxsum<1, 2, kSB>(mz, s, red);
        aux_digits<OpT, EPT>(w, c, cv, mz[0]);
        if (threadIdx.x == 0) {
            c.rz = s[0];
            c.r0 = sqrt(s[1]);
            c.phase = PH_CG;
            c.it = 0;
        }
        __syncthreads();
    }
    __syncthreads();
    if (threadIdx.x == 0) w.col[ci] = c;
}

__global__ void __launch_bounds__(kSB) compact_kernel(Work w) { compact_lists<kSB>(w); }

template <typename OpT, typename UT, int EPT, bool CI, int CE>
static hipError_t step_launch(const Work &w, hipStream_t st) {
    hipLaunchKernelGGL((solver_step_kernel<OpT, UT, EPT, CI, CE>), dim3(w.col_count), dim3(kSB), 0, st, w);
    return hipGetLastError();
}

// EPT elements per thread and chunk. When one chunk covers the longest
// column the subproblem step keeps x and g in registers between its two
// passes, and the LOBPCG step keeps its eight vectors for the second pass:
// in registers for short columns, beyond two elements per thread six of them
// in LDS. Longer columns take several chunks of 4 (6 or more elements per
// chunk would spill the gathered loads).
template <typename OpT, typename UT>
static hipError_t step_ept(const Work &w, int64_t nmax, hipStream_t st) {
    if (nmax <= 1 * kSB) return step_launch<OpT, UT, 1, true, 1>(w, st);
    if (nmax <= 2 * kSB) return step_launch<OpT, UT, 2, true, 1>(w, st);
    if (nmax <= 4 * kSB) return step_launch<OpT, UT, 4, true, 2>(w, st);
    if (nmax <= 6 * kSB) return step_launch<OpT, UT, 6, true, 2>(w, st);
    return step_launch<OpT, UT, 4, false, 0>(w, st);
}

hipError_t launch_solver_step(int optype, int utype, const Work &w, int64_t nmax, hipStream_t st) {
    if (optype == PSDP_I8 && utype == PSDP_I8) return step_ept<int8_t, int64_t>(w, nmax, st);
    if (optype == PSDP_F64 && utype == PSDP_F64) return step_ept<double, double>(w, nmax, st);
    if (optype == PSDP_F32 && utype == PSDP_F32) return step_ept<float, float>(w, nmax, st);
    if (optype == PSDP_BF16 && utype == PSDP_F32) return step_ept<__hip_bfloat16, float>(w, nmax, st);
    return hipErrorInvalidValue;
}

template <typename OpT>
static hipError_t init_launch(const Work &w, const double *X0, int use_cg, hipStream_t st) {
    hipLaunchKernelGGL((solver_init_kernel<OpT, 4>), dim3(w.col_count), dim3(kSB), 0, st, w, X0, use_cg);
    return hipGetLastError();
}

hipError_t launch_solver_init(int optype, const Work &w, const double *X0, int use_cg,
                              hipStream_t st) {
    if (optype == PSDP_I8) return init_launch<int8_t>(w, X0, use_cg, st);
    if (optype == PSDP_F64) return init_launch<double>(w, X0, use_cg, st);
    if (optype == PSDP_F32) return init_launch<float>(w, X0, use_cg, st);
    return init_launch<__hip_bfloat16>(w, X0, use_cg, st);
}

hipError_t launch_compact(const Work &w, hipStream_t st) {
    hipLaunchKernelGGL(compact_kernel, dim3(1), dim3(kSB), 0, st, w);
    return hipGetLastError();
}

}  // namespace psdp
