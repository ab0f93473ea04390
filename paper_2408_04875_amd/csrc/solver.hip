// Per-column solver state machine of the vectorized PSDP method.
//
// One workgroup owns one column (one start of one instance). Every sweep the
// Q.X kernels apply the off-diagonal part of the (perturbed) Q to one vector
// per live column; this kernel consumes that product according to the
// column's phase and prepares the next operand:
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
#include "common.hpp"

namespace psdp {

template <typename UT>
__device__ __forceinline__ double uval(const Work &w, int64_t idx) {
    const UT *U = (const UT *)w.U;
    double s = to_f64<UT>(U[idx]);
    for (int t = 1; t < w.ksplit; ++t) s += to_f64<UT>(U[(int64_t)t * w.slice + idx]);
    return s;
}

// Product for a lambda_min / CG column (FP64 buffers when precision is split).
template <typename UT>
__device__ __forceinline__ double uaux(const Work &w, int64_t idx) {
    if (!w.split) return uval<UT>(w, idx);
    double s = w.U_aux[idx];
    for (int t = 1; t < w.ksplit_aux; ++t) s += w.U_aux[(int64_t)t * w.slice_aux + idx];
    return s;
}

// Next operand of a lambda_min / CG column.
template <typename OpT>
__device__ __forceinline__ void put_aux(const Work &w, int64_t idx, double v) {
    if (w.split) w.op_aux[idx] = v;
    else ((OpT *)w.op)[idx] = from_f64<OpT>(v);
}

// Next operand of a subproblem column.
template <typename OpT>
__device__ __forceinline__ void put_main(const Work &w, int64_t idx, double v) {
    ((OpT *)w.op)[idx] = from_f64<OpT>(v);
}

__device__ __forceinline__ bool interior(double x) { return x > 0.0 && x < 1.0; }

// ---------------------------------------------------------------------------
// Outer loop head (Algorithm 3): exit tests, then start lambda_min.

template <typename OpT>
__device__ void outer_begin(const Work &w, Col &c, const Inst &in, double *red) {
    const int64_t n = c.n;
    const double *x = w.x + c.off;
    const double *p = w.p + c.off;
    const double *b = w.b + in.off, *gam = w.gam + in.off, *R = w.R + in.off, *dq = w.dq + in.off;
    double mx[4] = {0.0, 0.0, 0.0, 0.0};  // binary gap, pinned-at-half flag, row term, |b_r + p|
    double sm[2] = {0.0, 0.0};            // sum of z over I, |I|
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
        const double xi = x[i];
        mx[0] = fmax(mx[0], fmin(xi, 1.0 - xi));
        if (fabs(xi - 0.5) < 1e-9) mx[1] = 1.0;
        if (interior(xi)) {
            sm[0] += xi - xi * xi;
            sm[1] += 1.0;
        }
        const double A = (dq[i] + gam[i]) - p[i];
        mx[2] = fmax(mx[2], 2.0 * (R[i] + fabs(A)));
        mx[3] = fmax(mx[3], fabs((b[i] - gam[i]) + p[i]));
    }
    block_max<4>(mx, red);
    block_sum<2>(sm, red);
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
    // first LOBPCG vector: constant on I, normalized in the Z inner product
    const double v0 = 1.0 / sqrt(sm[0]);
    double *v = w.v + c.off;
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
        const double vi = interior(x[i]) ? v0 : 0.0;
        v[i] = vi;
        put_aux<OpT>(w, c.off + i, vi);
    }
}

// ---------------------------------------------------------------------------
// Penalty update: alpha = eta * max(lambda, floor * rho), p_I += alpha z_I
// (eqs. (pp1), (alpha1)); then the next subproblem starts from the same x.

template <typename OpT>
__device__ void eig_finish(const Work &w, Col &c, const Inst &in, double *red, double lam) {
    const int64_t n = c.n;
    const double *x = w.x + c.off;
    double *p = w.p + c.off;
    const double *b = w.b + in.off, *gam = w.gam + in.off, *R = w.R + in.off, *dq = w.dq + in.off;
    const double alpha = w.eta * fmax(lam, w.lambda_floor_rel * c.rho_outer);
    double mx[2] = {0.0, 0.0};
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
        const double xi = x[i];
        double pi = p[i];
        if (interior(xi)) {
            pi = pi + alpha * (xi - xi * xi);
            p[i] = pi;
        }
        const double A = (dq[i] + gam[i]) - pi;
        mx[0] = fmax(mx[0], 2.0 * (R[i] + fabs(A)));
        mx[1] = fmax(mx[1], fabs((b[i] - gam[i]) + pi));
        put_main<OpT>(w, c.off + i, xi);
    }
    block_max<2>(mx, red);
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
// End of a subproblem (Algorithm 3 after line 6).

template <typename OpT>
__device__ void end_subproblem(const Work &w, Col &c, const Inst &in, double *red, int ci,
                               bool moved, double rel) {
    if (threadIdx.x == 0) {
        c.stall = moved ? 0 : c.stall + 1;
        if (w.trace && c.ntrace < w.trace_cap) {
            double *t = w.trace + ((int64_t)ci * w.trace_cap + c.ntrace) * 6;
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
    outer_begin<OpT>(w, c, in, red);
}

// ---------------------------------------------------------------------------
// Subproblem iteration (Algorithms 1 and 2).

template <typename OpT, typename UT>
__device__ void inner_step(const Work &w, Col &c, const Inst &in, double *red, int ci) {
    const int64_t n = c.n;
    double *x = w.x + c.off, *xp = w.xp + c.off, *g = w.g + c.off, *gp = w.gp + c.off;
    const double *p = w.p + c.off;
    const double *b = w.b + in.off, *gam = w.gam + in.off, *R = w.R + in.off, *dq = w.dq + in.off;
    const int k = c.k;
    double mx[2] = {0.0, 0.0};       // cret, any nonzero step component
    double sm[3] = {0.0, 0.0, 0.0};  // s's, s'y, y'y
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
        const double xi = x[i];
        const double A = (dq[i] + gam[i]) - p[i];
        const double bbar = (b[i] - gam[i]) + p[i];
        const double gi = 2.0 * (uval<UT>(w, c.off + i) + A * xi) + bbar;
        g[i] = gi;
        double viol;
        if (interior(xi)) viol = fabs(gi);
        else if (xi == 0.0) viol = fmax(-gi, 0.0);
        else viol = fmax(gi, 0.0);
        mx[0] = fmax(mx[0], viol);
        if (k > 0) {
            const double s = xi - xp[i];
            const double y = gi - gp[i];
            sm[0] += s * s;
            sm[1] += s * y;
            sm[2] += y * y;
            if (s != 0.0) mx[1] = 1.0;
        }
    }
    block_max<2>(mx, red);
    if (k > 0) block_sum<3>(sm, red);
    const double rel = mx[0] / c.rho;
    if (threadIdx.x == 0) {
        c.evals += 1;
        c.final_rel = rel;
    }
    __syncthreads();
    if (rel < w.tol_kkt) {
        end_subproblem<OpT>(w, c, in, red, ci, k > 0, rel);
        return;
    }
    if (k > 0 && mx[1] == 0.0) {
        end_subproblem<OpT>(w, c, in, red, ci, true, rel);
        return;
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
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
        const double xi = x[i];
        const double gi = g[i];
        double xn;
        if (w.inner == PSDP_INNER_PABB) {
            xn = fmin(fmax(xi - alpha * gi, 0.0), 1.0);
        } else {
            const double hp = fmax((R[i] + fabs(dq[i] + gam[i])) - p[i], w.eps_hp);
            xn = fmin(fmax(xi + (-gi / (2.0 * hp)), 0.0), 1.0);
        }
        xp[i] = xi;
        gp[i] = gi;
        x[i] = xn;
        put_main<OpT>(w, c.off + i, xn);
    }
    if (k + 1 >= w.max_inner) {
        __syncthreads();
        end_subproblem<OpT>(w, c, in, red, ci, true, rel);
        return;
    }
    if (threadIdx.x == 0) c.k = k + 1;
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Small dense helpers for the LOBPCG Rayleigh-Ritz step (m <= 3).

__device__ bool chol3(int m, const double (&G)[3][3], double (&L)[3][3]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) L[i][j] = 0.0;
    for (int j = 0; j < m; ++j) {
        double d = G[j][j];
        for (int q = 0; q < j; ++q) d -= L[j][q] * L[j][q];
        if (!(d > 1e-12)) return false;  // near-dependent basis (G has unit diagonal)
        L[j][j] = sqrt(d);
        for (int i = j + 1; i < m; ++i) {
            double s = G[i][j];
            for (int q = 0; q < j; ++q) s -= L[i][q] * L[j][q];
            L[i][j] = s / L[j][j];
        }
    }
    return true;
}

// Cyclic Jacobi on a symmetric m x m matrix; returns the smallest eigenpair.
__device__ void jacobi_min(int m, double (&C)[3][3], double &theta, double (&y)[3]) {
    double V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int sweep = 0; sweep < 30; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                tot += C[i][j] * C[i][j];
                if (i != j) off += C[i][j] * C[i][j];
            }
        if (off <= 1e-32 * tot) break;
        for (int pq = 0; pq < m; ++pq)
            for (int qq = pq + 1; qq < m; ++qq) {
                const double apq = C[pq][qq];
                if (apq == 0.0) continue;
                const double tau = (C[qq][qq] - C[pq][pq]) / (2.0 * apq);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                const double cs = 1.0 / sqrt(1.0 + t * t), sn = t * cs;
                for (int r = 0; r < m; ++r) {
                    const double a = C[r][pq], bq = C[r][qq];
                    C[r][pq] = cs * a - sn * bq;
                    C[r][qq] = sn * a + cs * bq;
                }
                for (int r = 0; r < m; ++r) {
                    const double a = C[pq][r], bq = C[qq][r];
                    C[pq][r] = cs * a - sn * bq;
                    C[qq][r] = sn * a + cs * bq;
                }
                for (int r = 0; r < m; ++r) {
                    const double a = V[r][pq], bq = V[r][qq];
                    V[r][pq] = cs * a - sn * bq;
                    V[r][qq] = sn * a + cs * bq;
                }
            }
    }
    int best = 0;
    for (int i = 1; i < m; ++i)
        if (C[i][i] < C[best][best]) best = i;
    theta = C[best][best];
    for (int i = 0; i < 3; ++i) y[i] = i < m ? V[i][best] : 0.0;
}

// ---------------------------------------------------------------------------
// lambda_min: first LOBPCG vector applied.

template <typename OpT, typename UT>
__device__ void eig0_step(const Work &w, Col &c, const Inst &in, double *red) {
    const int64_t n = c.n;
    const double *x = w.x + c.off, *p = w.p + c.off;
    const double *gam = w.gam + in.off, *dq = w.dq + in.off;
    double *v = w.v + c.off, *Av = w.Av + c.off, *wv = w.w + c.off;
    double sm[2] = {0.0, 0.0};  // v'Av, v'Zv
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
        const double xi = x[i];
        double av = 0.0;
        if (interior(xi)) {
            const double A = (dq[i] + gam[i]) - p[i];
            av = uaux<UT>(w, c.off + i) + A * v[i];
            sm[0] += v[i] * av;
            sm[1] += (xi - xi * xi) * v[i] * v[i];
        }
        Av[i] = av;
    }
    block_sum<2>(sm, red);
    const double lam = sm[0] / sm[1];
    double rn[1] = {0.0};
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
        const double xi = x[i];
        double wi = 0.0;
        if (interior(xi)) {
            const double z = xi - xi * xi;
            const double A = (dq[i] + gam[i]) - p[i];
            const double r = Av[i] - lam * z * v[i];
            rn[0] += r * r / z;
            wi = r / (A != 0.0 ? fabs(A) : 1.0);
        }
        wv[i] = wi;
        put_aux<OpT>(w, c.off + i, wi);
    }
    block_sum<1>(rn, red);
    if (threadIdx.x == 0) {
        c.aux += 1;
        c.it = 1;
        c.lam = lam;
        c.hasP = 0;
    }
    __syncthreads();
    if (sqrt(rn[0] / sm[1]) <= w.eig_tol * fabs(lam) || w.eig_maxit <= 1) {
        eig_finish<OpT>(w, c, in, red, lam);
        return;
    }
    if (threadIdx.x == 0) c.phase = PH_EIG;
    __syncthreads();
}

// ---------------------------------------------------------------------------
// lambda_min: one LOBPCG iteration (Rayleigh-Ritz on span{v, w, P}).

template <typename OpT, typename UT>
__device__ void eig_step(const Work &w, Col &c, const Inst &in, double *red) {
    const int64_t n = c.n;
    const double *x = w.x + c.off, *p = w.p + c.off;
    const double *gam = w.gam + in.off, *dq = w.dq + in.off;
    double *v = w.v + c.off, *Av = w.Av + c.off, *P = w.P + c.off, *AP = w.AP + c.off;
    double *wv = w.w + c.off, *Aw = w.g + c.off;  // g is free during lambda_min
    const bool hasP = c.hasP != 0;
    // Gram matrices: B = Z-inner products, A = Qbar-inner products
    double sm[12];
#pragma unroll
    for (int j = 0; j < 12; ++j) sm[j] = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
        const double xi = x[i];
        double aw = 0.0;
        if (interior(xi)) {
            const double z = xi - xi * xi;
            const double A = (dq[i] + gam[i]) - p[i];
            const double wi = wv[i], vi = v[i];
            aw = uaux<UT>(w, c.off + i) + A * wi;
            sm[0] += z * vi * vi;
            sm[1] += z * vi * wi;
            sm[2] += z * wi * wi;
            sm[6] += vi * Av[i];
            sm[7] += vi * aw;
            sm[8] += wi * aw;
            if (hasP) {
                const double pi = P[i];
                sm[3] += z * vi * pi;
                sm[4] += z * wi * pi;
                sm[5] += z * pi * pi;
                sm[9] += vi * AP[i];
                sm[10] += wi * AP[i];
                sm[11] += pi * AP[i];
            }
        }
        Aw[i] = aw;
    }
    block_sum<12>(sm, red);
    // Rayleigh-Ritz, computed identically by every thread
    int m = hasP ? 3 : 2;
    double d[3] = {1.0 / sqrt(sm[0]), 1.0 / sqrt(sm[2]), hasP ? 1.0 / sqrt(sm[5]) : 0.0};
    double G0[3][3] = {{sm[0], sm[1], sm[3]}, {sm[1], sm[2], sm[4]}, {sm[3], sm[4], sm[5]}};
    double H0[3][3] = {{sm[6], sm[7], sm[9]}, {sm[7], sm[8], sm[10]}, {sm[9], sm[10], sm[11]}};
    double G[3][3], H[3][3], L[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            G[i][j] = G0[i][j] * d[i] * d[j];
            H[i][j] = H0[i][j] * d[i] * d[j];
        }
    bool ok = chol3(m, G, L);
    if (!ok && m == 3) {
        m = 2;
        ok = chol3(m, G, L);
    }
    const bool w_ok = sm[2] > 0.0 && isfinite(d[1]);
    if (!ok || !w_ok) {
        // the residual direction is numerically inside span{v}: converged
        if (threadIdx.x == 0) c.aux += 1;
        __syncthreads();
        eig_finish<OpT>(w, c, in, red, c.lam);
        return;
    }
    // C = L^-1 H L^-T
    double Li[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int j = 0; j < m; ++j) {
        Li[j][j] = 1.0 / L[j][j];
        for (int i = j + 1; i < m; ++i) {
            double s = 0.0;
            for (int q = j; q < i; ++q) s -= L[i][q] * Li[q][j];
            Li[i][j] = s / L[i][i];
        }
    }
    double T[3][3], C[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int q = 0; q < m; ++q) s += Li[i][q] * H[q][j];
            T[i][j] = (i < m && j < m) ? s : 0.0;
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int q = 0; q < m; ++q) s += T[i][q] * Li[j][q];
            C[i][j] = (i < m && j < m) ? s : 0.0;
        }
    for (int i = 0; i < m; ++i)
        for (int j = i + 1; j < m; ++j) {
            const double s = 0.5 * (C[i][j] + C[j][i]);
            C[i][j] = s;
            C[j][i] = s;
        }
    double theta, y[3];
    jacobi_min(m, C, theta, y);
    double a[3] = {0.0, 0.0, 0.0};  // a = D L^-T y
    for (int i = 0; i < m; ++i) {
        double s = 0.0;
        for (int q = 0; q < m; ++q) s += Li[q][i] * y[q];
        a[i] = s * d[i];
    }
    double rn[2] = {0.0, 0.0};  // ||r||^2_{Z^-1}, v'Zv
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
        const double xi = x[i];
        double wn = 0.0;
        if (interior(xi)) {
            const double z = xi - xi * xi;
            const double A = (dq[i] + gam[i]) - p[i];
            const double pi = hasP ? P[i] : 0.0, api = hasP ? AP[i] : 0.0;
            const double vn = a[0] * v[i] + a[1] * wv[i] + a[2] * pi;
            const double avn = a[0] * Av[i] + a[1] * Aw[i] + a[2] * api;
            const double pn = a[1] * wv[i] + a[2] * pi;
            const double apn = a[1] * Aw[i] + a[2] * api;
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
        put_aux<OpT>(w, c.off + i, wn);
    }
    block_sum<2>(rn, red);
    const int it = c.it + 1;
    if (threadIdx.x == 0) {
        c.aux += 1;
        c.it = it;
        c.lam = theta;
        c.hasP = 1;
    }
    __syncthreads();
    if (sqrt(rn[0] / rn[1]) <= w.eig_tol * fabs(theta) || it >= w.eig_maxit) {
        eig_finish<OpT>(w, c, in, red, theta);
    }
}

// ---------------------------------------------------------------------------
// x^0 by Jacobi-preconditioned CG on K = 2 (Q + Diag gamma).

template <typename OpT, typename UT>
__device__ void cg_step(const Work &w, Col &c, const Inst &in, double *red) {
    const int64_t n = c.n;
    double *x = w.x + c.off;
    double *r = w.v + c.off, *d = w.w + c.off, *Kd = w.Av + c.off;
    const double *gam = w.gam + in.off, *dq = w.dq + in.off;
    double s1[1] = {0.0};
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
        const double kd = 2.0 * (uaux<UT>(w, c.off + i) + (dq[i] + gam[i]) * d[i]);
        Kd[i] = kd;
        s1[0] += d[i] * kd;
    }
    block_sum<1>(s1, red);
    const double a = c.rz / s1[0];
    double s2[2] = {0.0, 0.0};  // r'M^-1 r, r'r
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
        x[i] = x[i] + a * d[i];
        const double ri = r[i] - a * Kd[i];
        r[i] = ri;
        const double zz = ri / (2.0 * (dq[i] + gam[i]));
        s2[0] += ri * zz;
        s2[1] += ri * ri;
    }
    block_sum<2>(s2, red);
    const int it = c.it + 1;
    if (threadIdx.x == 0) {
        c.aux += 1;
        c.it = it;
    }
    __syncthreads();
    if (sqrt(s2[1]) <= w.cg_tol * c.r0 || it >= w.cg_maxit) {
        outer_begin<OpT>(w, c, in, red);
        return;
    }
    const double beta = s2[0] / c.rz;
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
        const double zz = r[i] / (2.0 * (dq[i] + gam[i]));
        const double dn = zz + beta * d[i];
        d[i] = dn;
        put_aux<OpT>(w, c.off + i, dn);
    }
    if (threadIdx.x == 0) c.rz = s2[0];
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Kernels.

template <typename OpT, typename UT>
__global__ void __launch_bounds__(kBlock) solver_step_kernel(Work w) {
    const int ci = blockIdx.x;
    if (ci >= w.ncol || w.col[ci].phase == PH_DONE) return;
    __shared__ Col c;
    __shared__ Inst in;
    __shared__ double red[12 * kWaves];
    if (threadIdx.x == 0) {
        c = w.col[ci];
        in = w.inst[c.inst];
    }
    __syncthreads();
    switch (c.phase) {
        case PH_INNER: inner_step<OpT, UT>(w, c, in, red, ci); break;
        case PH_EIG0: eig0_step<OpT, UT>(w, c, in, red); break;
        case PH_EIG: eig_step<OpT, UT>(w, c, in, red); break;
        case PH_CG: cg_step<OpT, UT>(w, c, in, red); break;
        default: break;
    }
    __syncthreads();
    if (threadIdx.x == 0) w.col[ci] = c;
}

// Column set-up: x from X0 (column ci of an n x B matrix with leading
// dimension n) and the first outer step, or the CG start x = 0, r = gamma - b.
template <typename OpT>
__global__ void __launch_bounds__(kBlock) solver_init_kernel(Work w, const double *X0, int use_cg) {
    const int ci = blockIdx.x;
    if (ci >= w.ncol) return;
    __shared__ Col c;
    __shared__ Inst in;
    __shared__ double red[12 * kWaves];
    if (threadIdx.x == 0) {
        c = w.col[ci];
        in = w.inst[c.inst];
    }
    __syncthreads();
    const int64_t n = c.n;
    double *x = w.x + c.off;
    if (!use_cg) {
        for (int64_t i = threadIdx.x; i < n; i += kBlock) x[i] = X0[(int64_t)ci * n + i];
        __syncthreads();
        outer_begin<OpT>(w, c, in, red);
    } else {
        const double *b = w.b + in.off, *gam = w.gam + in.off, *dq = w.dq + in.off;
        double *r = w.v + c.off, *d = w.w + c.off;
        double s[2] = {0.0, 0.0};
        for (int64_t i = threadIdx.x; i < n; i += kBlock) {
            x[i] = 0.0;
            const double ri = gam[i] - b[i];
            const double zz = ri / (2.0 * (dq[i] + gam[i]));
            r[i] = ri;
            d[i] = zz;
            put_aux<OpT>(w, c.off + i, zz);
            s[0] += ri * zz;
            s[1] += ri * ri;
        }
        block_sum<2>(s, red);
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

// Live-column lists for the next sweep, in column order; also counts sweeps.
// Split precision: `active` gets the subproblem columns and `active_aux` the
// lambda_min / CG columns; otherwise `active` gets every live column.
__global__ void __launch_bounds__(kBlock) compact_kernel(Work w, int64_t *sweeps) {
    __shared__ int32_t cnt[2][kBlock];
    const int ncol = w.ncol;
    const int chunk = (ncol + kBlock - 1) / kBlock;
    const int lo = threadIdx.x * chunk;
    const int hi = min(ncol, lo + chunk);
    int my0 = 0, my1 = 0;
    for (int ci = lo; ci < hi; ++ci) {
        const int ph = w.col[ci].phase;
        if (ph == PH_DONE) continue;
        if (w.split && ph != PH_INNER) ++my1;
        else ++my0;
    }
    cnt[0][threadIdx.x] = my0;
    cnt[1][threadIdx.x] = my1;
    __syncthreads();
    if (threadIdx.x == 0) {
        int a0 = 0, a1 = 0;
        for (int t = 0; t < kBlock; ++t) {
            const int v0 = cnt[0][t], v1 = cnt[1][t];
            cnt[0][t] = a0;
            cnt[1][t] = a1;
            a0 += v0;
            a1 += v1;
        }
        *w.nactive = a0;
        if (w.split) *w.nactive_aux = a1;
        if (sweeps) *sweeps += 1;
    }
    __syncthreads();
    int p0 = cnt[0][threadIdx.x], p1 = cnt[1][threadIdx.x];
    for (int ci = lo; ci < hi; ++ci) {
        const int ph = w.col[ci].phase;
        if (ph == PH_DONE) continue;
        if (w.split && ph != PH_INNER) w.active_aux[p1++] = ci;
        else w.active[p0++] = ci;
    }
}

template <typename OpT, typename UT>
static hipError_t step_launch(const Work &w, hipStream_t st) {
    hipLaunchKernelGGL((solver_step_kernel<OpT, UT>), dim3(w.ncol), dim3(kBlock), 0, st, w);
    return hipGetLastError();
}

hipError_t launch_solver_step(int optype, int utype, const Work &w, hipStream_t st) {
    if (optype == PSDP_F64 && utype == PSDP_F64) return step_launch<double, double>(w, st);
    if (optype == PSDP_F32 && utype == PSDP_F32) return step_launch<float, float>(w, st);
    if (optype == PSDP_BF16 && utype == PSDP_F32) return step_launch<__hip_bfloat16, float>(w, st);
    return hipErrorInvalidValue;
}

hipError_t launch_solver_init(int optype, const Work &w, const double *X0, int use_cg,
                              hipStream_t st) {
    if (optype == PSDP_F64)
        hipLaunchKernelGGL(solver_init_kernel<double>, dim3(w.ncol), dim3(kBlock), 0, st, w, X0, use_cg);
    else if (optype == PSDP_F32)
        hipLaunchKernelGGL(solver_init_kernel<float>, dim3(w.ncol), dim3(kBlock), 0, st, w, X0, use_cg);
    else
        hipLaunchKernelGGL(solver_init_kernel<__hip_bfloat16>, dim3(w.ncol), dim3(kBlock), 0, st, w,
                           X0, use_cg);
    return hipGetLastError();
}

hipError_t launch_compact(const Work &w, hipStream_t st) {
    hipLaunchKernelGGL(compact_kernel, dim3(1), dim3(kBlock), 0, st, w, (int64_t *)nullptr);
    return hipGetLastError();
}

hipError_t launch_compact_count(const Work &w, int64_t *sweeps, hipStream_t st) {
    hipLaunchKernelGGL(compact_kernel, dim3(1), dim3(kBlock), 0, st, w, sweeps);
    return hipGetLastError();
}

}  // namespace psdp
