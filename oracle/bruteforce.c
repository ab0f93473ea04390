/* Exhaustive minimization of f(x) = x^T Q x + b^T x over x in {0,1}^n.
 *
 * TEST INFRASTRUCTURE ONLY (part of the CPU oracle): it pins the objective
 * of Section 2, eq. (bqp), by enumeration, independently of any solver.
 *
 * The 2^n vectors are visited in reflected Gray-code order, so consecutive
 * vectors differ in one bit k and f changes by
 *   (1 - 2 x_k) * (Q_kk + b_k + 2 * sum_{j != k} Q_kj x_j)
 * which is tracked exactly in int64 together with s = Q x. Ties keep the
 * vector with the smallest binary value (bit i = x_i).
 */
#include <stdint.h>

int ubqp_bruteforce(int n, const int64_t *Q, const int64_t *b,
                    int64_t *best_obj, uint64_t *best_mask)
{
    if (n < 1 || n > 30) return -1;
    int64_t s[32];
    for (int i = 0; i < n; ++i) s[i] = 0;          /* s = Q x, x = 0 */
    uint64_t mask = 0;
    int64_t f = 0;
    int64_t bestf = 0;
    uint64_t bestm = 0;
    uint64_t total = (uint64_t)1 << n;
    for (uint64_t step = 1; step < total; ++step) {
        int k = __builtin_ctzll(step);             /* bit flipped by Gray code */
        int64_t off = s[k] - Q[(int64_t)k * n + k] * (int64_t)((mask >> k) & 1);
        int64_t d = Q[(int64_t)k * n + k] + b[k] + 2 * off;
        if ((mask >> k) & 1) {
            f -= d;
            mask &= ~((uint64_t)1 << k);
            for (int i = 0; i < n; ++i) s[i] -= Q[(int64_t)i * n + k];
        } else {
            f += d;
            mask |= (uint64_t)1 << k;
            for (int i = 0; i < n; ++i) s[i] += Q[(int64_t)i * n + k];
        }
        if (f < bestf || (f == bestf && mask < bestm)) {
            bestf = f;
            bestm = mask;
        }
    }
    *best_obj = bestf;
    *best_mask = bestm;
    return 0;
}
