/*
 * qap_oracle.c -- plain, slow, single-threaded CPU oracle for simulated
 * annealing (SA) on the quadratic assignment problem (QAP), following
 * G. Paul, "A GPU implementation of the Simulated Annealing Heuristic for the
 * Quadratic Assignment Problem" (arXiv 1208.2675).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker, not the product: only
 * the test-suite, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no code, header, table or constant generator with the
 * device library, and it never calls it.
 *
 * What it computes, and the passage each part follows:
 *   orc_cost                     Eq. (1), Sec. 1: C = sum_ij A_ij B_{p(i),p(j)}.
 *   orc_swap_cost_by_definition  the cost of swapping the locations of two
 *                                facilities (Sec. 2.1): C(p o (r s)) - C(p), two
 *                                literal evaluations of Eq. (1).
 *   orc_swap_cost                the same number in O(N): Eq. (1) differenced
 *                                over the terms whose indices meet {r, s}; this
 *                                is the "from scratch" per-proposal cost of the
 *                                traditional SA the paper contrasts with (Sec. 2.1).
 *   orc_delta_matrix             step (a) of the Delta-matrix approach (Sec. 2.2):
 *                                the swap cost of every pair r < s for the current p.
 *   orc_philox4x32_10            the counter-based generator Philox-4x32 with 10
 *                                rounds of Salmon, Moraes, Dror and Shaw, "Parallel
 *                                random numbers: as easy as 1, 2, 3" (SC'11),
 *                                written from that paper's definition.
 *   orc_uniform                  the r of Eq. (2): uniform in (0, 1), one draw per
 *                                iteration from counter (t, chain) and a 64-bit key.
 *   orc_temperature_tables /
 *   orc_temperature              the cooling schedule (Sec. 2.1 leaves its form
 *                                open): geometric, T_t = T0 * alpha^t, evaluated
 *                                as a product of three table entries (reading
 *                                below).
 *   orc_sa_run                   steps (b)-(e) of Sec. 2.2 with the Metropolis test
 *                                of Eq. (2); every proposal's cost is recomputed
 *                                from scratch, so the trajectory does not depend on
 *                                any maintained Delta matrix.
 *   orc_random_pair_index /
 *   orc_sa_run_order             the same run with the pairs drawn at random
 *                                (Sec. 2.1 lets the next swap be chosen randomly
 *                                or sequentially): iteration t proposes a pair
 *                                drawn from its own counter (reading below).
 *   orc_tabu_run                 tabu search over the same swap costs, the heuristic
 *                                whose Delta bookkeeping (Taillard) the method takes
 *                                over (Sec. 2.2, Sec. 2.4): every iteration evaluates
 *                                all swaps and makes the best admissible one
 *                                (reading below).
 *   orc_brute_force              the exact optimum over all N! permutations (N <= 10).
 *
 * Readings where the paper is silent (each is also listed in the design notes):
 *   - p(i) is the location of facility i (pinned by a library QAP routine in the tests).
 *   - Proposals run through the pairs r < s in row-major order, cyclically; one
 *     proposal is one iteration, accepted or not (Sec. 2.1 allows a sequential
 *     enumeration; step (b) of Sec. 2.2 increments per proposal).
 *   - Eq. (2) in floating point: delta <= 0 accepts (r < 1 makes e^0 > r); for
 *     delta > 0, z = fl(fl(delta / T_t) + fl(log r_t)) and the swap is made iff
 *     z < 0.  |z| < 1e-12 is logged as a near tie.
 *   - r_t = (2 u + 1) 2^-53 with u the 52 bits (x0 << 20) | (x1 >> 12) of the
 *     generator output for counter (lo32 t, hi32 t, chain, 0), key (lo32 seed,
 *     hi32 seed); exact in binary64 and strictly inside (0, 1).
 *   - Random order: iteration t proposes pair number floor(x2 M / 2^32) of the
 *     row-major enumeration (M = n(n-1)/2), x2 being the third output word of
 *     the same generator call that gives r_t.  Each of the M pairs takes
 *     floor(2^32 / M) or that plus one of the 2^32 values of x2.
 *   - Tabu search (the paper names it, after Taillard, but fixes no rules):
 *     when facility i leaves location l at iteration t, assigning i to l is
 *     tabu for the iterations t' < t + tenure.  The swap (r, s) is tabu at t
 *     when both of its new assignments, r to p(s) and s to p(r), are; a tabu
 *     swap is still admissible when it gives a cost below the best seen.
 *     Iteration t makes the admissible swap of least cost change, the lowest
 *     row-major pair number among equals; if none is admissible, the swap of
 *     least cost change among all.  Every iteration makes one swap.
 *   - T_t = ((T0 * H[t >> 20]) * M[(t >> 10) & 1023]) * L[t & 1023] with
 *     L[j] = L[j-1] alpha, M[j] = M[j-1] (L[1023] alpha),
 *     H[j] = H[j-1] (M[1023] L[1023] alpha), all three starting at 1.
 *
 * Integer arithmetic is int64 throughout; orc_check_bounds states when that
 * is exact.  Build with -ffp-contract=off and without fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_INVAL (-1)
#define ORC_E_NOT_PERM (-2)
#define ORC_E_RANGE (-3)

/* ------------------------------------------------------------------ Eq. (1) */

int64_t orc_cost(int32_t n, const int32_t *A, const int32_t *B, const int32_t *p)
{
    int64_t c = 0;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < n; ++j)
            c += (int64_t)A[(int64_t)i * n + j] * (int64_t)B[(int64_t)p[i] * n + p[j]];
    return c;
}

/* Cost change of swapping the locations of facilities r and s: C(p o (r s)) - C(p). */
int64_t orc_swap_cost_by_definition(int32_t n, const int32_t *A, const int32_t *B,
                                    const int32_t *p, int32_t r, int32_t s)
{
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!q) return INT64_MIN;
    memcpy(q, p, sizeof(int32_t) * (size_t)n);
    int32_t tmp = q[r];
    q[r] = q[s];
    q[s] = tmp;
    int64_t d = orc_cost(n, A, B, q) - orc_cost(n, A, B, p);
    free(q);
    return d;
}

/*
 * The same swap cost in O(N).  With q = p o (r s), only the terms of Eq. (1)
 * with i or j in {r, s} differ between C(q) and C(p):
 *   i, j both in {r, s}:  (A_rr - A_ss)(B_{ps ps} - B_{pr pr}) + (A_rs - A_sr)(B_{ps pr} - B_{pr ps})
 *   j = k, k not in {r,s}, i in {r, s}:  (A_rk - A_sk)(B_{ps pk} - B_{pr pk})
 *   i = k, k not in {r,s}, j in {r, s}:  (A_kr - A_ks)(B_{pk ps} - B_{pk pr})
 * where pr = p(r), ps = p(s), pk = p(k).
 */
int64_t orc_swap_cost(int32_t n, const int32_t *A, const int32_t *B, const int32_t *p,
                      int32_t r, int32_t s)
{
    const int64_t N = n;
    const int64_t pr = p[r], ps = p[s];
    int64_t d = ((int64_t)A[r * N + r] - A[s * N + s]) * ((int64_t)B[ps * N + ps] - B[pr * N + pr])
              + ((int64_t)A[r * N + s] - A[s * N + r]) * ((int64_t)B[ps * N + pr] - B[pr * N + ps]);
    for (int64_t k = 0; k < N; ++k) {
        if (k == r || k == s) continue;
        const int64_t pk = p[k];
        d += ((int64_t)A[r * N + k] - A[s * N + k]) * ((int64_t)B[ps * N + pk] - B[pr * N + pk]);
        d += ((int64_t)A[k * N + r] - A[k * N + s]) * ((int64_t)B[pk * N + ps] - B[pk * N + pr]);
    }
    return d;
}

/* Step (a): swap cost of every pair r < s, stored row-major (the proposal order). */
void orc_delta_matrix(int32_t n, const int32_t *A, const int32_t *B, const int32_t *p,
                      int64_t *delta_out)
{
    int64_t idx = 0;
    for (int32_t r = 0; r < n; ++r)
        for (int32_t s = r + 1; s < n; ++s)
            delta_out[idx++] = orc_swap_cost(n, A, B, p, r, s);
}

/* T0 reading: mean |Delta| over the n(n-1)/2 pairs, as an int64 sum and one division. */
double orc_mean_abs_delta(int32_t n, const int64_t *delta, int64_t *sum_out)
{
    const int64_t m = (int64_t)n * (n - 1) / 2;
    int64_t s = 0;
    for (int64_t i = 0; i < m; ++i) s += delta[i] < 0 ? -delta[i] : delta[i];
    if (sum_out) *sum_out = s;
    return (double)s / (double)m;
}

/*
 * Every int64 quantity above stays exact when
 *   n^2 * max|A| * max|B| < 2^62   (the cost) and
 *   (2n + 8) * range(A) * range(B) < 2^62  (any swap cost and any difference of two).
 * Returns ORC_OK or ORC_E_RANGE.  The check multiplies in 128 bits so that
 * it cannot overflow itself.
 */
int orc_check_bounds(int32_t n, const int32_t *A, const int32_t *B)
{
    int64_t amin = INT32_MAX, amax = INT32_MIN, bmin = INT32_MAX, bmax = INT32_MIN;
    const int64_t nn = (int64_t)n * n;
    for (int64_t i = 0; i < nn; ++i) {
        if (A[i] < amin) amin = A[i];
        if (A[i] > amax) amax = A[i];
        if (B[i] < bmin) bmin = B[i];
        if (B[i] > bmax) bmax = B[i];
    }
    const int64_t amag = amax > -amin ? amax : -amin;
    const int64_t bmag = bmax > -bmin ? bmax : -bmin;
    const __int128 lim = (__int128)1 << 62;
    if ((__int128)nn * amag * bmag >= lim) return ORC_E_RANGE;
    if ((__int128)(2 * (int64_t)n + 8) * (amax - amin) * (bmax - bmin) >= lim) return ORC_E_RANGE;
    return ORC_OK;
}

/* ------------------------------------------------------ Philox-4x32, 10 rounds */
/*
 * One round maps (x0, x1, x2, x3) under round key (k0, k1) to
 *   (hi(M1 x2) ^ x1 ^ k0,  lo(M1 x2),  hi(M0 x0) ^ x3 ^ k1,  lo(M0 x0))
 * with the two 32-bit multipliers M0, M1 of the SC'11 paper; the key is
 * advanced by the Weyl constants W0, W1 between rounds.
 */
#define ORC_PHILOX_M0 0xD2511F53u
#define ORC_PHILOX_M1 0xCD9E8D57u
#define ORC_PHILOX_W0 0x9E3779B9u
#define ORC_PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        const uint64_t prod0 = (uint64_t)ORC_PHILOX_M0 * x0;
        const uint64_t prod1 = (uint64_t)ORC_PHILOX_M1 * x2;
        const uint32_t y0 = (uint32_t)(prod1 >> 32) ^ x1 ^ k0;
        const uint32_t y1 = (uint32_t)prod1;
        const uint32_t y2 = (uint32_t)(prod0 >> 32) ^ x3 ^ k1;
        const uint32_t y3 = (uint32_t)prod0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += ORC_PHILOX_W0;
        k1 += ORC_PHILOX_W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* r_t of Eq. (2) for iteration t of chain `chain` under 64-bit key `seed`. */
double orc_uniform(uint64_t seed, uint32_t chain, uint64_t t)
{
    const uint32_t ctr[4] = {(uint32_t)t, (uint32_t)(t >> 32), chain, 0u};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    const uint64_t u = ((uint64_t)x[0] << 20) | (uint64_t)(x[1] >> 12);
    return (double)(2 * u + 1) * 0x1p-53;
}

/* Pair number proposed at iteration t under random order (m = n(n-1)/2 pairs). */
uint64_t orc_random_pair_index(uint64_t seed, uint32_t chain, uint64_t t, uint64_t m)
{
    const uint32_t ctr[4] = {(uint32_t)t, (uint32_t)(t >> 32), chain, 0u};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    return ((uint64_t)x[2] * m) >> 32;
}

/* ------------------------------------------------------------ cooling schedule */

/* alpha of a geometric schedule that falls by `ratio` over `iters` iterations. */
double orc_geometric_alpha(uint64_t iters, double ratio)
{
    if (iters <= 1) return 1.0;
    return pow(ratio, 1.0 / (double)(iters - 1));
}

uint64_t orc_temperature_table_len(uint64_t iters)
{
    uint64_t nh = (iters + ((uint64_t)1 << 20) - 1) >> 20;
    return nh ? nh : 1;
}

/* L, M: 1024 entries each; H: orc_temperature_table_len(iters) entries. */
void orc_temperature_tables(double alpha, uint64_t iters, double *L, double *M, double *H)
{
    L[0] = 1.0;
    for (int j = 1; j < 1024; ++j) L[j] = L[j - 1] * alpha;
    const double step_m = L[1023] * alpha;           /* alpha^1024  */
    M[0] = 1.0;
    for (int j = 1; j < 1024; ++j) M[j] = M[j - 1] * step_m;
    const double step_h = M[1023] * step_m;          /* alpha^(2^20) */
    const uint64_t nh = orc_temperature_table_len(iters);
    H[0] = 1.0;
    for (uint64_t j = 1; j < nh; ++j) H[j] = H[j - 1] * step_h;
}

double orc_temperature(double T0, const double *L, const double *M, const double *H, uint64_t t)
{
    const double th = T0 * H[t >> 20];
    const double tm = th * M[(t >> 10) & 1023];
    return tm * L[t & 1023];
}

/* ------------------------------------------------------------------ SA run */

typedef struct {
    uint64_t t;          /* next iteration index                                  */
    uint64_t accepts;    /* swaps made so far                                     */
    uint64_t near_ties;  /* Metropolis tests with |z| < 1e-12 so far              */
    uint64_t hash;       /* sum of orc_accept_fingerprint over accepted swaps      */
    int64_t cost;        /* Eq. (1) at the current p, tracked incrementally       */
    int64_t best_cost;   /* lowest cost seen                                      */
    uint64_t best_iter;  /* iterations completed when best_cost was first reached */
} orc_state;

/*
 * Trajectory hash (a checksum for comparing runs, not part of the method): the
 * sum mod 2^64 over accepted swaps of fp(t, r, s, delta) =
 * f(f(f(t) ^ (r << 32 | s)) ^ delta), with f the output function of splitmix64
 * (Steele, Lea, Flood, "Fast splittable pseudorandom number generators",
 * OOPSLA 2014).  Distinct accepted swaps have distinct t, so the sum still
 * identifies the sequence.
 */
static uint64_t orc_splitmix_out(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t orc_accept_fingerprint(uint64_t t, int32_t r, int32_t s, int64_t delta)
{
    uint64_t h = orc_splitmix_out(t);
    h = orc_splitmix_out(h ^ (((uint64_t)(uint32_t)r << 32) | (uint64_t)(uint32_t)s));
    return orc_splitmix_out(h ^ (uint64_t)delta);
}

/* Fresh chain state for permutation p: cost by Eq. (1), empty logs. */
void orc_state_init(int32_t n, const int32_t *A, const int32_t *B, const int32_t *p, orc_state *st)
{
    st->t = 0;
    st->accepts = 0;
    st->near_ties = 0;
    st->hash = 0;
    st->cost = orc_cost(n, A, B, p);
    st->best_cost = st->cost;
    st->best_iter = 0;
}

static int orc_is_perm(int32_t n, const int32_t *p)
{
    unsigned char *seen = (unsigned char *)calloc((size_t)n, 1);
    int ok = seen != NULL;
    for (int32_t i = 0; ok && i < n; ++i) {
        if (p[i] < 0 || p[i] >= n || seen[p[i]]) ok = 0;
        else seen[p[i]] = 1;
    }
    free(seen);
    return ok;
}

/* (r, s) of pair number idx in row-major r < s order. */
static void orc_pair_of_index(int32_t n, uint64_t idx, int32_t *r, int32_t *s)
{
    int32_t row = 0;
    while (idx >= (uint64_t)(n - 1 - row)) { idx -= (uint64_t)(n - 1 - row); ++row; }
    *r = row;
    *s = row + 1 + (int32_t)idx;
}

/*
 * Iterations st->t .. t_end-1 of an SA run of length `iters` (Sec. 2.1-2.2).
 * Iteration t proposes a pair (r, s), computes its swap cost from scratch,
 * applies Eq. (2) with T_t and r_t, and on acceptance swaps p(r), p(s) and adds
 * the swap cost to the tracked cost.  order 0: pair number (t mod n(n-1)/2) in
 * row-major r < s order.  order 1: pair number orc_random_pair_index(t).
 *
 * acc_log (optional): 4 int64 per accepted swap (t, r, s, delta), the first
 *   acc_cap of them counted from st->accepts == 0.
 * tie_t / tie_z (optional): the first tie_cap near ties (|z| < 1e-12): t and z.
 */
int orc_sa_run_order(int32_t n, const int32_t *A, const int32_t *B, int32_t *p, orc_state *st,
                     uint64_t iters, uint64_t t_end, double T0, double alpha,
                     uint64_t seed, uint32_t chain, int32_t order,
                     int64_t *acc_log, uint64_t acc_cap,
                     uint64_t *tie_t, double *tie_z, uint64_t tie_cap)
{
    if (n < 2 || t_end > iters || st->t > t_end || !(T0 > 0.0) || !(alpha > 0.0) || alpha > 1.0 ||
        (order != 0 && order != 1))
        return ORC_E_INVAL;
    if (!orc_is_perm(n, p)) return ORC_E_NOT_PERM;
    if (orc_check_bounds(n, A, B) != ORC_OK) return ORC_E_RANGE;

    const uint64_t m = (uint64_t)n * (uint64_t)(n - 1) / 2;
    const uint64_t nh = orc_temperature_table_len(iters);
    double *L = (double *)malloc(1024 * sizeof(double));
    double *M = (double *)malloc(1024 * sizeof(double));
    double *H = (double *)malloc(nh * sizeof(double));
    if (!L || !M || !H) { free(L); free(M); free(H); return ORC_E_INVAL; }
    orc_temperature_tables(alpha, iters, L, M, H);

    /* the pair proposed at iteration st->t in row-major order */
    int32_t r, s;
    orc_pair_of_index(n, st->t % m, &r, &s);

    for (uint64_t t = st->t; t < t_end; ++t) {
        if (order == 1) orc_pair_of_index(n, orc_random_pair_index(seed, chain, t, m), &r, &s);
        const int64_t delta = orc_swap_cost(n, A, B, p, r, s);
        int accept;
        if (delta <= 0) {
            accept = 1;
        } else {
            const double T = orc_temperature(T0, L, M, H, t);
            const double x = (double)delta / T;
            const double y = log(orc_uniform(seed, chain, t));
            const double z = x + y;
            if (fabs(z) < 1e-12) {
                if (st->near_ties < tie_cap) {
                    if (tie_t) tie_t[st->near_ties] = t;
                    if (tie_z) tie_z[st->near_ties] = z;
                }
                st->near_ties++;
            }
            accept = z < 0.0;
        }
        if (accept) {
            const int32_t tmp = p[r];
            p[r] = p[s];
            p[s] = tmp;
            st->cost += delta;
            if (acc_log && st->accepts < acc_cap) {
                int64_t *e = acc_log + 4 * st->accepts;
                e[0] = (int64_t)t; e[1] = r; e[2] = s; e[3] = delta;
            }
            st->accepts++;
            st->hash += orc_accept_fingerprint(t, r, s, delta);
            if (st->cost < st->best_cost) {
                st->best_cost = st->cost;
                st->best_iter = t + 1;
            }
        }
        /* next pair in row-major order, wrapping to (0, 1) */
        if (++s == n) {
            if (++r == n - 1) r = 0;
            s = r + 1;
        }
    }
    st->t = t_end;
    free(L); free(M); free(H);
    return ORC_OK;
}

/* The row-major run (order 0). */
int orc_sa_run(int32_t n, const int32_t *A, const int32_t *B, int32_t *p, orc_state *st,
               uint64_t iters, uint64_t t_end, double T0, double alpha,
               uint64_t seed, uint32_t chain,
               int64_t *acc_log, uint64_t acc_cap,
               uint64_t *tie_t, double *tie_z, uint64_t tie_cap)
{
    return orc_sa_run_order(n, A, B, p, st, iters, t_end, T0, alpha, seed, chain, 0,
                            acc_log, acc_cap, tie_t, tie_z, tie_cap);
}

/* ------------------------------------------------------------- tabu search */

/*
 * Iterations st->t .. t_end-1 of a tabu search (rules in the header).  tabu:
 * n*n int64, tabu[i*n + l] = the first iteration at which facility i may again
 * be assigned to location l (all zero before the first iteration).  Every
 * swap cost is computed from scratch (orc_swap_cost) at every iteration.
 * acc_log (optional): 4 int64 per swap (t, r, s, delta), as for orc_sa_run.
 */
int orc_tabu_run(int32_t n, const int32_t *A, const int32_t *B, int32_t *p, orc_state *st,
                 uint64_t t_end, int64_t tenure, int64_t *tabu, int64_t *acc_log, uint64_t acc_cap)
{
    if (n < 2 || st->t > t_end || tenure < 0 || !tabu) return ORC_E_INVAL;
    if (!orc_is_perm(n, p)) return ORC_E_NOT_PERM;
    if (orc_check_bounds(n, A, B) != ORC_OK) return ORC_E_RANGE;
    for (uint64_t t = st->t; t < t_end; ++t) {
        int found = 0, found_any = 0;
        int32_t br = 0, bs = 1, ar = 0, as = 1;
        int64_t bd = 0, ad = 0;
        for (int32_t r = 0; r < n - 1; ++r) {
            for (int32_t s = r + 1; s < n; ++s) {
                const int64_t d = orc_swap_cost(n, A, B, p, r, s);
                if (!found_any || d < ad) { found_any = 1; ad = d; ar = r; as = s; }
                const int is_tabu = tabu[(int64_t)r * n + p[s]] > (int64_t)t &&
                                    tabu[(int64_t)s * n + p[r]] > (int64_t)t;
                const int admissible = !is_tabu || st->cost + d < st->best_cost;
                if (admissible && (!found || d < bd)) { found = 1; bd = d; br = r; bs = s; }
            }
        }
        if (!found) { bd = ad; br = ar; bs = as; }
        /* the facilities leave their locations: returning is tabu for `tenure` iterations */
        tabu[(int64_t)br * n + p[br]] = (int64_t)t + tenure;
        tabu[(int64_t)bs * n + p[bs]] = (int64_t)t + tenure;
        const int32_t tmp = p[br];
        p[br] = p[bs];
        p[bs] = tmp;
        st->cost += bd;
        if (acc_log && st->accepts < acc_cap) {
            int64_t *e = acc_log + 4 * st->accepts;
            e[0] = (int64_t)t; e[1] = br; e[2] = bs; e[3] = bd;
        }
        st->accepts++;
        st->hash += orc_accept_fingerprint(t, br, bs, bd);
        if (st->cost < st->best_cost) {
            st->best_cost = st->cost;
            st->best_iter = t + 1;
        }
    }
    st->t = t_end;
    return ORC_OK;
}

/* ------------------------------------------------------------ brute force */

/* Exact optimum of Eq. (1) over all n! permutations (Heap's algorithm), n <= 10. */
int64_t orc_brute_force(int32_t n, const int32_t *A, const int32_t *B, int32_t *p_best,
                        uint64_t *n_visited)
{
    if (n < 1 || n > 10) return INT64_MIN;
    int32_t q[10], c[10];
    for (int32_t i = 0; i < n; ++i) { q[i] = i; c[i] = 0; }
    int64_t best = orc_cost(n, A, B, q);
    memcpy(p_best, q, sizeof(int32_t) * (size_t)n);
    uint64_t visited = 1;
    int32_t i = 1;
    while (i < n) {
        if (c[i] < i) {
            const int32_t j = (i % 2 == 0) ? 0 : c[i];
            const int32_t tmp = q[j];
            q[j] = q[i];
            q[i] = tmp;
            ++visited;
            const int64_t cq = orc_cost(n, A, B, q);
            if (cq < best) {
                best = cq;
                memcpy(p_best, q, sizeof(int32_t) * (size_t)n);
            }
            c[i] += 1;
            i = 1;
        } else {
            c[i] = 0;
            ++i;
        }
    }
    if (n_visited) *n_visited = visited;
    return best;
}
