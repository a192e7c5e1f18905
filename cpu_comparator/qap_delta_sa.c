/*
 * qap_delta_sa.c -- single-threaded CPU simulated annealing for the QAP with
 * the Delta matrix, the comparator type of G. Paul, "A GPU implementation of
 * the Simulated Annealing Heuristic for the Quadratic Assignment Problem"
 * (arXiv 1208.2675): the efficient non-parallel Delta-matrix SA the paper
 * times its GPU against (Sec. 2.2, Sec. 4).
 *
 * A TIMING BASELINE ONLY.  It is neither the product nor the correctness
 * oracle: the benchmark times it on the host beside the GPU, and the tests
 * check that it walks the oracle's trajectory.  It shares no code with the
 * device library or with the oracle.
 *
 * Like the paper's comparator it computes each proposal's swap cost from
 * scratch in O(N) while most proposals are accepted, and moves to the Delta
 * matrix of Sec. 2.2 (steps (a)-(d)) once acceptance falls: an accepted swap
 * then costs O(N^2) (the Taillard correction for pairs disjoint from the
 * swap, an O(N) recomputation for the 2N-3 pairs that meet it) and a rejected
 * proposal O(1).  Both modes give the same swap costs, so the switch never
 * changes the run.  The run itself follows the same readings as the rest of
 * the repository: row-major cyclic proposals, r_t from Philox-4x32-10 (Salmon
 * et al., SC'11) at counter (t, chain) and key seed, Eq. (2) in binary64 with
 * |z| < 1e-12 counted as a near tie, the geometric schedule evaluated as a
 * product of three table entries, and the accept checksum built from the
 * splitmix64 output function (Steele, Lea, Flood, OOPSLA 2014).
 *
 * Build: gcc -O3 -march=native -ffp-contract=off -fno-fast-math -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t t, accepts, near_ties, hash;
    int64_t cost, best_cost;
    uint64_t best_iter;
    uint64_t delta_mode_at;   /* iteration at which the Delta matrix was built (or ~0) */
} cmp_state;

/* ------------------------------------------------------------ generator */

static void philox10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    for (int i = 0; i < 10; ++i) {
        const uint64_t pa = (uint64_t)0xD2511F53u * c[0];
        const uint64_t pb = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(pb >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(pa >> 32) ^ c[3] ^ k1;
        c[1] = (uint32_t)pb;
        c[3] = (uint32_t)pa;
        c[0] = n0;
        c[2] = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

static double draw_r(uint64_t seed, uint32_t chain, uint64_t t)
{
    uint32_t c[4] = {(uint32_t)t, (uint32_t)(t >> 32), chain, 0u};
    philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const uint64_t u = ((uint64_t)c[0] << 20) | (uint64_t)(c[1] >> 12);
    return (double)(2 * u + 1) * 0x1p-53;
}

static uint64_t mix(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static uint64_t fingerprint(uint64_t t, int32_t r, int32_t s, int64_t d)
{
    uint64_t h = mix(t);
    h = mix(h ^ (((uint64_t)(uint32_t)r << 32) | (uint32_t)s));
    return mix(h ^ (uint64_t)d);
}

/* ------------------------------------------------------------- chain data */

typedef struct {
    int n;
    const int32_t *A;   /* flows, row-major            */
    int32_t *At;        /* A transposed                */
    int32_t *Bp;        /* B'[i][j] = B[p(i)][p(j)]     */
    int32_t *Bt;        /* B' transposed               */
    int64_t *D;         /* packed Delta, row-major r<s */
    int64_t *rowoff;    /* packed offset of row r      */
} chain;

/* Swap cost of (r, s) in O(N) from rows of A, A^T, B', B'^T. */
static int64_t swap_cost(const chain *c, int r, int s)
{
    const int n = c->n;
    const int32_t *ar = c->A + (int64_t)r * n, *as = c->A + (int64_t)s * n;
    const int32_t *cr = c->At + (int64_t)r * n, *cs = c->At + (int64_t)s * n;
    const int32_t *br = c->Bp + (int64_t)r * n, *bs = c->Bp + (int64_t)s * n;
    const int32_t *dr = c->Bt + (int64_t)r * n, *ds = c->Bt + (int64_t)s * n;
    int64_t acc = 0;
#define TERM(k) (((int64_t)ar[k] - as[k]) * ((int64_t)bs[k] - br[k]) + ((int64_t)cr[k] - cs[k]) * ((int64_t)ds[k] - dr[k]))
    for (int k = 0; k < n; ++k) acc += TERM(k);
    /* the k = r and k = s terms above belong to neither sum; the two terms of
       Eq. (1) with both indices in {r, s} are added instead */
    acc -= TERM(r) + TERM(s);
#undef TERM
    acc += ((int64_t)ar[r] - as[s]) * ((int64_t)bs[s] - br[r]) + ((int64_t)ar[s] - as[r]) * ((int64_t)bs[r] - br[s]);
    return acc;
}

static void swap_int(int32_t *x, int32_t *y)
{
    const int32_t t = *x;
    *x = *y;
    *y = t;
}

/* B' (and its transpose) after the swap (u, v): rows and columns u, v exchanged. */
static void apply_swap(chain *c, int u, int v)
{
    const int n = c->n;
    int32_t *M[2] = {c->Bp, c->Bt};
    for (int m = 0; m < 2; ++m) {
        int32_t *X = M[m];
        for (int k = 0; k < n; ++k) swap_int(X + (int64_t)u * n + k, X + (int64_t)v * n + k);
        for (int k = 0; k < n; ++k) swap_int(X + (int64_t)k * n + u, X + (int64_t)k * n + v);
    }
}

static void build_delta(chain *c)
{
    const int n = c->n;
    for (int r = 0; r < n - 1; ++r)
        for (int s = r + 1; s < n; ++s) c->D[c->rowoff[r] + s - r - 1] = swap_cost(c, r, s);
}

/* Delta after the accepted swap (u, v), with B' already swapped: O(1) for the
   pairs disjoint from {u, v}, O(N) for the pairs that meet it. */
static void update_delta(chain *c, int u, int v, int64_t d_uv, int64_t *x, int64_t *y, int64_t *h, int64_t *w)
{
    const int n = c->n;
    for (int k = 0; k < n; ++k) {
        x[k] = (int64_t)c->At[(int64_t)u * n + k] - c->At[(int64_t)v * n + k];   /* A[k][u] - A[k][v]   */
        y[k] = (int64_t)c->A[(int64_t)u * n + k] - c->A[(int64_t)v * n + k];     /* A[u][k] - A[v][k]   */
        h[k] = (int64_t)c->Bt[(int64_t)u * n + k] - c->Bt[(int64_t)v * n + k];   /* B'[k][u] - B'[k][v] */
        w[k] = (int64_t)c->Bp[(int64_t)u * n + k] - c->Bp[(int64_t)v * n + k];   /* B'[u][k] - B'[v][k] */
    }
    for (int r = 0; r < n - 1; ++r) {
        if (r == u || r == v) continue;
        int64_t *row = c->D + c->rowoff[r] - r - 1;
        const int64_t xr = x[r], yr = y[r], hr = h[r], wr = w[r];
        for (int s = r + 1; s < n; ++s)
            row[s] += (xr - x[s]) * (h[s] - hr) + (yr - y[s]) * (w[s] - wr);
    }
    for (int k = 0; k < n; ++k) {
        if (k == u || k == v) continue;
        for (int e = 0; e < 2; ++e) {
            const int a = e ? v : u;
            const int lo = k < a ? k : a, hi = k < a ? a : k;
            c->D[c->rowoff[lo] + hi - lo - 1] = swap_cost(c, lo, hi);
        }
    }
    const int lo = u < v ? u : v, hi = u < v ? v : u;
    c->D[c->rowoff[lo] + hi - lo - 1] = -d_uv;
}

/*
 * Iterations st->t .. t_end-1 of a run of length iters.  The chain moves to
 * the Delta matrix (for good) when fewer than switch_num proposals in
 * switch_den were accepted over the last 8192 iterations (switch_num = 0:
 * never; switch_num < 0: from the first iteration).  Returns 0, or -1 on bad
 * arguments or memory.
 */
int cmp_sa_run(int32_t n, const int32_t *A, const int32_t *B, int32_t *p, cmp_state *st, uint64_t iters,
               uint64_t t_end, double T0, double alpha, uint64_t seed, uint32_t chain_id, int32_t switch_num,
               int32_t switch_den)
{
    if (n < 2 || t_end > iters || st->t > t_end || !(T0 > 0.0) || !(alpha > 0.0) || alpha > 1.0 || switch_den <= 0)
        return -1;
    const int64_t nn = (int64_t)n * n, m = (int64_t)n * (n - 1) / 2;
    chain c;
    c.n = n;
    c.A = A;
    c.At = malloc(sizeof(int32_t) * nn);
    c.Bp = malloc(sizeof(int32_t) * nn);
    c.Bt = malloc(sizeof(int32_t) * nn);
    c.D = malloc(sizeof(int64_t) * (m > 0 ? m : 1));
    c.rowoff = malloc(sizeof(int64_t) * n);
    int64_t *vec = malloc(sizeof(int64_t) * 4 * n);
    const uint64_t nh = ((iters + (1ull << 20) - 1) >> 20) ? ((iters + (1ull << 20) - 1) >> 20) : 1;
    double *L = malloc(sizeof(double) * (2048 + nh));
    if (!c.At || !c.Bp || !c.Bt || !c.D || !c.rowoff || !vec || !L) {
        free(c.At); free(c.Bp); free(c.Bt); free(c.D); free(c.rowoff); free(vec); free(L);
        return -1;
    }
    double *M = L + 1024, *H = L + 2048;
    L[0] = 1.0;
    for (int j = 1; j < 1024; ++j) L[j] = L[j - 1] * alpha;
    const double sm = L[1023] * alpha;
    M[0] = 1.0;
    for (int j = 1; j < 1024; ++j) M[j] = M[j - 1] * sm;
    const double sh = M[1023] * sm;
    H[0] = 1.0;
    for (uint64_t j = 1; j < nh; ++j) H[j] = H[j - 1] * sh;

    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            c.At[(int64_t)j * n + i] = A[(int64_t)i * n + j];
            const int32_t b = B[(int64_t)p[i] * n + p[j]];
            c.Bp[(int64_t)i * n + j] = b;
            c.Bt[(int64_t)j * n + i] = b;
        }
    for (int r = 0; r < n; ++r) c.rowoff[r] = (int64_t)r * (2 * n - r - 1) / 2;

    int delta_mode = switch_num < 0;
    if (delta_mode) { build_delta(&c); st->delta_mode_at = st->t; }
    int64_t idx = (int64_t)(st->t % (uint64_t)m);
    int r = 0;
    while (idx >= c.rowoff[r] + (n - 1 - r)) ++r;
    int s = r + 1 + (int)(idx - c.rowoff[r]);
    uint32_t win_it = 0, win_acc = 0;

    for (uint64_t t = st->t; t < t_end; ++t) {
        const int64_t d = delta_mode ? c.D[idx] : swap_cost(&c, r, s);
        int accept = d <= 0;
        if (!accept) {
            const double T = ((T0 * H[t >> 20]) * M[(t >> 10) & 1023]) * L[t & 1023];
            /* log r > -36.74 for every draw: a larger delta / T is rejected
               without the draw (the margin covers the rounding of both sides) */
            if ((double)d <= 36.8 * T * 1.000001) {
                const double z = (double)d / T + log(draw_r(seed, chain_id, t));
                if (fabs(z) < 1e-12) st->near_ties++;
                accept = z < 0.0;
            }
        }
        if (accept) {
            const int32_t tmp = p[r];
            p[r] = p[s];
            p[s] = tmp;
            apply_swap(&c, r, s);
            if (delta_mode) update_delta(&c, r, s, d, vec, vec + n, vec + 2 * n, vec + 3 * n);
            st->cost += d;
            st->accepts++;
            st->hash += fingerprint(t, r, s, d);
            if (st->cost < st->best_cost) { st->best_cost = st->cost; st->best_iter = t + 1; }
            win_acc++;
        }
        if (++s == n) {
            if (++r == n - 1) r = 0;
            s = r + 1;
        }
        if (++idx == m) idx = 0;
        if (!delta_mode && switch_num > 0 && ++win_it == 8192) {
            if ((int64_t)win_acc * switch_den < (int64_t)switch_num * 8192) {
                build_delta(&c);
                delta_mode = 1;
                st->delta_mode_at = t + 1;
            }
            win_it = win_acc = 0;
        }
    }
    st->t = t_end;
    free(c.At); free(c.Bp); free(c.Bt); free(c.D); free(c.rowoff); free(vec); free(L);
    return 0;
}

/* Fresh state at p: the cost of Eq. (1). */
void cmp_state_init(int32_t n, const int32_t *A, const int32_t *B, const int32_t *p, cmp_state *st)
{
    int64_t cost = 0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) cost += (int64_t)A[(int64_t)i * n + j] * B[(int64_t)p[i] * n + p[j]];
    memset(st, 0, sizeof *st);
    st->cost = st->best_cost = cost;
    st->delta_mode_at = ~0ull;
}
