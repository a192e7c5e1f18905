// qapsa_chain_wg.hip -- one annealing chain per workgroup, whole state in LDS.
//
// Steps (b)-(e) of Sec. 2.2 for instances whose A and B' value ranges fit a
// byte (entries are stored shifted by their minimum: every swap cost is a sum
// of products of differences of A entries and of B' entries, so the shift
// changes nothing) and whose matrices fit one CU's LDS (N up to about 155
// asymmetric, 195 symmetric).
//
// Two interchangeable ways to produce the swap cost of a proposal; both give
// exactly Delta(r,s) = C(p o (r s)) - C(p), so the run does not depend on which
// one is active:
//   scratch mode   the swap cost of each proposal is computed when it is met,
//                  in O(N) (the "traditional" evaluation of Sec. 2.1).  One
//                  wave per proposal; a workgroup tests as many consecutive
//                  proposals as it has waves and keeps the first acceptance.
//                  Used while the acceptance rate is high, where the Delta
//                  matrix would cost O(N^2) per accepted swap.
//   Delta mode     steps (b)-(d) of Sec. 2.2: Delta(r,s) is kept for every pair;
//                  the scan tests many proposals against the unchanged matrix
//                  and keeps the first acceptance (Sec. 3 (ii)); after an
//                  accepted swap (u,v) pairs disjoint from {u,v} get an O(1)
//                  correction from four staged vectors and pairs that meet
//                  {u,v} are recomputed in O(N) (Sec. 3 (i)).
// A chain starts in scratch mode and moves to Delta mode once the acceptance
// rate over a window of iterations falls under a threshold (or is pinned to one
// mode by a flag).
//
// The swap cost in O(N) uses dot products of byte rows (v_dot4_u32_u8):
//   sum_k (a_kr - a_ks)(b_ks - b_kr) = <a.r, b.s> + <a.s, b.r> - <a.r, b.r> - <a.s, b.s>
// over columns (rows of the transposes A^T, B'^T) plus the same over rows,
// less the k = r and k = s terms, plus the two terms of Eq. (1) whose indices
// both lie in {r, s}.
#include <hip/hip_runtime.h>
#include <limits.h>

#include "qapsa_device.hpp"
#include "qapsa_internal.hpp"

namespace qapsa {

namespace {

constexpr int kRing = 1024;          // thresholds tau_t kept ahead in scratch mode
constexpr int kRec = 64;             // accepted swaps buffered before they are hashed
constexpr int kSwitchWindow = 8192;  // iterations between acceptance-rate checks

typedef short v2i16 __attribute__((ext_vector_type(2)));

struct Rec {
    uint64_t t;
    uint32_t uv;   // u << 16 | v
    int32_t d;
};

struct Wg {
    uint8_t* Ab;   // A - a_min, rows of P bytes
    uint8_t* At;   // (A - a_min)^T             (asymmetric only)
    uint8_t* Bb;   // B' - b_min
    uint8_t* Bt;   // (B' - b_min)^T            (asymmetric only)
    int32_t* D;    // packed Delta
    uint32_t* abp; // staged (A[k][u]-A[k][v], A[u][k]-A[v][k]) as int16 pairs
    uint32_t* bbp; // staged (B'[k][u]-B'[k][v], B'[u][k]-B'[v][k])
    int32_t* tu;
    int32_t* tv;
    int32_t* tau;  // ring of acceptance thresholds
    int16_t* ps;   // p
    Rec* rec;
};

__host__ __device__ inline size_t a16(size_t x) { return (x + 15) & ~(size_t)15; }

// LDS layout of one chain.  With `gbase` (global scratch of wg_global_bytes)
// the read-only byte copies of A and A^T live there and Delta stays in the
// caller's buffer `gdelta`, so only B', B'^T and small vectors use LDS.
__host__ __device__ inline size_t wg_layout(int n, int q, bool sym, char* base, Wg* L,
                                           char* gbase = nullptr, int32_t* gdelta = nullptr, bool gmem = false)
{
    const size_t m = (size_t)n * (n - 1) / 2, P = 4 * (size_t)q;
    size_t off = 0;
    auto take = [&](size_t bytes) { char* p = base ? base + off : nullptr; off = a16(off + bytes); return p; };
    char* ab = gmem ? gbase : take(n * P);
    char* at = sym ? nullptr : (gmem ? (gbase ? gbase + n * P : nullptr) : take(n * P));
    char* bb = take(n * P);
    char* bt = sym ? nullptr : take(n * P);
    char* d = gmem ? (char*)gdelta : take(4 * m);
    char* abp = take(4 * (size_t)n);
    char* bbp = take(4 * (size_t)n);
    char* tu = take(4 * (size_t)n);
    char* tv = take(4 * (size_t)n);
    char* tau = take(4 * (size_t)kRing);
    char* ps = take(2 * (size_t)n);
    char* rec = take(sizeof(Rec) * kRec);
    if (L) {
        L->Ab = (uint8_t*)ab; L->At = (uint8_t*)at; L->Bb = (uint8_t*)bb; L->Bt = (uint8_t*)bt;
        L->D = (int32_t*)d; L->abp = (uint32_t*)abp; L->bbp = (uint32_t*)bbp;
        L->tu = (int32_t*)tu; L->tv = (int32_t*)tv; L->tau = (int32_t*)tau;
        L->ps = (int16_t*)ps; L->rec = (Rec*)rec;
    }
    return off;
}

__device__ __forceinline__ uint32_t dot4(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_udot4(a, b, c, false);
}

// Sum over the 64 lanes of a wave (DPP row shifts and broadcasts); every lane
// receives the total.
__device__ __forceinline__ int wave_sum(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);
    return __builtin_amdgcn_readlane(v, 63);
}

// Terms that the all-k dot products get wrong or miss for the pair (r, s):
// the k = r and k = s terms are dropped and the two terms of Eq. (1) with both
// indices in {r, s} are added.  Arguments are the shifted entries at the four
// positions (r,r), (r,s), (s,r), (s,s).
template <bool SYM>
__device__ __forceinline__ int finish_delta(int S, int arr, int ars, int asr, int ass,
                                            int brr, int brs, int bsr, int bss)
{
    const int corner = (arr - ass) * (bss - brr) + (ars - asr) * (bsr - brs);
    const int row_r = (arr - asr) * (bsr - brr);   // (a_rk - a_sk)(b_sk - b_rk) at k = r
    const int row_s = (ars - ass) * (bss - brs);   // ... at k = s
    if constexpr (SYM) {
        return 2 * (S - row_r - row_s) + corner;
    } else {
        const int col_r = (arr - ars) * (brs - brr);   // (a_kr - a_ks)(b_ks - b_kr) at k = r
        const int col_s = (asr - ass) * (bss - bsr);   // ... at k = s
        return S - row_r - row_s - col_r - col_s + corner;
    }
}

// Wave-uniform copies of values (scalar registers).
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Packed offset of row r (32-bit; the one-workgroup kernel has n <= 256).
__device__ __forceinline__ uint32_t rs32(int n, int r) { return (uint32_t)r * (uint32_t)(2 * n - r - 1) >> 1; }

// Pair (r, s) of packed index idx by binary search over row offsets.
__device__ __forceinline__ void pair_of_u(int n, uint32_t idx, int& r, int& s)
{
    int lo = 0, hi = n - 2;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (rs32(n, mid) <= idx) lo = mid; else hi = mid - 1;
    }
    r = lo;
    s = lo + 1 + (int)(idx - rs32(n, lo));
}

// Next pair in row-major cyclic order, k times.
__device__ __forceinline__ void advance_pair(int n, int& r, int& s, int k)
{
    for (int i = 0; i < k; ++i) {
        if (++s == n) {
            if (++r == n - 1) r = 0;
            s = r + 1;
        }
    }
}

inline size_t wg_global_bytes(int n, int q, bool sym) { return (sym ? 1 : 2) * (size_t)n * 4 * q; }

template <bool SYM, bool GMEM>
struct Chain {
    const ChainArgs& a;
    Wg L;
    int n, q, P;
    uint32_t m;
    int tid, nt, lane, wave, nwaves;

    __device__ Chain(const ChainArgs& args, char* smem) : a(args)
    {
        n = a.n;
        q = a.quads;
        P = 4 * q;
        m = (uint32_t)((int64_t)n * (n - 1) / 2);
        tid = threadIdx.x; nt = blockDim.x;
        lane = tid & 63; wave = uni(tid >> 6); nwaves = nt >> 6;
        wg_layout(n, q, SYM, smem, &L, (char*)a.gscratch, a.delta, GMEM);
    }

    __device__ __forceinline__ int Ae(int i, int j) const { return L.Ab[i * P + j]; }
    __device__ __forceinline__ int Be(int i, int j) const { return L.Bb[i * P + j]; }
    __device__ __forceinline__ const uint32_t* row(const uint8_t* M, int i) const
    {
        return (const uint32_t*)(M + i * P);
    }

    // Swap cost of pair (r, s), r != s (wave-uniform), for the current B'; one
    // wave, every lane returns it.
    __device__ int pair_delta(int r, int s) const
    {
        const uint32_t *ar = row(L.Ab, r), *as = row(L.Ab, s), *br = row(L.Bb, r), *bs = row(L.Bb, s);
        const uint32_t *cr = nullptr, *cs = nullptr, *dr = nullptr, *ds = nullptr;
        if constexpr (!SYM) { cr = row(L.At, r); cs = row(L.At, s); dr = row(L.Bt, r); ds = row(L.Bt, s); }
        uint32_t pos = 0, neg = 0;
        for (int k = lane; k < q; k += 64) {
            const uint32_t xr = ar[k], xs = as[k], yr = br[k], ys = bs[k];
            pos = dot4(xr, ys, pos); pos = dot4(xs, yr, pos);
            neg = dot4(xr, yr, neg); neg = dot4(xs, ys, neg);
            if constexpr (!SYM) {
                const uint32_t zr = cr[k], zs = cs[k], wr = dr[k], ws = ds[k];
                pos = dot4(zr, ws, pos); pos = dot4(zs, wr, pos);
                neg = dot4(zr, wr, neg); neg = dot4(zs, ws, neg);
            }
        }
        const int S = wave_sum((int)(pos - neg));
        return finish_delta<SYM>(S, Ae(r, r), Ae(r, s), Ae(s, r), Ae(s, s), Be(r, r), Be(r, s), Be(s, r), Be(s, s));
    }

    // For every s: tu[s] += (all-k dot sums of pair (u, s)) less the self terms
    // of u, likewise tv for v.  Lanes run over s; the quads of k are split into
    // chunks over the waves; partial sums meet in LDS atomics (tu, tv zero on
    // entry).
    __device__ void gemv_two(int u, int v) const
    {
        const uint32_t *au = row(L.Ab, u), *av = row(L.Ab, v), *bu = row(L.Bb, u), *bv = row(L.Bb, v);
        const uint32_t *cu = nullptr, *cv = nullptr, *du = nullptr, *dv = nullptr;
        if constexpr (!SYM) { cu = row(L.At, u); cv = row(L.At, v); du = row(L.Bt, u); dv = row(L.Bt, v); }
        const int sgroups = (n + 63) >> 6;
        const int nchunks = max(1, nwaves / sgroups);
        for (int item = wave; item < sgroups * nchunks; item += nwaves) {
            const int c = item / sgroups, g = item - c * sgroups;
            const int s = (g << 6) + lane;
            const int k0 = q * c / nchunks, k1 = q * (c + 1) / nchunks;
            if (s >= n) continue;
            const uint32_t *as = row(L.Ab, s), *bs = row(L.Bb, s);
            const uint32_t *cs = nullptr, *ds = nullptr;
            if constexpr (!SYM) { cs = row(L.At, s); ds = row(L.Bt, s); }
            uint32_t pu = 0, pv = 0, ng = 0;
#pragma unroll 4
            for (int k = k0; k < k1; ++k) {
                const uint32_t xs = as[k], ys = bs[k];
                const uint32_t xu = au[k], yu = bu[k], xv = av[k], yv = bv[k];
                pu = dot4(xu, ys, pu); pu = dot4(xs, yu, pu);
                pv = dot4(xv, ys, pv); pv = dot4(xs, yv, pv);
                ng = dot4(xs, ys, ng);
                if constexpr (!SYM) {
                    const uint32_t zs = cs[k], ws = ds[k];
                    const uint32_t zu = cu[k], wu = du[k], zv = cv[k], wv = dv[k];
                    pu = dot4(zu, ws, pu); pu = dot4(zs, wu, pu);
                    pv = dot4(zv, ws, pv); pv = dot4(zs, wv, pv);
                    ng = dot4(zs, ws, ng);
                }
            }
            atomicAdd(&L.tu[s], (int)(pu - ng));
            atomicAdd(&L.tv[s], (int)(pv - ng));
        }
    }

    // Self terms <a.x, b.x> (+ transposed) of row x, one wave.
    __device__ int self_dot(int x) const
    {
        const uint32_t *ax = row(L.Ab, x), *bx = row(L.Bb, x);
        const uint32_t *cx = nullptr, *dx = nullptr;
        if constexpr (!SYM) { cx = row(L.At, x); dx = row(L.Bt, x); }
        uint32_t acc = 0;
        for (int k = lane; k < q; k += 64) {
            acc = dot4(ax[k], bx[k], acc);
            if constexpr (!SYM) acc = dot4(cx[k], dx[k], acc);
        }
        return wave_sum((int)acc);
    }

    __device__ __forceinline__ int finish_row(int u, int s, int Su) const
    {
        return finish_delta<SYM>(Su, Ae(u, u), Ae(u, s), Ae(s, u), Ae(s, s), Be(u, u), Be(u, s), Be(s, u), Be(s, s));
    }

    // The full Delta matrix from scratch, two rows per pass.
    __device__ void build_delta(int* s_self)
    {
        for (int r0 = 0; r0 < n - 1; r0 += 2) {
            const int r1 = min(r0 + 1, n - 1);
            for (int s = tid; s < n; s += nt) { L.tu[s] = 0; L.tv[s] = 0; }
            if (wave == 0) { const int x = self_dot(r0); if (lane == 0) s_self[0] = x; }
            if (wave == (nwaves > 1 ? 1 : 0)) { const int x = self_dot(r1); if (lane == 0) s_self[1] = x; }
            __syncthreads();
            gemv_two(r0, r1);
            __syncthreads();
            const uint32_t b0 = rs32(n, r0) - r0 - 1, b1 = rs32(n, r1) - r1 - 1;
            for (int s = tid; s < n; s += nt) {
                if (s > r0) L.D[b0 + s] = finish_row(r0, s, L.tu[s] - s_self[0]);
                if (r1 != r0 && s > r1) L.D[b1 + s] = finish_row(r1, s, L.tv[s] - s_self[1]);
            }
            __syncthreads();
        }
    }

    // Swap rows u, v and columns u, v of B' (and of its transpose).
    __device__ void swap_bprime(int u, int v) const
    {
        uint8_t* B = L.Bb;
        uint8_t* T = L.Bt;
        for (int k = tid; k < n; k += nt) {
            if (k == u || k == v) continue;
            uint8_t x = B[u * P + k]; B[u * P + k] = B[v * P + k]; B[v * P + k] = x;
            x = B[k * P + u]; B[k * P + u] = B[k * P + v]; B[k * P + v] = x;
            if constexpr (!SYM) {
                x = T[u * P + k]; T[u * P + k] = T[v * P + k]; T[v * P + k] = x;
                x = T[k * P + u]; T[k * P + u] = T[k * P + v]; T[k * P + v] = x;
            }
        }
        if (tid == nt - 1) {   // the four corners, away from thread 0's scalar work
            uint8_t x = B[u * P + u]; B[u * P + u] = B[v * P + v]; B[v * P + v] = x;
            x = B[u * P + v]; B[u * P + v] = B[v * P + u]; B[v * P + u] = x;
            if constexpr (!SYM) {
                x = T[u * P + u]; T[u * P + u] = T[v * P + v]; T[v * P + v] = x;
                x = T[u * P + v]; T[u * P + v] = T[v * P + u]; T[v * P + u] = x;
            }
        }
    }

    // Acceptance threshold of iteration t: the largest Delta that Eq. (2) accepts
    // (Eq. (2) is monotone in Delta).  *exact is set when T_t is so large that
    // near ties cannot be located from the threshold alone.
    __device__ int32_t threshold(uint64_t t, bool* exact) const
    {
        const double T = temperature(a.temps, a.T0, t);
        const double y = log(uniform_r(a.seed, a.chain_id, t));
        if (!(T <= 1e9)) *exact = true;
        const double xs = -y * T;
        int64_t d = xs >= 2147483647.0 ? 2147483647 : (int64_t)xs;
        auto acc = [&](int64_t dd) { return dd <= 0 || ((double)dd / T + y) < 0.0; };
        while (d < 2147483647 && acc(d + 1)) ++d;
        while (d > 0 && !acc(d)) --d;
        return (int32_t)d;
    }
};

template <bool SYM, bool GMEM>
__device__ void chain_run(const ChainArgs& a, char* smem)
{
    // Cross-wave exchange only; the chain's scalars live in registers of every
    // thread (all threads follow the same uniform control flow and apply the
    // same updates).
    __shared__ unsigned long long s_key[3];   // (winner << 32 | its Delta), min-reduced
    __shared__ unsigned long long s_ties;
    __shared__ int s_flag;
    __shared__ int s_self[2];
    __shared__ unsigned long long s_prof[QAP_PHASES];

    Chain<SYM, GMEM> C(a, smem);
    const Wg& L = C.L;
    const int n = C.n, P = C.P, tid = C.tid, nt = C.nt, lane = C.lane, wave = C.wave, nwaves = C.nwaves;
    const uint32_t m = C.m;

    // phase counters: thread 0 adds to LDS without waiting for the result
    const bool prof = a.prof != nullptr;
    if (tid < QAP_PHASES) s_prof[tid] = 0;
    unsigned long long prof_last = prof ? clock64() : 0;
    const unsigned long long prof_start = prof_last;
    auto mark = [&](int k) {
        if (prof) {
            const unsigned long long now = clock64();
            atomicAdd(&s_prof[k], now - prof_last);
            prof_last = now;
        }
    };
    auto bump = [&](int k, unsigned long long x) { if (prof) atomicAdd(&s_prof[k], x); };

    // ------------------------------------------------------------------ load
    const qap_chain_state st0 = *a.state;
    if (tid == 0) { s_flag = 0; s_ties = st0.near_ties; }
    __syncthreads();
    for (int e = tid; e < n * P; e += nt) {
        const int i = e / P, j = e - i * P;
        int av = 0, bv = 0, at = 0, bt = 0;
        if (j < n) {
            av = a.A[i * n + j] - a.a_min;
            bv = a.Bp[i * n + j] - a.b_min;
            at = a.A[j * n + i] - a.a_min;
            bt = a.Bp[j * n + i] - a.b_min;
            if ((av | bv | at | bt) & ~0xff) s_flag = 1;
        }
        L.Ab[e] = (uint8_t)av;
        L.Bb[e] = (uint8_t)bv;
        if constexpr (!SYM) { L.At[e] = (uint8_t)at; L.Bt[e] = (uint8_t)bt; }
    }
    for (int i = tid; i < n; i += nt) L.ps[i] = (int16_t)a.p[i];
    if (tid < 3) s_key[tid] = ~0ull;
    __syncthreads();
    const int status = st0.status != QAP_OK ? st0.status : (s_flag ? (int)QAP_E_RANGE : (int)QAP_OK);
    if (status != QAP_OK) {
        if (tid == 0) a.state->status = status;
        return;
    }
    int mode = (a.flags & kFlagDeltaOnly) ? 1 : (a.flags & kFlagScratchOnly) ? 0 : st0.mode;
    if (mode == 1 && !GMEM) {   // the caller's Delta is valid for p after qap_delta_init and after every run
        for (uint32_t i = tid; i < m; i += nt) L.D[i] = a.delta[i];
        __syncthreads();
    }
    mark(QAP_PH_IO);

    const uint64_t t_end = a.t_end;
    const double T0 = a.T0;
    const double* __restrict__ temps = a.temps;
    const uint32_t nt_mod = (uint32_t)nt % m;
    uint64_t t = st0.t;
    unsigned long long accepts = st0.accepts, hash = st0.hash, best_iter = st0.best_iter;
    long long cost = st0.cost, best = st0.best_cost;
    int nrec = 0;
    uint32_t idx0 = (uint32_t)(t % m);      // packed index proposed at iteration t
    int r0, s0;                              // its pair
    pair_of_u(n, idx0, r0, s0);
    int buf = 0;
    int step_e = 1;
    uint64_t tau_base = ~0ull;               // the threshold ring covers [tau_base, tau_base + kRing)
    bool ring_exact = false;
    uint64_t win_iters = 0, win_acc = 0;
    int kround = nwaves < 4 ? nwaves : 4;    // proposals per scratch round (adapted to the acceptance rate)

    // hash the buffered accept records (wave 0); the 64-bit sum over lanes is
    // taken in three 22-bit slices so that no slice can carry out
    auto flush = [&]() {
        if (wave == 0) {
            uint64_t h = 0;
            if (lane < nrec) {
                const Rec r = L.rec[lane];
                h = accept_fingerprint(r.t, (int)(r.uv >> 16), (int)(r.uv & 0xffff), r.d);
            }
            const uint64_t x0 = (uint32_t)wave_sum((int)(h & 0x3fffff));
            const uint64_t x1 = (uint32_t)wave_sum((int)((h >> 22) & 0x3fffff));
            const uint64_t x2 = (uint32_t)wave_sum((int)(h >> 44));
            hash += x0 + (x1 << 22) + (x2 << 44);
        }
        nrec = 0;
    };

    // the swap (u, v) at iteration tt with cost change d: scalars, p and B'
    auto accept_common = [&](uint64_t tt, int u, int v, int d) {
        if (tid == 0) {
            const int16_t pu = L.ps[u], pv = L.ps[v];
            L.ps[u] = pv; L.ps[v] = pu;
            if (a.acc_log && accepts < a.acc_cap) {
                int64_t* e = a.acc_log + 4 * accepts;
                e[0] = (int64_t)tt; e[1] = u; e[2] = v; e[3] = d;
            }
            L.rec[nrec] = Rec{tt, ((uint32_t)u << 16) | (uint32_t)v, d};
        }
        cost += d;
        accepts += 1;
        nrec += 1;
        if (cost < best) { best = cost; best_iter = tt + 1; }
        C.swap_bprime(u, v);
    };

    auto advance = [&](uint64_t k) {   // move the proposal cursor k iterations on
        t += k;
        if (k >= m) k %= m;
        idx0 += (uint32_t)k;
        if (idx0 >= m) idx0 -= m;
        if (k < 64) advance_pair(n, r0, s0, (int)k);
        else pair_of_u(n, idx0, r0, s0);
    };

    auto take_key = [&]() -> unsigned long long {
        const unsigned long long key = s_key[buf];
        if (tid == 0) s_key[buf == 0 ? 2 : buf - 1] = ~0ull;   // the buffer of the step before, read by all
        buf = buf == 2 ? 0 : buf + 1;
        return key;
    };

    while (t < t_end) {
        if (mode == 0) {
            // ------------------------------------------------------ scratch mode
            const int K = (int)min<uint64_t>((uint64_t)kround, t_end - t);
            if (tau_base == ~0ull || t + K > tau_base + kRing) {
                tau_base = t;
                if (tid == 0) s_flag = 0;
                __syncthreads();
                bool ex = false;
                for (int i = tid; i < kRing; i += nt) {
                    const uint64_t tt = tau_base + i;
                    L.tau[i] = tt < a.iters ? C.threshold(tt, &ex) : 0;
                }
                if (ex) s_flag = 1;
                __syncthreads();
                ring_exact = s_flag != 0;
                if (tid == 0) mark(QAP_PH_SCRATCH_THRESH), bump(QAP_PH_N_THRESH, 1);
            }
            bool tie = false;
            double zt = 0.0;
            int dw = 0;
            if (wave < K) {
                int r = r0, s = s0;
                advance_pair(n, r, s, wave);
                const int32_t tau = L.tau[(uint32_t)(t - tau_base) + wave];
                dw = C.pair_delta(r, s);
                if (lane == 0) {
                    bool acc = dw <= tau;
                    if (dw > 0 && (ring_exact || (dw >= tau - 1 && dw <= tau + 2))) {
                        const uint64_t tw = t + wave;
                        const bool ex_acc = metropolis_positive(dw, temperature(temps, T0, tw),
                                                                uniform_r(a.seed, a.chain_id, tw), &zt);
                        if (ring_exact) acc = ex_acc;
                        tie = fabs(zt) < kNearTie;
                    }
                    if (acc) atomicMin(&s_key[buf], ((unsigned long long)wave << 32) | (uint32_t)dw);
                }
            }
            __syncthreads();
            const unsigned long long key = take_key();
            const int w = key == ~0ull ? -1 : (int)(key >> 32);
            if (tid == 0) mark(QAP_PH_SCRATCH_EVAL), bump(QAP_PH_N_ROUNDS, 1);
            if (tie && (w < 0 || wave <= w)) {   // near ties among the proposals a sequential run evaluates
                const unsigned long long slot = atomicAdd(&s_ties, 1ull);
                if (a.ties && slot < a.tie_cap) a.ties[slot] = qap_near_tie{t + wave, (int64_t)dw, zt};
            }
            if (w < 0) {
                advance(K);
                win_iters += K;
            } else {
                int u = r0, v = s0;
                advance_pair(n, u, v, w);
                accept_common(t + w, u, v, (int)(uint32_t)key);
                __syncthreads();
                if (nrec == kRec) flush();
                advance(w + 1);
                win_iters += w + 1;
                win_acc += 1;
                if (tid == 0) mark(QAP_PH_SCRATCH_ACCEPT), bump(QAP_PH_N_SCRATCH_ACC, 1);
            }
            if (win_iters >= kSwitchWindow) {
                // at high acceptance a few proposals per round suffice; at lower
                // acceptance every wave tests one
                kround = win_acc * 8 >= win_iters ? min(4, nwaves) : nwaves;
                if (!(a.flags & kFlagScratchOnly) && win_acc * 1000 < win_iters * (uint64_t)a.switch_permille) {
                    C.build_delta(s_self);
                    mode = 1;
                    step_e = 1;
                    if (tid == 0) mark(QAP_PH_BUILD), bump(QAP_PH_SWITCH_T, t);
                }
                win_iters = win_acc = 0;
            }
            continue;
        }

        // ------------------------------------------------------------ Delta mode
        const uint64_t rem = t_end - t;
        const uint64_t cap = (uint64_t)step_e * nt;
        const uint32_t W = (uint32_t)(rem < cap ? rem : cap);
        const int32_t bound = reject_bound(temperature(temps, T0, t));
        uint32_t idx_l = idx0 + tid;
        while (idx_l >= m) idx_l -= m;
        bool tie = false;
        {
            uint32_t idx = idx_l;
            unsigned long long mine = ~0ull;
            for (int e = 0; e < step_e; e += 4) {
                // four proposals per lane loaded together, then tested in order
                int32_t dv[4];
                uint32_t jv[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    jv[k] = (uint32_t)(e + k) * nt + tid;
                    dv[k] = (e + k < step_e && jv[k] < W) ? L.D[idx] : INT_MAX;
                    idx += nt_mod;
                    if (idx >= m) idx -= m;
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int32_t d = dv[k];
                    if (mine != ~0ull || d == INT_MAX) continue;
                    bool acc = d <= 0;
                    if (!acc && d <= bound) {
                        const uint64_t tt = t + jv[k];
                        double z;
                        acc = metropolis_positive(d, temperature(temps, T0, tt), uniform_r(a.seed, a.chain_id, tt), &z);
                        tie |= fabs(z) < kNearTie;
                    }
                    if (acc) mine = ((unsigned long long)jv[k] << 32) | (uint32_t)d;
                }
                if (mine != ~0ull) break;
            }
            if (mine != ~0ull) atomicMin(&s_key[buf], mine);
        }
        __syncthreads();
        const unsigned long long key = take_key();
        const uint32_t jstar = key == ~0ull ? UINT_MAX : (uint32_t)(key >> 32);
        if (tie) {
            const uint32_t limit = jstar == UINT_MAX ? W - 1 : jstar;
            uint32_t idx = idx_l;
            for (int e = 0; e < step_e; ++e) {
                const uint32_t j = (uint32_t)e * nt + tid;
                if (j > limit) break;
                const int32_t d = L.D[idx];
                if (d > 0 && d <= bound) {
                    const uint64_t tt = t + j;
                    double z;
                    metropolis_positive(d, temperature(temps, T0, tt), uniform_r(a.seed, a.chain_id, tt), &z);
                    if (fabs(z) < kNearTie) {
                        const unsigned long long slot = atomicAdd(&s_ties, 1ull);
                        if (a.ties && slot < a.tie_cap) a.ties[slot] = qap_near_tie{tt, (int64_t)d, z};
                    }
                }
                idx += nt_mod;
                if (idx >= m) idx -= m;
            }
        }
        if (tid == 0) {
            mark(QAP_PH_DELTA_SCAN);
            bump(QAP_PH_N_SCAN_STEPS, 1);
            bump(QAP_PH_N_SCANNED, jstar == UINT_MAX ? W : jstar + 1);
        }
        if (jstar == UINT_MAX) {
            advance(W);
            step_e = min(step_e * 2, a.max_step);
            continue;
        }
        step_e = 1;
        uint32_t istar = idx0 + (jstar % m);
        if (istar >= m) istar -= m;
        int u, v;
        pair_of_u(n, istar, u, v);
        const int dstar = (int)(uint32_t)key;
        accept_common(t + jstar, u, v, dstar);
        for (int k = tid; k < n; k += nt) { L.tu[k] = 0; L.tv[k] = 0; }
        __syncthreads();

        // staged differences (after the swap) and the self terms of u and v
        for (int k = tid; k < n; k += nt) {
            int a1, a2, b1, b2;
            if constexpr (SYM) {
                a1 = a2 = C.Ae(u, k) - C.Ae(v, k);
                b1 = b2 = C.Be(u, k) - C.Be(v, k);
            } else {
                a1 = L.At[u * P + k] - L.At[v * P + k];   // A[k][u] - A[k][v]
                a2 = C.Ae(u, k) - C.Ae(v, k);             // A[u][k] - A[v][k]
                b1 = L.Bt[u * P + k] - L.Bt[v * P + k];
                b2 = C.Be(u, k) - C.Be(v, k);
            }
            L.abp[k] = (uint32_t)(uint16_t)a1 | ((uint32_t)(uint16_t)a2 << 16);
            L.bbp[k] = (uint32_t)(uint16_t)b1 | ((uint32_t)(uint16_t)b2 << 16);
        }
        if (wave == 0) { const int x = C.self_dot(u); if (lane == 0) s_self[0] = x; }
        if (wave == (nwaves > 1 ? 1 : 0)) { const int x = C.self_dot(v); if (lane == 0) s_self[1] = x; }
        if (nrec == kRec) flush();
        __syncthreads();

        // pairs disjoint from {u, v}: lanes own columns s, waves walk rows r < s,
        // four rows at a time so that their loads overlap
        {
            const int nb = (n + 63) >> 6;
            for (int b = 0; b < nb; ++b) {
                const int s = (b << 6) + lane;
                const bool col_ok = s < n && s != u && s != v;
                const v2i16 as = __builtin_bit_cast(v2i16, col_ok ? L.abp[s] : 0u);
                const v2i16 bs = __builtin_bit_cast(v2i16, col_ok ? L.bbp[s] : 0u);
                const int rmax = min(n - 1, (b << 6) + 63);
                for (int r = wave; r < rmax; r += 4 * nwaves) {
                    int32_t dv[4];
                    v2i16 ar[4], br[4];
                    bool ok[4];
                    uint32_t off[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int rr = r + k * nwaves;
                        ok[k] = col_ok && rr < rmax && s > rr && rr != u && rr != v;
                        const int rc = rr < rmax ? rr : 0;
                        ar[k] = __builtin_bit_cast(v2i16, L.abp[rc]);
                        br[k] = __builtin_bit_cast(v2i16, L.bbp[rc]);
                        off[k] = rs32(n, rc) - rc - 1 + s;
                        dv[k] = ok[k] ? L.D[off[k]] : 0;
                    }
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (ok[k]) L.D[off[k]] = __builtin_amdgcn_sdot2(ar[k] - as, bs - br[k], dv[k], false);
                }
            }
        }
        // pairs that meet {u, v}
        C.gemv_two(u, v);
        __syncthreads();
        {
            const int su = s_self[0], sv = s_self[1];
            for (int s = tid; s < n; s += nt) {
                if (s == u || s == v) continue;
                const int lu = min(u, s), hu = max(u, s), lv = min(v, s), hv = max(v, s);
                const int du = C.finish_row(u, s, L.tu[s] - su);
                const int dv = C.finish_row(v, s, L.tv[s] - sv);
                L.D[rs32(n, lu) + hu - lu - 1] = du;
                L.D[rs32(n, lv) + hv - lv - 1] = dv;
            }
        }
        if (tid == 0) L.D[istar] = -dstar;
        __syncthreads();
        advance(jstar + 1);
        if (tid == 0) mark(QAP_PH_DELTA_UPDATE), bump(QAP_PH_N_DELTA_ACC, 1);
    }

    // ------------------------------------------------------------ write back
    __syncthreads();
    if (nrec > 0) flush();
    if (tid == 0) mark(QAP_PH_IO);
    if (mode == 0) C.build_delta(s_self);   // the caller's Delta stays valid in either mode
    __syncthreads();
    if (tid == 0) mark(QAP_PH_BUILD);
    if (!GMEM)
        for (uint32_t i = tid; i < m; i += nt) a.delta[i] = L.D[i];
    for (int e = tid; e < n * n; e += nt) {
        const int i = e / n, j = e - i * n;
        a.Bp[e] = (int32_t)L.Bb[i * P + j] + a.b_min;
    }
    for (int i = tid; i < n; i += nt) a.p[i] = L.ps[i];
    if (tid == 0) {
        qap_chain_state st;
        st.t = t; st.accepts = accepts; st.near_ties = s_ties; st.hash = hash;
        st.cost = cost; st.best_cost = best; st.best_iter = best_iter;
        st.status = QAP_OK;
        st.mode = mode;
        *a.state = st;
        mark(QAP_PH_IO);
        bump(QAP_PH_TOTAL, clock64() - prof_start);
    }
    if (prof) {
        __syncthreads();
        if (tid < QAP_PHASES) atomicAdd((unsigned long long*)&a.prof[tid], s_prof[tid]);
    }
}

template <bool SYM, bool GMEM>
__global__ void __launch_bounds__(1024) k_chain_wg(ChainArgs a)
{
    extern __shared__ __align__(16) char smem[];
    chain_run<SYM, GMEM>(a, smem);
}

// Many independent chains in one persistent launch: each workgroup takes the
// next chain from a device-wide queue and runs it (or its next slice) with the
// one-workgroup routine above.  One instantiation serves the chains whose
// state is all in LDS, the other those that keep Delta and A in device memory
// (a per-chain scratch); each skips the other kind, so both can walk the same
// descriptor array concurrently.
template <bool GMEM>
__global__ void __launch_bounds__(256) k_chain_batch(BatchArgs b)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ int s_idx;
    unsigned* next = &b.ws->next[GMEM ? 1 : 0];
    for (;;) {
        if (threadIdx.x == 0) s_idx = (int)atomicAdd(next, 1u);
        __syncthreads();
        const int idx = s_idx;
        __syncthreads();
        if (idx >= b.n_chains) break;
        const int c = b.order ? b.order[idx] : idx;
        const qap_chain_desc d = b.descs[c];
        if ((d.scratch != nullptr) != GMEM) continue;
        ChainArgs a{};
        a.n = d.n;
        a.quads = ((d.n + 3) / 4) | 1;
        a.max_step = 16;
        a.flags = d.flags;
        a.switch_permille = d.switch_permille ? d.switch_permille : 20;
        a.a_min = d.a_min;
        a.b_min = d.b_min;
        a.A = d.A; a.Bp = d.Bp; a.p = d.p; a.delta = d.delta; a.state = d.state;
        a.temps = d.temps;
        a.ties = d.ties; a.tie_cap = d.tie_cap;
        a.prof = b.prof;
        a.iters = d.iters;
        const uint64_t t_now = d.state->t;
        a.t_end = (b.slice && t_now + b.slice < d.t_end) ? t_now + b.slice : d.t_end;
        if (a.t_end < t_now) a.t_end = t_now;
        a.T0 = d.T0;
        a.seed = d.seed;
        a.chain_id = d.chain_id;
        a.gscratch = d.scratch;
        if (d.symmetric) chain_run<true, GMEM>(a, smem);
        else chain_run<false, GMEM>(a, smem);
        __syncthreads();
    }
}

__global__ void k_batch_reset(BatchWs* ws) { ws->next[0] = 0; ws->next[1] = 0; }

}  // namespace

int launch_chain_batch(const BatchArgs& b, int groups, int count_lds, int count_gmem, int threads,
                       size_t lds_bytes, size_t gmem_lds_bytes, hipStream_t stream)
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return QAP_E_DEVICE;
    auto size = [&](const void* fn, size_t bytes, int count, int* out) -> int {
        *out = 0;
        if (count == 0) return QAP_OK;
        if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess)
            return QAP_E_DEVICE;
        int g = groups;
        if (g <= 0) {
            int per_cu = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, bytes) != hipSuccess)
                return QAP_E_DEVICE;
            g = (per_cu < 1 ? 1 : per_cu) * cus;
        }
        *out = g > count ? count : g;
        return QAP_OK;
    };
    int groups_lds = 0, groups_gmem = 0;
    if (size((const void*)k_chain_batch<false>, lds_bytes, count_lds, &groups_lds) != QAP_OK ||
        size((const void*)k_chain_batch<true>, gmem_lds_bytes, count_gmem, &groups_gmem) != QAP_OK)
        return QAP_E_DEVICE;
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, stream, b.ws);
    BatchArgs args = b;
    void* kargs[] = {&args};
    if (groups_lds > 0 && groups_gmem > 0) {
        // the two kinds run side by side: fork onto a second stream, join back
        hipStream_t side;
        hipEvent_t fork, join;
        if (side_stream(&side, &fork, &join) != QAP_OK) return QAP_E_DEVICE;
        if (hipEventRecord(fork, stream) != hipSuccess || hipStreamWaitEvent(side, fork, 0) != hipSuccess)
            return QAP_E_DEVICE;
        if (hipLaunchKernel((const void*)k_chain_batch<true>, dim3(groups_gmem), dim3(threads), kargs,
                            gmem_lds_bytes, side) != hipSuccess)
            return QAP_E_DEVICE;
        if (hipLaunchKernel((const void*)k_chain_batch<false>, dim3(groups_lds), dim3(threads), kargs, lds_bytes,
                            stream) != hipSuccess)
            return QAP_E_DEVICE;
        if (hipEventRecord(join, side) != hipSuccess || hipStreamWaitEvent(stream, join, 0) != hipSuccess)
            return QAP_E_DEVICE;
        return QAP_OK;
    }
    if (groups_lds > 0 && hipLaunchKernel((const void*)k_chain_batch<false>, dim3(groups_lds), dim3(threads), kargs,
                                          lds_bytes, stream) != hipSuccess)
        return QAP_E_DEVICE;
    if (groups_gmem > 0 && hipLaunchKernel((const void*)k_chain_batch<true>, dim3(groups_gmem), dim3(threads), kargs,
                                           gmem_lds_bytes, stream) != hipSuccess)
        return QAP_E_DEVICE;
    return QAP_OK;
}

int wg_quads(int n)
{
    return ((n + 3) / 4) | 1;   // odd dword pitch: strided row reads hit distinct banks
}

size_t lds_wg_bytes(int n, bool symmetric, bool gmem)
{
    return wg_layout(n, wg_quads(n), symmetric, nullptr, nullptr, nullptr, nullptr, gmem);
}

size_t wg_scratch_bytes(int n, bool symmetric) { return wg_global_bytes(n, wg_quads(n), symmetric); }

int launch_chain_wg(const ChainArgs& a, bool symmetric, int threads, hipStream_t stream)
{
    const bool gmem = a.gscratch != nullptr;
    const size_t bytes = lds_wg_bytes(a.n, symmetric, gmem);
    const void* fn = symmetric ? (gmem ? (const void*)k_chain_wg<true, true> : (const void*)k_chain_wg<true, false>)
                               : (gmem ? (const void*)k_chain_wg<false, true> : (const void*)k_chain_wg<false, false>);
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess)
        return QAP_E_DEVICE;
    ChainArgs args = a;
    args.quads = wg_quads(a.n);
    void* kargs[] = {&args};
    if (hipLaunchKernel(fn, dim3(1), dim3(threads), kargs, bytes, stream) != hipSuccess) return QAP_E_DEVICE;
    return QAP_OK;
}

}  // namespace qapsa
