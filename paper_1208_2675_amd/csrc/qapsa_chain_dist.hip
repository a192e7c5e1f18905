// qapsa_chain_dist.hip -- one annealing chain spread over G workgroups, for
// symmetric instances too large for one CU (N up to about 3000 on 256 CUs).
//
// Steps (b)-(e) of Sec. 2.2 with the Delta matrix kept for every pair.  The
// state is split by rows: workgroup w owns rows r = w, w + G, w + 2G, ... of
// the full symmetric Delta matrix (both halves are stored, so a workgroup
// holds complete rows), of A and of B', all resident in its LDS; p is
// replicated.  Nothing of size O(N^2) crosses workgroups.  Per accepted swap
// (u, v):
//   - every workgroup reads rows u and v of A and of B (through the new p),
//     which are read-only in device memory and so need no exchange;
//   - it swaps columns u, v of its B' rows, corrects its pairs disjoint from
//     {u, v} in O(1) each (Sec. 3 (ii): only rows u, v of A and B' are needed,
//     the symmetric case) and recomputes Delta(r, u), Delta(r, v) of its rows
//     in O(N) (Sec. 3 (i)), publishing these 2 values per row;
//   - the owners of rows u and v are then stale for those rows; they copy the
//     published values in after the next grid barrier.  Until then the scan
//     reads a pair (r, s) from row r instead of row s when s is stale.
// The scan (Sec. 3 (ii)) tests a window of proposals against the current
// Delta: proposal (r, s), r < s, is tested by the owner of row s, so one
// window spreads over all workgroups; each contributes its first acceptance to
// a device-wide minimum.  One grid barrier (Sec. 3 (iii)) per scan window is
// the only synchronisation; the launch is cooperative, so every workgroup is
// resident (the paper's "blocks no more than multiprocessors").
#include <hip/hip_runtime.h>
#include <limits.h>

#include "qapsa_device.hpp"
#include "qapsa_internal.hpp"

namespace qapsa {

namespace {

typedef short v2i16 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint32_t dot4(uint32_t a, uint32_t b, uint32_t c) { return __builtin_amdgcn_udot4(a, b, c, false); }

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

__device__ __forceinline__ unsigned long long wave_min64(unsigned long long v)
{
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ uint32_t rs32(int n, int r) { return (uint32_t)r * (uint32_t)(2 * n - r - 1) >> 1; }

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

__device__ __forceinline__ int finish_sym(int S, int arr, int ars, int asr, int ass, int brr, int brs, int bsr, int bss)
{
    const int corner = (arr - ass) * (bss - brr) + (ars - asr) * (bsr - brs);
    const int row_r = (arr - asr) * (bsr - brr);
    const int row_s = (ars - ass) * (bss - brs);
    return 2 * (S - row_r - row_s) + corner;
}

// Wait until this wave's global stores have completed (vmcnt = 0).
__device__ __forceinline__ void wait_stores() { __builtin_amdgcn_s_waitcnt(0x0F70); }

__device__ __forceinline__ void put(int* p, int v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ __forceinline__ int get(int* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

struct Lds {
    int32_t* D;      // [R][n] full rows of Delta
    uint8_t* Ab;     // [R][P] rows of A - a_min
    uint8_t* Bb;     // [R][P] rows of B' - b_min
    uint8_t* Su;     // [P] row u of A - a_min
    uint8_t* Sv;
    uint8_t* Tu;     // [P] row u of B' - b_min after the swap
    uint8_t* Tv;
    uint32_t* abp;   // [n] (A[u][k]-A[v][k]) twice, as int16 pair
    uint32_t* bbp;   // [n] (B'[u][k]-B'[v][k]) twice
    int16_t* ps;     // [n]
};

__host__ __device__ inline size_t a16(size_t x) { return (x + 15) & ~(size_t)15; }

__host__ __device__ inline size_t dist_layout(int n, int G, int q, char* base, Lds* L)
{
    const size_t R = (size_t)(n + G - 1) / G, P = 4 * (size_t)q;
    size_t off = 0;
    auto take = [&](size_t b) { char* p = base ? base + off : nullptr; off = a16(off + b); return p; };
    char* d = take(4 * R * n);
    char* ab = take(R * P);
    char* bb = take(R * P);
    char* su = take(P);
    char* sv = take(P);
    char* tu = take(P);
    char* tv = take(P);
    char* abp = take(4 * (size_t)n);
    char* bbp = take(4 * (size_t)n);
    char* ps = take(2 * (size_t)n);
    if (L) {
        L->D = (int32_t*)d; L->Ab = (uint8_t*)ab; L->Bb = (uint8_t*)bb;
        L->Su = (uint8_t*)su; L->Sv = (uint8_t*)sv; L->Tu = (uint8_t*)tu; L->Tv = (uint8_t*)tv;
        L->abp = (uint32_t*)abp; L->bbp = (uint32_t*)bbp; L->ps = (int16_t*)ps;
    }
    return off;
}

constexpr int kRec = 64;
struct Rec {
    uint64_t t;
    uint32_t uv;
    int32_t d;
};

__global__ void __launch_bounds__(1024) k_chain_dist(DistArgs a)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ unsigned long long s_key;
    __shared__ int s_ok;
    __shared__ int s_self[2];
    __shared__ int s_ntie;
    __shared__ unsigned long long s_tie_j[8];
    __shared__ int s_tie_d[8];
    __shared__ double s_tie_z[8];
    __shared__ Rec s_rec[kRec];
    __shared__ unsigned long long s_prof[QAP_PHASES];

    const int n = a.n, G = gridDim.x, w = blockIdx.x;
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = uni(tid >> 6), nwaves = nt >> 6;
    const int q = a.quads, P = 4 * q;
    const int Rw = (n - w + G - 1) / G;          // rows owned by this workgroup
    const int C = Rw;                             // columns s = w + G c of this workgroup (same count)
    const uint32_t m = (uint32_t)((int64_t)n * (n - 1) / 2);
    Lds L;
    dist_layout(n, G, q, smem, &L);
    DistWs* ws = a.ws;
    int* X = a.X;                                 // [2 parities][2 rows][n]

    const bool prof = a.prof != nullptr && w == 0;
    if (tid < QAP_PHASES) s_prof[tid] = 0;
    unsigned long long prof_last = prof ? clock64() : 0;
    const unsigned long long prof_start = prof_last;
    auto mark = [&](int k) {
        if (prof && tid == 0) {
            const unsigned long long now = clock64();
            atomicAdd(&s_prof[k], now - prof_last);
            prof_last = now;
        }
    };
    auto bump = [&](int k, unsigned long long x) { if (prof && tid == 0) atomicAdd(&s_prof[k], x); };

    // ---------------------------------------------------------------- load
    if (tid == 0) { s_ok = 1; s_ntie = 0; }
    __syncthreads();
    for (int e = tid; e < Rw * n; e += nt) {
        const int lr = e / n, s = e - lr * n, r = w + G * lr;
        int d = 0;
        if (s > r) d = a.delta[rs32(n, r) + s - r - 1];
        else if (s < r) d = a.delta[rs32(n, s) + r - s - 1];
        L.D[e] = d;
    }
    for (int e = tid; e < Rw * P; e += nt) {
        const int lr = e / P, k = e - lr * P, r = w + G * lr;
        int av = 0, bv = 0;
        if (k < n) {
            av = a.A[r * n + k] - a.a_min;
            bv = a.Bp[r * n + k] - a.b_min;
            if ((av | bv) & ~0xff) s_ok = 0;
        }
        L.Ab[e] = (uint8_t)av;
        L.Bb[e] = (uint8_t)bv;
    }
    for (int k = tid; k < P; k += nt) { L.Su[k] = 0; L.Sv[k] = 0; L.Tu[k] = 0; L.Tv[k] = 0; }
    for (int i = tid; i < n; i += nt) {
        const int pi = a.p[i];
        if (pi < 0 || pi >= n) s_ok = 0;   // p indexes B below
        L.ps[i] = (int16_t)pi;
    }
    const qap_chain_state st0 = *a.state;
    __syncthreads();
    if (!s_ok || st0.status != QAP_OK) {
        if (w == 0 && tid == 0) a.state->status = st0.status != QAP_OK ? st0.status : QAP_E_INVAL;
        return;   // every workgroup takes the same branch: the instance and state are shared
    }
    if (tid == 0) mark(QAP_PH_IO);

    const uint64_t t_end = a.t_end;
    const double T0 = a.T0;
    const double* __restrict__ temps = a.temps;
    uint64_t t = st0.t;
    unsigned long long accepts = st0.accepts, hash = st0.hash, best_iter = st0.best_iter;
    long long cost = st0.cost, best = st0.best_cost;
    uint32_t idx0 = (uint32_t)(t % m);
    int r0, s0;
    pair_of_u(n, idx0, r0, s0);
    unsigned long long epoch = 0;
    int kb = 0, par = 0;
    int pu = -1, pv = -1, pd = 0, ppar = 0;       // stale rows of the last swap, its Delta, its X parity
    uint32_t kwin = a.kmin;
    int nrec = 0;
    bool alive = true;

    auto grid_sync = [&]() -> bool {
        wait_stores();
        __syncthreads();
        if (tid == 0) {
            epoch += 1;
            const unsigned long long target = epoch * (unsigned long long)G;
            __hip_atomic_fetch_add(&ws->count, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            uint64_t spins = 0;
            int ok = 1;
            while (__hip_atomic_load(&ws->count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > a.spin_limit || get(&ws->err)) { ok = 0; break; }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            if (!ok) put(&ws->err, 1);
            s_ok = ok;
        }
        __syncthreads();
        return s_ok != 0;
    };

    auto flush = [&]() {
        if (w == 0 && wave == 0) {
            uint64_t h = 0;
            if (lane < nrec) {
                const Rec r = s_rec[lane];
                h = accept_fingerprint(r.t, (int)(r.uv >> 16), (int)(r.uv & 0xffff), r.d);
            }
            const uint64_t x0 = (uint32_t)wave_sum((int)(h & 0x3fffff));
            const uint64_t x1 = (uint32_t)wave_sum((int)((h >> 22) & 0x3fffff));
            const uint64_t x2 = (uint32_t)wave_sum((int)(h >> 44));
            hash += x0 + (x1 << 22) + (x2 << 44);
        }
        nrec = 0;
    };

    auto refresh = [&]() {   // copy the published Delta(., u), Delta(., v) into stale own rows
        if (pu < 0) return;
        for (int which = 0; which < 2; ++which) {
            const int x = which == 0 ? pu : pv, y = which == 0 ? pv : pu;
            if (x % G != w) continue;
            int32_t* row = L.D + (x / G) * n;
            int* src = X + (ppar * 2 + which) * n;
            for (int s = tid; s < n; s += nt) {
                if (s == x) row[s] = 0;
                else if (s == y) row[s] = -pd;
                else row[s] = get(src + s);
            }
        }
        pu = pv = -1;
        __syncthreads();
    };

    while (alive && t < t_end) {
        // ------------------------------------------------------------ scan
        const uint32_t W = (uint32_t)min<uint64_t>(min<uint64_t>((uint64_t)kwin, t_end - t), (uint64_t)m);
        const int32_t bound = reject_bound(temperature(temps, T0, t));
        unsigned long long mine = ~0ull;
        __syncthreads();   // everyone has read the previous window's LDS results
        if (tid == 0) { s_key = ~0ull; s_ntie = 0; }
        __syncthreads();
        auto test = [&](uint32_t j, int d) {
            bool acc = d <= 0;
            if (!acc && d <= bound) {
                const uint64_t tt = t + j;
                double z;
                acc = metropolis_positive(d, temperature(temps, T0, tt), uniform_r(a.seed, a.chain_id, tt), &z);
                if (fabs(z) < kNearTie) {
                    const int slot = atomicAdd(&s_ntie, 1);
                    if (slot < 8) { s_tie_j[slot] = j; s_tie_d[slot] = d; s_tie_z[slot] = z; }
                }
            }
            if (acc) {
                const unsigned long long key = ((unsigned long long)j << 32) | (uint32_t)d;
                mine = key < mine ? key : mine;
            }
        };
        // proposals (r, s) with s owned here, r < s, in the window.  The rows of
        // the window are r0, r0 + 1, ... cyclically; row offset n - 1 is row r0
        // again, for a window that wraps round to the pairs before (r0, s0).
        if (C > 0) {
            const int rows_per_pass = max(1, nt / C);
            const int i_loc = tid / C, c = tid - i_loc * C;
            const int s = w + G * c;
            for (int ib = 0; ib <= n - 1; ib += rows_per_pass) {
                if (ib > 0) {
                    const int rb = (r0 + ib) % (n - 1);
                    const uint32_t jb = (rs32(n, rb) + m - idx0) % m;
                    if (jb >= W) break;
                }
                const int i = ib + i_loc;
                if (i_loc >= rows_per_pass || i > n - 1) continue;
                const int r = (r0 + i) % (n - 1);
                bool ok = s > r && s < n;
                if (i == 0) ok = ok && s >= s0;
                if (i == n - 1) ok = ok && s < s0;
                if (!ok) continue;
                const uint32_t j = (rs32(n, r) + (uint32_t)(s - r - 1) + m - idx0) % m;
                if (j >= W) continue;
                if (s != pu && s != pv) test(j, L.D[(s / G) * n + r]);
                else if (r == pu && s == pv) test(j, -pd);
            }
        }
        // proposals (r, x) with x a stale row and r owned here: read from row r
        if (pu >= 0) {
            for (int lr = tid; lr < 2 * Rw; lr += nt) {
                const int rr = w + G * (lr >> 1), x = (lr & 1) ? pv : pu;
                if (rr == pu || rr == pv || x <= rr) continue;
                const uint32_t j = (rs32(n, rr) + (uint32_t)(x - rr - 1) + m - idx0) % m;
                if (j < W) test(j, L.D[(lr >> 1) * n + x]);
            }
        }
        mine = wave_min64(mine);
        if (lane == 0 && mine != ~0ull) atomicMin(&s_key, mine);
        __syncthreads();
        if (tid == 0 && s_key != ~0ull)
            __hip_atomic_fetch_min(&ws->key[kb], s_key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (tid == 0) mark(QAP_PH_DELTA_SCAN);
        alive = grid_sync();
        if (!alive) break;
        const unsigned long long key = __hip_atomic_load(&ws->key[kb], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (w == 0 && tid == 0)   // the buffer of two windows ago: everyone has read it by now
            __hip_atomic_store(&ws->key[kb == 0 ? 2 : kb - 1], ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        kb = kb == 2 ? 0 : kb + 1;
        const uint32_t jstar = key == ~0ull ? UINT_MAX : (uint32_t)(key >> 32);
        // near ties a sequential run would have met
        const int ntie = min(s_ntie, 8);
        if (tid < ntie && s_tie_j[tid] <= (jstar == UINT_MAX ? W - 1 : jstar)) {
            const unsigned long long slot = atomicAdd((unsigned long long*)&ws->nties, 1ull);
            if (a.ties && st0.near_ties + slot < a.tie_cap)
                a.ties[st0.near_ties + slot] = qap_near_tie{t + s_tie_j[tid], (int64_t)s_tie_d[tid], s_tie_z[tid]};
        }
        if (tid == 0) { mark(QAP_PH_RESERVED); bump(QAP_PH_N_SCAN_STEPS, 1); }
        refresh();
        if (jstar == UINT_MAX) {
            t += W;
            idx0 = (uint32_t)(((uint64_t)idx0 + W) % m);
            pair_of_u(n, idx0, r0, s0);
            kwin = min<uint64_t>((uint64_t)kwin * 2, (uint64_t)a.kmax);
            continue;
        }

        // ------------------------------------------------------------ accept
        const int dstar = (int)(uint32_t)key;
        const uint64_t tstar = t + jstar;
        uint32_t istar = idx0 + jstar;
        if (istar >= m) istar -= m;
        int u, v;
        pair_of_u(n, istar, u, v);
        cost += dstar;
        accepts += 1;
        if (cost < best) { best = cost; best_iter = tstar + 1; }
        if (w == 0 && tid == 0) {
            if (a.acc_log && accepts - 1 < a.acc_cap) {
                int64_t* e = a.acc_log + 4 * (accepts - 1);
                e[0] = (int64_t)tstar; e[1] = u; e[2] = v; e[3] = dstar;
            }
            s_rec[nrec] = Rec{tstar, ((uint32_t)u << 16) | (uint32_t)v, dstar};
        }
        nrec += 1;
        if (tid == 0) { const int16_t x = L.ps[u]; L.ps[u] = L.ps[v]; L.ps[v] = x; }
        __syncthreads();
        const int pu_new = L.ps[u], pv_new = L.ps[v];
        for (int k = tid; k < n; k += nt) {
            const int pk = L.ps[k];
            L.Su[k] = (uint8_t)(a.A[u * n + k] - a.a_min);
            L.Sv[k] = (uint8_t)(a.A[v * n + k] - a.a_min);
            L.Tu[k] = (uint8_t)(a.B[pu_new * n + pk] - a.b_min);
            L.Tv[k] = (uint8_t)(a.B[pv_new * n + pk] - a.b_min);
        }
        __syncthreads();
        // own rows of B': rows u, v are replaced, the others swap columns u, v
        for (int e = tid; e < Rw * n; e += nt) {
            const int lr = e / n, k = e - lr * n, r = w + G * lr;
            uint8_t* row = L.Bb + lr * P;
            if (r == u) row[k] = L.Tu[k];
            else if (r == v) row[k] = L.Tv[k];
            else if (k == u) { const uint8_t x = row[u]; row[u] = row[v]; row[v] = x; }
        }
        for (int k = tid; k < n; k += nt) {
            const int da = (int)L.Su[k] - (int)L.Sv[k], db = (int)L.Tu[k] - (int)L.Tv[k];
            L.abp[k] = (uint32_t)(uint16_t)da | ((uint32_t)(uint16_t)da << 16);
            L.bbp[k] = (uint32_t)(uint16_t)db | ((uint32_t)(uint16_t)db << 16);
        }
        if (wave == 0 || wave == (nwaves > 1 ? 1 : 0)) {
            const uint8_t* x = (wave == 0) ? L.Su : L.Sv;
            const uint8_t* y = (wave == 0) ? L.Tu : L.Tv;
            uint32_t acc = 0;
            for (int k = lane; k < q; k += 64) acc = dot4(((const uint32_t*)x)[k], ((const uint32_t*)y)[k], acc);
            const int sd = wave_sum((int)acc);
            if (lane == 0) s_self[wave == 0 ? 0 : 1] = sd;
            if (nwaves == 1) {
                uint32_t acc2 = 0;
                for (int k = lane; k < q; k += 64) acc2 = dot4(((const uint32_t*)L.Sv)[k], ((const uint32_t*)L.Tv)[k], acc2);
                const int sd2 = wave_sum((int)acc2);
                if (lane == 0) s_self[1] = sd2;
            }
        }
        if (nrec == kRec) flush();
        __syncthreads();

        // pairs of own rows disjoint from {u, v}
        for (int e = tid; e < Rw * n; e += nt) {
            const int lr = e / n, s = e - lr * n, r = w + G * lr;
            if (r == u || r == v || s == u || s == v || s == r) continue;
            const v2i16 ar = __builtin_bit_cast(v2i16, L.abp[r]), as = __builtin_bit_cast(v2i16, L.abp[s]);
            const v2i16 br = __builtin_bit_cast(v2i16, L.bbp[r]), bs = __builtin_bit_cast(v2i16, L.bbp[s]);
            L.D[e] = __builtin_amdgcn_sdot2(ar - as, bs - br, L.D[e], false);
        }
        // Delta(r, u), Delta(r, v) of own rows: one wave per row
        {
            const int su = s_self[0], sv = s_self[1];
            for (int lr = wave; lr < Rw; lr += nwaves) {
                const int r = w + G * lr;
                if (r == u || r == v) continue;
                const uint32_t* ar = (const uint32_t*)(L.Ab + lr * P);
                const uint32_t* br = (const uint32_t*)(L.Bb + lr * P);
                uint32_t pu_ = 0, pv_ = 0, self = 0;
                for (int k = lane; k < q; k += 64) {
                    const uint32_t xa = ar[k], xb = br[k];
                    pu_ = dot4(xa, ((const uint32_t*)L.Tu)[k], pu_);
                    pu_ = dot4(((const uint32_t*)L.Su)[k], xb, pu_);
                    pv_ = dot4(xa, ((const uint32_t*)L.Tv)[k], pv_);
                    pv_ = dot4(((const uint32_t*)L.Sv)[k], xb, pv_);
                    self = dot4(xa, xb, self);
                }
                const int Pu = wave_sum((int)pu_), Pv = wave_sum((int)pv_), Sr = wave_sum((int)self);
                if (lane == 0) {
                    const uint8_t* A_r = L.Ab + lr * P;
                    const uint8_t* B_r = L.Bb + lr * P;
                    const int du = finish_sym(Pu - Sr - su, A_r[r], A_r[u], L.Su[r], L.Su[u], B_r[r], B_r[u], L.Tu[r], L.Tu[u]);
                    const int dv = finish_sym(Pv - Sr - sv, A_r[r], A_r[v], L.Sv[r], L.Sv[v], B_r[r], B_r[v], L.Tv[r], L.Tv[v]);
                    L.D[lr * n + u] = du;
                    L.D[lr * n + v] = dv;
                    put(X + (par * 2 + 0) * n + r, du);
                    put(X + (par * 2 + 1) * n + r, dv);
                }
            }
        }
        __syncthreads();
        pu = u; pv = v; pd = dstar; ppar = par;
        par ^= 1;
        t = tstar + 1;
        idx0 = istar + 1 == m ? 0 : istar + 1;
        r0 = u; s0 = v;
        if (++s0 == n) { if (++r0 == n - 1) r0 = 0; s0 = r0 + 1; }
        kwin = a.kmin;
        if (tid == 0) { mark(QAP_PH_DELTA_UPDATE); bump(QAP_PH_N_DELTA_ACC, 1); }
    }

    // ------------------------------------------------------------ write back
    if (alive) alive = grid_sync();   // the last swap's published values
    if (alive) refresh();
    if (w == 0 && nrec > 0) flush();
    for (int e = tid; e < Rw * n; e += nt) {
        const int lr = e / n, s = e - lr * n, r = w + G * lr;
        if (s > r) a.delta[rs32(n, r) + s - r - 1] = L.D[e];
    }
    for (int e = tid; e < Rw * n; e += nt) {
        const int lr = e / n, k = e - lr * n, r = w + G * lr;
        a.Bp[r * n + k] = (int32_t)L.Bb[lr * P + k] + a.b_min;
    }
    if (w == 0) {
        for (int i = tid; i < n; i += nt) a.p[i] = L.ps[i];
        if (tid == 0) {
            qap_chain_state st;
            st.t = t; st.accepts = accepts; st.hash = hash;
            st.near_ties = st0.near_ties + __hip_atomic_load((unsigned long long*)&ws->nties, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT);
            st.cost = cost; st.best_cost = best; st.best_iter = best_iter;
            st.status = alive ? QAP_OK : QAP_E_TIMEOUT;
            st.mode = QAP_MODE_DELTA;
            *a.state = st;
            mark(QAP_PH_IO);
            bump(QAP_PH_TOTAL, clock64() - prof_start);
        }
        if (prof) {
            __syncthreads();
            if (tid < QAP_PHASES) atomicAdd((unsigned long long*)&a.prof[tid], s_prof[tid]);
        }
    }
}

__global__ void k_ws_reset(DistWs* ws)
{
    ws->count = 0;
    ws->key[0] = ws->key[1] = ws->key[2] = ~0ull;
    ws->err = 0;
    ws->nties = 0;
}

}  // namespace

int dist_quads(int n) { return (n + 3) / 4; }

size_t lds_dist_bytes(int n, int G)
{
    return dist_layout(n, G, dist_quads(n), nullptr, nullptr);
}

int launch_chain_dist(const DistArgs& a0, int G, int threads, hipStream_t stream)
{
    DistArgs a = a0;
    a.quads = dist_quads(a.n);
    const size_t bytes = lds_dist_bytes(a.n, G);
    const void* fn = (const void*)k_chain_dist;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess)
        return QAP_E_DEVICE;
    hipLaunchKernelGGL(k_ws_reset, dim3(1), dim3(1), 0, stream, a.ws);
    void* kargs[] = {&a};
    if (hipLaunchCooperativeKernel(fn, dim3(G), dim3(threads), kargs, (unsigned)bytes, stream) != hipSuccess)
        return QAP_E_DEVICE;
    return QAP_OK;
}

}  // namespace qapsa
