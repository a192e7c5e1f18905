// qapsa_chain_lds.hip -- one annealing chain per workgroup with its whole
// state (Delta, B', p and, when it fits, A) resident in LDS.
//
// This is steps (b)-(e) of Sec. 2.2 for instances small enough for one CU
// (N up to about 200 with 16-bit A and B' values):
//   scan    Sec. 3 (ii): the workgroup tests the next proposals in parallel
//           against the unchanged Delta and keeps the one that sequential
//           evaluation would have met first (smallest t).  Each lane tests
//           proposals t + e*threads + lane, so every step covers a contiguous
//           range of t; the first step with any acceptance holds the answer.
//   accept  swap p(u), p(v); swap rows u, v and columns u, v of B' (Eq. (3)).
//   update  Sec. 3 (i)-(ii): pairs disjoint from {u, v} get an O(1) correction
//           from four staged vectors; pairs that meet {u, v} are recomputed in
//           O(N) each (the general asymmetric form); Delta(u, v) becomes -Delta.
// Only workgroup barriers are needed; nothing leaves the CU until the end of
// the call, when Delta, B', p and the chain state are written back.
#include <hip/hip_runtime.h>
#include <limits.h>

#include "qapsa_device.hpp"
#include "qapsa_internal.hpp"

namespace qapsa {

namespace {

struct ChainLds {
    int32_t* D;     // packed Delta, m entries
    int16_t* Bs;    // B', n rows of `pitch`
    int16_t* As;    // A, n rows of `pitch` (null when A is read from global memory)
    int16_t* al1;   // A[k][u] - A[k][v]          (after the swap)
    int16_t* be1;   // B'[k][u] - B'[k][v]
    int16_t* al2;   // A[u][k] - A[v][k]          (asymmetric only)
    int16_t* be2;   // B'[u][k] - B'[v][k]
    int32_t* tu;    // partial sums of the touched pairs (u, s)
    int32_t* tv;    // and (v, s)
    int16_t* ps;    // p
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

__host__ __device__ inline size_t chain_layout(int n, int pitch, bool sym, bool a_lds, char* base,
                                               ChainLds* L)
{
    const size_t m = (size_t)n * (n - 1) / 2;
    size_t off = 0;
    auto take = [&](size_t bytes) { char* p = base ? base + off : nullptr; off = align16(off + bytes); return p; };
    char* d = take(4 * m);
    char* bs = take(2 * (size_t)n * pitch);
    char* as = a_lds ? take(2 * (size_t)n * pitch) : nullptr;
    char* al1 = take(2 * (size_t)n);
    char* be1 = take(2 * (size_t)n);
    char* al2 = sym ? nullptr : take(2 * (size_t)n);
    char* be2 = sym ? nullptr : take(2 * (size_t)n);
    char* tu = take(4 * (size_t)n);
    char* tv = take(4 * (size_t)n);
    char* ps = take(2 * (size_t)n);
    if (L) {
        L->D = (int32_t*)d; L->Bs = (int16_t*)bs; L->As = (int16_t*)as;
        L->al1 = (int16_t*)al1; L->be1 = (int16_t*)be1; L->al2 = (int16_t*)al2; L->be2 = (int16_t*)be2;
        L->tu = (int32_t*)tu; L->tv = (int32_t*)tv; L->ps = (int16_t*)ps;
    }
    return off;
}

template <typename T>
__device__ __forceinline__ void swap_lds(T& x, T& y) { T t = x; x = y; y = t; }

template <bool SYM, bool A_LDS>
__device__ void chain_body(const ChainArgs& a, char* smem)
{
    __shared__ unsigned long long s_t, s_acc, s_ties, s_hash, s_best_iter;
    __shared__ long long s_cost, s_best;
    __shared__ unsigned s_min[3];
    __shared__ int s_status;

    const int n = a.n;
    const uint32_t m = (uint32_t)((int64_t)n * (n - 1) / 2);
    const int P = a.pitch;
    const int tid = threadIdx.x, nt = blockDim.x;
    ChainLds L;
    chain_layout(n, P, SYM, A_LDS, smem, &L);

    auto Ag = [&](int i, int j) -> int {
        if constexpr (A_LDS) return L.As[i * P + j];
        else return a.A[(int64_t)i * n + j];
    };
    auto Bg = [&](int i, int j) -> int { return L.Bs[i * P + j]; };

    // ---------------------------------------------------------------- load
    for (uint32_t i = tid; i < m; i += nt) L.D[i] = a.delta[i];
    for (int e = tid; e < n * n; e += nt) {
        const int i = e / n, j = e - i * n;
        L.Bs[i * P + j] = (int16_t)a.Bp[e];
        if constexpr (A_LDS) L.As[i * P + j] = (int16_t)a.A[e];
    }
    for (int i = tid; i < n; i += nt) L.ps[i] = (int16_t)a.p[i];
    if (tid == 0) {
        const qap_chain_state st = *a.state;
        s_t = st.t; s_acc = st.accepts; s_ties = st.near_ties; s_hash = st.hash;
        s_cost = st.cost; s_best = st.best_cost; s_best_iter = st.best_iter;
        s_status = st.status != QAP_OK ? st.status : (st.mode == QAP_MODE_SCRATCH_STALE ? (int)QAP_E_STATE : QAP_OK);
        if (st.status == QAP_OK && s_status != QAP_OK) a.state->status = s_status;
        s_min[0] = s_min[1] = s_min[2] = UINT_MAX;
    }
    __syncthreads();
    if (s_status != QAP_OK) return;

    const uint64_t t_end = a.t_end;
    const double T0 = a.T0;
    const double* __restrict__ temps = a.temps;
    const uint32_t nt_mod = (uint32_t)nt % m;
    uint64_t t = s_t;
    uint32_t idx0 = (uint32_t)(t % m);
    const bool rnd = (a.flags & QAP_FLAG_RANDOM_ORDER) != 0;
    // pair number proposed at iteration t + j; idx is that of the row-major cursor
    auto pair_at = [&](uint32_t j, uint32_t idx) -> uint32_t {
        return rnd ? random_pair_index(a.seed, a.chain_id, t + j, m) : idx;
    };
    int step_e = 1;
    int buf = 0;

    while (t < t_end) {
        // ------------------------------------------------------------ scan
        const uint64_t rem = t_end - t;
        const uint64_t cap = (uint64_t)step_e * nt;
        const uint32_t W = (uint32_t)(rem < cap ? rem : cap);
        const int32_t bound = reject_bound(temperature(temps, T0, t));
        uint32_t cand = UINT_MAX;
        bool tie = false;
        {
            uint32_t idx = (uint32_t)(((uint64_t)idx0 + tid) % m);
            for (int e = 0; e < step_e; ++e) {
                const uint32_t j = (uint32_t)e * nt + tid;
                if (j >= W) break;
                const int32_t d = L.D[pair_at(j, idx)];
                bool acc = d <= 0;
                if (!acc && d <= bound) {
                    const uint64_t tt = t + j;
                    double z;
                    acc = metropolis_positive(d, temperature(temps, T0, tt),
                                              uniform_r(a.seed, a.chain_id, tt), &z);
                    tie |= fabs(z) < kNearTie;
                }
                if (acc) { cand = j; break; }
                idx += nt_mod;
                if (idx >= m) idx -= m;
            }
        }
        if (cand != UINT_MAX) atomicMin(&s_min[buf], cand);
        __syncthreads();
        const uint32_t jstar = s_min[buf];
        if (tid == 0) s_min[(buf + 2) % 3] = UINT_MAX;
        buf = (buf + 1) % 3;

        if (tie) {
            // near ties among the proposals a sequential run evaluates
            const uint32_t limit = jstar == UINT_MAX ? W - 1 : jstar;
            uint32_t idx = (uint32_t)(((uint64_t)idx0 + tid) % m);
            for (int e = 0; e < step_e; ++e) {
                const uint32_t j = (uint32_t)e * nt + tid;
                if (j > limit) break;
                const int32_t d = L.D[pair_at(j, idx)];
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

        if (jstar == UINT_MAX) {
            t += W;
            idx0 = (uint32_t)(((uint64_t)idx0 + W) % m);
            step_e = min(step_e * 2, a.max_step);
            continue;
        }

        // ---------------------------------------------------------- accept
        step_e = 1;
        const uint64_t tstar = t + jstar;
        const uint32_t istar = pair_at(jstar, (uint32_t)(((uint64_t)idx0 + jstar) % m));
        int u, v;
        pair_of(n, istar, u, v);
        const int32_t dstar = L.D[istar];

        if (tid == 0) {
            swap_lds(L.ps[u], L.ps[v]);
            s_cost += dstar;
            if (a.acc_log && s_acc < a.acc_cap) {
                int64_t* e = a.acc_log + 4 * s_acc;
                e[0] = (int64_t)tstar; e[1] = u; e[2] = v; e[3] = dstar;
            }
            s_acc += 1;
            s_hash += accept_fingerprint(tstar, u, v, dstar);
            if (s_cost < s_best) { s_best = s_cost; s_best_iter = tstar + 1; }
            swap_lds(L.Bs[u * P + u], L.Bs[v * P + v]);
            swap_lds(L.Bs[u * P + v], L.Bs[v * P + u]);
        }
        for (int k = tid; k < n; k += nt) {
            if (k != u && k != v) {
                swap_lds(L.Bs[u * P + k], L.Bs[v * P + k]);
                swap_lds(L.Bs[k * P + u], L.Bs[k * P + v]);
            }
            L.tu[k] = 0;
            L.tv[k] = 0;
        }
        __syncthreads();

        for (int k = tid; k < n; k += nt) {
            L.al1[k] = (int16_t)(Ag(k, u) - Ag(k, v));
            L.be1[k] = (int16_t)(Bg(k, u) - Bg(k, v));
            if constexpr (!SYM) {
                L.al2[k] = (int16_t)(Ag(u, k) - Ag(v, k));
                L.be2[k] = (int16_t)(Bg(u, k) - Bg(v, k));
            }
        }
        __syncthreads();

        // disjoint pairs: one wave per row r, lanes over s > r
        {
            const int wave = tid >> 6, lane = tid & 63, nwaves = nt >> 6;
            for (int r = wave; r < n - 1; r += nwaves) {
                if (r == u || r == v) continue;
                const int a1r = L.al1[r], b1r = L.be1[r];
                int a2r = 0, b2r = 0;
                if constexpr (!SYM) { a2r = L.al2[r]; b2r = L.be2[r]; }
                int32_t* Drow = L.D + (row_start(n, r) - (r + 1));
                for (int s = r + 1 + lane; s < n; s += 64) {
                    if (s == u || s == v) continue;
                    int32_t inc;
                    if constexpr (SYM) {
                        inc = 2 * (a1r - L.al1[s]) * (b1r - L.be1[s]);
                    } else {
                        inc = (a1r - L.al1[s]) * (b1r - L.be1[s]) + (a2r - L.al2[s]) * (b2r - L.be2[s]);
                    }
                    Drow[s] -= inc;
                }
            }
        }
        // touched pairs (u, s) and (v, s): lanes over s, k split into chunks
        {
            const int ns = (n + 63) & ~63;
            const int nchunks = nt >= ns ? nt / ns : 1;
            for (int slot = tid; slot < ns * nchunks; slot += nt) {
                const int c = slot / ns, s = slot - c * ns;
                if (s >= n) continue;
                const int k0 = (int)((int64_t)n * c / nchunks);
                const int k1 = (int)((int64_t)n * (c + 1) / nchunks);
                int32_t su = 0, sv = 0;
                for (int k = k0; k < k1; ++k) {
                    const int aks = Ag(k, s), bks = Bg(k, s);
                    const int aku = Ag(k, u), bku = Bg(k, u);
                    const int akv = Ag(k, v), bkv = Bg(k, v);
                    int xu = (aku - aks) * (bks - bku);
                    int xv = (akv - aks) * (bks - bkv);
                    if constexpr (!SYM) {
                        const int ask = Ag(s, k), bsk = Bg(s, k);
                        xu += (Ag(u, k) - ask) * (bsk - Bg(u, k));
                        xv += (Ag(v, k) - ask) * (bsk - Bg(v, k));
                    }
                    su += (k != u && k != s) ? xu : 0;
                    sv += (k != v && k != s) ? xv : 0;
                }
                atomicAdd(&L.tu[s], su);
                atomicAdd(&L.tv[s], sv);
            }
        }
        __syncthreads();

        for (int s = tid; s < n; s += nt) {
            if (s == u || s == v) continue;
            const int mul = SYM ? 2 : 1;
            {
                int val = mul * L.tu[s] + (Ag(u, u) - Ag(s, s)) * (Bg(s, s) - Bg(u, u));
                if constexpr (!SYM) val += (Ag(u, s) - Ag(s, u)) * (Bg(s, u) - Bg(u, s));
                const int lo = min(u, s), hi = max(u, s);
                L.D[row_start(n, lo) + hi - lo - 1] = val;
            }
            {
                int val = mul * L.tv[s] + (Ag(v, v) - Ag(s, s)) * (Bg(s, s) - Bg(v, v));
                if constexpr (!SYM) val += (Ag(v, s) - Ag(s, v)) * (Bg(s, v) - Bg(v, s));
                const int lo = min(v, s), hi = max(v, s);
                L.D[row_start(n, lo) + hi - lo - 1] = val;
            }
        }
        if (tid == 0) L.D[istar] = -dstar;
        __syncthreads();

        t = tstar + 1;
        idx0 = istar + 1 == m ? 0 : istar + 1;
    }

    // ------------------------------------------------------------ write back
    __syncthreads();
    for (uint32_t i = tid; i < m; i += nt) a.delta[i] = L.D[i];
    for (int e = tid; e < n * n; e += nt) {
        const int i = e / n, j = e - i * n;
        a.Bp[e] = L.Bs[i * P + j];
    }
    for (int i = tid; i < n; i += nt) a.p[i] = L.ps[i];
    if (tid == 0) {
        qap_chain_state st;
        st.t = t; st.accepts = s_acc; st.near_ties = s_ties; st.hash = s_hash;
        st.cost = s_cost; st.best_cost = s_best; st.best_iter = s_best_iter;
        st.status = QAP_OK; st.mode = QAP_MODE_DELTA;
        *a.state = st;
    }
}

template <bool SYM, bool A_LDS>
__global__ void __launch_bounds__(1024) k_chain_lds(ChainArgs a)
{
    extern __shared__ __align__(16) char smem[];
    chain_body<SYM, A_LDS>(a, smem);
}

}  // namespace

size_t lds_chain_bytes(int n, bool symmetric, bool a_in_lds)
{
    return chain_layout(n, n | 1, symmetric, a_in_lds, nullptr, nullptr);
}

int launch_chain_lds(const ChainArgs& a, bool symmetric, bool a_in_lds, int threads, hipStream_t stream)
{
    const size_t bytes = lds_chain_bytes(a.n, symmetric, a_in_lds);
    const void* fn;
    if (symmetric) fn = a_in_lds ? (const void*)k_chain_lds<true, true> : (const void*)k_chain_lds<true, false>;
    else fn = a_in_lds ? (const void*)k_chain_lds<false, true> : (const void*)k_chain_lds<false, false>;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess)
        return QAP_E_DEVICE;
    ChainArgs args = a;
    void* kargs[] = {&args};
    if (hipLaunchKernel(fn, dim3(1), dim3(threads), kargs, bytes, stream) != hipSuccess) return QAP_E_DEVICE;
    return QAP_OK;
}

}  // namespace qapsa
