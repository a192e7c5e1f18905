// qapsa_chain_wg.hip -- one annealing chain per workgroup of four waves (one
// per SIMD), state in LDS.
//
// Steps (b)-(e) of Sec. 2.2 for instances whose A and B' value ranges fit a
// byte (entries are stored shifted by their minimum: every swap cost is a sum
// of products of differences of A entries and of B' entries, so the shift
// changes nothing).  Where the state outgrows one CU's LDS, Delta (placement
// 1) and then also A (placement 2) move to device memory; B' always stays in
// LDS.
//
// Two interchangeable ways to produce the swap cost of a proposal; both give
// exactly Delta(r,s) = C(p o (r s)) - C(p), so the run does not depend on which
// one is active:
//   scratch mode   the swap cost of each proposal is computed when it is met,
//                  in O(N) (the "traditional" evaluation of Sec. 2.1).  A round
//                  tests 4 KW consecutive proposals, KW per wave: their
//                  partial dot products are summed across lanes together
//                  (cross-lane swaps, then row sums), one lane per proposal
//                  finishes its swap cost and compares it with the
//                  acceptance threshold of its iteration, and a ballot picks
//                  the wave's first acceptance; the waves meet once per round.
//                  KW follows the acceptance rate (few proposals per round
//                  while most are accepted).
//   Delta mode     steps (b)-(d) of Sec. 2.2: Delta(r,s) is kept for every pair;
//                  the scan tests many proposals against the unchanged matrix
//                  and keeps the first acceptance (Sec. 3 (ii)); after an
//                  accepted swap (u,v) pairs disjoint from {u,v} get an O(1)
//                  correction from two staged vectors and pairs that meet
//                  {u,v} are recomputed in O(N) (Sec. 3 (i)).
// A chain starts in scratch mode and moves to Delta mode once the acceptance
// rate over a window of iterations falls under a threshold (or is pinned to one
// mode by a flag).  Proposals run in row-major order, or at random with
// QAP_FLAG_RANDOM_ORDER (drawn pairs kept beside the acceptance thresholds).
// The same routine with a tabu flag runs tabu search over the same Delta: the
// best admissible swap per iteration instead of the first accepted one.
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

constexpr int kThreads = 256;        // four waves, one per SIMD
constexpr int kWaves = kThreads / 64;
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
    uint2* stg;    // staged, as int16 pairs: .x (A[k][u]-A[k][v], A[u][k]-A[v][k]),
                   // .y (B'[k][u]-B'[k][v], B'[u][k]-B'[v][k])
    int32_t* part; // [2][kWaves][n] per-wave partial sums of the pairs (u, s) and (v, s)
    int32_t* tau;  // ring of acceptance thresholds
    int16_t* ps;   // p
    Rec* rec;
};

__host__ __device__ inline size_t a16(size_t x) { return (x + 15) & ~(size_t)15; }

// Byte layout of one chain.  Placement 0: everything in LDS (`base`).
// Placement 1: Delta is the caller's buffer `gdelta`.  Placement 2: also the
// read-only byte copies of A and A^T, in the global scratch `gbase`.
// Placement 3: also B' and B'^T, after them in the scratch.
constexpr int kPlacements = 4;

__host__ __device__ inline size_t wg_layout(int n, int q, bool sym, int place, char* base, Wg* L,
                                           char* gbase = nullptr, int32_t* gdelta = nullptr)
{
    const size_t m = (size_t)n * (n - 1) / 2, P = 4 * (size_t)q;
    size_t off = 0, goff = 0;
    auto take = [&](size_t bytes) { char* p = base ? base + off : nullptr; off = a16(off + bytes); return p; };
    auto gtake = [&](size_t bytes) { char* p = gbase ? gbase + goff : nullptr; goff += bytes; return p; };
    char* ab = place >= 2 ? gtake(n * P) : take(n * P);
    char* at = sym ? nullptr : (place >= 2 ? gtake(n * P) : take(n * P));
    char* bb = place >= 3 ? gtake(n * P) : take(n * P);
    char* bt = sym ? nullptr : (place >= 3 ? gtake(n * P) : take(n * P));
    char* d = place >= 1 ? (char*)gdelta : take(4 * m);
    char* stg = take(8 * (size_t)n);
    char* part = take(4 * 2 * (size_t)kWaves * n);
    char* tau = take(4 * (size_t)kRing);
    char* ps = take(2 * (size_t)n);
    char* rec = take(sizeof(Rec) * kRec);
    if (L) {
        L->Ab = (uint8_t*)ab; L->At = (uint8_t*)at; L->Bb = (uint8_t*)bb; L->Bt = (uint8_t*)bt;
        L->D = (int32_t*)d; L->stg = (uint2*)stg; L->part = (int32_t*)part;
        L->tau = (int32_t*)tau; L->ps = (int16_t*)ps; L->rec = (Rec*)rec;
    }
    return off;
}

__host__ __device__ inline int wg_quads_of(int n) { return ((n + 3) / 4) | 1; }

// Smallest placement whose LDS part fits one workgroup, or -1.
__host__ __device__ inline int wg_placement(int n, bool sym)
{
    for (int pl = 0; pl < kPlacements; ++pl)
        if (wg_layout(n, wg_quads_of(n), sym, pl, nullptr, nullptr) <= kLdsLimit - kLdsStaticReserve) return pl;
    return -1;
}

// Device scratch of a placement: the byte matrices it keeps outside LDS.
inline size_t wg_global_bytes(int n, int q, bool sym, int place)
{
    const size_t mats = place >= 3 ? 2 : (place == 2 ? 1 : 0);
    return mats * (sym ? 1 : 2) * (size_t)n * 4 * q;
}

__device__ __forceinline__ uint32_t dot4(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_udot4(a, b, c, false);
}

// Sum over the 64 lanes (DPP row shifts and broadcasts); every lane receives it.
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

// Row sums: lane 15 of each 16-lane row receives the total of its row.
__device__ __forceinline__ int row_sums(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);
    return v;
}

// Lane sums of two values at once: v_permlane32_swap exchanges the upper half
// of x with the lower half of y, so that after one add lanes 0-31 hold
// pairwise partial sums of x and lanes 32-63 those of y.
__device__ __forceinline__ int half_fold(int x, int y)
{
    const auto s = __builtin_amdgcn_permlane32_swap((unsigned)x, (unsigned)y, false, false);
    return (int)(s[0] + s[1]);
}
// ... and v_permlane16_swap exchanges odd 16-lane rows of x with even rows of
// y: rows of the sum are x rows 0+1, y rows 0+1, x rows 2+3, y rows 2+3.
__device__ __forceinline__ int row_fold(int x, int y)
{
    const auto s = __builtin_amdgcn_permlane16_swap((unsigned)x, (unsigned)y, false, false);
    return (int)(s[0] + s[1]);
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ unsigned long long dpp_min_step(unsigned long long v)
{
    const uint32_t lo = __builtin_amdgcn_update_dpp(0xffffffffu, (uint32_t)v, CTRL, ROW_MASK, 0xf, false);
    const uint32_t hi = __builtin_amdgcn_update_dpp(0xffffffffu, (uint32_t)(v >> 32), CTRL, ROW_MASK, 0xf, false);
    const unsigned long long o = ((unsigned long long)hi << 32) | lo;
    return o < v ? o : v;
}

// Minimum over the 64 lanes, returned to every lane.
__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v)
{
    v = dpp_min_step<0x111, 0xf>(v);
    v = dpp_min_step<0x112, 0xf>(v);
    v = dpp_min_step<0x114, 0xf>(v);
    v = dpp_min_step<0x118, 0xf>(v);
    v = dpp_min_step<0x142, 0xa>(v);
    v = dpp_min_step<0x143, 0xc>(v);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, 63);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), 63);
    return ((unsigned long long)hi << 32) | lo;
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

// Wave-uniform copies of values (scalar registers).  Values the whole
// workgroup agrees on but that come back from LDS would otherwise be treated
// as per-lane, and everything derived from them (the proposal cursor, row
// addresses) would run on the vector unit.
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint32_t uni(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }
__device__ __forceinline__ unsigned long long uni64(unsigned long long x)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

// Packed offset of row r (32-bit; the one-workgroup kernel has n <= 512).
__host__ __device__ __forceinline__ uint32_t rs32(int n, int r) { return (uint32_t)r * (uint32_t)(2 * n - r - 1) >> 1; }

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

// The pair k places on in row-major cyclic order (k < n(n-1)/2): one step per
// row crossed.
__device__ __forceinline__ void advance_by(int n, int& r, int& s, int k)
{
    s += k;
    while (s >= n) {
        const int over = s - n;
        if (++r == n - 1) r = 0;
        s = r + 1 + over;
    }
}

// Eq. (2) for Delta > 0 at iteration t, out of line: it is the rare path of
// the scratch rounds and of the scan, and inlined copies of the FP64 log and
// the generator cost scalar registers everywhere else.  Returns
// z = fl(Delta / T_t + log r_t); the swap is accepted iff z < 0.  (A value, not
// a pointer argument, so that callers keep no stack slot.)
__device__ __noinline__ double exact_z(int d, const double* temps, double T0, uint64_t seed, uint32_t chain,
                                       uint64_t t)
{
    double z;
    metropolis_positive(d, temperature(temps, T0, t), uniform_r(seed, chain, t), &z);
    return z;
}

// inf_draw_clear out of line: it is evaluated only when T0 = +inf, and an
// inlined copy of the generator keeps its constants and key schedule in
// registers for the whole run.
__device__ __noinline__ bool inf_clear(uint64_t seed, uint32_t chain, uint64_t t)
{
    return inf_draw_clear(seed, chain, t);
}

// Acceptance threshold of iteration t: the largest Delta that Eq. (2) accepts
// (Eq. (2) is monotone in Delta), in .x; .y is set when T_t is so large that
// near ties cannot be located from the threshold alone.
__device__ __noinline__ int2 threshold_at(const double* temps, double T0, uint64_t seed, uint32_t chain,
                                          uint64_t t)
{
    const double T = temperature(temps, T0, t);
    const double y = log(uniform_r(seed, chain, t));
    const double xs = -y * T;
    int64_t d = xs >= 2147483647.0 ? 2147483647 : (int64_t)xs;
    auto acc = [&](int64_t dd) { return dd <= 0 || ((double)dd / T + y) < 0.0; };
    while (d < 2147483647 && acc(d + 1)) ++d;
    while (d > 0 && !acc(d)) --d;
    return make_int2((int32_t)d, !(T <= 1e9) ? 1 : 0);
}

template <bool SYM, int PL>
struct Chain {
    Wg L;
    int n, q, P;
    uint32_t m;
    int tid, lane, wave;

    __device__ Chain(const ChainArgs& a, char* smem)
    {
        n = a.n;
        q = a.quads;
        P = 4 * q;
        m = (uint32_t)((int64_t)n * (n - 1) / 2);
        tid = threadIdx.x;
        lane = tid & 63;
        wave = uni(tid >> 6);
        wg_layout(n, q, SYM, PL, smem, &L, (char*)a.gscratch, a.delta);
    }

    __device__ __forceinline__ int Ae(int i, int j) const { return L.Ab[i * P + j]; }
    __device__ __forceinline__ int Be(int i, int j) const { return L.Bb[i * P + j]; }
    __device__ __forceinline__ const uint32_t* row(const uint8_t* M, int i) const
    {
        return (const uint32_t*)(M + i * P);
    }
    // packed index of the pair {x, y}, x != y
    __device__ __forceinline__ uint32_t pidx(int x, int y) const
    {
        const int lo = min(x, y), hi = max(x, y);
        return rs32(n, lo) + (uint32_t)(hi - lo - 1);
    }

    // This lane's share of the all-k dot sums of the pair (r, s) (wave-uniform
    // r != s) for the current B': <A_r - A_s, B'_s - B'_rb> over rows (and the
    // same over columns), with rb = r.  With rb = y, the same sums for the
    // state after the swap (r, y), up to the two entries x = r, y that the
    // swap exchanges (see finish_after).
    __device__ __forceinline__ int lane_part(int r, int s, int rb = -1) const
    {
        if (rb < 0) rb = r;
        int out[1];
        const int rr[1] = {r}, ss[1] = {s}, bb[1] = {rb};
        lane_parts<1>(rr, ss, bb, out);
        return out[0];
    }

    // lane_part of NP pairs (r[i], s[i]) with rows rb[i] of B', in one pass
    // over k: every LDS read of the pass is issued before the first product.
    // For q <= 64 (n <= 256) each lane takes one k, clamped to q - 1 so that
    // every read stays inside its row, and lanes past q contribute nothing.
    template <int NP>
    __device__ __forceinline__ void lane_parts(const int (&r)[NP], const int (&s)[NP], const int (&rb)[NP],
                                               int (&out)[NP]) const
    {
        uint32_t pos[NP], neg[NP];
#pragma unroll
        for (int i = 0; i < NP; ++i) pos[i] = neg[i] = 0;
        auto body = [&](int k) __attribute__((always_inline)) {
            uint32_t xr[NP], xs[NP], yr[NP], ys[NP], zr[NP], zs[NP], wr[NP], ws[NP];
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                xr[i] = row(L.Ab, r[i])[k]; xs[i] = row(L.Ab, s[i])[k];
                yr[i] = row(L.Bb, rb[i])[k]; ys[i] = row(L.Bb, s[i])[k];
                if constexpr (!SYM) {
                    zr[i] = row(L.At, r[i])[k]; zs[i] = row(L.At, s[i])[k];
                    wr[i] = row(L.Bt, rb[i])[k]; ws[i] = row(L.Bt, s[i])[k];
                }
            }
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                pos[i] = dot4(xr[i], ys[i], pos[i]); pos[i] = dot4(xs[i], yr[i], pos[i]);
                neg[i] = dot4(xr[i], yr[i], neg[i]); neg[i] = dot4(xs[i], ys[i], neg[i]);
                if constexpr (!SYM) {
                    pos[i] = dot4(zr[i], ws[i], pos[i]); pos[i] = dot4(zs[i], wr[i], pos[i]);
                    neg[i] = dot4(zr[i], wr[i], neg[i]); neg[i] = dot4(zs[i], ws[i], neg[i]);
                }
            }
        };
        if (q <= 64) {
            body(min(lane, q - 1));
#pragma unroll
            for (int i = 0; i < NP; ++i) out[i] = lane < q ? (int)(pos[i] - neg[i]) : 0;
        } else {
            for (int k = lane; k < q; k += 64) body(k);
#pragma unroll
            for (int i = 0; i < NP; ++i) out[i] = (int)(pos[i] - neg[i]);
        }
    }

    // Swap cost of the pair (r, s) held by this lane, from its all-k sum S.
    __device__ __forceinline__ int finish_pair(int S, int r, int s) const
    {
        return finish_delta<SYM>(S, Ae(r, r), Ae(r, s), Ae(s, r), Ae(s, s), Be(r, r), Be(r, s), Be(s, r), Be(s, s));
    }

    // Swap cost of the pair (r, s) in the state after the swap (r, y) (s not
    // in {r, y}), from S = lane sums of lane_part(r, s, y).  The swap permutes
    // rows and columns of B' by sigma = (r y): B''[i][j] = B'[sigma(i)][sigma(j)],
    // so row s of B'' minus row r is (B'_s - B'_y) with entries r, y exchanged,
    // and <g, f o sigma> = <g, f> + (g_r - g_y)(f_y - f_r) (the same for
    // columns); then the k in {r, s} terms and the corner, with B'' entries.
    // With y = r (no swap before) this is finish_pair.
    __device__ __forceinline__ int finish_after(int S, int r, int s, int y) const
    {
        return fin_eval(S, fin_load(r, s, y));
    }

    // The entries of A and B' that finish_after(S, r, s, y) reads, loaded
    // apart from the arithmetic so that a round can issue the reads before
    // its dot products and find them there when the lane sums are in.
    struct Fin {
        int arr, ars, asr, ass, ary, asy, ayr, ays;   // A at (r,r), (r,s), (s,r), (s,s), (r,y), (s,y), (y,r), (y,s)
        int bsr, byr, bsy, byy, bys, bss, brs, bry;   // B' at (s,r), (y,r), (s,y), (y,y), (y,s), (s,s), (r,s), (r,y)
    };
    __device__ __forceinline__ Fin fin_load(int r, int s, int y) const
    {
        Fin f;
        f.arr = Ae(r, r); f.ars = Ae(r, s); f.asr = Ae(s, r); f.ass = Ae(s, s);
        f.ary = Ae(r, y); f.asy = Ae(s, y);
        f.bsr = Be(s, r); f.byr = Be(y, r); f.bsy = Be(s, y); f.byy = Be(y, y); f.bys = Be(y, s); f.bss = Be(s, s);
        if constexpr (!SYM) {
            f.ayr = Ae(y, r); f.ays = Ae(y, s);
            f.brs = Be(r, s); f.bry = Be(r, y);
        } else {
            f.ayr = f.ays = f.brs = f.bry = 0;
        }
        return f;
    }
    __device__ __forceinline__ int fin_eval(int S, const Fin& f) const
    {
        const int gx = f.arr - f.asr, gy = f.ary - f.asy;
        const int fx = f.bsr - f.byr, fy = f.bsy - f.byy;
        int Sc = S + (gx - gy) * (fy - fx);
        if constexpr (!SYM) {   // columns: g = A[.][r] - A[.][s], f = B'[.][s] - B'[.][y]
            const int hx = f.arr - f.ars, hy = f.ayr - f.ays;
            const int ex = f.brs - f.bry, ey = f.bys - f.byy;
            Sc += (hx - hy) * (ey - ex);
        }
        // B'' at (r,r), (r,s), (s,r), (s,s): B' at (y,y), (y,s), (s,y), (s,s)
        return finish_delta<SYM>(Sc, f.arr, f.ars, f.asr, f.ass, f.byy, f.bys, f.bsy, f.bss);
    }

    // This wave's share of the swap (u, v) applied to B' (and B'^T).
    __device__ __forceinline__ void swap_part(int u, int v) const
    {
        const int x[2] = {u, v}, src[2] = {v, u};
        permute_part<2>(x, src);
    }

    // This wave's share of B'new[i][j] = B'[pi(i)][pi(j)] for a permutation pi
    // that moves only the NC indices x[c], with pi(x[c]) = src[c] (a swap, or
    // the 3-cycle of two swaps (r a), (r b) made in one pass: pi = (r a)(r b)
    // maps r -> b, b -> a, a -> r).  Rows x[c] take rows src[c] (whole
    // dwords; then lanes c * NC + e write the NC * NC entries in columns x,
    // read with the rows), and in every other row the entries in columns x
    // are permuted.  Each share issues all of its reads before its first
    // write (a wave's LDS accesses are ordered); shares touch disjoint bytes.
    template <int NC>
    __device__ __forceinline__ void permute_part(const int (&x)[NC], const int (&src)[NC]) const
    {
        static_assert(NC == 2 || NC == 3, "a swap or a 3-cycle");
        // the indices as plain values, so that the per-lane picks below stay
        // selects (picks from an array would put the array in memory)
        const int x0 = uni(x[0]), x1 = uni(x[1]), s0 = uni(src[0]), s1 = uni(src[1]);
        int x2 = 0, s2 = 0;
        if constexpr (NC == 3) { x2 = uni(x[2]); s2 = uni(src[2]); }
        auto pick = [](int c, int a0, int a1, int a2) __attribute__((always_inline)) {
            return c == 0 ? a0 : (c == 1 ? a1 : a2);
        };
        auto rows = [&](uint8_t* M) __attribute__((always_inline)) {
            const int l = lane < NC * NC ? lane : 0;   // lane l: corner entry (l / NC, l % NC)
            const int ci = l / NC, ce = l - ci * NC;
            const uint8_t corner = M[pick(ci, s0, s1, s2) * P + pick(ce, s0, s1, s2)];
            for (int k = lane; k < q; k += 64) {
                uint32_t w[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) w[c] = row(M, src[c])[k];
#pragma unroll
                for (int c = 0; c < NC; ++c) ((uint32_t*)(M + x[c] * P))[k] = w[c];
            }
            if (lane < NC * NC) M[pick(ci, x0, x1, x2) * P + pick(ce, x0, x1, x2)] = corner;
        };
        auto cols = [&](uint8_t* M, int i0, int step) __attribute__((always_inline)) {
            for (int i = i0; i < n; i += 4 * step) {
                uint8_t e[4][NC];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int ii = min(i + j * step, n - 1);
#pragma unroll
                    for (int c = 0; c < NC; ++c) e[j][c] = M[ii * P + src[c]];
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int ii = i + j * step;
                    bool own = ii < n;
#pragma unroll
                    for (int c = 0; c < NC; ++c) own = own && ii != x[c];
                    if (own) {
#pragma unroll
                        for (int c = 0; c < NC; ++c) M[ii * P + x[c]] = e[j][c];
                    }
                }
            }
        };
        if constexpr (SYM) {
            if (wave == 0) rows(L.Bb);
            else cols(L.Bb, (wave - 1) * 64 + lane, (kWaves - 1) * 64);
        } else {
            if (wave == 0) rows(L.Bb);
            else if (wave == 1) rows(L.Bt);
            else if (wave == 2) cols(L.Bb, lane, 64);
            else cols(L.Bt, lane, 64);
        }
    }

    // Staged differences after the swap (u, v), threads over k.
    __device__ void stage(int u, int v) const
    {
        for (int k = tid; k < n; k += kThreads) {
            int a1, a2, b1, b2;
            if constexpr (SYM) {
                a1 = a2 = Ae(u, k) - Ae(v, k);
                b1 = b2 = Be(u, k) - Be(v, k);
            } else {
                a1 = L.At[u * P + k] - L.At[v * P + k];   // A[k][u] - A[k][v]
                a2 = Ae(u, k) - Ae(v, k);                 // A[u][k] - A[v][k]
                b1 = L.Bt[u * P + k] - L.Bt[v * P + k];
                b2 = Be(u, k) - Be(v, k);
            }
            L.stg[k] = make_uint2((uint32_t)(uint16_t)a1 | ((uint32_t)(uint16_t)a2 << 16),
                                  (uint32_t)(uint16_t)b1 | ((uint32_t)(uint16_t)b2 << 16));
        }
    }

    // Pairs disjoint from {u, v}: the O(1) correction of Sec. 3 (i) from the
    // staged vectors.  The packed triangle is folded into a rectangle n wide:
    // folded row f holds row f of the triangle in columns c < n-1-f (the pair
    // (f, f+1+c)) and row n-2-f after it (the pair (n-2-f, c)).  Read in
    // order and cut after the M = n(n-1)/2 entries, the rectangle covers every
    // pair once (for even n the middle row would otherwise come twice).  Lanes
    // take its entries in order, 64 to a wave and 256 to a step, carrying
    // (f, c) from step to step, so that every lane of every step but the last
    // does useful work whatever n is.  Four steps are loaded before any is
    // stored (a store to Delta may not move above a later load of it).  Pairs
    // that meet {u, v} are updated too, with a meaningless value:
    // finish_rows rewrites all of them after the next barrier, and skipping
    // them would cost a mask per entry.
    __device__ void taillard() const
    {
        constexpr int kStep = 64 * kWaves, U = 4;
        const uint32_t m = __umul24((uint32_t)n, (uint32_t)(n - 1)) >> 1;
        const int fq = kStep / n, cq = kStep - fq * n;     // one step, as folded rows and columns
        int f = 0, c = wave * 64 + lane;
        while (c >= n) { c -= n; ++f; }                    // at most 255 / n + 1 times
        auto next = [&]() __attribute__((always_inline)) {
            f += fq;
            c += cq;
            if (c >= n) { c -= n; ++f; }
        };
        // entry (f, c) of the folded rectangle: Delta offset and the pair's staged differences
        auto locate = [&](uint32_t& off, v2i16& x, v2i16& y) __attribute__((always_inline)) {
            const bool first = c < n - 1 - f;
            const int r = first ? f : n - 2 - f;
            const int s = first ? f + 1 + c : c;
            off = (__umul24((uint32_t)r, (uint32_t)(2 * n - 1 - r)) >> 1) + (uint32_t)(s - r - 1);
            const uint2 gr = L.stg[r], gs = L.stg[s];
            x = __builtin_bit_cast(v2i16, gr.x) - __builtin_bit_cast(v2i16, gs.x);
            y = __builtin_bit_cast(v2i16, gs.y) - __builtin_bit_cast(v2i16, gr.y);
        };
        uint32_t kb = (uint32_t)(wave * 64);                // this wave's first entry of the step
        for (; kb + (U - 1) * kStep + 64 <= m; kb += U * kStep) {
            uint32_t off[U];
            int32_t dv[U];
            v2i16 x[U], y[U];
#pragma unroll
            for (int j = 0; j < U; ++j) {
                locate(off[j], x[j], y[j]);
                dv[j] = L.D[off[j]];
                next();
            }
#pragma unroll
            for (int j = 0; j < U; ++j) L.D[off[j]] = __builtin_amdgcn_sdot2(x[j], y[j], dv[j], false);
        }
        for (; kb < m; kb += kStep) {
            if (kb + (uint32_t)lane < m) {
                uint32_t off;
                v2i16 x, y;
                locate(off, x, y);
                L.D[off] = __builtin_amdgcn_sdot2(x, y, L.D[off], false);
            }
            next();
        }
    }

    // Partial sums, over this wave's quarter of the quads k, of the all-k dot
    // sums of the pairs (x, s) and (y, s) for every s, less the self terms of s:
    // part[0][wave][s] and part[1][wave][s].  (At s = x the first one is the
    // self term of x.)
    __device__ void gemv_part(int x, int y) const
    {
        const int k0 = q * wave / kWaves, k1 = q * (wave + 1) / kWaves;
        const uint32_t *ax = row(L.Ab, x), *ay = row(L.Ab, y), *bx = row(L.Bb, x), *by = row(L.Bb, y);
        const uint32_t *cx = nullptr, *cy = nullptr, *dx = nullptr, *dy = nullptr;
        if constexpr (!SYM) { cx = row(L.At, x); cy = row(L.At, y); dx = row(L.Bt, x); dy = row(L.Bt, y); }
        int32_t* px = L.part + wave * n;
        int32_t* py = L.part + (kWaves + wave) * n;
        for (int s = lane; s < n; s += 64) {
            const uint32_t *as = row(L.Ab, s), *bs = row(L.Bb, s);
            const uint32_t *cs = nullptr, *ds = nullptr;
            if constexpr (!SYM) { cs = row(L.At, s); ds = row(L.Bt, s); }
            uint32_t pu = 0, pv = 0, ng = 0;
#pragma unroll 2
            for (int k = k0; k < k1; ++k) {
                const uint32_t xs = as[k], ys = bs[k];
                pu = dot4(ax[k], ys, pu); pu = dot4(xs, bx[k], pu);
                pv = dot4(ay[k], ys, pv); pv = dot4(xs, by[k], pv);
                ng = dot4(xs, ys, ng);
                if constexpr (!SYM) {
                    const uint32_t zs = cs[k], ws = ds[k];
                    pu = dot4(cx[k], ws, pu); pu = dot4(zs, dx[k], pu);
                    pv = dot4(cy[k], ws, pv); pv = dot4(zs, dy[k], pv);
                    ng = dot4(zs, ws, ng);
                }
            }
            px[s] = (int)(pu - ng);
            py[s] = (int)(pv - ng);
        }
    }

    // Delta of the pairs (x, s) and (y, s) from the partial sums, threads over
    // s.  Update (build = false): every s outside {x, y}; the pair (x, y) is
    // the caller's.  Build (build = true, y = x + 1 or y = x = n - 1): the
    // pairs above the diagonal of rows x and y.
    __device__ void finish_rows(int x, int y, bool build) const
    {
        const int32_t* p0 = L.part;
        const int32_t* p1 = L.part + kWaves * n;
        int sx = 0, sy = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) { sx += p0[w * n + x]; sy += p1[w * n + y]; }
        sx = uni(sx);
        sy = uni(sy);
        for (int s = tid; s < n; s += kThreads) {
            int tx = 0, ty = 0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) { tx += p0[w * n + s]; ty += p1[w * n + s]; }
            if (build) {
                if (s > x) L.D[pidx(x, s)] = finish_pair(tx - sx, x, s);
                if (y != x && s > y) L.D[pidx(y, s)] = finish_pair(ty - sy, y, s);
            } else if (s != x && s != y) {
                L.D[pidx(x, s)] = finish_pair(tx - sx, x, s);
                L.D[pidx(y, s)] = finish_pair(ty - sy, y, s);
            }
        }
    }

    // The full Delta matrix from scratch, two rows per pass (all threads).
    __device__ void build_delta() const
    {
        for (int r0 = 0; r0 < n - 1; r0 += 2) {
            const int r1 = min(r0 + 1, n - 1);
            gemv_part(r0, r1);
            __syncthreads();
            finish_rows(r0, r1, true);
            __syncthreads();
        }
    }
};

template <int V> struct IC { static constexpr int value = V; };

// TABU: tabu search over the same Delta instead of annealing (every iteration
// takes the best admissible swap; rules at the tabu loop below).  PROF = false
// compiles the phase counters out (for launches without them).
template <bool SYM, int PL, bool TABU = false, bool PROF = true>
__device__ void chain_run(const ChainArgs& a_in, char* smem)
{
    // The chain's hot scalars live in scalar registers of every wave (all
    // threads follow the same uniform control flow and apply the same
    // updates).  Scalar registers are scarce (102), so cold arguments are read
    // from an LDS copy where they are used and the running statistics are
    // kept by thread 0 alone.
    // per-wave first acceptance (j << 32 | Delta), by round parity; entries
    // kWaves.. hold the same for the proposals after the window's first (see
    // scratch_round_ahead), so that one read pass takes both
    __shared__ unsigned long long s_wkey[2][2 * kWaves];
    __shared__ unsigned long long s_ties;
    __shared__ int s_flag;
    __shared__ unsigned long long s_prof[QAP_PHASES];
    __shared__ ChainArgs s_arg;
    __shared__ long long s_asp;   // tabu search: best - cost, the aspiration bound of the next iteration

    if (threadIdx.x == 0) s_arg = a_in;
    __syncthreads();
    const ChainArgs& a = s_arg;
    Chain<SYM, PL> C(a, smem);
    const Wg& L = C.L;
    const int n = C.n, P = C.P, tid = C.tid, lane = C.lane, wave = C.wave;
    const uint32_t m = C.m;

    // phase counters: thread 0 adds to LDS without waiting for the result
    const bool prof = PROF && a.prof != nullptr;
    if (tid < QAP_PHASES) s_prof[tid] = 0;
    unsigned long long prof_last = prof ? clock64() : 0;
    const unsigned long long prof_start = prof_last;
    auto mark = [&](int k) __attribute__((always_inline)) {
        if (prof && tid == 0) {
            const unsigned long long now = clock64();
            atomicAdd(&s_prof[k], now - prof_last);
            prof_last = now;
        }
    };
    auto bump = [&](int k, unsigned long long x) __attribute__((always_inline)) {
        if (prof && tid == 0) atomicAdd(&s_prof[k], x);
    };

    // ------------------------------------------------------------------ load
    // rows of A and B' are read coalesced; the transposes are written in place
    const qap_chain_state st0 = *a.state;
    if (tid == 0) { s_flag = 0; s_ties = st0.near_ties; }
    __syncthreads();
#pragma unroll 4
    for (int e = tid; e < n * n; e += kThreads) {
        const int i = e / n, j = e - i * n;
        const int av = a.A[e] - a.a_min, bv = a.Bp[e] - a.b_min;
        if ((av | bv) & ~0xff) s_flag = 1;
        L.Ab[i * P + j] = (uint8_t)av;
        L.Bb[i * P + j] = (uint8_t)bv;
        if constexpr (!SYM) { L.At[j * P + i] = (uint8_t)av; L.Bt[j * P + i] = (uint8_t)bv; }
    }
    for (int e = tid; e < n * (P - n); e += kThreads) {   // zero padding after each row
        const int i = e / (P - n), j = n + (e - i * (P - n));
        L.Ab[i * P + j] = 0;
        L.Bb[i * P + j] = 0;
        if constexpr (!SYM) { L.At[i * P + j] = 0; L.Bt[i * P + j] = 0; }
    }
    for (int i = tid; i < n; i += kThreads) L.ps[i] = (int16_t)a.p[i];
    if (tid < 2 * kWaves) s_wkey[tid / kWaves][tid % kWaves] = ~0ull;
    __syncthreads();
    const int status = st0.status != QAP_OK ? st0.status : (s_flag ? (int)QAP_E_RANGE : (int)QAP_OK);
    if (status != QAP_OK) {
        if (tid == 0) a.state->status = status;
        return;
    }
    const bool delta_current = st0.mode != QAP_MODE_SCRATCH_STALE;
    int mode = (a.flags & kFlagDeltaOnly) ? 1 : (a.flags & kFlagScratchOnly) ? 0 : (st0.mode == QAP_MODE_DELTA);
    if constexpr (TABU) mode = 1;
    if (mode == 1) {
        if (!delta_current) C.build_delta();
        else if (PL == 0) {   // the caller's Delta is valid for p after qap_delta_init and after every run
            for (uint32_t i = tid; i < m; i += kThreads) L.D[i] = a.delta[i];
            __syncthreads();
        }
    }
    mark(QAP_PH_IO);

    // hot arguments as plain values
    const uint64_t t_end = uni64(a.t_end);
    const double T0 = a.T0;
    const double* __restrict__ temps = a.temps;
    const uint64_t seed = a.seed;
    const uint32_t chain_id = a.chain_id;
    const bool t0_inf = __builtin_isinf(T0);
    // random proposal order: the ring's second half holds the drawn pairs
    // ((r << 16) | s) of the iterations whose thresholds the first half holds
    const bool rnd = (uni(a.flags) & QAP_FLAG_RANDOM_ORDER) != 0;
    const uint32_t ring_len = rnd ? kRing / 2 : kRing;
    uint32_t* const ring_pairs = (uint32_t*)L.tau + kRing / 2;

    const uint32_t nt_mod = (uint32_t)kThreads % m;
    uint64_t t = uni64(st0.t);
    // running statistics: thread 0's registers only
    unsigned long long accepts = 0, hash = 0, best_iter = 0;
    long long cost = 0, best = 0;
    if (tid == 0) {
        accepts = st0.accepts; hash = st0.hash; best_iter = st0.best_iter;
        cost = st0.cost; best = st0.best_cost;
    }
    int nrec = 0;
    uint32_t idx0 = (uint32_t)(t % m);      // packed index proposed at iteration t
    int r0, s0;                              // its pair
    pair_of_u(n, idx0, r0, s0);
    int buf = 0;
    int step_e = 1;
    int kw = 1;                              // proposals per wave in a scratch round
    uint64_t tau_base = ~0ull;               // the threshold ring covers [tau_base, tau_base + kRing)
    bool ring_exact = false;
    uint32_t win = 0;   // the switch window: iterations (low 16 bits) and accepted swaps (high 16)

    // hash the buffered accept records (wave 0); the 64-bit sum over lanes is
    // taken in three 22-bit slices so that no slice can carry out
    auto flush = [&]() __attribute__((always_inline)) {
        if (wave == 0) {
            uint64_t h = 0;
            if (lane < nrec) {
                const Rec r = L.rec[lane];
                h = accept_fingerprint(r.t, (int)(r.uv >> 16), (int)(r.uv & 0xffff), r.d);
            }
            const uint64_t x0 = (uint32_t)wave_sum((int)(h & 0x3fffff));
            const uint64_t x1 = (uint32_t)wave_sum((int)((h >> 22) & 0x3fffff));
            const uint64_t x2 = (uint32_t)wave_sum((int)(h >> 44));
            if (tid == 0) hash += x0 + (x1 << 22) + (x2 << 44);
        }
        nrec = 0;
    };

    // the swap (u, v) at iteration tt with cost change d: scalars, p, the
    // record (B' is the caller's)
    auto book = [&](uint64_t tt, int u, int v, int d) __attribute__((always_inline)) {
        if (tid == 0) {
            const int16_t pu = L.ps[u], pv = L.ps[v];
            L.ps[u] = pv; L.ps[v] = pu;
            int64_t* const acc_log = a.acc_log;
            if (acc_log && accepts < a.acc_cap) {
                int64_t* e = acc_log + 4 * accepts;
                e[0] = (int64_t)tt; e[1] = u; e[2] = v; e[3] = d;
            }
            L.rec[nrec] = Rec{tt, ((uint32_t)u << 16) | (uint32_t)v, d};
            cost += d;
            accepts += 1;
            if (cost < best) { best = cost; best_iter = tt + 1; }
        }
        nrec += 1;
    };
    // ... and B'
    auto accept_common = [&](uint64_t tt, int u, int v, int d) __attribute__((always_inline)) {
        book(tt, u, v, d);
        C.swap_part(u, v);
    };

    auto advance = [&](uint32_t k) __attribute__((always_inline)) {   // move the proposal cursor k iterations on
        k = uni(k);
        t = uni64(t + k);
        if (k >= m) k %= m;
        idx0 += k;
        if (idx0 >= m) idx0 -= m;
        idx0 = uni(idx0);
        if (k < 64) advance_by(n, r0, s0, (int)k);
        else pair_of_u(n, idx0, r0, s0);
        r0 = uni(r0);
        s0 = uni(s0);
    };

    auto log_tie = [&](uint64_t tt, int d, double z) __attribute__((always_inline)) {
        const unsigned long long slot = atomicAdd(&s_ties, 1ull);
        qap_near_tie* const ties = a.ties;
        if (ties && slot < a.tie_cap) ties[slot] = qap_near_tie{tt, (int64_t)d, z};
    };

    auto min_key = [&]() __attribute__((always_inline)) -> unsigned long long {
        unsigned long long key = s_wkey[buf][0];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) {
            const unsigned long long x = s_wkey[buf][w];
            key = x < key ? x : key;
        }
        buf ^= 1;   // the other set is written next; everyone read this one before the next barrier
        return uni64(key);
    };

    auto refill = [&]() __attribute__((always_inline)) {
        tau_base = t;
        if (tid == 0) s_flag = 0;
        __syncthreads();
        bool ex = false;
        const uint64_t iters = a.iters;
        for (int i = tid; i < (int)ring_len; i += kThreads) {
            const uint64_t tt = tau_base + i;
            int2 th = make_int2(0, 0);
            if (tt < iters) th = threshold_at(temps, T0, seed, chain_id, tt);
            L.tau[i] = th.x;
            ex |= th.y != 0;
            if (rnd) {
                int r = 0, s = 1;
                if (tt < iters) pair_of_u(n, random_pair_index(seed, chain_id, tt, m), r, s);
                ring_pairs[i] = ((uint32_t)r << 16) | (uint32_t)s;
            }
        }
        if (ex) s_flag = 1;
        __syncthreads();
        ring_exact = uni(s_flag) != 0;
        mark(QAP_PH_SCRATCH_THRESH);
        bump(QAP_PH_N_THRESH, 1);
    };

    // One scratch-mode round: KW proposals per wave, the first acceptance wins.
    auto scratch_round = [&](auto kw_tag) __attribute__((always_inline)) {
        constexpr int KW = decltype(kw_tag)::value;
        constexpr int K = kWaves * KW;
        const uint32_t rem = (uint32_t)min<uint64_t>((uint64_t)K, t_end - t);
        if (tau_base == ~0ull || t + K > tau_base + ring_len) refill();
        int pr[KW], pc[KW];
        if (rnd) {
            const uint32_t* const pk = ring_pairs + (uint32_t)(t - tau_base) + wave * KW;
#pragma unroll
            for (int i = 0; i < KW; ++i) {
                const uint32_t x = uni(pk[i]);
                pr[i] = (int)(x >> 16);
                pc[i] = (int)(x & 0xffffu);
            }
        } else {
            int r = r0, s = s0;
            advance_by(n, r, s, wave * KW);
#pragma unroll
            for (int i = 0; i < KW; ++i) {
                pr[i] = uni(r); pc[i] = uni(s);
                if (i + 1 < KW) advance_by(n, r, s, 1);
            }
        }
        // lane i < KW finishes proposal i of this wave: its entries of A and
        // B' and its threshold are read first, the dot products after them
        int my_r = pr[0], my_s = pc[0];
#pragma unroll
        for (int i = 1; i < KW; ++i)
            if (lane == i) { my_r = pr[i]; my_s = pc[i]; }
        const int jl = wave * KW + (lane < KW ? lane : 0);
        const int32_t tau = L.tau[(uint32_t)(t - tau_base) + (uint32_t)jl];
        const auto fin = C.fin_load(my_r, my_s, my_r);
        int S[KW];
        {
            int part[KW];
            C.template lane_parts<KW>(pr, pc, pr, part);
            if constexpr (KW == 1) {
                S[0] = wave_sum(part[0]);
            } else if constexpr (KW == 2) {
                const int z = row_sums(half_fold(part[0], part[1]));
                S[0] = __builtin_amdgcn_readlane(z, 15) + __builtin_amdgcn_readlane(z, 31);
                S[1] = __builtin_amdgcn_readlane(z, 47) + __builtin_amdgcn_readlane(z, 63);
            } else {
                const int z = row_sums(row_fold(half_fold(part[0], part[2]), half_fold(part[1], part[3])));
                S[0] = __builtin_amdgcn_readlane(z, 15);
                S[1] = __builtin_amdgcn_readlane(z, 31);
                S[2] = __builtin_amdgcn_readlane(z, 47);
                S[3] = __builtin_amdgcn_readlane(z, 63);
            }
        }
        int my_S = S[0];
#pragma unroll
        for (int i = 1; i < KW; ++i)
            if (lane == i) my_S = S[i];
        const int dl = C.fin_eval(my_S, fin);
        const bool valid = lane < KW && (uint32_t)jl < rem;
        bool acc = valid && dl <= tau;
        bool tie = false;
        double zt = 0.0;
        if (valid && dl > 0 && (ring_exact || (dl >= tau - 1 && dl <= tau + 2)) &&
            !(t0_inf && inf_clear(seed, chain_id, t + jl))) {
            zt = exact_z(dl, temps, T0, seed, chain_id, t + jl);
            if (ring_exact) acc = zt < 0.0;
            tie = fabs(zt) < kNearTie;
        }
        const unsigned long long mask = __ballot(acc);
        unsigned long long wkey = ~0ull;
        if (mask) {
            const int f = __builtin_ctzll(mask);
            wkey = ((unsigned long long)(wave * KW + f) << 32) | (uint32_t)__builtin_amdgcn_readlane(dl, f);
        }
        if (lane == 0) s_wkey[buf][wave] = wkey;
        __syncthreads();
        const unsigned long long key = min_key();
        const int jstar = key == ~0ull ? -1 : (int)(key >> 32);
        mark(QAP_PH_SCRATCH_EVAL);
        bump(QAP_PH_N_ROUNDS, 1);
        if (__ballot(tie)) {   // rare: log the near ties a sequential run meets
            if (tie && (jstar < 0 || jl <= jstar)) log_tie(t + jl, dl, zt);
        }
        if (jstar < 0) {
            advance(rem);
            win += rem;
        } else {
            int u = r0, v = s0;
            if (rnd) {
                const uint32_t x = uni(ring_pairs[(uint32_t)(t - tau_base) + (uint32_t)jstar]);
                u = (int)(x >> 16);
                v = (int)(x & 0xffffu);
            } else {
                advance_by(n, u, v, jstar);
            }
            u = uni(u);
            v = uni(v);
            accept_common(t + jstar, u, v, (int)(uint32_t)key);
            __syncthreads();
            if (nrec == kRec) flush();
            advance((uint32_t)jstar + 1);
            win += (uint32_t)jstar + 1 + (1u << 16);
            mark(QAP_PH_SCRATCH_ACCEPT);
            bump(QAP_PH_N_SCRATCH_ACC, 1);
        }
    };

    // A scratch round of four proposals (r0, s0 + w), one per wave w, that
    // also tests the four proposals that follow the first one, (r0, s0 + 1 + w),
    // in the state after the swap (r0, s0): when that first proposal is
    // accepted (about half the rounds while half the proposals are), the round
    // goes on to the first acceptance among them, and one round makes two
    // swaps.  Wave w sums both dot products together (lane_part with row s0 of
    // B' in place of row r0 gives the sums after the swap up to two exchanged
    // entries, which finish_after corrects).  For rounds inside one row of the
    // cyclic order (s0 + 4 < n), in row-major order, with all five iterations
    // in the slice.
    auto scratch_round_ahead = [&]() __attribute__((always_inline)) {
        constexpr int K = kWaves;
        if (tau_base == ~0ull || t + K + 1 > tau_base + ring_len) refill();
        const int r = r0, sn = uni(s0 + wave), sa = uni(s0 + 1 + wave);
        // lane 0: the window's proposal at t + w; lane 1: the one after the
        // swap, at t + 1 + w.  Their entries of A and B' and thresholds are
        // read first, the dot products after them.
        const bool after = lane == 1;
        const uint32_t jo = (uint32_t)wave + (after ? 1u : 0u);
        const int32_t tau = L.tau[(uint32_t)(t - tau_base) + jo];
        const auto fin = C.fin_load(r, after ? sa : sn, after ? s0 : r);
        int Sn, Sa;
        {
            const int rr[2] = {r, r}, ss[2] = {sn, sa}, bb[2] = {r, s0};
            int pp[2];
            C.template lane_parts<2>(rr, ss, bb, pp);
            const int z = row_sums(half_fold(pp[0], pp[1]));
            Sn = __builtin_amdgcn_readlane(z, 15) + __builtin_amdgcn_readlane(z, 31);
            Sa = __builtin_amdgcn_readlane(z, 47) + __builtin_amdgcn_readlane(z, 63);
        }
        const int dl = C.fin_eval(after ? Sa : Sn, fin);
        const bool valid = lane < 2;
        bool acc = valid && dl <= tau;
        bool tie = false;
        double zt = 0.0;
        if (valid && dl > 0 && (ring_exact || (dl >= tau - 1 && dl <= tau + 2)) &&
            !(t0_inf && inf_clear(seed, chain_id, t + jo))) {
            zt = exact_z(dl, temps, T0, seed, chain_id, t + jo);
            if (ring_exact) acc = zt < 0.0;
            tie = fabs(zt) < kNearTie;
        }
        const int dn = __builtin_amdgcn_readlane(dl, 0), da = __builtin_amdgcn_readlane(dl, 1);
        const unsigned long long mask = __ballot(acc);
        if (lane == 0) {
            s_wkey[buf][wave] = (mask & 1ull) ? (((unsigned long long)wave << 32) | (uint32_t)dn) : ~0ull;
            s_wkey[buf][kWaves + wave] = (mask & 2ull) ? (((unsigned long long)wave << 32) | (uint32_t)da) : ~0ull;
        }
        __syncthreads();
        unsigned long long kv[2 * kWaves];
#pragma unroll
        for (int w = 0; w < 2 * kWaves; ++w) kv[w] = s_wkey[buf][w];
        buf ^= 1;   // the other set is written next; everyone read this one before the next barrier
        unsigned long long key = kv[0], akey = kv[kWaves];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) {
            key = kv[w] < key ? kv[w] : key;
            akey = kv[kWaves + w] < akey ? kv[kWaves + w] : akey;
        }
        key = uni64(key);
        akey = uni64(akey);
        const int jstar = key == ~0ull ? -1 : (int)(key >> 32);
        const int istar = (jstar != 0 || akey == ~0ull) ? -1 : (int)(akey >> 32);
        mark(QAP_PH_SCRATCH_EVAL);
        bump(QAP_PH_N_ROUNDS, 1);
        // near ties a sequential run meets: the window's proposals up to the
        // first acceptance, and those after the swap when it is the first one
        if (__ballot(tie)) {   // rare
            if (tie && !after && (jstar < 0 || wave <= jstar)) log_tie(t + jo, dl, zt);
            if (tie && after && jstar == 0 && (istar < 0 || wave <= istar)) log_tie(t + jo, dl, zt);
        }
        if (jstar < 0) {
            advance(K);
            win += K;
            return;
        }
        uint32_t used;
        if (jstar == 0 && istar >= 0) {
            // both swaps (r, s0) and (r, b): one pass permutes B' by their product
            const int b = s0 + 1 + istar;
            book(t, r, s0, (int)(uint32_t)key);
            if (nrec == kRec) flush();
            book(t + 1 + istar, r, b, (int)(uint32_t)akey);
            const int x[3] = {r, s0, b}, src[3] = {b, r, s0};
            C.template permute_part<3>(x, src);
            __syncthreads();
            if (nrec == kRec) flush();
            used = (uint32_t)istar + 2;
            win += 2u << 16;
            bump(QAP_PH_N_SCRATCH_ACC, 1);
        } else {
            accept_common(t + jstar, r, s0 + jstar, (int)(uint32_t)key);
            __syncthreads();
            if (nrec == kRec) flush();
            // after a first acceptance at j = 0, the four proposals after the swap were all rejected
            used = jstar == 0 ? (uint32_t)K + 1 : (uint32_t)jstar + 1;
            win += 1u << 16;
        }
        advance(used);
        win += used;
        mark(QAP_PH_SCRATCH_ACCEPT);
        bump(QAP_PH_N_SCRATCH_ACC, 1);
    };

    // One Delta-mode step: scan up to step_e proposals per thread against the
    // unchanged Delta; on an acceptance, swap and update Delta.
    auto delta_step = [&]() __attribute__((always_inline)) {
        const uint64_t remain = t_end - t;
        const uint64_t cap = (uint64_t)step_e * kThreads;
        const uint32_t W = (uint32_t)(remain < cap ? remain : cap);
        const int32_t bound = reject_bound(temperature(temps, T0, t));
        uint32_t idx_l = idx0 + tid;
        while (idx_l >= m) idx_l -= m;
        bool tie = false;
        unsigned long long mine = ~0ull;
        {
            uint32_t idx = idx_l;
            for (int e = 0; e < step_e; e += 4) {
                // four proposals per lane loaded together, then tested in order
                int32_t dv[4];
                uint32_t jv[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    jv[k] = (uint32_t)(e + k) * kThreads + tid;
                    const uint32_t ix = rnd ? random_pair_index(seed, chain_id, t + jv[k], m) : idx;
                    dv[k] = (e + k < step_e && jv[k] < W) ? L.D[ix] : INT_MAX;
                    idx += nt_mod;
                    if (idx >= m) idx -= m;
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int32_t d = dv[k];
                    if (mine != ~0ull || d == INT_MAX) continue;
                    bool acc = d <= 0;
                    if (!acc && t0_inf && inf_clear(seed, chain_id, t + jv[k])) {
                        acc = true;   // T = +inf: accepted, and no near tie
                    } else if (!acc && d <= bound) {
                        const double z = exact_z(d, temps, T0, seed, chain_id, t + jv[k]);
                        acc = z < 0.0;
                        tie |= fabs(z) < kNearTie;
                    }
                    if (acc) mine = ((unsigned long long)jv[k] << 32) | (uint32_t)d;
                }
                if (mine != ~0ull) break;
            }
        }
        {
            const unsigned long long wk = __ballot(mine != ~0ull) ? wave_min_u64(mine) : ~0ull;
            if (lane == 0) s_wkey[buf][wave] = wk;
        }
        __syncthreads();
        const unsigned long long key = min_key();
        const uint32_t jstar = key == ~0ull ? UINT_MAX : (uint32_t)(key >> 32);
        if (tie) {   // rare: log the near ties a sequential run meets
            const uint32_t limit = jstar == UINT_MAX ? W - 1 : jstar;
            uint32_t idx = idx_l;
            for (int e = 0; e < step_e; ++e) {
                const uint32_t j = (uint32_t)e * kThreads + tid;
                if (j > limit) break;
                const int32_t d = L.D[rnd ? random_pair_index(seed, chain_id, t + j, m) : idx];
                if (d > 0 && d <= bound) {
                    const double z = exact_z(d, temps, T0, seed, chain_id, t + j);
                    if (fabs(z) < kNearTie) log_tie(t + j, d, z);
                }
                idx += nt_mod;
                if (idx >= m) idx -= m;
            }
        }
        mark(QAP_PH_DELTA_SCAN);
        bump(QAP_PH_N_SCAN_STEPS, 1);
        bump(QAP_PH_N_SCANNED, jstar == UINT_MAX ? W : jstar + 1);
        if (jstar == UINT_MAX) {
            advance(W);
            step_e = min(step_e * 2, uni(a.max_step));
            return;
        }
        step_e = 1;
        uint32_t istar = idx0 + (jstar % m);
        if (istar >= m) istar -= m;
        if (rnd) istar = random_pair_index(seed, chain_id, t + jstar, m);
        istar = uni(istar);
        int u, v;
        pair_of_u(n, istar, u, v);
        u = uni(u);
        v = uni(v);
        const int dstar = (int)(uint32_t)key;
        accept_common(t + jstar, u, v, dstar);
        __syncthreads();
        C.stage(u, v);
        if (nrec == kRec) flush();
        __syncthreads();
        C.taillard();
        C.gemv_part(u, v);
        __syncthreads();
        C.finish_rows(u, v, false);
        if (tid == 0) L.D[istar] = -dstar;
        __syncthreads();
        advance(jstar + 1);
        mark(QAP_PH_DELTA_UPDATE);
        bump(QAP_PH_N_DELTA_ACC, 1);
    };

    if constexpr (TABU) {
        // Tabu search.  When facility i leaves location l at iteration t,
        // returning i to l is tabu until iteration t + tenure; the swap (r, s)
        // is tabu when both its new assignments, r to p(s) and s to p(r), are,
        // and a tabu swap is still admissible when cost + Delta < best cost.
        // Each iteration makes the admissible swap of least Delta (lowest
        // packed index among equals), or the least Delta of all when none is
        // admissible.  Keys (Delta with the sign bit flipped, packed index)
        // order exactly so, as unsigned 64-bit numbers.
        int32_t* const T = a.tabu;
        const int32_t tenure = a.tenure;
        if (tid == 0) s_asp = best - cost;
        __syncthreads();
        const int fq = kThreads / n, cq = kThreads - fq * n;   // one step of the folded walk
        int f0 = 0, c0 = tid;
        while (c0 >= n) { c0 -= n; ++f0; }
        while (t < t_end) {
            const long long asp = s_asp;
            const int32_t tt = (int32_t)t;
            unsigned long long k_adm = ~0ull, k_all = ~0ull;
            int f = f0, c = c0;
            for (uint32_t k = tid; k < m; k += kThreads) {
                const bool first = c < n - 1 - f;
                const int r = first ? f : n - 2 - f;
                const int s = first ? f + 1 + c : c;
                const uint32_t off = rs32(n, r) + (uint32_t)(s - r - 1);
                const int32_t d = L.D[off];
                const unsigned long long key = ((unsigned long long)((uint32_t)d ^ 0x80000000u) << 32) | off;
                k_all = key < k_all ? key : k_all;
                const bool tabu = T[r * n + L.ps[s]] > tt && T[s * n + L.ps[r]] > tt;
                if ((!tabu || (long long)d < asp) && key < k_adm) k_adm = key;
                f += fq;
                c += cq;
                if (c >= n) { c -= n; ++f; }
            }
            k_adm = wave_min_u64(k_adm);
            k_all = wave_min_u64(k_all);
            if (lane == 0) { s_wkey[0][wave] = k_adm; s_wkey[1][wave] = k_all; }
            __syncthreads();
            unsigned long long ka = s_wkey[0][0], kl = s_wkey[1][0];
#pragma unroll
            for (int w = 1; w < kWaves; ++w) {
                ka = s_wkey[0][w] < ka ? s_wkey[0][w] : ka;
                kl = s_wkey[1][w] < kl ? s_wkey[1][w] : kl;
            }
            const unsigned long long key = uni64(ka != ~0ull ? ka : kl);
            const uint32_t istar = uni((uint32_t)key);
            const int dstar = (int)((uint32_t)(key >> 32) ^ 0x80000000u);
            mark(QAP_PH_DELTA_SCAN);
            int u, v;
            pair_of_u(n, istar, u, v);
            u = uni(u);
            v = uni(v);
            if (tid == 0) {   // before the swap moves them: u and v leave their locations
                T[u * n + L.ps[u]] = tt + tenure;
                T[v * n + L.ps[v]] = tt + tenure;
            }
            accept_common(t, u, v, dstar);
            __syncthreads();
            C.stage(u, v);
            if (nrec == kRec) flush();
            __syncthreads();
            C.taillard();
            C.gemv_part(u, v);
            __syncthreads();
            C.finish_rows(u, v, false);
            if (tid == 0) {
                L.D[istar] = -dstar;
                s_asp = best - cost;
            }
            __threadfence_block();   // the tabu entries written above, for the next iteration's reads
            __syncthreads();
            t = uni64(t + 1);
            mark(QAP_PH_DELTA_UPDATE);
            bump(QAP_PH_N_DELTA_ACC, 1);
        }
    } else
    while (t < t_end) {
        if (mode == 0) {
            if (kw == 1) {
                if (!rnd && s0 + kWaves < n && t + kWaves + 1 <= t_end) scratch_round_ahead();
                else scratch_round(IC<1>{});
            } else if (kw == 2) {
                scratch_round(IC<2>{});
            } else {
                scratch_round(IC<4>{});
            }
            if ((win & 0xffffu) >= kSwitchWindow) {
                const uint32_t win_iters = win & 0xffffu, win_acc = win >> 16;
                // few proposals per round while most are accepted, more as acceptance
                // falls: 1 per wave above 1/4, 2 above 1/8, else 4 (the cut points
                // measured fastest for the N = 150 chain among 1/2..1/8 and 1/6..1/32)
                kw = win_acc * 4 >= win_iters ? 1 : (win_acc * 8 >= win_iters ? 2 : 4);
                const uint32_t flags = uni(a.flags), switch_permille = uni(a.switch_permille);
                if (!(flags & kFlagScratchOnly) && win_acc * 1000u < win_iters * switch_permille) {
                    C.build_delta();
                    mode = 1;
                    step_e = 1;
                    mark(QAP_PH_BUILD);
                    bump(QAP_PH_SWITCH_T, t);
                }
                win = 0;
            }
        } else {
            delta_step();
        }
    }

    // ------------------------------------------------------------ write back
    __syncthreads();
    if (nrec > 0) flush();
    mark(QAP_PH_IO);
    // Delta is current in Delta mode; in scratch mode it is rebuilt when the
    // schedule ends and otherwise left stale
    int out_mode = mode == 1 ? QAP_MODE_DELTA : QAP_MODE_SCRATCH_STALE;
    if (mode == 0 && t >= a.iters) {
        C.build_delta();
        out_mode = QAP_MODE_SCRATCH;
    }
    __syncthreads();
    mark(QAP_PH_BUILD);
    if (PL == 0 && out_mode != QAP_MODE_SCRATCH_STALE)
        for (uint32_t i = tid; i < m; i += kThreads) a.delta[i] = L.D[i];
    for (int e = tid; e < n * n; e += kThreads) {
        const int i = e / n, j = e - i * n;
        a.Bp[e] = (int32_t)L.Bb[i * P + j] + a.b_min;
    }
    for (int i = tid; i < n; i += kThreads) a.p[i] = L.ps[i];
    if (tid == 0) {
        qap_chain_state st;
        st.t = t; st.accepts = accepts; st.near_ties = s_ties; st.hash = hash;
        st.cost = cost; st.best_cost = best; st.best_iter = best_iter;
        st.status = QAP_OK;
        st.mode = out_mode;
        *a.state = st;
        mark(QAP_PH_IO);
        bump(QAP_PH_TOTAL, clock64() - prof_start);
    }
    if (prof) {
        __syncthreads();
        if (tid < QAP_PHASES) atomicAdd((unsigned long long*)&a.prof[tid], s_prof[tid]);
    }
}

template <bool SYM, int PL, bool PROF>
__global__ void __launch_bounds__(kThreads) k_chain_wg(ChainArgs a)
{
    extern __shared__ __align__(16) char smem[];
    chain_run<SYM, PL, false, PROF>(a, smem);
}

template <bool SYM, int PL>
__global__ void __launch_bounds__(kThreads) k_tabu_wg(ChainArgs a)
{
    extern __shared__ __align__(16) char smem[];
    chain_run<SYM, PL, true>(a, smem);
}

// Many independent chains in one persistent launch: each workgroup takes the
// next chain from a device-wide queue and runs it (or its next slice) with the
// one-workgroup routine above.  One instantiation per placement; each skips
// the chains of the other placements, so all can walk the same descriptor
// array concurrently.  With an LDS split, a launch of the same placement runs
// either the chains whose LDS bytes exceed it (cls 1) or the others (cls 0),
// each kind with its own queue position.  PROF as for k_chain_wg.
template <int PL, bool PROF>
__global__ void __launch_bounds__(kThreads) k_chain_batch(BatchArgs b)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ int s_idx;
    unsigned* next = &b.ws->next[2 * PL + b.cls];
    for (;;) {
        if (threadIdx.x == 0) s_idx = (int)atomicAdd(next, 1u);
        __syncthreads();
        const int idx = s_idx;
        __syncthreads();
        if (idx >= b.n_chains) break;
        const int c = b.order ? b.order[idx] : idx;
        const qap_chain_desc d = b.descs[c];
        int pc = wg_placement(d.n, d.symmetric != 0);
        if (pc < b.min_place) pc = b.min_place;
        if (pc != PL) continue;
        if (b.lds_split && (wg_layout(d.n, wg_quads_of(d.n), d.symmetric != 0, pc, nullptr, nullptr) > b.lds_split) !=
                               (b.cls != 0))
            continue;
        ChainArgs a{};
        a.n = d.n;
        a.quads = wg_quads_of(d.n);
        a.max_step = 16;
        a.flags = d.flags;
        a.switch_permille = d.switch_permille ? d.switch_permille : kDefaultSwitchPermille;
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
        if (d.symmetric) chain_run<true, PL, false, PROF>(a, smem);
        else chain_run<false, PL, false, PROF>(a, smem);
        __syncthreads();
    }
}

__global__ void k_batch_reset(BatchWs* ws)
{
    for (int i = 0; i < kBatchKinds; ++i) ws->next[i] = 0;
}

// Holds its stream for `ticks` of the constant-rate wall clock, so that the
// kernel queued behind it is dispatched after those of the other streams.
__global__ void k_hold(uint64_t ticks)
{
    const uint64_t t0 = wall_clock64();
    while (wall_clock64() - t0 < ticks) __builtin_amdgcn_s_sleep(8);
}

}  // namespace

int wg_quads(int n) { return wg_quads_of(n); }   // odd dword pitch: strided row reads hit distinct banks

int wg_place(int n, bool symmetric) { return wg_placement(n, symmetric); }

size_t lds_wg_bytes(int n, bool symmetric, int place)
{
    return wg_layout(n, wg_quads_of(n), symmetric, place, nullptr, nullptr);
}

size_t wg_scratch_bytes(int n, bool symmetric, int place)
{
    return wg_global_bytes(n, wg_quads_of(n), symmetric, place);
}

int launch_chain_batch(const BatchArgs& b, int groups, const int count[kBatchKinds], int threads,
                       const size_t lds[kBatchKinds], hipStream_t stream)
{
    if (threads != kThreads) return QAP_E_INVAL;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return QAP_E_DEVICE;
    const void* const fns_all[2][kPlacements] = {
        {(const void*)k_chain_batch<0, false>, (const void*)k_chain_batch<1, false>,
         (const void*)k_chain_batch<2, false>, (const void*)k_chain_batch<3, false>},
        {(const void*)k_chain_batch<0, true>, (const void*)k_chain_batch<1, true>,
         (const void*)k_chain_batch<2, true>, (const void*)k_chain_batch<3, true>}};
    const void* const* fns = fns_all[b.prof ? 1 : 0];
    int g[kBatchKinds] = {};
    double full[kBatchKinds] = {};   // workgroups of the kind that fill the GPU
    int kinds = 0;
    for (int k = 0; k < kBatchKinds; ++k) {
        if (count[k] == 0) continue;
        kinds += 1;
        const void* fn = fns[k / 2];
        if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds[k]) != hipSuccess)
            return QAP_E_DEVICE;
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kThreads, lds[k]) != hipSuccess)
            return QAP_E_DEVICE;
        full[k] = (double)(per_cu < 1 ? 1 : per_cu) * cus;
        const int gg = groups > 0 ? groups : (int)full[k];
        g[k] = gg > count[k] ? count[k] : gg;
    }
    if (kinds > 4) return QAP_E_INVAL;   // the caller's stream and three side streams
    // The kernels run side by side, and the hardware may dispatch them in any
    // order.  So that none of them waits for another's workgroups to finish,
    // all of them must be resident at once: when their shares of the GPU add
    // up to more than one, the kinds of the smaller chains get fewer
    // (persistent) workgroups, each then running more chains in turn.
    if (groups <= 0 && kinds > 1) {
        double used = 0;
        for (int k = kBatchKinds - 1; k >= 0; --k) {
            if (g[k] == 0) continue;
            const double left = 1.0 - used;
            const int fit = (int)(left * full[k]);
            if (g[k] > fit) g[k] = fit < 1 ? 1 : fit;
            used += g[k] / full[k];
        }
    }
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, stream, b.ws);
    BatchArgs args[kBatchKinds];
    for (int k = 0; k < kBatchKinds; ++k) {
        args[k] = b;
        args[k].cls = k % 2;
    }
    // With LDS classes and one kind of small chains (class 0), that kind runs
    // last on the caller's stream, behind a 1 ms hold: the hardware may
    // dispatch side-by-side kernels in any order, and class-0 workgroups
    // dispatched first would take a little LDS on every CU and leave none
    // whole for the larger chains, which would then wait for them (3.2 s
    // instead of 2.5 s for the 512-chain mix).
    int small = -1, nsmall = 0;
    if (b.lds_split && kinds > 1)
        for (int k = 0; k < kBatchKinds; k += 2)
            if (g[k] > 0) { small = k; ++nsmall; }
    if (nsmall != 1) small = -1;
    // the other kinds run side by side: the first on the caller's stream
    // (when no small kind takes it), the others on side streams forked from
    // it and joined back.  The kinds of the largest chains are launched first,
    // so that their workgroups (the longest-running ones) are dispatched
    // before the small chains take the CUs.
    hipStream_t used[kBatchKinds];
    hipEvent_t joins[kBatchKinds];
    int nused = 0;
    for (int k = kBatchKinds - 1; k >= 0; --k) {
        if (g[k] == 0) continue;
        if (nused == 0 && small < 0) {
            used[nused++] = stream;
            continue;
        }
        if (k == small) continue;
        const int which = small < 0 ? nused - 1 : nused;
        hipStream_t side;
        hipEvent_t fork, join;
        if (side_stream(which, &side, &fork, &join) != QAP_OK) return QAP_E_DEVICE;
        if (hipEventRecord(fork, stream) != hipSuccess || hipStreamWaitEvent(side, fork, 0) != hipSuccess)
            return QAP_E_DEVICE;
        used[nused] = side;
        joins[nused] = join;
        ++nused;
    }
    int i = 0;
    for (int k = kBatchKinds - 1; k >= 0; --k) {
        if (g[k] == 0 || k == small) continue;
        void* kargs[] = {&args[k]};
        if (hipLaunchKernel(fns[k / 2], dim3(g[k]), dim3(kThreads), kargs, lds[k], used[i]) != hipSuccess)
            return QAP_E_DEVICE;
        ++i;
    }
    if (small >= 0) {
        int khz = 0;   // the wall clock's rate
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) khz = 100000;
        hipLaunchKernelGGL(k_hold, dim3(1), dim3(64), 0, stream, (uint64_t)khz);   // 1 ms
        void* kargs[] = {&args[small]};
        if (hipLaunchKernel(fns[small / 2], dim3(g[small]), dim3(kThreads), kargs, lds[small], stream) != hipSuccess)
            return QAP_E_DEVICE;
    }
    for (int j = small < 0 ? 1 : 0; j < nused; ++j)
        if (hipEventRecord(joins[j], used[j]) != hipSuccess || hipStreamWaitEvent(stream, joins[j], 0) != hipSuccess)
            return QAP_E_DEVICE;
    return QAP_OK;
}

int launch_chain_wg(const ChainArgs& a, bool symmetric, int place, hipStream_t stream, bool tabu)
{
    if (place < 0 || place >= kPlacements || (place >= 2 && a.gscratch == nullptr)) return QAP_E_INVAL;
    const size_t bytes = lds_wg_bytes(a.n, symmetric, place);
    // with and without the phase counters
    const void* fns[2][2][kPlacements] = {
        {{(const void*)k_chain_wg<false, 0, false>, (const void*)k_chain_wg<false, 1, false>,
          (const void*)k_chain_wg<false, 2, false>, (const void*)k_chain_wg<false, 3, false>},
         {(const void*)k_chain_wg<true, 0, false>, (const void*)k_chain_wg<true, 1, false>,
          (const void*)k_chain_wg<true, 2, false>, (const void*)k_chain_wg<true, 3, false>}},
        {{(const void*)k_chain_wg<false, 0, true>, (const void*)k_chain_wg<false, 1, true>,
          (const void*)k_chain_wg<false, 2, true>, (const void*)k_chain_wg<false, 3, true>},
         {(const void*)k_chain_wg<true, 0, true>, (const void*)k_chain_wg<true, 1, true>,
          (const void*)k_chain_wg<true, 2, true>, (const void*)k_chain_wg<true, 3, true>}}};
    const void* tfns[2][kPlacements] = {
        {(const void*)k_tabu_wg<false, 0>, (const void*)k_tabu_wg<false, 1>, (const void*)k_tabu_wg<false, 2>,
         (const void*)k_tabu_wg<false, 3>},
        {(const void*)k_tabu_wg<true, 0>, (const void*)k_tabu_wg<true, 1>, (const void*)k_tabu_wg<true, 2>,
         (const void*)k_tabu_wg<true, 3>}};
    const void* fn = tabu ? tfns[symmetric ? 1 : 0][place] : fns[a.prof ? 1 : 0][symmetric ? 1 : 0][place];
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess)
        return QAP_E_DEVICE;
    ChainArgs args = a;
    args.quads = wg_quads_of(a.n);
    void* kargs[] = {&args};
    if (hipLaunchKernel(fn, dim3(1), dim3(kThreads), kargs, bytes, stream) != hipSuccess) return QAP_E_DEVICE;
    return QAP_OK;
}

}  // namespace qapsa
