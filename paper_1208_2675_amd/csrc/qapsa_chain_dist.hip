// qapsa_chain_dist.hip -- one annealing chain spread over G workgroups, for
// instances too large for one CU (N up to about 2600 symmetric and 2000
// asymmetric on 256 CUs with byte-range values, less with wider values).
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
//   - the owners of rows u and v are then stale for those rows; they read the
//     published values (tagged with the update that wrote them) during the
//     next exchange.  Until then the scan reads a pair (r, s) from row r
//     instead of row s when s is stale.
// While windows accept their first proposal, the rows of the next window's
// first proposal are requested during the exchange (speculative staging).
// Random proposal order (QAP_FLAG_RANDOM_ORDER): every workgroup draws the
// whole window and tests the proposals it holds.
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

// Wave-uniform copies (scalar registers) of values the workgroup agrees on but
// that come back from LDS, so that what derives from them stays scalar.
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint32_t uni(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }
__device__ __forceinline__ unsigned long long uni64(unsigned long long x)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ uint32_t dot4(uint32_t a, uint32_t b, uint32_t c) { return __builtin_amdgcn_udot4(a, b, c, false); }

// Element types of A and B' (value minus the matrix minimum): bytes when both
// value ranges fit 0..255, 16-bit words up to 65535, else 32-bit words.  Every
// swap cost is a combination of products of such values that the Delta bound
// keeps inside int32, so all sums are taken modulo 2^32 (wrapping dot products
// and multiplies) and come out exact.
template <typename E> struct Elem;
template <> struct Elem<uint8_t> {
    static constexpr uint32_t kMax = 0xffu;
    // four products of a word's bytes, added to c modulo 2^32
    static __device__ __forceinline__ uint32_t dot(uint32_t a, uint32_t b, uint32_t c) { return __builtin_amdgcn_udot4(a, b, c, false); }
};
template <> struct Elem<uint16_t> {
    static constexpr uint32_t kMax = 0xffffu;
    static __device__ __forceinline__ uint32_t dot(uint32_t a, uint32_t b, uint32_t c)
    {
        typedef unsigned short v2u16 __attribute__((ext_vector_type(2)));
        return __builtin_amdgcn_udot2(__builtin_bit_cast(v2u16, a), __builtin_bit_cast(v2u16, b), c, false);
    }
};
template <> struct Elem<uint32_t> {
    static constexpr uint32_t kMax = 0xffffffffu;
    static __device__ __forceinline__ uint32_t dot(uint32_t a, uint32_t b, uint32_t c) { return a * b + c; }
};

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

// Sum over the lanes with the same lane mod K (K = 4, 8 or 16), returned to
// every lane: rotations within 16-lane rows, then v_permlane16_swap and
// v_permlane32_swap fold the rows (no LDS round trips).
__device__ __forceinline__ uint32_t stride_sum(uint32_t v, uint32_t K)
{
    if (K <= 4) v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x124, 0xf, 0xf, false);   // row_ror:4
    if (K <= 8) v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xf, 0xf, false);   // row_ror:8
    const auto a = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    v = a[0] + a[1];
    const auto b = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return b[0] + b[1];
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

// Swap cost of (r, s) from the all-k sums S over rows and columns (general
// form): the k = r and k = s terms are dropped and the two terms of Eq. (1)
// with both indices in {r, s} are added.  Arguments are shifted entries at
// (r,r), (r,s), (s,r), (s,s) of A and B'.
// (Arithmetic modulo 2^32: exact for every value width, see Elem.)
__device__ __forceinline__ int finish_gen(uint32_t S, uint32_t arr, uint32_t ars, uint32_t asr, uint32_t ass,
                                          uint32_t brr, uint32_t brs, uint32_t bsr, uint32_t bss)
{
    const uint32_t corner = (arr - ass) * (bss - brr) + (ars - asr) * (bsr - brs);
    const uint32_t row_r = (arr - asr) * (bsr - brr);
    const uint32_t row_s = (ars - ass) * (bss - brs);
    const uint32_t col_r = (arr - ars) * (brs - brr);
    const uint32_t col_s = (asr - ass) * (bss - bsr);
    return (int)(S - row_r - row_s - col_r - col_s + corner);
}

__device__ __forceinline__ int finish_sym(uint32_t S, uint32_t arr, uint32_t ars, uint32_t asr, uint32_t ass,
                                          uint32_t brr, uint32_t brs, uint32_t bsr, uint32_t bss)
{
    const uint32_t corner = (arr - ass) * (bss - brr) + (ars - asr) * (bsr - brs);
    const uint32_t row_r = (arr - asr) * (bsr - brr);
    const uint32_t row_s = (ars - ass) * (bss - brs);
    return (int)(2u * (S - row_r - row_s) + corner);
}

// Wait until this wave's global stores have completed (vmcnt = 0).
__device__ __forceinline__ void wait_stores() { __builtin_amdgcn_s_waitcnt(0x0F70); }

__device__ __forceinline__ int get(int* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// Failure codes of a run in DistWs::err; the larger one wins when several
// workgroups fail at once (every other workgroup stops at its next exchange).
constexpr int kErrTimeout = 1;
constexpr int kErrTieOverflow = 2;
__device__ __forceinline__ void raise_err(int* p, int code)
{
    __hip_atomic_fetch_max(p, code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Rows are P elements (4 q bytes, zero padded); see Elem for the element types.
struct Lds {
    int32_t* D;      // [R][n] full rows of Delta
    char* Ab;        // [R][P] rows of A - a_min (symmetric form; the general form reads A from device memory)
    char* Bb;        // [R][P] rows of B' - b_min
    char* Bt;        // [R][P] columns of B' - b_min (general form)
    char* Su;        // [P] row u of A - a_min
    char* Sv;
    char* Tu;        // [P] row u of B' - b_min after the swap
    char* Tv;
    char* Scu;       // [P] column u of A - a_min (general form)
    char* Scv;
    char* Tcu;       // [P] column u of B' - b_min after the swap (general form)
    char* Tcv;
    // per k: (A[k][u]-A[k][v], A[u][k]-A[v][k]) and (B'[k][u]-B'[k][v], B'[u][k]-B'[v][k])
    // after the swap (equal halves when symmetric): int16 pairs for bytes, int32 pairs otherwise
    char* abp;
    char* bbp;
    int16_t* ps;     // [n]
    // scratch-mode launches (no Delta rows, no staging)
    char* Ar;        // [R][P] own rows of A - a_min (general form)
    char* Ac;        // [R][P] own columns of A - a_min (general form)
    int32_t* dg;     // [2][n] diagonals of A and B
};

__host__ __device__ inline size_t a16(size_t x) { return (x + 15) & ~(size_t)15; }

// LDS layout of one workgroup.  The general (asymmetric) form keeps its own
// columns of B' beside its rows and stages columns u, v as well as rows; its
// rows and columns of A are read from byte copies in device memory instead
// (they never change), so that N = 2000 still fits one CU's LDS.  A
// scratch-mode launch keeps no Delta and stages nothing: its own rows (and
// columns) of A and B', the diagonals of A and B, and p.
__host__ __device__ inline size_t dist_layout(int n, int G, int q, int esize, bool sym, bool scratch, char* base,
                                              Lds* L)
{
    const size_t R = (size_t)(n + G - 1) / G, P = 4 * (size_t)q;   // P: row bytes here
    const size_t pw = esize == 1 ? 4 : 8;                          // bytes of one difference pair
    size_t off = 0;
    auto take = [&](size_t b) { char* p = base ? base + off : nullptr; off = a16(off + b); return p; };
    if (scratch) {
        char* ab = sym ? take(R * P) : nullptr;
        char* ar = sym ? nullptr : take(R * P);
        char* ac = sym ? nullptr : take(R * P);
        char* bb = take(R * P);
        char* bt = sym ? nullptr : take(R * P);
        char* dg = take(8 * (size_t)n);
        char* ps = take(2 * (size_t)n);
        if (L) {
            *L = Lds{};
            L->Ab = ab; L->Ar = ar; L->Ac = ac; L->Bb = bb; L->Bt = bt;
            L->dg = (int32_t*)dg; L->ps = (int16_t*)ps;
        }
        return off;
    }
    char* d = take(4 * R * n);
    char* ab = sym ? take(R * P) : nullptr;
    char* bb = take(R * P);
    char* bt = sym ? nullptr : take(R * P);
    char* su = take(P);
    char* sv = take(P);
    char* tu = take(P);
    char* tv = take(P);
    char* scu = sym ? nullptr : take(P);
    char* scv = sym ? nullptr : take(P);
    char* tcu = sym ? nullptr : take(P);
    char* tcv = sym ? nullptr : take(P);
    char* abp = take(pw * (size_t)n);
    char* bbp = take(pw * (size_t)n);
    char* ps = take(2 * (size_t)n);
    if (L) {
        *L = Lds{};
        L->D = (int32_t*)d; L->Ab = ab; L->Bb = bb; L->Bt = bt;
        L->Su = su; L->Sv = sv; L->Tu = tu; L->Tv = tv;
        L->Scu = scu; L->Scv = scv; L->Tcu = tcu; L->Tcv = tcv;
        L->abp = abp; L->bbp = bbp; L->ps = (int16_t*)ps;
    }
    return off;
}

constexpr int kRec = 64;
struct Rec {
    uint64_t t;
    uint32_t uv;
    int32_t d;
};

// Exchange slots: bits 63..54 the window number (mod 1024), 53..32 the window
// offset j of the workgroup's first acceptance, 31..0 its Delta; a workgroup
// without acceptance publishes all ones in bits 53..0.  The minimum over slots of the
// low 54 bits is the window's first acceptance.
constexpr unsigned long long kKeyBits = (1ull << 54) - 1;
constexpr unsigned long long kNone = kKeyBits;

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ unsigned long long dpp_min_step(unsigned long long v)
{
    const uint32_t lo = __builtin_amdgcn_update_dpp(0xffffffffu, (uint32_t)v, CTRL, ROW_MASK, 0xf, false);
    const uint32_t hi = __builtin_amdgcn_update_dpp(0xffffffffu, (uint32_t)(v >> 32), CTRL, ROW_MASK, 0xf, false);
    const unsigned long long o = ((unsigned long long)hi << 32) | lo;
    return o < v ? o : v;
}

// Minimum over the 64 lanes (DPP row shifts and broadcasts; lanes that read
// outside their row see the identity), returned to every lane from lane 63.
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

__device__ __forceinline__ void put64(unsigned long long* p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long get64(unsigned long long* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int kMaxPerThread = 8;   // n <= 8 * threads
constexpr int kTieSlots = 16;      // near ties one workgroup records per scan window
constexpr int kMaxOwnRows = 64;    // rows per workgroup (n <= 64 G)

// Eq. (2) for Delta > 0 at iteration t, out of line (keeps the FP64 log and the
// generator from occupying scalar registers across the kernel).
__device__ __noinline__ bool exact_test(int d, const double* temps, double T0, uint64_t seed, uint32_t chain,
                                        uint64_t t, double* z)
{
    return metropolis_positive(d, temperature(temps, T0, t), uniform_r(seed, chain, t), z);
}
// The three cooling-table entries of T_t, read apart from the products that
// make T_t (temperature()) so that their latency can overlap other work.
struct TempParts {
    double h, m, l;
};
__device__ __forceinline__ TempParts temp_parts(const double* __restrict__ temps, uint64_t t)
{
    return TempParts{temps[2048 + (t >> 20)], temps[1024 + ((t >> 10) & 1023u)], temps[t & 1023u]};
}
// T_t from its table entries, in the order temperature() multiplies them
__device__ __forceinline__ double temp_of(double T0, const TempParts& p) { return ((T0 * p.h) * p.m) * p.l; }

// The pair `steps` places after (r, s) in the cyclic row-major order.
__device__ __forceinline__ void advance_pair(int n, int& r, int& s, int steps)
{
    s += steps;
    while (s >= n) {
        const int off = s - n;
        r = r + 1 == n - 1 ? 0 : r + 1;
        s = r + 1 + off;
    }
}

// SCR: the scratch-mode instantiation (returns at once when the chain is to
// run in Delta mode); otherwise the Delta-mode one.  Two instantiations keep
// the registers of each mode to themselves.
template <bool SYM, typename E, bool SCR>
__global__ void __launch_bounds__(512) k_chain_dist(DistArgs a)
{
    constexpr bool kByte = sizeof(E) == 1;
    constexpr int kEpw = 4 / (int)sizeof(E);   // elements per 32-bit word
    extern __shared__ __align__(16) char smem[];
    __shared__ unsigned long long s_wkey[16];    // first acceptance per wave of the window
    __shared__ unsigned long long s_key;         // the grid-wide first acceptance
    __shared__ int s_ok;
    __shared__ int s_rf_bad;                     // a published value did not arrive within the spin bound
    __shared__ int s_selfw[16][2];               // per-wave partial self terms of u, v
    __shared__ int s_pub[2 * kMaxOwnRows];       // this workgroup's published Delta(r, u), Delta(r, v), row-major
    __shared__ int s_ntie[2];                    // near ties of the window, by window parity
    __shared__ unsigned long long s_tie_j[2][kTieSlots];
    __shared__ int s_tie_d[2][kTieSlots];
    __shared__ double s_tie_z[2][kTieSlots];
    __shared__ Rec s_rec[kRec];
    __shared__ unsigned long long s_prof[QAP_PHASES];
    __shared__ uint32_t s_gsum[16][kScratchK];   // scratch mode: per-wave sums of the gathered partials
    __shared__ int s_swap[4];                     // scratch mode: u, v and their new p values

    const int n = a.n, G = gridDim.x, w = blockIdx.x;
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = uni(tid >> 6), nwaves = nt >> 6;
    const int q = a.quads, P = kEpw * q;      // words and elements per row
    const int Rw = (n - w + G - 1) / G;          // rows owned by this workgroup
    const int Rmax = (n + G - 1) / G;
    const int C = Rw;                             // columns s = w + G c of this workgroup (same count)
    const uint32_t m = (uint32_t)((int64_t)n * (n - 1) / 2);
    Lds L_;
    dist_layout(n, G, q, (int)sizeof(E), SYM, SCR, smem, &L_);
    // the LDS arrays as plain pointer values
    int32_t* const lD = L_.D;
    E* const lAb = (E*)L_.Ab;
    E* const lBb = (E*)L_.Bb;
    E* const lBt = (E*)L_.Bt;
    E* const lSu = (E*)L_.Su;
    E* const lSv = (E*)L_.Sv;
    E* const lTu = (E*)L_.Tu;
    E* const lTv = (E*)L_.Tv;
    E* const lScu = (E*)L_.Scu;
    E* const lScv = (E*)L_.Scv;
    E* const lTcu = (E*)L_.Tcu;
    E* const lTcv = (E*)L_.Tcv;
    uint32_t* const labp = (uint32_t*)L_.abp;   // bytes: int16 pairs
    uint32_t* const lbbp = (uint32_t*)L_.bbp;
    uint2* const labp2 = (uint2*)L_.abp;        // wider values: int32 pairs
    uint2* const lbbp2 = (uint2*)L_.bbp;
    // general form: copies (value - minimum, rows padded to P) in device memory
    const E* __restrict__ const gA = (const E*)a.Ab;     // A
    const E* __restrict__ const gAt = (const E*)a.Atb;   // A^T
    const E* __restrict__ const gBt = (const E*)a.Btb;   // B^T
    int16_t* const lps = L_.ps;
    DistWs* ws = a.ws;
    // published values, workgroup-major: [2 parities][G workgroups][Rmax own rows][2]
    unsigned long long* X = a.X;

    const bool prof = a.prof != nullptr && w == 0;
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
    auto bump = [&](int k, unsigned long long x) __attribute__((always_inline)) { if (prof && tid == 0) atomicAdd(&s_prof[k], x); };

    // ---------------------------------------------------------------- load
    // A call with nothing to do (failed chain, or t already at t_end) leaves
    // everything as it is.  The scratch-mode instantiation runs when scratch
    // mode is forced, or when the chain's state says Delta is not being kept
    // and Delta mode is not forced; it keeps no Delta and holds its own rows
    // and columns of A in LDS (the general form).
    const qap_chain_state st0 = *a.state;
    if (st0.status != QAP_OK || st0.t >= a.t_end) return;
    const bool scr = SCR && ((a.flags & kFlagDeltaOnly) ? false : (a.flags & kFlagScratchOnly) ? true
                                                                                             : st0.mode != QAP_MODE_DELTA);
    if (SCR && !scr) return;
    constexpr bool a_lds = !SYM && SCR;           // scratch mode: own rows and columns of A in LDS
    E* const lAr = (E*)L_.Ar;                     // [R][P] own rows of A - a_min (general form, scratch mode)
    E* const lAc = (E*)L_.Ac;                     // [R][P] own columns of A - a_min
    if (tid == 0) { s_ok = 1; s_rf_bad = 0; s_ntie[0] = 0; s_ntie[1] = 0; }
    __syncthreads();
    for (int lr = 0; lr < Rw; ++lr) {
        const int r = w + G * lr;
        const int32_t* up = a.delta + rs32(n, r) - r - 1;   // row r, s > r
        if constexpr (!SCR)
            for (int s = tid; s < n; s += nt) {
                int d = 0;
                if (s > r) d = up[s];
                else if (s < r) d = a.delta[rs32(n, s) + r - s - 1];
                lD[lr * n + s] = d;
            }
        for (int k = tid; k < P; k += nt) {
            uint32_t av = 0, bv = 0, cv = 0, ac = 0;
            if (k < n) {
                av = (uint32_t)a.A[r * n + k] - (uint32_t)a.a_min;
                bv = (uint32_t)a.Bp[r * n + k] - (uint32_t)a.b_min;
                if (!SYM) cv = (uint32_t)a.Bp[k * n + r] - (uint32_t)a.b_min;   // column r of B'
                if (a_lds) ac = (uint32_t)a.A[k * n + r] - (uint32_t)a.a_min;   // column r of A
                if (av > Elem<E>::kMax || bv > Elem<E>::kMax || cv > Elem<E>::kMax || ac > Elem<E>::kMax) s_ok = 0;
            }
            if constexpr (SYM) lAb[lr * P + k] = (E)av;
            lBb[lr * P + k] = (E)bv;
            if constexpr (!SYM) lBt[lr * P + k] = (E)cv;
            if constexpr (a_lds) { lAr[lr * P + k] = (E)av; lAc[lr * P + k] = (E)ac; }
        }
    }
    if constexpr (!SCR)
        for (int k = tid; k < P; k += nt) {
            lSu[k] = 0; lSv[k] = 0; lTu[k] = 0; lTv[k] = 0;
            if constexpr (!SYM) { lScu[k] = 0; lScv[k] = 0; lTcu[k] = 0; lTcv[k] = 0; }
        }
    for (int i = tid; i < n; i += nt) {
        const int pi = a.p[i];
        if (pi < 0 || pi >= n) s_ok = 0;   // p indexes B below
        lps[i] = (int16_t)pi;
        if constexpr (SCR) { L_.dg[i] = a.A[i * n + i]; L_.dg[n + i] = a.B[i * n + i]; }
    }
    __syncthreads();
    if (!s_ok || (!scr && st0.mode == QAP_MODE_SCRATCH_STALE)) {
        if (w == 0 && tid == 0) a.state->status = s_ok ? QAP_E_STATE : QAP_E_INVAL;
        return;   // every workgroup takes the same branch: the instance and state are shared
    }
    if (tid == 0) mark(QAP_PH_IO);

    // kernel arguments used inside the helpers below, as plain values
    const uint64_t t_end = a.t_end;
    const double T0 = a.T0;
    const double* __restrict__ temps = a.temps;
    const uint64_t seed = a.seed;
    const uint32_t chain_id = a.chain_id;
    const uint64_t spin_limit = a.spin_limit;
    const bool t0_inf = __builtin_isinf(T0);
    const bool rnd = a.random_order != 0;
    unsigned long long* const slot_base = a.slots;
    uint64_t t = st0.t;
    unsigned long long accepts = st0.accepts, hash = st0.hash, best_iter = st0.best_iter;
    long long cost = st0.cost, best = st0.best_cost;
    uint32_t idx0 = (uint32_t)(t % m);
    int r0, s0;
    pair_of_u(n, idx0, r0, s0);
    unsigned long long epoch = 0;
    int par = 0;
    int pu = -1, pv = -1, pd = 0, ppar = 0;       // stale rows of the last swap, its Delta, its X parity
    uint32_t ptag = 0;                             // the tag its published values carry
    uint32_t kwin = a.kmin;
    int nrec = 0;
    int tb = 0;                                    // tie buffer of the current window
    bool alive = true;

    // Rows u, v of A and (through p) of B' after the swap (u, v): A[u][.],
    // A[v][.], B'[u][.] = B[p(v)][p(.)] and B'[v][.] = B[p(u)][p(.)], this
    // thread's columns, all loads issued before any result is used.
    const int nk = (n + nt - 1) / nt;   // columns per thread (uniform)
    // The general form also stages columns u, v of A and of B' (A[k][u],
    // A[k][v], B'[k][u], B'[k][v] from the copies of A^T and B^T): bytes packed
    // four to a register in ge here; wider values are read where they are
    // written to LDS (four more registers per column would spill).
    auto stage_loads = [&](int u, int v, int* ga, int* gb, int* gc, int* gd, uint32_t* ge)
        __attribute__((always_inline)) {
        const int pu_new = uni((int)lps[v]), pv_new = uni((int)lps[u]);
#pragma unroll
        for (int i = 0; i < kMaxPerThread; ++i) {
            if (i >= nk) break;
            const int k = min(tid + i * nt, n - 1);
            const int pk = k == u ? pu_new : (k == v ? pv_new : (int)lps[k]);
            ga[i] = a.A[u * n + k];
            gb[i] = a.A[v * n + k];
            gc[i] = a.B[pu_new * n + pk];
            gd[i] = a.B[pv_new * n + pk];
            if constexpr (!SYM && kByte) {
                ge[i] = (uint32_t)gAt[(size_t)u * P + k] | ((uint32_t)gAt[(size_t)v * P + k] << 8) |
                        ((uint32_t)gBt[(size_t)pu_new * P + pk] << 16) | ((uint32_t)gBt[(size_t)pv_new * P + pk] << 24);
            }
        }
    };
    // Speculative staging: while the previous window accepted its first
    // proposal (every proposal accepted, or a high acceptance rate), the rows
    // of this window's first proposal (r0, s0) are requested during the
    // exchange, so that their latency overlaps it; they are used only when
    // that proposal is the one accepted, and requested again otherwise.
    bool last_j0 = false;
    int ga[kMaxPerThread], gb[kMaxPerThread], gc[kMaxPerThread], gd[kMaxPerThread];
    uint32_t ge[kMaxPerThread];

    // Stale own rows take the published Delta(., u), Delta(., v) of the last
    // swap.  Each published value carries the tag of the update that wrote it,
    // so a reader needs no ordering with the writer's slot: it reads until the
    // tag is the expected one.  This runs inside the exchange, on the waves
    // that do not poll (threads first, first + step, ...), so that its loads
    // overlap the exchange instead of following it.
    auto refresh_part = [&](int first, int step) __attribute__((always_inline)) {
        if (pu < 0) return;
        for (int which = 0; which < 2; ++which) {
            const int x = which == 0 ? pu : pv, y = which == 0 ? pv : pu;
            if (x % G != w) continue;
            int32_t* row = lD + (x / G) * n;
            unsigned long long* src = X + ppar * G * Rmax * 2 + which;
            for (int s = first; s < n; s += step) {
                if (s == x) { row[s] = 0; continue; }
                if (s == y) { row[s] = -pd; continue; }
                unsigned long long* e = src + ((s % G) * Rmax + s / G) * 2;
                unsigned long long xv = get64(e);
                uint64_t spins = 0;
                while ((uint32_t)(xv >> 32) != ptag) {
                    if (++spins > spin_limit || ((spins & 63) == 0 && get(&ws->err))) { s_rf_bad = 1; break; }
                    __builtin_amdgcn_s_sleep(1);
                    xv = get64(e);
                }
                row[s] = (int32_t)(uint32_t)xv;
            }
        }
    };

    // Publish this workgroup's first acceptance of the window (the minimum of
    // its waves' keys, or none without a scan) and wait for every workgroup's;
    // returns the grid-wide minimum (kNone if there is no acceptance).
    // The caller's global stores (published Delta values) are complete before
    // the slot is written, so a workgroup that has seen every slot of this
    // window also sees them.  Slots alternate by window parity: a workgroup
    // can be at most one window ahead of the slowest.
    auto exchange = [&](bool with_scan, bool spec) __attribute__((always_inline)) -> unsigned long long {
        wait_stores();   // the published values of the last update have landed
        __syncthreads();
        epoch += 1;
        const unsigned long long tag = (epoch & 1023ull) << 54;
        unsigned long long* slots = slot_base + (epoch & 1) * kMaxGroups;
        if (wave != 0) {
            if (spec) stage_loads(r0, s0, ga, gb, gc, gd, ge);
            refresh_part(tid - 64, nt - 64);
        }
        if (wave == 0) {
            unsigned long long wk = ~0ull;
            if (with_scan)
                for (int i = lane; i < nwaves; i += 64) wk = s_wkey[i];
            wk = wave_min_u64(wk);
            const unsigned long long own = wk == ~0ull ? kNone : (wk & kKeyBits);
            if (lane == 0) put64(&slots[w], tag | own);
            if (spec) stage_loads(r0, s0, ga, gb, gc, gd, ge);
            uint64_t spins = 0;
            bool ok = true;
            unsigned long long best_key;
            for (;;) {
                best_key = kNone;
                bool all = true;
                for (int i = lane; i < G; i += 64) {
                    const unsigned long long x = get64(&slots[i]);
                    all = all && (x >> 54) == (epoch & 1023ull);
                    const unsigned long long k = x & kKeyBits;
                    best_key = k < best_key ? k : best_key;
                }
                if (__all(all)) break;
                // another workgroup's failure is checked every 64 polls: a load
                // of its own on every poll would add a round trip to each
                if (++spins > spin_limit || ((spins & 63) == 0 && get(&ws->err))) { ok = false; break; }
                __builtin_amdgcn_s_sleep(1);
            }
            best_key = wave_min_u64(best_key);
            if (lane == 0) {
                if (!ok) raise_err(&ws->err, kErrTimeout);
                s_ok = ok;
                s_key = best_key;
            }
            if (nwaves == 1) refresh_part(tid, nt);
        }
        __syncthreads();
        pu = pv = -1;   // refreshed
        if (s_rf_bad && tid == 0) { s_ok = 0; raise_err(&ws->err, kErrTimeout); }
        __syncthreads();
        return uni64(s_key);
    };

    auto flush = [&]() __attribute__((always_inline)) {
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

    // ---------------------------------------------------------------- scratch mode
    // Each proposal's swap cost is computed when it is met (Sec. 2.2 (c)),
    // split over the workgroups by rows: a window of K proposals is taken in
    // order, every workgroup sums the terms k of its own rows (k not in
    // {r, s}) for each of them and publishes K tagged partial sums, and every
    // workgroup adds up all partials and the two terms with both indices in
    // {r, s}, so that all of them take the same decisions.  The first accepted
    // proposal of the window is made and the window restarts after it.  A swap
    // (u, v) changes p, columns u, v of every row of B' (local), and rows u, v
    // of B' (read again through p by their owners).  Delta is not kept: the
    // run leaves it stale, and returns as soon as the acceptance rate over
    // the last 8192 or more iterations falls below switch_permille per 1000,
    // for Delta to be rebuilt and the run continued in Delta mode.
    if constexpr (SCR) {
        uint32_t K = 4;                           // proposals per window: 4, 8 or 16
        uint64_t win_iters = 0, win_acc = 0;
        const uint32_t flags = a.flags, switch_permille = a.switch_permille;
        unsigned long long* const Pbase = a.Pp;
        const int32_t* const ldA = L_.dg;         // diagonal of A
        const int32_t* const ldB = L_.dg + n;     // diagonal of B
        // Every workgroup writes its partial sums to `reps` copies and reads
        // copy w mod reps: fewer readers per line (7% faster at N = 2000 with
        // four copies than with one)
        const int reps = scratch_reps(G);
        // Rows of B' read off the critical path, after this workgroup's
        // partial sums are out and while the exchange runs: the owner of the
        // v of a candidate (r0, v) reads row (and column) r0, which becomes
        // row v when (r0, v) is accepted (two entries change places); the
        // owner of u of an accepted swap reads its new row u in the next
        // window (before its partial sums only when a proposal needs the row).
        // One element of each of this thread's columns k = tid + i * nt.
        uint32_t sp_row[kMaxPerThread], sp_col[kMaxPerThread];
        uint32_t pd_row[kMaxPerThread], pd_col[kMaxPerThread];
        int spec_r = -1;    // row read ahead into sp_*, or -1
        int pend = -1;      // own row to be read again through p (after a swap), or -1
        // row x of B' (and column x, general form) from registers; the
        // entries at ua and va change places (none when ua < 0)
        auto write_row = [&](int x, const uint32_t* vr, const uint32_t* vc, int ua, int va)
            __attribute__((always_inline)) {
            E* row = lBb + (x / G) * P;
#pragma unroll
            for (int i = 0; i < kMaxPerThread; ++i) {
                if (i >= nk) break;
                const int k = tid + i * nt;
                if (k >= n) continue;
                const int dst = k == ua ? va : (k == va ? ua : k);
                row[dst] = (E)vr[i];
                if constexpr (!SYM) (lBt + (x / G) * P)[dst] = (E)vc[i];
            }
        };
        // row x of B' after the swap (u, v) (p' = p o (u v)), read through p':
        // B'[x][k] = B[p'(x)][p'(k)], and column x, B[p'(k)][p'(x)]
        auto read_row = [&](int px, int u, int v, int pu_new, int pv_new, uint32_t* vr, uint32_t* vc)
            __attribute__((always_inline)) {
#pragma unroll
            for (int i = 0; i < kMaxPerThread; ++i) {
                if (i >= nk) break;
                const int k = min(tid + i * nt, n - 1);
                const int pk = k == u ? pu_new : (k == v ? pv_new : (int)lps[k]);
                vr[i] = (uint32_t)a.B[px * n + pk] - (uint32_t)a.b_min;
                if constexpr (!SYM) vc[i] = gBt[(size_t)px * P + pk];
            }
        };
        while (alive && t < t_end) {
            const uint32_t W = (uint32_t)min<uint64_t>(min<uint64_t>((uint64_t)K, t_end - t), (uint64_t)m);
            epoch += 1;
            const uint32_t tag = (uint32_t)epoch;
            unsigned long long* const Pw = Pbase + (size_t)(epoch & 1) * kMaxGroups * kScratchK;
            // which rows of this workgroup the window needs: the pending row is
            // needed by proposals (r, s) with r not that row; a candidate (r0, v)
            // with v owned here has row r0 read ahead
            bool spec = false, need_pend = pend >= 0 && rnd;
            if (!rnd && s0 + (int)W <= n) {
                // the usual case: (r0, s0), ..., (r0, s0 + W - 1), owners of s0, s0 + 1, ... in turn
                const int s0_own = uni(s0 % G);
                int lag = w - s0_own;
                if (lag < 0) lag += G;
                spec = (uint32_t)lag < W;
                need_pend = pend >= 0 && pend != r0;
            } else if (!rnd) {
                int rr = r0, ss = s0;
                for (uint32_t jj = 0; jj < W; ++jj) {
                    if (jj) advance_pair(n, rr, ss, 1);
                    if (rr == r0 && ss % G == w) spec = true;
                    if (pend >= 0 && rr != pend) need_pend = true;
                }
            }
            if (need_pend) {
                read_row((int)lps[pend], -1, -1, 0, 0, pd_row, pd_col);
                write_row(pend, pd_row, pd_col, -1, -1);
                pend = -1;
                __syncthreads();
            }
            spec_r = spec ? r0 : -1;
            // wave 0: this workgroup's partial sums, one proposal per lane j < K
            // (lanes j, j + K, ... split the own rows).  The owner of row s
            // adds the two terms with both indices in {r, s}; the symmetric
            // form counts each row term twice (rows and columns alike).
            const int j = lane & (int)(K - 1);
            int r = r0, s = s0;
            TempParts tp{0.0, 0.0, 0.0};
            double ylog = 0.0;
            if (wave == 0) {
                if (rnd) pair_of_u(n, random_pair_index(seed, chain_id, t + (uint64_t)j, m), r, s);
                else advance_pair(n, r, s, j);
                if ((uint32_t)j < W) tp = temp_parts(temps, t + (uint64_t)j);   // read now, used after the exchange
                uint32_t part = 0;   // modulo 2^32 (see Elem)
                if ((uint32_t)j < W) {
                    const int pr = lps[r], ps = lps[s];
                    for (int lr = lane / (int)K; lr < Rw; lr += 64 / (int)K) {
                        const int k = w + G * lr;
                        if (k == r) continue;
                        const E* Bk = lBb + lr * P;   // row k of B'
                        if constexpr (SYM) {
                            const E* Ak = lAb + lr * P;
                            if (k == s) {
                                part += ((uint32_t)ldA[r] - (uint32_t)ldA[s]) * ((uint32_t)ldB[ps] - (uint32_t)ldB[pr]);
                                continue;
                            }
                            part += 2u * (((uint32_t)Ak[r] - (uint32_t)Ak[s]) * ((uint32_t)Bk[s] - (uint32_t)Bk[r]));
                        } else {
                            // row k of A, column k of A (Ck[x] = A[x][k]) and column k of B' (Dk[x] = B'[x][k])
                            const E* Ak = a_lds ? lAr + lr * P : gA + (size_t)k * P;
                            const E* Ck = a_lds ? lAc + lr * P : gAt + (size_t)k * P;
                            const E* Dk = lBt + lr * P;
                            if (k == s) {
                                part += ((uint32_t)ldA[r] - (uint32_t)ldA[s]) * ((uint32_t)ldB[ps] - (uint32_t)ldB[pr]);
                                part += ((uint32_t)Ck[r] - (uint32_t)Ak[r]) * ((uint32_t)Bk[r] - (uint32_t)Dk[r]);
                                continue;
                            }
                            part += ((uint32_t)Ak[r] - (uint32_t)Ak[s]) * ((uint32_t)Bk[s] - (uint32_t)Bk[r]);
                            part += ((uint32_t)Ck[r] - (uint32_t)Ck[s]) * ((uint32_t)Dk[s] - (uint32_t)Dk[r]);
                        }
                    }
                }
                part = stride_sum(part, K);
                if (lane < (int)K)
                    for (int rr = 0; rr < reps; ++rr) put64(Pw + rr * G * K + w * K + lane, ((unsigned long long)tag << 32) | part);
                // log r_t of Eq. (2) while the exchange runs
                if ((uint32_t)j < W && !t0_inf) ylog = log(uniform_r(seed, chain_id, t + (uint64_t)j));
            }
            // rows read now: the old row r0 for a candidate's v (current p), and
            // the pending row (not read by this window's partial sums)
            if (spec) read_row((int)lps[r0], -1, -1, 0, 0, sp_row, sp_col);
            if (pend >= 0) {
                read_row((int)lps[pend], -1, -1, 0, 0, pd_row, pd_col);
                write_row(pend, pd_row, pd_col, -1, -1);
                pend = -1;
            }
            if (tid == 0) mark(QAP_PH_SCRATCH_EVAL);
            // every workgroup's partials of this window (thread tid takes
            // proposal tid mod K: the block size is a multiple of K)
            {
                const int total = G * (int)K;
                unsigned long long* const Pr = Pw + (w % reps) * total;
                uint32_t acc = 0;
                bool bad = false;
                for (int e0 = tid; e0 < total && !bad; e0 += 8 * nt) {
                    unsigned long long x[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const int e = e0 + i * nt;
                        x[i] = e < total ? get64(Pr + e) : ((unsigned long long)tag << 32);
                    }
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const int e = e0 + i * nt;
                        uint64_t spins = 0;
                        while (!bad && (uint32_t)(x[i] >> 32) != tag) {
                            if (++spins > spin_limit || ((spins & 63) == 0 && get(&ws->err))) { bad = true; break; }
                            __builtin_amdgcn_s_sleep(1);
                            x[i] = get64(Pr + e);
                        }
                        if (e < total) acc += (uint32_t)x[i];
                    }
                }
                if (bad) s_rf_bad = 1;
                acc = stride_sum(acc, K);
                if (lane < (int)K) s_gsum[wave][lane] = acc;
            }
            __syncthreads();
            if (s_rf_bad) {
                if (tid == 0) raise_err(&ws->err, kErrTimeout);
                alive = false;
                break;
            }
            if (tid == 0) mark(QAP_PH_GRID_SYNC);
            // wave 0: the swap costs, Eq. (2) and the first acceptance
            if (wave == 0) {
                uint32_t S = 0;
                for (int i = 0; i < nwaves; ++i) S += s_gsum[i][j];
                const int d = (int)S;
                bool acc = false, tie = false;
                double z = 0.0;
                if (lane < (int)W) {
                    acc = d <= 0;
                    const double Tj = temp_of(T0, tp);
                    if (!acc && t0_inf && inf_draw_clear(seed, chain_id, t + (uint64_t)j)) {
                        acc = true;
                    } else if (!acc && d <= reject_bound(Tj)) {
                        if (t0_inf) ylog = log(uniform_r(seed, chain_id, t + (uint64_t)j));
                        z = (double)d / Tj + ylog;   // the operations of metropolis_positive
                        acc = z < 0.0;
                        tie = fabs(z) < kNearTie;
                    }
                }
                const unsigned long long bal = __ballot(acc);
                const int js = bal ? __builtin_ctzll(bal) : 64;
                if (w == 0 && tie && j <= js) {
                    const unsigned long long slot = atomicAdd((unsigned long long*)&ws->nties, 1ull);
                    if (a.ties && st0.near_ties + slot < a.tie_cap)
                        a.ties[st0.near_ties + slot] = qap_near_tie{t + (uint64_t)j, (int64_t)d, z};
                }
                if (lane == 0) s_key = bal ? (((unsigned long long)js << 32) | (uint32_t)__builtin_amdgcn_readlane(d, js)) : ~0ull;
                if (bal && lane == js) {
                    s_swap[0] = r; s_swap[1] = s;
                    s_swap[2] = lps[s]; s_swap[3] = lps[r];   // p(u), p(v) after the swap
                }
            }
            __syncthreads();
            if (tid == 0) bump(QAP_PH_N_ROUNDS, 1);
            const unsigned long long key = uni64(s_key);
            if (key == ~0ull) {
                t += W;
                win_iters += W;
                advance_pair(n, r0, s0, (int)W);
                r0 = uni(r0);
                s0 = uni(s0);
            } else {
                const uint32_t jstar = (uint32_t)(key >> 32);
                const int dstar = (int)(uint32_t)key;
                const uint64_t tstar = t + jstar;
                const int u = uni(s_swap[0]), v = uni(s_swap[1]);
                const int pu_new = uni(s_swap[2]), pv_new = uni(s_swap[3]);
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
                // columns u, v of own rows (and rows u, v of own columns) change places
                for (int lr = tid; lr < Rw; lr += nt) {
                    const int k = w + G * lr;
                    if (k == u || k == v) continue;
                    E* row = lBb + lr * P;
                    const E x = row[u];
                    row[u] = row[v];
                    row[v] = x;
                    if constexpr (!SYM) {
                        E* col = lBt + lr * P;
                        const E y = col[u];
                        col[u] = col[v];
                        col[v] = y;
                    }
                }
                // own row v: the row read ahead (old row u, entries u and v
                // exchanged) when it is this window's, else read now (not
                // reading p at u or v, which thread 0 changes meanwhile); own
                // row u: read in the next window, through the new p
                if (v % G == w) {
                    if (spec_r == u) {
                        write_row(v, sp_row, sp_col, u, v);
                    } else {
                        read_row(pv_new, u, v, pu_new, pv_new, sp_row, sp_col);
                        write_row(v, sp_row, sp_col, -1, -1);
                    }
                }
                if (u % G == w) pend = u;
                if (tid == 0) { lps[u] = (int16_t)pu_new; lps[v] = (int16_t)pv_new; }
                t = tstar + 1;
                win_iters += jstar + 1;
                win_acc += 1;
                r0 = u;
                s0 = v;
                advance_pair(n, r0, s0, 1);
                r0 = uni(r0);
                s0 = uni(s0);
                __syncthreads();
                if (nrec == kRec) flush();
                if (tid == 0) { mark(QAP_PH_SCRATCH_ACCEPT); bump(QAP_PH_N_SCRATCH_ACC, 1); }
            }
            if (win_iters >= 8192) {
                // few proposals per window while most are accepted, more as acceptance falls
                K = win_acc * 4 >= win_iters ? 4u : (win_acc * 8 >= win_iters ? 8u : 16u);
                if (!(flags & kFlagScratchOnly) && win_acc * 1000u < win_iters * switch_permille) {
                    if (tid == 0) bump(QAP_PH_SWITCH_T, t);
                    break;
                }
                win_iters = win_acc = 0;
            }
        }
        if (pend >= 0) {
            __syncthreads();   // thread 0's last write of p is visible
            read_row((int)lps[pend], -1, -1, 0, 0, pd_row, pd_col);
            write_row(pend, pd_row, pd_col, -1, -1);
        }
        // write back: B' rows, p and the state; Delta is left stale
        __syncthreads();
        if (w == 0 && nrec > 0) flush();
        for (int lr = 0; lr < Rw; ++lr) {
            const int r = w + G * lr;
            for (int k = tid; k < n; k += nt) a.Bp[r * n + k] = (int32_t)((uint32_t)lBb[lr * P + k] + (uint32_t)a.b_min);
        }
        if (w == 0) {
            for (int i = tid; i < n; i += nt) a.p[i] = lps[i];
            if (tid == 0) {
                qap_chain_state st;
                st.t = t; st.accepts = accepts; st.hash = hash;
                st.near_ties = st0.near_ties + __hip_atomic_load((unsigned long long*)&ws->nties, __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_AGENT);
                st.cost = cost; st.best_cost = best; st.best_iter = best_iter;
                const int err = get(&ws->err);
                st.status = alive && err == 0 ? QAP_OK : (err == kErrTieOverflow ? QAP_E_TIE_OVERFLOW : QAP_E_TIMEOUT);
                st.mode = QAP_MODE_SCRATCH_STALE;
                *a.state = st;
                mark(QAP_PH_IO);
                bump(QAP_PH_TOTAL, clock64() - prof_start);
            }
            if (prof) {
                __syncthreads();
                if (tid < QAP_PHASES) atomicAdd((unsigned long long*)&a.prof[tid], s_prof[tid]);
            }
        }
        return;
    }

    while (alive && t < t_end) {
        // ------------------------------------------------------------ scan
        const uint32_t W = (uint32_t)min<uint64_t>(min<uint64_t>((uint64_t)kwin, t_end - t), (uint64_t)m);
        const int32_t bound = reject_bound(temperature(temps, T0, t));
        unsigned long long mine = ~0ull;
        auto test = [&](uint32_t j, int d) __attribute__((always_inline)) {
            bool acc = d <= 0;
            if (!acc && t0_inf && inf_draw_clear(seed, chain_id, t + j)) {
                acc = true;   // T = +inf: accepted, and no near tie (see inf_draw_clear)
            } else if (!acc && d <= bound) {
                double z;
                acc = exact_test(d, temps, T0, seed, chain_id, t + j, &z);
                if (fabs(z) < kNearTie) {
                    const int slot = atomicAdd(&s_ntie[tb], 1);
                    if (slot < kTieSlots) { s_tie_j[tb][slot] = j; s_tie_d[tb][slot] = d; s_tie_z[tb][slot] = z; }
                }
            }
            if (acc) {
                const unsigned long long key = ((unsigned long long)j << 32) | (uint32_t)d;
                mine = key < mine ? key : mine;
            }
        };
        __syncthreads();   // the last update's LDS writes are visible
        if (rnd) {
            // random order: every workgroup draws the whole window and tests the
            // proposals it holds -- (r, s) from row s, or from row r where row s
            // is stale -- so that each proposal is tested exactly once
            for (uint32_t j = tid; j < W; j += nt) {
                int r, s;
                pair_of_u(n, random_pair_index(seed, chain_id, t + j, m), r, s);
                const bool s_stale = s == pu || s == pv;
                if (!s_stale) {
                    if (s % G == w) test(j, lD[(s / G) * n + r]);
                } else if (r == pu && s == pv) {
                    if (s % G == w) test(j, -pd);
                } else if (r != pu && r != pv && r % G == w) {
                    test(j, lD[(r / G) * n + s]);
                }
            }
        }
        // proposals (r, s) with s owned here, r < s, in the window.  The rows of
        // the window are r0, r0 + 1, ... cyclically; row offset n - 1 is row r0
        // again, for a window that wraps round to the pairs before (r0, s0).
        if (!rnd && C > 0) {
            const int rows_per_pass = max(1, nt / C);
            const int i_loc = tid / C, c = tid - i_loc * C;
            const int s = w + G * c;
            for (int ib = 0; ib <= n - 1; ib += rows_per_pass) {
                if (ib > 0) {
                    const int rb = r0 + ib >= n - 1 ? r0 + ib - (n - 1) : r0 + ib;
                    uint32_t jb = rs32(n, rb) + m - idx0;
                    if (jb >= m) jb -= m;
                    if (jb >= W) break;
                }
                const int i = ib + i_loc;
                if (i_loc >= rows_per_pass || i > n - 1) continue;
                const int r = r0 + i >= n - 1 ? r0 + i - (n - 1) : r0 + i;
                bool ok = s > r && s < n;
                if (i == 0) ok = ok && s >= s0;
                if (i == n - 1) ok = ok && s < s0;
                if (!ok) continue;
                uint32_t j = rs32(n, r) + (uint32_t)(s - r - 1) + m - idx0;
                if (j >= m) j -= m;
                if (j >= W) continue;
                if (s != pu && s != pv) test(j, lD[(s / G) * n + r]);
                else if (r == pu && s == pv) test(j, -pd);
            }
        }
        // proposals (r, x) with x a stale row and r owned here: read from row r
        if (!rnd && pu >= 0) {
            for (int lr = tid; lr < 2 * Rw; lr += nt) {
                const int rr = w + G * (lr >> 1), x = (lr & 1) ? pv : pu;
                if (rr == pu || rr == pv || x <= rr) continue;
                uint32_t j = rs32(n, rr) + (uint32_t)(x - rr - 1) + m - idx0;
                if (j >= m) j -= m;
                if (j < W) test(j, lD[(lr >> 1) * n + x]);
            }
        }
        {
            const bool any = __ballot(mine != ~0ull) != 0;
            const unsigned long long wk = any ? wave_min_u64(mine) : ~0ull;
            if (lane == 0) s_wkey[wave] = wk;
        }
        if (tid == 0) mark(QAP_PH_DELTA_SCAN);
        const bool spec = !rnd && last_j0;
        const unsigned long long key = exchange(true, spec);
        alive = uni(s_ok) != 0;
        if (!alive) break;
        const uint32_t jstar = key == kNone ? UINT_MAX : (uint32_t)(key >> 32);
        last_j0 = jstar == 0;
        // near ties a sequential run would have met; the other buffer, read
        // by everyone before this window's exchange, is cleared for the next.
        // A workgroup that met more ties in the window than it recorded cannot
        // tell how many of them lie before the first acceptance: the run stops
        // with an error instead of reporting a count that may be too low.
        const int ntie_all = s_ntie[tb];
        if (ntie_all > kTieSlots) {
            if (tid == 0) raise_err(&ws->err, kErrTieOverflow);
            alive = false;
            break;
        }
        if (tid < ntie_all && s_tie_j[tb][tid] <= (jstar == UINT_MAX ? W - 1 : jstar)) {
            const unsigned long long slot = atomicAdd((unsigned long long*)&ws->nties, 1ull);
            if (a.ties && st0.near_ties + slot < a.tie_cap)
                a.ties[st0.near_ties + slot] =
                    qap_near_tie{t + s_tie_j[tb][tid], (int64_t)s_tie_d[tb][tid], s_tie_z[tb][tid]};
        }
        if (tid == 0) s_ntie[tb ^ 1] = 0;
        tb ^= 1;
        if (tid == 0) { mark(QAP_PH_GRID_SYNC); bump(QAP_PH_N_SCAN_STEPS, 1); }
        if (jstar == UINT_MAX) {
            t += W;
            idx0 = uni((uint32_t)(((uint64_t)idx0 + W) % m));
            pair_of_u(n, idx0, r0, s0);
            r0 = uni(r0);
            s0 = uni(s0);
            kwin = min<uint64_t>((uint64_t)kwin * 2, (uint64_t)a.kmax);
            continue;
        }

        // ------------------------------------------------------------ accept
        const int dstar = (int)(uint32_t)key;
        const uint64_t tstar = t + jstar;
        uint32_t istar = idx0 + jstar;
        if (istar >= m) istar -= m;
        if (rnd) istar = random_pair_index(seed, chain_id, tstar, m);
        istar = uni(istar);
        int u, v;
        pair_of_u(n, istar, u, v);
        u = uni(u);
        v = uni(v);
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
        // staged rows after the swap (requested during the exchange when the
        // accepted proposal is the window's first and that was speculated)
        const int pu_new = uni((int)lps[v]), pv_new = uni((int)lps[u]);
        if (!(spec && jstar == 0)) stage_loads(u, v, ga, gb, gc, gd, ge);
        // staged bytes, packed differences and this thread's share of the self
        // terms <A[x][.], B'[x][.]> of x = u, v
        uint32_t self_u = 0, self_v = 0;   // modulo 2^32 (see Elem)
#pragma unroll
        for (int i = 0; i < kMaxPerThread; ++i) {
            if (i >= nk) break;
            const int k = tid + i * nt;
            if (k < n) {
                const uint32_t su = (uint32_t)ga[i] - (uint32_t)a.a_min, sv = (uint32_t)gb[i] - (uint32_t)a.a_min;
                const uint32_t tu = (uint32_t)gc[i] - (uint32_t)a.b_min, tv = (uint32_t)gd[i] - (uint32_t)a.b_min;
                lSu[k] = (E)su;
                lSv[k] = (E)sv;
                lTu[k] = (E)tu;
                lTv[k] = (E)tv;
                const uint32_t da = su - sv, db = tu - tv;
                uint32_t dc = da, dt = db;   // column differences (the row ones when symmetric)
                if constexpr (SYM) {
                    self_u += su * tu;
                    self_v += sv * tv;
                } else {
                    uint32_t cu, cv, tcu, tcv;
                    if constexpr (kByte) {
                        cu = ge[i] & 0xff; cv = (ge[i] >> 8) & 0xff; tcu = (ge[i] >> 16) & 0xff; tcv = ge[i] >> 24;
                    } else {
                        const int pk = k == u ? pu_new : (k == v ? pv_new : (int)lps[k]);
                        cu = gAt[(size_t)u * P + k];
                        cv = gAt[(size_t)v * P + k];
                        tcu = gBt[(size_t)pu_new * P + pk];
                        tcv = gBt[(size_t)pv_new * P + pk];
                    }
                    lScu[k] = (E)cu;
                    lScv[k] = (E)cv;
                    lTcu[k] = (E)tcu;
                    lTcv[k] = (E)tcv;
                    dc = cu - cv;
                    dt = tcu - tcv;
                    self_u += su * tu + cu * tcu;
                    self_v += sv * tv + cv * tcv;
                }
                if constexpr (kByte) {
                    labp[k] = (uint32_t)(uint16_t)dc | ((uint32_t)(uint16_t)da << 16);
                    lbbp[k] = (uint32_t)(uint16_t)dt | ((uint32_t)(uint16_t)db << 16);
                } else {
                    labp2[k] = make_uint2(dc, da);
                    lbbp2[k] = make_uint2(dt, db);
                }
            }
        }
        self_u = (uint32_t)wave_sum((int)self_u);
        self_v = (uint32_t)wave_sum((int)self_v);
        if (lane == 0) { s_selfw[wave][0] = (int)self_u; s_selfw[wave][1] = (int)self_v; }
        // own rows of B' other than u, v swap columns u, v (thread lr for own
        // row lr); nothing reads B' between the exchange and the touched pass
        for (int lr = tid; lr < Rw; lr += nt) {
            const int r = w + G * lr;
            if (r != u && r != v) {
                E* row = lBb + lr * P;
                const E x = row[u];
                row[u] = row[v];
                row[v] = x;
                if constexpr (!SYM) {   // column r of B': its entries u, v change places too
                    E* col = lBt + lr * P;
                    const E y = col[u];
                    col[u] = col[v];
                    col[v] = y;
                }
            }
        }
        __syncthreads();   // staged rows and B' columns complete; everyone has read p
        if (tid == 0) { lps[u] = (int16_t)pu_new; lps[v] = (int16_t)pv_new; }
        // own rows u, v of B' are replaced by the staged rows (whole rows, all
        // threads); the touched pass below skips them
        for (int which = 0; which < 2; ++which) {
            const int x = which == 0 ? u : v;
            if (x % G != w) continue;
            E* row = lBb + (x / G) * P;
            const E* src = which == 0 ? lTu : lTv;
            for (int k = tid; k < n; k += nt) row[k] = src[k];
            if constexpr (!SYM) {
                E* col = lBt + (x / G) * P;
                const E* srcc = which == 0 ? lTcu : lTcv;
                for (int k = tid; k < n; k += nt) col[k] = srcc[k];
            }
        }
        if (nrec == kRec) flush();
        // No barrier between the correction of the disjoint pairs and the
        // touched pass: the first reads neither B' nor p and writes Delta only,
        // the second reads own rows of A and B' other than u, v and the staged
        // rows and writes its results to s_pub only, so a wave that finishes its
        // share of the first goes on to its touched row while others still
        // work.  Columns u, v of Delta take the touched values from s_pub after
        // the barrier that ends both passes.

        // pairs of own rows disjoint from {u, v}: the entries of up to eight
        // own rows in two of this thread's columns are loaded before any is
        // stored (a store to Delta may not move above a later load of it).
        // Entries in columns u, v and in rows u, v get a meaningless value:
        // the first are rewritten below (after a barrier), the rows are stale
        // and refreshed from the published values, and the diagonal is never
        // read.  So the only mask is the end of the row.
        {
            constexpr int kRowBatch = 8;
            if constexpr (kByte) {
            for (int lr0 = 0; lr0 < Rw; lr0 += kRowBatch) {
                v2i16 ar[kRowBatch], br[kRowBatch];
#pragma unroll
                for (int h = 0; h < kRowBatch; ++h) {
                    const int lr = lr0 + h < Rw ? lr0 + h : Rw - 1;
                    const int r = w + G * lr;
                    ar[h] = __builtin_bit_cast(v2i16, labp[r]);
                    br[h] = __builtin_bit_cast(v2i16, lbbp[r]);
                }
                // four of this thread's columns at a time (all of them at n <= 4 * threads)
                constexpr int kCols = 4;
                for (int i0 = 0; i0 < nk; i0 += kCols) {
                    v2i16 as[kCols], bs[kCols];
                    int32_t dv[kCols][kRowBatch];
#pragma unroll
                    for (int i = 0; i < kCols; ++i) {
                        const int s = tid + (i0 + i) * nt;
                        const int sc = s < n ? s : 0;
                        as[i] = __builtin_bit_cast(v2i16, labp[sc]);
                        bs[i] = __builtin_bit_cast(v2i16, lbbp[sc]);
#pragma unroll
                        for (int h = 0; h < kRowBatch; ++h) {
                            const int lr = lr0 + h < Rw ? lr0 + h : Rw - 1;
                            dv[i][h] = lD[lr * n + sc];
                        }
                    }
#pragma unroll
                    for (int i = 0; i < kCols; ++i) {
                        const int s = tid + (i0 + i) * nt;
                        if (s >= n) continue;
#pragma unroll
                        for (int h = 0; h < kRowBatch; ++h)
                            if (lr0 + h < Rw)
                                lD[(lr0 + h) * n + s] =
                                    __builtin_amdgcn_sdot2(ar[h] - as[i], bs[i] - br[h], dv[i][h], false);
                    }
                }
            }
            } else {
            // wider values: the two products in 32-bit arithmetic modulo 2^32
            for (int lr0 = 0; lr0 < Rw; lr0 += kRowBatch) {
                uint2 ar[kRowBatch], br[kRowBatch];
#pragma unroll
                for (int h = 0; h < kRowBatch; ++h) {
                    const int lr = lr0 + h < Rw ? lr0 + h : Rw - 1;
                    const int r = w + G * lr;
                    ar[h] = labp2[r];
                    br[h] = lbbp2[r];
                }
                for (int i = 0; i < nk; ++i) {
                    const int s = tid + i * nt;
                    if (s >= n) continue;
                    const uint2 as = labp2[s], bs = lbbp2[s];
                    uint32_t dv[kRowBatch];
#pragma unroll
                    for (int h = 0; h < kRowBatch; ++h) {
                        const int lr = lr0 + h < Rw ? lr0 + h : Rw - 1;
                        dv[h] = (uint32_t)lD[lr * n + s];
                    }
#pragma unroll
                    for (int h = 0; h < kRowBatch; ++h)
                        if (lr0 + h < Rw)
                            lD[(lr0 + h) * n + s] = (int32_t)(dv[h] + (ar[h].x - as.x) * (bs.x - br[h].x) +
                                                              (ar[h].y - as.y) * (bs.y - br[h].y));
                }
            }
            }
        }
        // Delta(r, u), Delta(r, v) of own rows: one wave per row
        {
            uint32_t su = 0, sv = 0;
            for (int i = 0; i < nwaves; ++i) { su += (uint32_t)s_selfw[i][0]; sv += (uint32_t)s_selfw[i][1]; }
            su = uni(su);
            sv = uni(sv);
            for (int lr = wave; lr < Rw; lr += nwaves) {
                const int r = w + G * lr;
                if (r == u || r == v) continue;
                // own row r of A: LDS (symmetric form) or the byte copy in device memory
                const E* A_r = SYM ? lAb + lr * P : gA + (size_t)r * P;
                const uint32_t* ar = (const uint32_t*)A_r;
                const uint32_t* br = (const uint32_t*)(lBb + lr * P);
                const E* B_r = lBb + lr * P;
                const uint32_t arr = A_r[r], aru = A_r[u], arv = A_r[v], brr = B_r[r], bru = B_r[u], brv = B_r[v];
                const uint32_t sur = lSu[r], suu = lSu[u], svr = lSv[r], svv = lSv[v];
                const uint32_t tur = lTu[r], tuu = lTu[u], tvr = lTv[r], tvv = lTv[v];
                auto dot = [](uint32_t x, uint32_t y, uint32_t c) { return Elem<E>::dot(x, y, c); };
                uint32_t pu_ = 0, pv_ = 0, self = 0;
                if constexpr (SYM) {
                    for (int k = lane; k < q; k += 64) {
                        const uint32_t xa = ar[k], xb = br[k];
                        pu_ = dot(xa, ((const uint32_t*)lTu)[k], pu_);
                        pu_ = dot(((const uint32_t*)lSu)[k], xb, pu_);
                        pv_ = dot(xa, ((const uint32_t*)lTv)[k], pv_);
                        pv_ = dot(((const uint32_t*)lSv)[k], xb, pv_);
                        self = dot(xa, xb, self);
                    }
                } else {
                    // rows and columns: column r of A from the copy of A^T, column r of B' in LDS
                    const uint32_t* cr = (const uint32_t*)(gAt + (size_t)r * P);
                    const uint32_t* dr = (const uint32_t*)(lBt + lr * P);
                    for (int k = lane; k < q; k += 64) {
                        const uint32_t xa = ar[k], xb = br[k], xc = cr[k], xd = dr[k];
                        pu_ = dot(xa, ((const uint32_t*)lTu)[k], pu_);
                        pu_ = dot(((const uint32_t*)lSu)[k], xb, pu_);
                        pu_ = dot(xc, ((const uint32_t*)lTcu)[k], pu_);
                        pu_ = dot(((const uint32_t*)lScu)[k], xd, pu_);
                        pv_ = dot(xa, ((const uint32_t*)lTv)[k], pv_);
                        pv_ = dot(((const uint32_t*)lSv)[k], xb, pv_);
                        pv_ = dot(xc, ((const uint32_t*)lTcv)[k], pv_);
                        pv_ = dot(((const uint32_t*)lScv)[k], xd, pv_);
                        self = dot(xa, xb, self);
                        self = dot(xc, xd, self);
                    }
                }
                const uint32_t Pu = (uint32_t)wave_sum((int)pu_), Pv = (uint32_t)wave_sum((int)pv_);
                const uint32_t Sr = (uint32_t)wave_sum((int)self);
                if (lane == 0) {
                    if constexpr (SYM) {
                        s_pub[2 * lr] = finish_sym(Pu - Sr - su, arr, aru, sur, suu, brr, bru, tur, tuu);
                        s_pub[2 * lr + 1] = finish_sym(Pv - Sr - sv, arr, arv, svr, svv, brr, brv, tvr, tvv);
                    } else {
                        s_pub[2 * lr] = finish_gen(Pu - Sr - su, arr, aru, sur, suu, brr, bru, tur, tuu);
                        s_pub[2 * lr + 1] = finish_gen(Pv - Sr - sv, arr, arv, svr, svv, brr, brv, tvr, tvv);
                    }
                }
            }
        }
        // columns u, v of own rows take the touched values, and this
        // workgroup's touched values are published as one contiguous block;
        // the stores complete during the next scan.  Rows u, v (if own) keep
        // whatever the correction wrote: they are stale and refreshed from the
        // published values in the next exchange.
        __syncthreads();
        {
            unsigned long long* dst = X + ((par * G + w) * Rmax) * 2;
            const unsigned long long tag = (unsigned long long)(uint32_t)epoch << 32;
            for (int i = tid; i < 2 * Rw; i += nt) {
                const int lr = i >> 1, r = w + G * lr;
                if (r != u && r != v) lD[lr * n + ((i & 1) ? v : u)] = s_pub[i];
                put64(dst + i, tag | (uint32_t)s_pub[i]);
            }
        }
        pu = u; pv = v; pd = dstar; ppar = par; ptag = (uint32_t)epoch;
        par ^= 1;
        t = tstar + 1;
        idx0 = istar + 1 == m ? 0 : istar + 1;
        r0 = u; s0 = v;
        if (++s0 == n) { if (++r0 == n - 1) r0 = 0; s0 = r0 + 1; }
        kwin = a.kmin;
        if (tid == 0) { mark(QAP_PH_DELTA_UPDATE); bump(QAP_PH_N_DELTA_ACC, 1); }
    }

    // ------------------------------------------------------------ write back
    if (alive) {   // the last swap's published values
        exchange(false, false);
        alive = s_ok != 0;
    }
    __syncthreads();
    if (w == 0 && nrec > 0) flush();
    for (int lr = 0; lr < Rw; ++lr) {
        const int r = w + G * lr;
        int32_t* up = a.delta + rs32(n, r) - r - 1;
        for (int s = r + 1 + tid; s < n; s += nt) up[s] = lD[lr * n + s];
        for (int k = tid; k < n; k += nt) a.Bp[r * n + k] = (int32_t)((uint32_t)lBb[lr * P + k] + (uint32_t)a.b_min);
    }
    if (w == 0) {
        for (int i = tid; i < n; i += nt) a.p[i] = lps[i];
        if (tid == 0) {
            qap_chain_state st;
            st.t = t; st.accepts = accepts; st.hash = hash;
            st.near_ties = st0.near_ties + __hip_atomic_load((unsigned long long*)&ws->nties, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT);
            st.cost = cost; st.best_cost = best; st.best_iter = best_iter;
            const int err = get(&ws->err);
            st.status = alive && err == 0 ? QAP_OK : (err == kErrTieOverflow ? QAP_E_TIE_OVERFLOW : QAP_E_TIMEOUT);
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

// Slots, published values and partial sums start from tag 0, which no window
// or update of this launch uses (epochs start at 1), so nothing left by an
// earlier launch or another chain can be taken for this launch's data.
__global__ void k_ws_reset(DistWs* ws, unsigned long long* slots, unsigned long long* X, int nx,
                           unsigned long long* Pp, int np)
{
    for (int i = threadIdx.x; i < 2 * kMaxGroups; i += blockDim.x) slots[i] = 0;   // window 0 is never used
    for (int i = threadIdx.x; i < nx; i += blockDim.x) X[i] = 0;
    for (int i = threadIdx.x; i < 2 * np; i += blockDim.x) Pp[(i >= np ? kMaxGroups * kScratchK - np : 0) + i] = 0;
    if (threadIdx.x == 0) {
        ws->err = 0;
        ws->nties = 0;
    }
}

// General form: copies (value - minimum, element type E) of A, A^T and B^T
// with rows padded to P elements (zeros), read by the staging loads and the
// touched pass.  One thread per padded entry; grid-stride.
template <typename E>
__global__ void k_dist_copies(int n, int P, const int32_t* __restrict__ A, const int32_t* __restrict__ B,
                              int a_min, int b_min, E* Ab, E* Atb, E* Btb)
{
    const size_t total = (size_t)n * P;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / P), j = (int)(e - (size_t)i * P);
        E a = 0, at = 0, bt = 0;
        if (j < n) {
            a = (E)((uint32_t)A[(size_t)i * n + j] - (uint32_t)a_min);
            at = (E)((uint32_t)A[(size_t)j * n + i] - (uint32_t)a_min);
            bt = (E)((uint32_t)B[(size_t)j * n + i] - (uint32_t)b_min);
        }
        Ab[e] = a;
        Atb[e] = at;
        Btb[e] = bt;
    }
}

template <typename E>
int launch_dist_typed(DistArgs& a, bool symmetric, int G, int Gs, int threads, size_t bytes, size_t bytes_s,
                      hipStream_t stream)
{
    const void* fn_s = symmetric ? (const void*)k_chain_dist<true, E, true> : (const void*)k_chain_dist<false, E, true>;
    const void* fn_d = symmetric ? (const void*)k_chain_dist<true, E, false> : (const void*)k_chain_dist<false, E, false>;
    // the static __shared__ variables come on top of the dynamic layout
    hipFuncAttributes fa_s, fa_d;
    if (hipFuncGetAttributes(&fa_s, fn_s) != hipSuccess || hipFuncGetAttributes(&fa_d, fn_d) != hipSuccess)
        return QAP_E_DEVICE;
    if (fa_s.sharedSizeBytes + bytes_s > kLdsLimit || fa_d.sharedSizeBytes + bytes > kLdsLimit) return QAP_E_UNSUPPORTED;
    if (hipFuncSetAttribute(fn_s, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes_s) != hipSuccess ||
        hipFuncSetAttribute(fn_d, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess)
        return QAP_E_DEVICE;
    if (!symmetric) {   // the copies precede the run on the same stream
        if (!a.Ab || !a.Atb || !a.Btb) return QAP_E_INVAL;
        const int P = a.quads * (4 / (int)sizeof(E));
        const size_t total = (size_t)a.n * P;
        const int blocks = (int)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
        hipLaunchKernelGGL(k_dist_copies<E>, dim3(blocks), dim3(256), 0, stream, a.n, P, a.A, a.B, a.a_min, a.b_min,
                           (E*)a.Ab, (E*)a.Atb, (E*)a.Btb);
    }
    auto run = [&](const void* fn, int g, size_t b) -> int {
        const int rmax = (a.n + g - 1) / g;
        hipLaunchKernelGGL(k_ws_reset, dim3(1), dim3(256), 0, stream, a.ws, a.slots, a.X, 2 * 2 * g * rmax, a.Pp,
                           scratch_reps(g) * g * kScratchK);
        void* kargs[] = {&a};
        if (hipLaunchCooperativeKernel(fn, dim3(g), dim3(threads), kargs, (unsigned)b, stream) != hipSuccess)
            return QAP_E_DEVICE;
        return QAP_OK;
    };
    // Delta mode alone: Delta rebuilt first if the chain left it stale.
    // Otherwise scratch mode runs first (a launch that returns at once when
    // the chain keeps Delta), and where it stopped early (acceptance fell) or
    // at the end of the schedule Delta is rebuilt and Delta mode continues;
    // the rebuild and the second launch read the chain state on the device
    // and do nothing when there is nothing to do.
    int rc = QAP_OK;
    if (!(a.flags & kFlagDeltaOnly)) rc = run(fn_s, Gs, bytes_s);
    if (rc == QAP_OK) rc = launch_delta_rebuild(a.n, a.A, a.Bp, a.delta, a.state, a.t_end, a.iters, stream);
    if (rc == QAP_OK && !(a.flags & kFlagScratchOnly)) rc = run(fn_d, G, bytes);
    return rc;
}

}  // namespace

int dist_words(int n, int esize) { return (int)(((size_t)n * esize + 3) / 4); }

size_t lds_dist_bytes(int n, int G, bool symmetric, int esize, bool scratch)
{
    return dist_layout(n, G, dist_words(n, esize), esize, symmetric, scratch, nullptr, nullptr);
}

constexpr int kScratchRows = 16;   // own rows per workgroup sought for scratch-mode launches

// Workgroups of a scratch-mode launch: about kScratchRows own rows each
// where the LDS allows (N = 2000: 125 workgroups, against 250 for Delta
// mode), never more than the Delta-mode launch's G.  Measured at N = 2000
// over the first 1e6 iterations: 16 rows 2.49 s symmetric and 2.73 s
// asymmetric, 8 rows 2.56 and 2.75, 32 rows 2.56 and 2.82.
int dist_scratch_groups(int n, int G, bool symmetric, int esize, size_t budget)
{
    int gs = (n + kScratchRows - 1) / kScratchRows;
    if (gs < 2) gs = 2;
    while (gs < G && lds_dist_bytes(n, gs, symmetric, esize, true) > budget) ++gs;
    return gs < G ? gs : G;
}

int launch_chain_dist(const DistArgs& a0, bool symmetric, int esize, int G, int threads, hipStream_t stream)
{
    DistArgs a = a0;
    a.quads = dist_words(a.n, esize);
    const size_t bytes = lds_dist_bytes(a.n, G, symmetric, esize, false);
    const int Gs = dist_scratch_groups(a.n, G, symmetric, esize, kLdsLimit - kDistStaticReserve);
    const size_t bytes_s = lds_dist_bytes(a.n, Gs, symmetric, esize, true);
    if (G > kMaxGroups || threads > 512 || threads % 64 != 0 || a.n > kMaxPerThread * threads ||
        (a.n + G - 1) / G > kMaxOwnRows)
        return QAP_E_INVAL;
    switch (esize) {
    case 1: return launch_dist_typed<uint8_t>(a, symmetric, G, Gs, threads, bytes, bytes_s, stream);
    case 2: return launch_dist_typed<uint16_t>(a, symmetric, G, Gs, threads, bytes, bytes_s, stream);
    case 4: return launch_dist_typed<uint32_t>(a, symmetric, G, Gs, threads, bytes, bytes_s, stream);
    default: return QAP_E_INVAL;
    }
}

}  // namespace qapsa
