// qapsa_device.hpp -- device-side building blocks shared by the kernels of
// libqapsa: the Philox-4x32-10 generator, r_t of Eq. (2), the cooling table
// lookup, the Metropolis test, the accept hash and packed-pair indexing.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/qapsa.h"

namespace qapsa {

// ----------------------------------------------------------------- Philox
// Philox-4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11): each round
// multiplies words 0 and 2 by two fixed 32-bit constants, feeds the high halves
// (xor'ed with words 1, 3 and the round key) and the low halves into the next
// round, and the key advances by two Weyl increments.
struct PhiloxConst {
    static constexpr uint32_t kMulA = 0xD2511F53u;
    static constexpr uint32_t kMulB = 0xCD9E8D57u;
    static constexpr uint32_t kWeylA = 0x9E3779B9u;
    static constexpr uint32_t kWeylB = 0xBB67AE85u;
};

__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint32_t hA = __umulhi(PhiloxConst::kMulA, c.x);
        const uint32_t lA = PhiloxConst::kMulA * c.x;
        const uint32_t hB = __umulhi(PhiloxConst::kMulB, c.z);
        const uint32_t lB = PhiloxConst::kMulB * c.z;
        c = make_uint4(hB ^ c.y ^ k0, lB, hA ^ c.w ^ k1, lA);
        k0 += PhiloxConst::kWeylA;
        k1 += PhiloxConst::kWeylB;
    }
    return c;
}

// r_t in (0, 1): (2u + 1) 2^-53, u = the top 52 bits of words 0 and 1.
__device__ __forceinline__ double uniform_r(uint64_t seed, uint32_t chain, uint64_t t)
{
    const uint4 x = philox10(make_uint4((uint32_t)t, (uint32_t)(t >> 32), chain, 0u),
                             (uint32_t)seed, (uint32_t)(seed >> 32));
    const uint64_t u = ((uint64_t)x.x << 20) | (uint64_t)(x.y >> 12);
    return (double)(2ull * u + 1ull) * 0x1p-53;
}

// Random proposal order: iteration t proposes pair number floor(x2 M / 2^32)
// of the row-major enumeration (M = n(n-1)/2 pairs), x2 being the third output
// word of the same generator call that gives r_t.
__device__ __forceinline__ uint32_t random_pair_index(uint64_t seed, uint32_t chain, uint64_t t, uint32_t m)
{
    const uint4 x = philox10(make_uint4((uint32_t)t, (uint32_t)(t >> 32), chain, 0u),
                             (uint32_t)seed, (uint32_t)(seed >> 32));
    return __umulhi(x.z, m);
}

// ---------------------------------------------------------------- cooling
// temps = [L(1024) | M(1024) | H(...)], T_t = ((T0 * H) * M) * L.
__device__ __forceinline__ double temperature(const double* __restrict__ temps, double T0, uint64_t t)
{
    const double th = T0 * temps[2048 + (t >> 20)];
    const double tm = th * temps[1024 + ((t >> 10) & 1023u)];
    return tm * temps[t & 1023u];
}

// Any Delta above this bound is rejected by Eq. (2) at every t' >= t of a
// non-increasing schedule: log r >= log 2^-53 > -36.74, so Delta / T > 36.75
// makes z > 0.  The factor 1 + 1e-6 covers the last-bit wobble of the table
// product between neighbouring iterations.
__device__ __forceinline__ int32_t reject_bound(double T)
{
    const double b = 36.8 * T * 1.000001;
    return b >= 2147483647.0 ? 2147483647 : (int32_t)b;  // floor for b >= 0
}

// Eq. (2) for Delta > 0.  Returns the decision; *z receives fl(x + y).
__device__ __forceinline__ bool metropolis_positive(int64_t delta, double T, double r, double* z)
{
    const double x = (double)delta / T;
    const double y = log(r);
    const double zz = x + y;
    *z = zz;
    return zz < 0.0;
}

constexpr double kNearTie = 1e-12;

// At T = +inf (T0 = +inf makes every T_t infinite) Eq. (2) accepts every
// Delta > 0 and z = fl(0 + log r) = log r.  A near tie |z| < 1e-12 then needs
// r > 1 - 1e-12; every draw with u <= 2^52 - 9008, i.e. r <= 1 - 2.0001e-12,
// is clear of that band whatever the last bit of log, so only draws above
// it need the FP64 evaluation.
__device__ __forceinline__ bool inf_draw_clear(uint64_t seed, uint32_t chain, uint64_t t)
{
    const uint4 x = philox10(make_uint4((uint32_t)t, (uint32_t)(t >> 32), chain, 0u),
                             (uint32_t)seed, (uint32_t)(seed >> 32));
    const uint64_t u = ((uint64_t)x.x << 20) | (uint64_t)(x.y >> 12);
    return u <= (1ull << 52) - 9008ull;
}

// ------------------------------------------------------------------- hash
// The trajectory hash is the sum mod 2^64 over accepted swaps of a fingerprint
// of (t, r, s, Delta); the sum does not depend on the order in which swaps are
// folded in, so it can be accumulated in bulk.  The fingerprint chains three
// rounds of the splitmix64 output function (Steele, Lea, Flood, OOPSLA 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t accept_fingerprint(uint64_t t, int32_t r, int32_t s, int64_t d)
{
    uint64_t h = mix64(t);
    h = mix64(h ^ (((uint64_t)(uint32_t)r << 32) | (uint32_t)s));
    return mix64(h ^ (uint64_t)d);
}

// ------------------------------------------------------------ pair index
// Packed index of pair r < s in row-major order: rowstart(r) + s - r - 1.
__host__ __device__ __forceinline__ int64_t row_start(int64_t n, int64_t r)
{
    return r * (2 * n - r - 1) / 2;
}

__device__ __forceinline__ void pair_of(int n, int64_t idx, int& r, int& s)
{
    const double b = 2.0 * n - 1.0;
    int rr = (int)((b - sqrt(b * b - 8.0 * (double)idx)) * 0.5);
    if (rr < 0) rr = 0;
    if (rr > n - 2) rr = n - 2;
    while (rr > 0 && row_start(n, rr) > idx) --rr;
    while (rr < n - 2 && row_start(n, rr + 1) <= idx) ++rr;
    r = rr;
    s = rr + 1 + (int)(idx - row_start(n, rr));
}

}  // namespace qapsa
