// qapsa_init.hip -- one-off kernels of libqapsa: Eq. (1), B' (Eq. (3)),
// step (a) of Sec. 2.2 (the full Delta matrix), instance checks and the
// cooling tables.  None of this is on the per-iteration path.
#include <hip/hip_runtime.h>
#include <limits.h>

#include "qapsa_device.hpp"
#include "qapsa_internal.hpp"

namespace qapsa {

namespace {

__global__ void k_info_reset(qap_instance_info* info)
{
    info->cost = 0;
    info->sum_abs_delta = 0;
    info->a_min = INT_MAX;
    info->a_max = INT_MIN;
    info->b_min = INT_MAX;
    info->b_max = INT_MIN;
    info->symmetric = 1;
    info->status = QAP_OK;
}

// Value ranges, symmetry and the permutation check, one thread per (i, j).
// p is a permutation iff every entry is in range and no two entries are equal.
__global__ void __launch_bounds__(256) k_scan_inputs(int n, const int32_t* __restrict__ A,
                                                     const int32_t* __restrict__ B,
                                                     const int32_t* __restrict__ p,
                                                     qap_instance_info* info)
{
    const int64_t nn = (int64_t)n * n;
    int amin = INT_MAX, amax = INT_MIN, bmin = INT_MAX, bmax = INT_MIN;
    int sym = 1, perm = 1;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nn;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / n), j = (int)(e % n);
        const int a = A[e], b = B[e];
        amin = min(amin, a); amax = max(amax, a);
        bmin = min(bmin, b); bmax = max(bmax, b);
        if (a != A[(int64_t)j * n + i] || b != B[(int64_t)j * n + i]) sym = 0;
        if (j == 0 && (p[i] < 0 || p[i] >= n)) perm = 0;
        if (i < j && p[i] == p[j]) perm = 0;
    }
    // wave reductions, then one atomic per wave
    for (int off = 32; off > 0; off >>= 1) {
        amin = min(amin, __shfl_xor(amin, off));
        amax = max(amax, __shfl_xor(amax, off));
        bmin = min(bmin, __shfl_xor(bmin, off));
        bmax = max(bmax, __shfl_xor(bmax, off));
        sym &= __shfl_xor(sym, off);
        perm &= __shfl_xor(perm, off);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMin(&info->a_min, amin);
        atomicMax(&info->a_max, amax);
        atomicMin(&info->b_min, bmin);
        atomicMax(&info->b_max, bmax);
        if (!sym) atomicAnd(&info->symmetric, 0);
        if (!perm) atomicCAS(&info->status, (int)QAP_OK, (int)QAP_E_NOT_PERM);
    }
}

// The int32 bound of the Delta entries and the int64 bound of the cost.
__global__ void k_check_bounds(int n, qap_instance_info* info)
{
    if (info->status != QAP_OK) return;
    const long long ra = (long long)info->a_max - info->a_min;
    const long long rb = (long long)info->b_max - info->b_min;
    const long long ma = max(llabs((long long)info->a_max), llabs((long long)info->a_min));
    const long long mb = max(llabs((long long)info->b_max), llabs((long long)info->b_min));
    const __int128 d_bound = (__int128)(2 * (long long)n + 8) * ra * rb;
    const __int128 c_bound = (__int128)n * n * ma * mb;
    if (d_bound >= ((__int128)1 << 31) || c_bound >= ((__int128)1 << 62)) info->status = QAP_E_RANGE;
}

// Eq. (3): Bp[i][j] = B[p[i]][p[j]].
__global__ void __launch_bounds__(256) k_bprime(int n, const int32_t* __restrict__ B,
                                                const int32_t* __restrict__ p,
                                                int32_t* __restrict__ Bp,
                                                const qap_instance_info* info)
{
    if (info->status == QAP_E_NOT_PERM) return;
    const int64_t nn = (int64_t)n * n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nn;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / n), j = (int)(e % n);
        Bp[e] = B[(int64_t)p[i] * n + p[j]];
    }
}

// Eq. (1) as sum_ij A[i][j] * B[p[i]][p[j]] with int64 products; entries of p
// outside 0..n-1 contribute 0.
__global__ void __launch_bounds__(256) k_cost_gather(int n, const int32_t* __restrict__ A,
                                                     const int32_t* __restrict__ B,
                                                     const int32_t* __restrict__ p,
                                                     int64_t* __restrict__ out)
{
    const int64_t nn = (int64_t)n * n;
    long long acc = 0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nn;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / n), j = (int)(e % n);
        const int pi = p[i], pj = p[j];
        if (pi >= 0 && pi < n && pj >= 0 && pj < n)
            acc += (long long)A[e] * (long long)B[(int64_t)pi * n + pj];
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) atomicAdd((unsigned long long*)out, (unsigned long long)acc);
}

__global__ void k_zero64(int64_t* x) { *x = 0; }

// Step (a): every Delta(r,s), r < s, from
//   (A_rr - A_ss)(B'_ss - B'_rr) + (A_rs - A_sr)(B'_sr - B'_rs)
//   + sum_{k != r,s} (A_kr - A_ks)(B'_ks - B'_kr) + (A_rk - A_sk)(B'_sk - B'_rk)
// (Eq. (1) differenced over the terms that meet {r, s}), accumulated in int64.
// A 32 x 32 tile of (r, s) per workgroup; k runs in chunks of 32 staged in LDS,
// columns r and s of A and B' (rows k) and rows r and s (columns k).
constexpr int kTile = 32;

// Body of the Delta build for one tile; returns this thread's sum of |Delta|
// and sets *overflow when an entry does not fit int32.
__device__ __forceinline__ long long delta_tile(int n, const int32_t* __restrict__ A, const int32_t* __restrict__ Bp,
                                                int32_t* __restrict__ delta, int* overflow_out)
{
    // tiles (tr, ts) with ts >= tr, enumerated in row-major order of the tile triangle
    const int nt = (n + kTile - 1) / kTile;
    int tr = 0;
    int64_t b = blockIdx.x;
    while (b >= nt - tr) { b -= nt - tr; ++tr; }
    const int ts = tr + (int)b;
    const int r0 = tr * kTile, s0 = ts * kTile;

    __shared__ int32_t cAr[kTile][kTile + 1], cAs[kTile][kTile + 1];  // [k][r], [k][s]
    __shared__ int32_t cBr[kTile][kTile + 1], cBs[kTile][kTile + 1];
    __shared__ int32_t wAr[kTile][kTile + 1], wAs[kTile][kTile + 1];  // [r][k], [s][k]
    __shared__ int32_t wBr[kTile][kTile + 1], wBs[kTile][kTile + 1];

    const int tid = threadIdx.x;
    const int lr = tid >> 3;          // 0..31: this thread's r within the tile
    const int ls0 = tid & 7;          // s = s0 + ls0 + 8q, q = 0..3
    long long acc[4] = {0, 0, 0, 0};

    for (int k0 = 0; k0 < n; k0 += kTile) {
        for (int e = tid; e < kTile * kTile; e += 256) {
            const int a = e >> 5, c = e & 31;   // a: row within chunk, c: column within tile
            const int k = k0 + a;
            const bool kin = k < n;
            cAr[a][c] = (kin && r0 + c < n) ? A[(int64_t)k * n + r0 + c] : 0;
            cAs[a][c] = (kin && s0 + c < n) ? A[(int64_t)k * n + s0 + c] : 0;
            cBr[a][c] = (kin && r0 + c < n) ? Bp[(int64_t)k * n + r0 + c] : 0;
            cBs[a][c] = (kin && s0 + c < n) ? Bp[(int64_t)k * n + s0 + c] : 0;
            const int kk = k0 + c;              // row a of the tile, column kk
            const bool kkin = kk < n;
            wAr[a][c] = (kkin && r0 + a < n) ? A[(int64_t)(r0 + a) * n + kk] : 0;
            wAs[a][c] = (kkin && s0 + a < n) ? A[(int64_t)(s0 + a) * n + kk] : 0;
            wBr[a][c] = (kkin && r0 + a < n) ? Bp[(int64_t)(r0 + a) * n + kk] : 0;
            wBs[a][c] = (kkin && s0 + a < n) ? Bp[(int64_t)(s0 + a) * n + kk] : 0;
        }
        __syncthreads();
        const int kmax = min(kTile, n - k0);
        const int r = r0 + lr;
        for (int kc = 0; kc < kmax; ++kc) {
            const int k = k0 + kc;
            const long long akr = cAr[kc][lr], bkr = cBr[kc][lr];
            const long long ark = wAr[lr][kc], brk = wBr[lr][kc];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int ls = ls0 + 8 * q;
                const int s = s0 + ls;
                const long long aks = cAs[kc][ls], bks = cBs[kc][ls];
                const long long ask = wAs[ls][kc], bsk = wBs[ls][kc];
                const long long term = (akr - aks) * (bks - bkr) + (ark - ask) * (bsk - brk);
                acc[q] += (k != r && k != s) ? term : 0;
            }
        }
        __syncthreads();
    }

    const int r = r0 + lr;
    long long local_abs = 0;
    int overflow = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int s = s0 + ls0 + 8 * q;
        if (r < n && s < n && r < s) {
            const long long arr = A[(int64_t)r * n + r], ass = A[(int64_t)s * n + s];
            const long long ars = A[(int64_t)r * n + s], asr = A[(int64_t)s * n + r];
            const long long brr = Bp[(int64_t)r * n + r], bss = Bp[(int64_t)s * n + s];
            const long long brs = Bp[(int64_t)r * n + s], bsr = Bp[(int64_t)s * n + r];
            const long long d = acc[q] + (arr - ass) * (bss - brr) + (ars - asr) * (bsr - brs);
            if (d > INT_MAX || d < INT_MIN) overflow = 1;
            delta[row_start(n, r) + (s - r - 1)] = (int32_t)d;
            local_abs += d < 0 ? -d : d;
        }
    }
    *overflow_out = overflow;
    return local_abs;
}

__global__ void __launch_bounds__(256) k_delta_init(int n, const int32_t* __restrict__ A,
                                                    const int32_t* __restrict__ Bp,
                                                    int32_t* __restrict__ delta,
                                                    qap_instance_info* info)
{
    if (info->status != QAP_OK) return;
    int overflow = 0;
    long long local_abs = delta_tile(n, A, Bp, delta, &overflow);
    const int tid = threadIdx.x;
    for (int off = 32; off > 0; off >>= 1) {
        local_abs += __shfl_xor(local_abs, off);
        overflow |= __shfl_xor(overflow, off);
    }
    if ((tid & 63) == 0) {
        atomicAdd((unsigned long long*)&info->sum_abs_delta, (unsigned long long)local_abs);
        if (overflow) atomicCAS(&info->status, (int)QAP_OK, (int)QAP_E_RANGE);
    }
}

// A chain that stopped in scratch mode (Delta left stale) either to move to
// Delta mode before t_end or at the end of its schedule gets its Delta matrix
// rebuilt for the current p from B' (kept current by every run); any other
// chain is left alone.  The condition is read from the device state, so a
// caller can queue the rebuild without knowing whether it is needed.
__device__ __forceinline__ bool needs_rebuild(const qap_chain_state* st, uint64_t t_end, uint64_t iters)
{
    return st->status == QAP_OK && st->mode == QAP_MODE_SCRATCH_STALE && (st->t < t_end || st->t >= iters);
}

__global__ void __launch_bounds__(256) k_delta_rebuild(int n, const int32_t* __restrict__ A,
                                                       const int32_t* __restrict__ Bp, int32_t* __restrict__ delta,
                                                       const qap_chain_state* st, uint64_t t_end, uint64_t iters)
{
    if (!needs_rebuild(st, t_end, iters)) return;
    int overflow = 0;
    (void)delta_tile(n, A, Bp, delta, &overflow);   // the instance passed the bound check: no overflow
}

__global__ void k_rebuild_done(qap_chain_state* st, uint64_t t_end, uint64_t iters)
{
    if (needs_rebuild(st, t_end, iters)) st->mode = st->t >= iters ? QAP_MODE_SCRATCH : QAP_MODE_DELTA;
}

__global__ void k_state_reset(const qap_instance_info* info, qap_chain_state* st)
{
    st->t = 0;
    st->accepts = 0;
    st->near_ties = 0;
    st->hash = 0;
    st->cost = info->cost;
    st->best_cost = info->cost;
    st->best_iter = 0;
    st->status = info->status;
    st->mode = QAP_MODE_SCRATCH;
}

// Cooling tables of a geometric schedule: three serial recurrences (one thread).
__global__ void k_schedule_tables(uint64_t nh, double alpha, double* temps)
{
    double* L = temps;
    double* M = temps + 1024;
    double* H = temps + 2048;
    double x = 1.0;
    L[0] = 1.0;
    for (int j = 1; j < 1024; ++j) { x = x * alpha; L[j] = x; }
    const double step_m = L[1023] * alpha;
    x = 1.0;
    M[0] = 1.0;
    for (int j = 1; j < 1024; ++j) { x = x * step_m; M[j] = x; }
    const double step_h = M[1023] * step_m;
    x = 1.0;
    H[0] = 1.0;
    for (uint64_t j = 1; j < nh; ++j) { x = x * step_h; H[j] = x; }
}

// The launches below report failure through the thread's last-error slot,
// which also holds the last non-success code of any earlier runtime call of
// the process (a query that returned "not ready", say).  Reset it first so
// that the check after the launches sees only their own errors.
void clear_error() { (void)hipGetLastError(); }

int grid_for(int64_t work, int block)
{
    int64_t g = (work + block - 1) / block;
    if (g > 4096) g = 4096;
    return (int)(g < 1 ? 1 : g);
}

}  // namespace

int launch_cost(int n, const int32_t* A, const int32_t* B, const int32_t* p, int64_t* cost,
                hipStream_t stream)
{
    clear_error();
    hipLaunchKernelGGL(k_zero64, dim3(1), dim3(1), 0, stream, cost);
    hipLaunchKernelGGL(k_cost_gather, dim3(grid_for((int64_t)n * n, 256)), dim3(256), 0, stream,
                       n, A, B, p, cost);
    return hipGetLastError() == hipSuccess ? QAP_OK : QAP_E_DEVICE;
}

int launch_delta_init(int n, const int32_t* A, const int32_t* B, const int32_t* p, int32_t* Bp,
                      int32_t* delta, qap_instance_info* info, qap_chain_state* state,
                      hipStream_t stream)
{
    const int64_t nn = (int64_t)n * n;
    clear_error();
    hipLaunchKernelGGL(k_info_reset, dim3(1), dim3(1), 0, stream, info);
    hipLaunchKernelGGL(k_scan_inputs, dim3(grid_for(nn, 256)), dim3(256), 0, stream, n, A, B, p, info);
    hipLaunchKernelGGL(k_check_bounds, dim3(1), dim3(1), 0, stream, n, info);
    hipLaunchKernelGGL(k_bprime, dim3(grid_for(nn, 256)), dim3(256), 0, stream, n, B, p, Bp, info);
    hipLaunchKernelGGL(k_cost_gather, dim3(grid_for(nn, 256)), dim3(256), 0, stream, n, A, B, p,
                       &info->cost);
    const int nt = (n + kTile - 1) / kTile;
    const int tiles = nt * (nt + 1) / 2;
    hipLaunchKernelGGL(k_delta_init, dim3(tiles), dim3(256), 0, stream, n, A, Bp, delta, info);
    if (state) hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(1), 0, stream, info, state);
    return hipGetLastError() == hipSuccess ? QAP_OK : QAP_E_DEVICE;
}

int launch_delta_rebuild(int n, const int32_t* A, const int32_t* Bp, int32_t* delta, qap_chain_state* state,
                         uint64_t t_end, uint64_t iters, hipStream_t stream)
{
    clear_error();
    const int nt = (n + kTile - 1) / kTile;
    const int tiles = nt * (nt + 1) / 2;
    hipLaunchKernelGGL(k_delta_rebuild, dim3(tiles), dim3(256), 0, stream, n, A, Bp, delta, state, t_end, iters);
    hipLaunchKernelGGL(k_rebuild_done, dim3(1), dim3(1), 0, stream, state, t_end, iters);
    return hipGetLastError() == hipSuccess ? QAP_OK : QAP_E_DEVICE;
}

int launch_schedule_tables(uint64_t iters, double alpha, double* temps, hipStream_t stream)
{
    const uint64_t nh = temp_table_len(iters) - 2048;
    clear_error();
    hipLaunchKernelGGL(k_schedule_tables, dim3(1), dim3(1), 0, stream, nh, alpha, temps);
    return hipGetLastError() == hipSuccess ? QAP_OK : QAP_E_DEVICE;
}

}  // namespace qapsa
