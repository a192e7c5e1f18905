// qapsa_internal.hpp -- declarations shared by the translation units of libqapsa.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/qapsa.h"

namespace qapsa {

inline uint64_t temp_table_len(uint64_t iters)
{
    uint64_t nh = (iters + (1ull << 20) - 1) >> 20;
    return 2048 + (nh ? nh : 1);
}

// Everything one chain's kernel needs; passed by value.
constexpr uint32_t kFlagDeltaOnly = QAP_FLAG_DELTA_ONLY;
constexpr uint32_t kFlagScratchOnly = QAP_FLAG_SCRATCH_ONLY;

struct ChainArgs {
    int32_t n;
    int32_t pitch;        // LDS row pitch of A and B' (int16 elements, odd; 16-bit kernel)
    int32_t quads;        // LDS row pitch in dwords (odd; byte kernel)
    int32_t max_step;     // most proposals per lane in one scan step
    uint32_t flags;
    uint32_t switch_permille;
    int32_t a_min, b_min; // value shifts of the byte kernel
    const int32_t* A;
    int32_t* Bp;
    int32_t* p;
    int32_t* delta;
    qap_chain_state* state;
    const double* temps;
    qap_near_tie* ties;
    int64_t* acc_log;
    uint64_t acc_cap;
    uint64_t* prof;       // optional phase counters (QAP_PHASES)
    void* gscratch;       // byte kernel: global scratch for A and A^T bytes (Delta stays in `delta`)
    uint64_t iters;
    uint64_t t_end;
    double T0;
    uint64_t seed;
    uint32_t chain_id;
    uint32_t tie_cap;
    int32_t* tabu;        // tabu search: n*n table of the first iteration a facility may return to a location
    int32_t tenure;       // tabu search: iterations a left location stays tabu
    int32_t pad;
};

// LDS footprint (bytes) of the one-workgroup chain kernel.
size_t lds_chain_bytes(int n, bool symmetric, bool a_in_lds);
constexpr size_t kLdsLimit = 160 * 1024;
constexpr size_t kLdsStaticReserve = 2048;  // the kernels' static __shared__ variables
constexpr size_t kDistStaticReserve = 4096; // the multi-workgroup kernel's (about 2.6 KB)

int launch_cost(int n, const int32_t* A, const int32_t* B, const int32_t* p, int64_t* cost,
                hipStream_t stream);
int launch_delta_init(int n, const int32_t* A, const int32_t* B, const int32_t* p, int32_t* Bp,
                      int32_t* delta, qap_instance_info* info, qap_chain_state* state,
                      hipStream_t stream);
int launch_schedule_tables(uint64_t iters, double alpha, double* temps, hipStream_t stream);
// Delta for the current p of a chain whose state says it stopped in scratch
// mode before t_end or at the end of its schedule (read on the device; a no-op
// otherwise), then the mode: QAP_MODE_DELTA, or QAP_MODE_SCRATCH at t = iters.
int launch_delta_rebuild(int n, const int32_t* A, const int32_t* Bp, int32_t* delta, qap_chain_state* state,
                         uint64_t t_end, uint64_t iters, hipStream_t stream);
int launch_chain_lds(const ChainArgs& a, bool symmetric, bool a_in_lds, int threads,
                     hipStream_t stream);

// Global workspace of the multi-workgroup kernel (one per chain, caller memory).
struct DistWs {
    unsigned long long nties;    // near ties logged by this call
    int err;                     // a workgroup gave up waiting for the others
    int pad[13];
};
static_assert(sizeof(DistWs) == 64, "workspace header");

// Multi-workgroup exchange area: the header, two sets (by window parity) of
// one 64-bit slot per workgroup, then the published Delta values (two swap
// parities x G workgroups x ceil(n / G) own rows x {u, v}, at most
// 2 x 2 x (n + G) ints).
// The general (asymmetric) form adds copies (value - minimum, elements of
// esize bytes, rows padded to a multiple of 4 bytes) of A, A^T and B^T,
// 256-byte aligned after them.
constexpr int kMaxGroups = 1024;
inline size_t dist_row_bytes(int n, int esize) { return 4 * (((size_t)n * esize + 3) / 4); }
// proposals of one scratch-mode window at most; the partial sums of a window
// are exchanged through [2 parities][kMaxGroups * kScratchK] tagged entries,
// each parity holding scratch_reps(G) copies of G * K entries
constexpr int kScratchK = 16;
__host__ __device__ inline int scratch_reps(int G) { return G <= kMaxGroups / 4 ? 4 : (G <= kMaxGroups / 2 ? 2 : 1); }
inline size_t dist_ws_head(int n)
{
    const size_t b = sizeof(DistWs) + 2 * kMaxGroups * sizeof(unsigned long long) +
                     4 * sizeof(unsigned long long) * ((size_t)n + kMaxGroups) +
                     2 * (size_t)kMaxGroups * kScratchK * sizeof(unsigned long long);
    return (b + 255) & ~(size_t)255;
}
inline size_t dist_ws_bytes(int n, bool sym, int esize)
{
    return dist_ws_head(n) + (sym ? 0 : 3 * (size_t)n * dist_row_bytes(n, esize));
}
inline uint8_t* dist_bytes(void* ws, int n) { return (uint8_t*)ws + dist_ws_head(n); }
inline unsigned long long* dist_slots(void* ws) { return (unsigned long long*)((char*)ws + sizeof(DistWs)); }
// published Delta(r, u), Delta(r, v) of every row, two buffers by parity; each
// entry is (tag << 32) | value, the tag naming the update that wrote it
inline unsigned long long* dist_X(void* ws) { return dist_slots(ws) + 2 * kMaxGroups; }
// scratch-mode partial sums, after the published values (sized for any n)
inline unsigned long long* dist_P(void* ws, int n) { return dist_X(ws) + 4 * ((size_t)n + kMaxGroups); }

struct DistArgs {
    int32_t n;
    int32_t quads;               // 32-bit words per row of A and B' (set at launch)
    int32_t a_min, b_min;
    uint32_t kmin, kmax;         // scan window bounds (proposals)
    uint32_t random_order;       // 1: pairs drawn per iteration (QAP_FLAG_RANDOM_ORDER)
    uint32_t flags;              // QAP_FLAG_DELTA_ONLY / QAP_FLAG_SCRATCH_ONLY
    uint32_t switch_permille;    // scratch mode ends (the kernel returns, Delta stale) below this acceptance
    uint32_t pad2;
    uint64_t spin_limit;         // barrier polls before giving up
    const int32_t* A;
    const int32_t* B;
    int32_t* Bp;
    int32_t* p;
    int32_t* delta;
    qap_chain_state* state;
    const double* temps;
    qap_near_tie* ties;
    int64_t* acc_log;
    uint64_t acc_cap;
    uint64_t* prof;
    uint64_t iters;
    uint64_t t_end;
    double T0;
    uint64_t seed;
    uint32_t chain_id;
    uint32_t tie_cap;
    DistWs* ws;
    unsigned long long* slots;   // [2][kMaxGroups]
    unsigned long long* X;
    unsigned long long* Pp;      // [2][kMaxGroups][kScratchK] tagged scratch-mode partial sums
    const void* Ab;              // general form: copies of A, A^T, B^T (dist_bytes)
    const void* Atb;
    const void* Btb;
};

// Scratch-to-Delta switch threshold (per mille of accepted proposals over
// 8192 iterations) when the caller gives none: the fastest of 1-160 for the
// N = 150 asymmetric single chain over 1e8 iterations on MI355X (7-10; 20 was
// 1.3% slower, 160 60% slower).  The threshold never changes a run's result.
constexpr uint32_t kDefaultSwitchPermille = 10;
// the multi-workgroup kernel's scratch mode costs about one grid-wide exchange
// per window of up to 16 proposals, so Delta mode pays off sooner there
constexpr uint32_t kDefaultDistSwitchPermille = 30;

// element size of the multi-workgroup kernel for value ranges a_range, b_range:
// 1 (both <= 255), 2 (<= 65535) or 4
inline int dist_esize(int64_t a_range, int64_t b_range)
{
    const int64_t r = a_range > b_range ? a_range : b_range;
    return r <= 255 ? 1 : (r <= 65535 ? 2 : 4);
}
int dist_words(int n, int esize);
size_t lds_dist_bytes(int n, int G, bool symmetric, int esize, bool scratch = false);
int dist_scratch_groups(int n, int G, bool symmetric, int esize, size_t budget);
int launch_chain_dist(const DistArgs& a, bool symmetric, int esize, int G, int threads, hipStream_t stream);

// batched chains (one persistent launch, a device-wide work queue)
// Kinds of batched launch: placement x LDS class (class 1: the chains whose
// LDS bytes exceed BatchArgs::lds_split, class 0: the others), kind = 2 *
// placement + class.
constexpr int kBatchKinds = 2 * 4;
struct BatchWs {
    unsigned next[kBatchKinds];   // queue positions of the kernels of each kind
    unsigned pad[16 - kBatchKinds];
};
struct BatchArgs {
    int32_t n_chains;
    int32_t min_place;            // chains of a smaller placement run in this one
    const qap_chain_desc* descs;
    const int32_t* order;
    BatchWs* ws;
    uint64_t slice;
    uint64_t* prof;
    uint32_t lds_split;           // LDS bytes that separate the two classes (0: one class)
    int32_t cls;                  // the class this launch runs
};
// groups <= 0: as many workgroups as can be resident at once (occupancy of each
// kernel at its LDS size times the CU count), never more than its chains
int launch_chain_batch(const BatchArgs& b, int groups, const int count[kBatchKinds], int threads,
                       const size_t lds[kBatchKinds],
                       hipStream_t stream);
// a second stream (default priority) and two events of the current device, created once
int side_stream(int which, hipStream_t* side, hipEvent_t* fork, hipEvent_t* join);

// byte-valued chain kernel (scratch and Delta modes)
int wg_quads(int n);
// Placement of the one-workgroup kernel's state: 0 all in LDS, 1 Delta in
// device memory (the caller's buffer), 2 also the byte copies of A in a
// device scratch of wg_scratch_bytes, 3 also those of B'; -1 if the small
// per-chain vectors alone do not fit.
int wg_place(int n, bool symmetric);
size_t lds_wg_bytes(int n, bool symmetric, int place);
size_t wg_scratch_bytes(int n, bool symmetric, int place);
int launch_chain_wg(const ChainArgs& a, bool symmetric, int place, hipStream_t stream, bool tabu = false);

}  // namespace qapsa
