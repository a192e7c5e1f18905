/*
 * qapsa.h -- C ABI of libqapsa: Delta-matrix simulated annealing for the
 * quadratic assignment problem (QAP) on AMD Instinct MI355X (gfx950).
 *
 * Method: G. Paul, "A GPU implementation of the Simulated Annealing Heuristic
 * for the Quadratic Assignment Problem", arXiv 1208.2675.
 *   - Problem, Sec. 1, Eq. (1): N facilities are placed at N locations.
 *     A[i*N+j] is the flow between facilities i and j, B[k*N+l] the distance
 *     between locations k and l, and p[i] the location of facility i.  The cost
 *     of p is C(p) = sum_i sum_j A[i][j] * B[p[i]][p[j]].
 *   - Move, Sec. 2.1: swap the locations of two facilities r and s.  Its cost
 *     change is Delta(r,s) = C(p o (r s)) - C(p).
 *   - Acceptance, Sec. 2.1, Eq. (2): a proposed swap is made when Delta < 0 or
 *     exp(-Delta/T) > r, r uniform in (0, 1), T lowered after every iteration.
 *   - Delta-matrix approach, Sec. 2.2, steps (a)-(e): keep Delta(r,s) for all
 *     pairs; step through proposals; on an accepted swap update p and Delta.
 *   - B' matrix, Sec. 3, Eq. (3): B'[i][j] = B[p[i]][p[j]] is kept alongside p
 *     so that every term of an update reads A and B' at the same index.
 *
 * Readings fixed by this library where the paper leaves a choice open:
 *   - Proposals enumerate the pairs r < s in row-major order, cyclically;
 *     iteration t (0-based) proposes pair number t mod N(N-1)/2.  Every
 *     proposal is one iteration, accepted or not.
 *   - Delta is stored packed: the N(N-1)/2 pairs r < s in row-major order,
 *     which is also the proposal order.  Entries are int32; every cost is int64.
 *   - r_t of iteration t of a chain is (2u + 1) * 2^-53, where u is the 52-bit
 *     number (x0 << 20) | (x1 >> 12) and (x0, x1, x2, x3) is Philox-4x32-10
 *     (Salmon et al., SC'11) at counter (lo32 t, hi32 t, chain_id, 0) and key
 *     (lo32 seed, hi32 seed).
 *   - Eq. (2) in binary64: Delta <= 0 is accepted; otherwise with
 *     z = fl(fl(Delta / T_t) + fl(log r_t)) the swap is made iff z < 0.
 *     Evaluations with |z| < 1e-12 are reported as near ties.
 *   - Cooling: geometric, T_t = ((T0 * H[t >> 20]) * M[(t >> 10) & 1023]) * L[t & 1023]
 *     with L[0] = M[0] = H[0] = 1, L[j] = L[j-1] * alpha,
 *     M[j] = M[j-1] * (L[1023] * alpha), H[j] = H[j-1] * (M[1023] * L[1023] * alpha).
 *
 * Conventions for every call:
 *   - Pointers are DEVICE pointers unless the comment says host.  The caller
 *     owns all memory; the library allocates none.  Matrices are row-major.
 *   - Calls are asynchronous on `stream` and never synchronise it.  Errors in
 *     the arguments are returned at once as a negative qap_status.  Errors
 *     that only the device can see are written to a device status field
 *     (qap_instance_info.status, qap_chain_state.status).
 *   - Calls that share device buffers must be ordered by the caller (same
 *     stream or events); calls on disjoint buffers may run concurrently.
 */
#ifndef QAPSA_H
#define QAPSA_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QAP_API __attribute__((visibility("default")))

typedef enum {
    QAP_OK = 0,
    QAP_E_INVAL = -1,        /* bad argument (null pointer, n < 2, bad schedule, ...) */
    QAP_E_NOT_PERM = -2,     /* p is not a permutation of 0..n-1                      */
    QAP_E_RANGE = -3,        /* the instance's values overflow the int32 Delta bound  */
    QAP_E_NOMEM = -4,        /* a size exceeds what the chosen kernel can hold         */
    QAP_E_DEVICE = -5,       /* a HIP runtime call failed                              */
    QAP_E_UNSUPPORTED = -6,  /* no kernel in this build handles the request            */
    QAP_E_STATE = -7,        /* a chain state that is not ready (see qap_chain_state)  */
    QAP_E_TIMEOUT = -8,      /* a grid barrier of a multi-workgroup run did not complete */
    QAP_E_TIE_OVERFLOW = -9  /* more near ties of Eq. (2) in one scan window than the
                                multi-workgroup kernel can record exactly; the run stops
                                rather than report a near-tie count that is too low    */
} qap_status;

/* Facts about an instance and start permutation, written by qap_delta_init. */
typedef struct {
    int64_t cost;           /* Eq. (1) at p                                         */
    int64_t sum_abs_delta;  /* sum over r < s of |Delta(r,s)|; T0 = this / (n(n-1)/2) */
    int32_t a_min, a_max;   /* value range of A                                     */
    int32_t b_min, b_max;   /* value range of B                                     */
    int32_t symmetric;      /* 1 if A == A^T and B == B^T                           */
    int32_t status;         /* QAP_OK, QAP_E_NOT_PERM or QAP_E_RANGE                */
} qap_instance_info;

/* Device-resident state of one annealing chain; carried between calls. */
typedef struct {
    uint64_t t;          /* next iteration index                                      */
    uint64_t accepts;    /* swaps made so far                                         */
    uint64_t near_ties;  /* Eq. (2) evaluations with |z| < 1e-12 so far                */
    uint64_t hash;       /* sum mod 2^64 over accepted swaps (t, r, s, Delta) of
                            f(f(f(t) ^ (r << 32 | s)) ^ Delta), f the splitmix64 output
                            function; starts at 0                                      */
    int64_t cost;        /* Eq. (1) at the current p, tracked incrementally           */
    int64_t best_cost;   /* lowest cost reached so far                                */
    uint64_t best_iter;  /* iterations completed when best_cost was first reached     */
    int32_t status;      /* QAP_OK, or the first error the device saw                 */
    int32_t mode;        /* how swap costs are produced: QAP_MODE_SCRATCH (each proposal's
                            cost computed in O(N) when it is met) or QAP_MODE_DELTA (the
                            Delta matrix of Sec. 2.2 is kept), and whether the caller's
                            delta buffer holds Delta for the current p: it does in
                            QAP_MODE_SCRATCH and QAP_MODE_DELTA; QAP_MODE_SCRATCH_STALE
                            (scratch mode, delta left as it was) follows a call that
                            stopped in scratch mode before t = iters                   */
} qap_chain_state;

#define QAP_MODE_SCRATCH 0
#define QAP_MODE_DELTA 1
#define QAP_MODE_SCRATCH_STALE 2

/* One near tie of Eq. (2). */
typedef struct {
    uint64_t t;
    int64_t delta;
    double z;            /* fl(fl(delta / T_t) + fl(log r_t)) */
} qap_near_tie;

/* Schedule of one run (host struct). */
typedef struct {
    uint64_t iters;      /* I, the length of the whole schedule (Sec. 2.2 step (e))    */
    uint64_t t_end;      /* this call runs iterations state.t .. t_end-1; t_end <= iters */
    double T0;           /* start temperature; +inf accepts every proposal            */
    double alpha;        /* per-iteration cooling factor, 0 < alpha <= 1              */
    uint64_t seed;       /* generator key                                             */
    uint32_t chain_id;   /* third generator counter word                              */
    uint32_t flags;      /* 0 or QAP_FLAG_* below                                      */
    uint32_t switch_permille; /* a chain in scratch mode moves to Delta mode when fewer
                            than this many proposals per 1000 were accepted over the
                            last 8192 iterations; 0 selects the default (10 on one
                            workgroup, 30 over many workgroups)                        */
    uint32_t scan_window; /* the size of the subset of proposals tested at once against
                            the unchanged Delta (Sec. 3 (ii), an adjustable parameter):
                            multi-workgroup kernel, proposals in the first window after
                            an accepted swap (doubling while no window accepts; 2^4 to
                            2^21); one-workgroup kernel, the largest scan step (a
                            multiple of 256 up to 16384, steps doubling from 256 to it);
                            0 selects the defaults (256, and 512 in random order, on the
                            grid; 4096 on one workgroup).  Never changes the run's
                            result                                                    */
} qap_schedule;

/* qap_schedule.flags.  The run is the same whichever mode produces the swap
   costs; the flags only pin the mode. */
#define QAP_FLAG_DELTA_ONLY 1u    /* keep the Delta matrix from the first iteration (Sec. 2.2) */
#define QAP_FLAG_SCRATCH_ONLY 2u  /* never build the Delta matrix during the run              */
#define QAP_FLAG_MULTI_WG 4u      /* byte-valued instances: run on the multi-workgroup kernel
                                     even where one workgroup could hold the chain
                                     (qap_sa_run only; the result is the same)                */
#define QAP_FLAG_RANDOM_ORDER 8u  /* propose the pairs at random instead of in row-major order
                                     (Sec. 2.1): iteration t proposes pair number
                                     floor(x2 M / 2^32) of the row-major enumeration, x2 the
                                     third output word of the generator call that gives r_t.
                                     A different run from the default order; resumed slices
                                     must keep the flag                                       */
#define QAP_FLAG_SINGLE_WG 16u    /* run on one workgroup wherever one can hold the chain (with
                                     Delta, A and B' in bufs->workspace where LDS runs out),
                                     never on the multi-workgroup kernel (qap_sa_run only; the
                                     result is the same; excludes QAP_FLAG_MULTI_WG)          */

/* Device buffers a run reads or appends to (host struct of device pointers). */
typedef struct {
    const double* temps;     /* qap_temp_table_len(iters) doubles from qap_schedule_tables */
    qap_near_tie* ties;      /* optional: first tie_cap near ties, in no fixed order       */
    uint32_t tie_cap;
    uint32_t reserved;
    int64_t* accept_log;     /* optional: 4 int64 (t, r, s, Delta) per accepted swap,
                                entry k for the k-th swap of the chain (k < accept_cap)    */
    uint64_t accept_cap;
    uint64_t* phase_cycles;  /* optional: QAP_PHASES counters, added to (see below)         */
    void* workspace;         /* qap_workspace_bytes(n) bytes of device memory, required when
                                the run spreads over several workgroups (large n); the
                                library initialises it on every call                      */
    uint64_t workspace_bytes;
} qap_run_buffers;

/* Indices of qap_run_buffers.phase_cycles: shader-clock cycles spent per phase
   and event counts, accumulated over calls.  Recorded by the first thread of
   the workgroup that runs a chain; phases end at workgroup barriers. */
enum {
    QAP_PH_TOTAL = 0,          /* cycles in the iteration loop                     */
    QAP_PH_SCRATCH_THRESH = 1, /* cycles computing acceptance thresholds          */
    QAP_PH_SCRATCH_EVAL = 2,   /* cycles evaluating proposals from scratch        */
    QAP_PH_SCRATCH_ACCEPT = 3, /* cycles making swaps in scratch mode             */
    QAP_PH_DELTA_SCAN = 4,     /* cycles scanning Delta                            */
    QAP_PH_DELTA_UPDATE = 5,   /* cycles updating Delta after swaps                */
    QAP_PH_BUILD = 6,          /* cycles rebuilding Delta from scratch             */
    QAP_PH_IO = 7,             /* cycles loading and writing back state            */
    QAP_PH_N_ROUNDS = 8,       /* scratch-mode rounds                              */
    QAP_PH_N_SCRATCH_ACC = 9,  /* swaps made in scratch mode                       */
    QAP_PH_N_SCAN_STEPS = 10,  /* Delta-mode scan steps                            */
    QAP_PH_N_DELTA_ACC = 11,   /* swaps made in Delta mode                         */
    QAP_PH_N_THRESH = 12,      /* threshold refills                                */
    QAP_PH_SWITCH_T = 13,      /* iteration at which the chain entered Delta mode  */
    QAP_PH_N_SCANNED = 14,     /* proposals tested in Delta mode                   */
    QAP_PH_GRID_SYNC = 15,     /* cycles from a scan window to the grid-wide result (multi-workgroup) */
    QAP_PHASES = 16
};

/* Text for a qap_status value (static storage). */
QAP_API const char* qap_strerror(int status);

/*
 * Eq. (1): *cost = sum_ij A[i][j] * B[p[i]][p[j]] in int64.
 * A, B: n*n int32; p: n int32, a permutation (entries outside 0..n-1 are
 * counted as 0 and make *cost meaningless); cost: 1 int64.
 */
QAP_API int qap_cost(int32_t n, const int32_t* A, const int32_t* B, const int32_t* p,
                     int64_t* cost, hipStream_t stream);

/*
 * Step (a) of Sec. 2.2 with Eq. (3): for permutation p build
 *   Bp[i*n+j] = B[p[i]][p[j]]                              (n*n int32, written)
 *   delta[idx(r,s)] = C(p o (r s)) - C(p) for all r < s     (n(n-1)/2 int32, written)
 * and fill *info (device).  If state != NULL it is reset to a fresh chain at
 * t = 0 with cost = info->cost, in QAP_MODE_SCRATCH.
 * The whole Delta matrix is computed from Eq. (1) differenced over the terms
 * that meet {r, s}, in int64, and stored as int32.  info->status becomes
 * QAP_E_NOT_PERM if p is not a permutation and QAP_E_RANGE unless
 *   (2n + 8) * (a_max - a_min) * (b_max - b_min) < 2^31   and
 *   n^2 * max|A| * max|B| < 2^62;
 * in both cases Bp and delta are left unspecified.  O(n^3) work.
 */
QAP_API int qap_delta_init(int32_t n, const int32_t* A, const int32_t* B, const int32_t* p,
                           int32_t* Bp, int32_t* delta, qap_instance_info* info,
                           qap_chain_state* state, hipStream_t stream);

/* Bytes of device workspace a run of an n-facility instance may need
   (qap_run_buffers.workspace): the larger of the multi-workgroup area (the
   exchange slots, published values and scratch-mode partial sums, 311360 + 32 n
   rounded up to 256, plus
   for asymmetric instances byte copies of A, A^T and B^T, 3 n * 4 ceil(n/4))
   and the one-workgroup scratch for asymmetric chains (qap_chain_scratch_bytes(n, 0)). */
QAP_API uint64_t qap_workspace_bytes(int32_t n);

/* Number of doubles in the temperature table of a schedule of `iters` iterations:
   2048 + ceil(iters / 2^20) (at least one H entry). */
QAP_API uint64_t qap_temp_table_len(uint64_t iters);

/*
 * Fill temps (device, qap_temp_table_len(iters) doubles) with the cooling
 * tables L (1024), M (1024) and H of a geometric schedule with factor alpha
 * (see the reading above).  The cooling schedule of Sec. 2.1 is left open by
 * the paper; this is the geometric one, evaluable for any t in O(1).
 */
QAP_API int qap_schedule_tables(uint64_t iters, double alpha, double* temps, hipStream_t stream);

/*
 * The geometric cooling schedule of a run (host only, no device work).  The
 * paper lowers T after every iteration (Sec. 2.1) without fixing the form;
 * this library reads it as geometric from T0 to final_ratio * T0 over `iters`
 * iterations, with T0 the mean |Delta| of the starting Delta matrix (step (a)
 * of Sec. 2.2):
 *   T0    = (double) info->sum_abs_delta / (double) (n (n - 1) / 2), one IEEE division
 *   alpha = pow(final_ratio, 1 / (iters - 1)), or 1 when iters == 1
 *   n      instance size (>= 2), the one qap_delta_init was called with
 *   info   host copy of the qap_instance_info qap_delta_init wrote
 *   iters  I, the length of the whole schedule (>= 1)
 *   final_ratio  T_{I-1} / T0, in (0, 1]; 1e-3 for the standard workloads
 *   sched  host, written: iters, t_end (= iters), T0 and alpha; seed, chain_id,
 *          flags, switch_permille and scan_window are left as the caller set them
 * Returns QAP_E_INVAL for n < 2, iters == 0, a ratio outside (0, 1] or a null
 * pointer, info->status when it is not QAP_OK, and QAP_E_INVAL when T0 would
 * be 0 (every swap cost 0: the schedule of Eq. (2) is then undefined).
 */
QAP_API int qap_schedule_init(int32_t n, const qap_instance_info* info, uint64_t iters, double final_ratio,
                              qap_schedule* sched);

/*
 * Steps (b)-(e) of Sec. 2.2 for one chain: iterations state->t .. sched->t_end-1.
 *   A      n*n int32 flows (read)
 *   B      n*n int32 distances (read; rows of B' are regathered from B and p)
 *   Bp     n*n int32 B' for the current p (read, updated per accepted swap, Eq. (3))
 *   p      n int32 permutation (read, updated)
 *   delta  n(n-1)/2 int32 packed Delta for the current p (read, updated)
 *   state  chain state (read, updated); state->status must be QAP_OK
 *   sched  host: schedule (T0, alpha, iters, t_end, seed, chain_id)
 *   info   host: the qap_instance_info qap_delta_init wrote for this instance
 *          (copied back by the caller); selects the kernel and the value width
 *   bufs   host struct of device pointers: temperature table (required), logs
 * Each accepted swap (u, v) updates p and B' and adds Delta(u,v) to the cost.
 * In QAP_MODE_DELTA it also updates every Delta entry: pairs disjoint from
 * {u, v} by an O(1) correction, pairs that meet {u, v} by an O(n)
 * recomputation (the general asymmetric form).  In QAP_MODE_SCRATCH each
 * proposal's swap cost is computed in O(n) when it is met; Delta is rebuilt
 * when the chain moves to Delta mode and when a call ends the schedule
 * (t = iters), and is otherwise left stale (state->mode says which).  The
 * 16-bit kernel needs a current Delta and fails with QAP_E_STATE on a stale
 * one.  The multi-workgroup kernel runs both modes: in scratch mode every
 * workgroup sums its own rows' terms of the swap costs of a window of up to 16
 * proposals and the workgroups exchange these partial sums; when the chain
 * moves to Delta mode the call rebuilds Delta between two launches and goes
 * on.  The run is identical whatever the split of [0, iters) into calls and
 * whichever mode is active.
 * Kernels: one workgroup holds the chain when its B' fits one CU's LDS
 * (Delta and then A moving to device memory first); otherwise (symmetric
 * instances up to about 2600 facilities, asymmetric ones up to about 2000)
 * the chain is spread over many workgroups of one cooperative launch, which
 * needs bufs->workspace; larger ones that qap_single_workgroup accepts run on
 * one workgroup with Delta, A and B' in bufs->workspace.  QAP_FLAG_MULTI_WG
 * and QAP_FLAG_SINGLE_WG override the choice where the other kernel can take
 * the chain.  Returns QAP_E_UNSUPPORTED when no kernel of this build handles n
 * and the value ranges, QAP_E_RANGE when info->status says so.
 */
QAP_API int qap_sa_run(int32_t n, const int32_t* A, const int32_t* B, int32_t* Bp, int32_t* p, int32_t* delta,
                       qap_chain_state* state, const qap_schedule* sched,
                       const qap_instance_info* info, const qap_run_buffers* bufs,
                       hipStream_t stream);

/* ------------------------------------------------------ no-allocation run */

/* Bytes of the library's static device scratch (1 MiB per device). */
QAP_API uint64_t qap_static_scratch_bytes(void);

/*
 * qap_sa_run for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same run, identical results, but the workspace of the kernels that need one
 * (the multi-workgroup exchange area, the per-chain scratch of a one-workgroup
 * chain whose matrices outgrow LDS) is a device array inside the library,
 * qap_static_scratch_bytes() bytes, one per device, held until the process
 * ends.  Nothing is allocated on any call.
 *   arguments  as for qap_sa_run; bufs->workspace must be NULL and
 *              bufs->workspace_bytes 0 (QAP_E_INVAL otherwise)
 * Returns QAP_E_NOMEM, before any device work, when the chosen kernel needs
 * more workspace than the static scratch holds (symmetric multi-workgroup
 * chains fit at every size the kernel takes; one-workgroup chains with device
 * scratch up to about 500 facilities), and what qap_sa_run returns otherwise.
 * Every call on one device shares that device's array, which keeps the last
 * call's contents (each kernel initialises what it reads): calls that overlap
 * on one device, on any streams, race and give wrong results.  Order them.
 */
QAP_API int qap_sa_run_static(int32_t n, const int32_t* A, const int32_t* B, int32_t* Bp, int32_t* p,
                              int32_t* delta, qap_chain_state* state, const qap_schedule* sched,
                              const qap_instance_info* info, const qap_run_buffers* bufs, hipStream_t stream);

/* ------------------------------------------------------------- tabu search */

/* Schedule of a tabu search (host struct). */
typedef struct {
    uint64_t iters;      /* length of the whole search; iters + tenure < 2^31           */
    uint64_t t_end;      /* this call runs iterations state.t .. t_end-1; t_end <= iters */
    int32_t tenure;      /* iterations for which a facility may not return to a location
                            it left (>= 0)                                              */
    uint32_t reserved;   /* must be 0                                                   */
} qap_tabu_schedule;

/*
 * Tabu search over the same Delta matrix: the heuristic Sec. 2.2 and 2.4 name
 * as the source of the Delta bookkeeping, which evaluates every swap and makes
 * one each iteration (Sec. 2.4).  The paper fixes no tabu rules; these are:
 * when facility i leaves location l at iteration t, returning i to l is tabu
 * for iterations t' < t + tenure; the swap (r, s) is tabu when both of its new
 * assignments (r to p(s), s to p(r)) are; a tabu swap is admissible when it
 * gives a cost below the best seen.  Iteration t makes the admissible swap of
 * least Delta (lowest packed index among equals), or the least Delta of all
 * when none is admissible, and updates Delta, B', p and the cost exactly as
 * qap_sa_run does for an accepted swap.
 *   A, Bp, p, delta, state, info  as for qap_sa_run (state->accepts counts the
 *          swaps, one per iteration; a stale Delta is rebuilt first)
 *   tabu   device, n*n int32, caller-owned: entry i*n + l is the first
 *          iteration at which facility i may return to location l.  Zero it
 *          before the first call of a search; keep it between calls.
 *   bufs   accept_log, phase_cycles and, where qap_single_workgroup says 2,
 *          workspace (qap_chain_scratch_bytes) are used; temps may be NULL.
 * One workgroup runs the search: byte-valued instances that
 * qap_single_workgroup accepts; QAP_E_UNSUPPORTED otherwise.
 */
QAP_API int qap_tabu_run(int32_t n, const int32_t* A, int32_t* Bp, int32_t* p, int32_t* delta,
                         qap_chain_state* state, const qap_tabu_schedule* sched,
                         const qap_instance_info* info, int32_t* tabu, const qap_run_buffers* bufs,
                         hipStream_t stream);

/* ----------------------------------------------------------------- batches */

/* One chain of a batched run.  Every pointer is a device pointer; the fields
   copied from qap_instance_info and qap_schedule have the same meaning there. */
typedef struct {
    int32_t n;
    int32_t symmetric;          /* qap_instance_info.symmetric                      */
    int32_t a_min, a_max;       /* qap_instance_info value ranges                   */
    int32_t b_min, b_max;
    uint32_t flags;             /* qap_schedule.flags                               */
    uint32_t switch_permille;   /* qap_schedule.switch_permille                     */
    const int32_t* A;
    int32_t* Bp;
    int32_t* p;
    int32_t* delta;
    qap_chain_state* state;
    const double* temps;        /* the chain's cooling tables (qap_schedule_tables) */
    qap_near_tie* ties;         /* optional                                         */
    uint32_t tie_cap;
    uint32_t chain_id;
    uint64_t iters;
    uint64_t t_end;
    double T0;
    uint64_t seed;
    void* scratch;              /* NULL, or qap_chain_scratch_bytes(n, symmetric) bytes of device
                                   memory: the chain then keeps Delta in `delta` and byte copies
                                   of A in scratch, and only B' uses LDS (larger n fits)       */
} qap_chain_desc;

typedef struct {
    int32_t threads;            /* threads per workgroup, a multiple of 64 up to 256; 0 picks 256  */
    int32_t groups;             /* persistent workgroups; 0 fills the device (LDS permitting)     */
    uint64_t slice;             /* > 0: every chain stops after at most this many iterations,
                                   so one launch advances the whole batch by a slice            */
    uint64_t* phase_cycles;     /* optional QAP_PHASES counters summed over chains              */
} qap_batch_config;

/* 1 if one workgroup can hold a chain of n facilities whose A and B value
   ranges (max - min) are a_range and b_range entirely in LDS; 2 if it can with
   a per-chain scratch (qap_chain_desc.scratch); 0 otherwise. */
QAP_API int qap_single_workgroup(int32_t n, int32_t symmetric, int64_t a_range, int64_t b_range);

/* Bytes of the per-chain scratch of qap_chain_desc.scratch (and of the
   single-chain workspace when a chain needs it). */
QAP_API uint64_t qap_chain_scratch_bytes(int32_t n, int32_t symmetric);

/* Bytes of device workspace qap_sa_run_batch needs (64). */
QAP_API uint64_t qap_batch_workspace_bytes(void);

/*
 * Steps (b)-(e) of Sec. 2.2 for many independent chains of different sizes in
 * one persistent launch.  Each workgroup repeatedly takes the next chain
 * (order[i], or i when order is NULL) from a device-wide queue and advances it
 * to its t_end (or by cfg->slice iterations) exactly as qap_sa_run would, so
 * every chain's result is the same alone or in any batch and any slicing.
 *   host_descs  host copy of the n_chains descriptors (checked, sizes the launch)
 *   dev_descs   the same descriptors in device memory (read by the kernel)
 *   order       optional device array of n_chains chain indices (queue order)
 *   workspace   qap_batch_workspace_bytes() bytes of device memory
 * Each chain must be one a single workgroup can hold (byte value ranges; n up
 * to about 155 asymmetric or 195 symmetric in LDS, about 280 with a scratch,
 * see qap_single_workgroup); otherwise QAP_E_UNSUPPORTED.
 * With more chains than the device has CUs, chains that fit LDS entirely keep
 * Delta in their delta buffer instead (less LDS per workgroup, more chains at
 * once), and the chains whose LDS fits twice in a CU run in launches of their
 * own beside those of the larger chains; results do not change.
 * Chains in one batch must not share state, p, Bp or delta buffers.
 */
QAP_API int qap_sa_run_batch(int32_t n_chains, const qap_chain_desc* host_descs,
                             const qap_chain_desc* dev_descs, const int32_t* order,
                             const qap_batch_config* cfg, void* workspace, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* QAPSA_H */
