// qapsa_api.hip -- the extern "C" entry points of libqapsa: argument checks,
// kernel selection and launches.  No device memory is allocated here.
#include <hip/hip_runtime.h>
#include <math.h>

#include <mutex>

#include "qapsa_device.hpp"
#include "qapsa_internal.hpp"

using namespace qapsa;

namespace {

bool fits16(int32_t lo, int32_t hi)
{
    return lo >= -32768 && hi <= 32767 && (int64_t)hi - lo <= 32767;
}

int check_schedule(const qap_schedule* s)
{
    if (!s) return QAP_E_INVAL;
    if (s->iters == 0 || s->t_end > s->iters) return QAP_E_INVAL;
    if (!(s->T0 > 0.0)) return QAP_E_INVAL;                // rejects NaN and <= 0; +inf allowed
    if (!(s->alpha > 0.0) || s->alpha > 1.0) return QAP_E_INVAL;
    if ((s->flags & ~(QAP_FLAG_DELTA_ONLY | QAP_FLAG_SCRATCH_ONLY | QAP_FLAG_MULTI_WG | QAP_FLAG_RANDOM_ORDER |
                      QAP_FLAG_SINGLE_WG)) != 0)
        return QAP_E_INVAL;
    if ((s->flags & QAP_FLAG_DELTA_ONLY) && (s->flags & QAP_FLAG_SCRATCH_ONLY)) return QAP_E_INVAL;
    if ((s->flags & QAP_FLAG_MULTI_WG) && (s->flags & QAP_FLAG_SINGLE_WG)) return QAP_E_INVAL;
    if (s->switch_permille > 1000) return QAP_E_INVAL;
    if (s->scan_window != 0 && (s->scan_window < 16 || s->scan_window > (1u << 21))) return QAP_E_INVAL;
    return QAP_OK;
}

}  // namespace

namespace qapsa {

int side_stream(int which, hipStream_t* side, hipEvent_t* fork, hipEvent_t* join)
{
    static hipStream_t streams[64][3];
    static hipEvent_t forks[64][3], joins[64][3];
    static bool made[64][3];
    int dev = 0;
    if (which < 0 || which > 2) return QAP_E_INVAL;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return QAP_E_DEVICE;
    if (!made[dev][which]) {
        if (hipStreamCreateWithFlags(&streams[dev][which], hipStreamNonBlocking) != hipSuccess) return QAP_E_DEVICE;
        if (hipEventCreateWithFlags(&forks[dev][which], hipEventDisableTiming) != hipSuccess) return QAP_E_DEVICE;
        if (hipEventCreateWithFlags(&joins[dev][which], hipEventDisableTiming) != hipSuccess) return QAP_E_DEVICE;
        made[dev][which] = true;
    }
    *side = streams[dev][which];
    *fork = forks[dev][which];
    *join = joins[dev][which];
    return QAP_OK;
}

}  // namespace qapsa

extern "C" {

QAP_API const char* qap_strerror(int status)
{
    switch (status) {
    case QAP_OK: return "ok";
    case QAP_E_INVAL: return "invalid argument";
    case QAP_E_NOT_PERM: return "p is not a permutation of 0..n-1";
    case QAP_E_RANGE: return "instance values exceed the int32 Delta bound";
    case QAP_E_NOMEM: return "size exceeds what the kernel can hold";
    case QAP_E_DEVICE: return "HIP runtime error";
    case QAP_E_UNSUPPORTED: return "no kernel in this build handles the request";
    case QAP_E_STATE: return "chain state is not ready";
    case QAP_E_TIMEOUT: return "a grid barrier did not complete";
    case QAP_E_TIE_OVERFLOW: return "too many near ties in one scan window to record exactly";
    default: return "unknown status";
    }
}

QAP_API int qap_cost(int32_t n, const int32_t* A, const int32_t* B, const int32_t* p, int64_t* cost,
                     hipStream_t stream)
{
    if (n < 1 || n > 46340 || !A || !B || !p || !cost) return QAP_E_INVAL;
    return launch_cost(n, A, B, p, cost, stream);
}

QAP_API int qap_delta_init(int32_t n, const int32_t* A, const int32_t* B, const int32_t* p, int32_t* Bp,
                           int32_t* delta, qap_instance_info* info, qap_chain_state* state,
                           hipStream_t stream)
{
    if (n < 2 || n > 46340 || !A || !B || !p || !Bp || !delta || !info) return QAP_E_INVAL;
    return launch_delta_init(n, A, B, p, Bp, delta, info, state, stream);
}

QAP_API uint64_t qap_temp_table_len(uint64_t iters) { return temp_table_len(iters); }

QAP_API uint64_t qap_workspace_bytes(int32_t n)
{
    if (n < 2) return 0;
    // the multi-workgroup area at the widest value type whose LDS layout fits
    // at some grid size (at most 256 workgroups, one per CU of an MI355X)
    size_t bytes = dist_ws_bytes(n, false, 1);
    for (int esize = 1; esize <= 4; esize *= 2)
        for (int sym = 0; sym < 2; ++sym)
            if (lds_dist_bytes(n, 256, sym != 0, esize) <= kLdsLimit - kDistStaticReserve) {
                const size_t b = dist_ws_bytes(n, sym != 0, esize);
                if (b > bytes) bytes = b;
            }
    for (int sym = 0; sym < 2; ++sym) {
        const int place = wg_place(n, sym != 0);
        if (place >= 0) {
            const size_t b = wg_scratch_bytes(n, sym != 0, place);
            if (b > bytes) bytes = b;
        }
    }
    return bytes;
}

QAP_API uint64_t qap_chain_scratch_bytes(int32_t n, int32_t symmetric)
{
    if (n < 2) return 0;
    const int place = wg_place(n, symmetric != 0);
    return place < 0 ? 0 : (uint64_t)wg_scratch_bytes(n, symmetric != 0, place);
}

QAP_API int qap_schedule_tables(uint64_t iters, double alpha, double* temps, hipStream_t stream)
{
    if (iters == 0 || !temps || !(alpha > 0.0) || alpha > 1.0) return QAP_E_INVAL;
    return launch_schedule_tables(iters, alpha, temps, stream);
}

QAP_API int qap_schedule_init(int32_t n, const qap_instance_info* info, uint64_t iters, double final_ratio,
                              qap_schedule* sched)
{
    if (n < 2 || !info || !sched || iters == 0 || !(final_ratio > 0.0) || final_ratio > 1.0) return QAP_E_INVAL;
    if (info->status != QAP_OK) return info->status;
    if (info->sum_abs_delta <= 0) return QAP_E_INVAL;
    const int64_t m = (int64_t)n * (n - 1) / 2;
    sched->iters = iters;
    sched->t_end = iters;
    sched->T0 = (double)info->sum_abs_delta / (double)m;
    sched->alpha = iters == 1 ? 1.0 : pow(final_ratio, 1.0 / (double)(iters - 1));
    return QAP_OK;
}

}  // extern "C"

namespace {

// No-allocation variant of qap_sa_run: this file-scope device array replaces
// the caller's workspace.  Each device holds its own copy until the process
// ends; host code never passes the array's name to a kernel, only the address
// hipGetSymbolAddress returns for the current device (looked up once per
// device, below).
constexpr size_t kStaticScratchBytes = 1u << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

// Kernel selection and launch of one chain's run; the workspace comes from
// bufs (qap_sa_run) or from the library's static scratch (qap_sa_run_static).
// A workspace smaller than the chosen kernel needs is reported as ws_short.
int sa_run_impl(int32_t n, const int32_t* A, const int32_t* B, int32_t* Bp, int32_t* p, int32_t* delta,
                qap_chain_state* state, const qap_schedule* sched, const qap_instance_info* info,
                const qap_run_buffers* bufs, hipStream_t stream, int ws_short)
{
    const int rc = check_schedule(sched);
    if (rc != QAP_OK) return rc;
    if (info->status != QAP_OK) return info->status;
    const bool sym = info->symmetric != 0;
    const size_t budget = kLdsLimit - kLdsStaticReserve;

    ChainArgs a{};
    a.n = n;
    // largest Delta-mode scan step of the one-workgroup kernel, in steps of 256 proposals
    a.max_step = sched->scan_window ? (int)((sched->scan_window + 255) / 256) : 16;
    if (a.max_step > 64) a.max_step = 64;
    a.flags = sched->flags;
    a.switch_permille = sched->switch_permille ? sched->switch_permille : kDefaultSwitchPermille;
    a.a_min = info->a_min;
    a.b_min = info->b_min;
    a.A = A; a.Bp = Bp; a.p = p; a.delta = delta; a.state = state;
    a.temps = bufs->temps;
    a.ties = bufs->ties; a.tie_cap = bufs->tie_cap;
    a.acc_log = bufs->accept_log; a.acc_cap = bufs->accept_log ? bufs->accept_cap : 0;
    a.prof = bufs->phase_cycles;
    a.iters = sched->iters;
    a.t_end = sched->t_end;
    a.T0 = sched->T0;
    a.seed = sched->seed;
    a.chain_id = sched->chain_id;

    // byte-valued kernel: value ranges of A and B fit 0..255 after shifting
    const bool bytes_ok = (int64_t)info->a_max - info->a_min <= 255 && (int64_t)info->b_max - info->b_min <= 255;
    const bool multi = (sched->flags & QAP_FLAG_MULTI_WG) != 0;
    const bool single = (sched->flags & QAP_FLAG_SINGLE_WG) != 0;
    a.flags &= ~(QAP_FLAG_MULTI_WG | QAP_FLAG_SINGLE_WG);
    int place = bytes_ok && !multi ? wg_place(n, sym) : -1;
    // large chains (all their matrices outside LDS on one workgroup): many
    // workgroups share the Delta update, unless one is asked for
    if (place == 3 && !single) place = -1;
    // one workgroup: Delta, then A, then B' in device memory where LDS runs out
    if (place >= 0 && place <= 1) return launch_chain_wg(a, sym, place, stream);
    if (place >= 2) {
        if (!bufs->workspace) return QAP_E_INVAL;
        if (bufs->workspace_bytes < wg_scratch_bytes(n, sym, place)) return ws_short;
        a.gscratch = bufs->workspace;
        return launch_chain_wg(a, sym, place, stream);
    }
    // value ranges wider than a byte, small enough for one CU: the 16-bit
    // one-workgroup kernel (Delta mode only)
    if (!bytes_ok && !multi && fits16(info->a_min, info->a_max) && fits16(info->b_min, info->b_max)) {
        bool a_lds = false, fits = true;
        if (lds_chain_bytes(n, sym, true) <= budget) a_lds = true;
        else if (lds_chain_bytes(n, sym, false) > budget) fits = false;
        if (fits) {
            a.pitch = n | 1;
            const int threads = n >= 64 ? 1024 : 256;
            return launch_chain_lds(a, sym, a_lds, threads, stream);
        }
    }
    // many workgroups, one cooperative launch: A and B' as bytes, 16-bit or
    // 32-bit words by their value ranges
    if (!single) {
        const int esize = dist_esize((int64_t)info->a_max - info->a_min, (int64_t)info->b_max - info->b_min);
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return QAP_E_DEVICE;
        int G = (n + 7) / 8;                 // about eight rows per workgroup
        if (G > cus) G = cus;
        if (G < 2) G = 2;
        const size_t dbudget = kLdsLimit - kDistStaticReserve;
        while (G < cus && lds_dist_bytes(n, G, sym, esize) > dbudget) ++G;
        if (lds_dist_bytes(n, G, sym, esize) <= dbudget) {
            if (!bufs->workspace) return QAP_E_INVAL;
            if (bufs->workspace_bytes < dist_ws_bytes(n, sym, esize)) return ws_short;
            DistArgs d{};
            d.n = n;
            d.a_min = info->a_min;
            d.b_min = info->b_min;
            d.random_order = (sched->flags & QAP_FLAG_RANDOM_ORDER) ? 1u : 0u;
            // a random-order window is drawn whole by every workgroup: start it small
            // the first window after an accept: 256 proposals (one per workgroup or so at N = 2000)
            // measured fastest among 256-16384 on the N = 2000 schedule (11.8 against 12.2 us per
            // accepted swap at 4096); a random-order window is drawn whole by every workgroup
            d.kmin = sched->scan_window ? sched->scan_window : (d.random_order ? 512 : 256);
            d.kmax = (1u << 22) - 2;   // window offsets fit the 22-bit field of an exchange slot
            d.spin_limit = 1ull << 22;
            d.A = A; d.B = B; d.Bp = Bp; d.p = p; d.delta = delta; d.state = state;
            d.temps = bufs->temps;
            d.ties = bufs->ties; d.tie_cap = bufs->tie_cap;
            d.acc_log = a.acc_log; d.acc_cap = a.acc_cap;
            d.prof = bufs->phase_cycles;
            d.iters = sched->iters; d.t_end = sched->t_end; d.T0 = sched->T0;
            d.seed = sched->seed; d.chain_id = sched->chain_id;
            d.ws = (DistWs*)bufs->workspace;
            d.slots = dist_slots(bufs->workspace);
            d.X = dist_X(bufs->workspace);
            d.Pp = dist_P(bufs->workspace, n);
            d.flags = sched->flags & (QAP_FLAG_DELTA_ONLY | QAP_FLAG_SCRATCH_ONLY);
            d.switch_permille = sched->switch_permille ? sched->switch_permille : kDefaultDistSwitchPermille;
            if (!sym) {
                uint8_t* copies = dist_bytes(bufs->workspace, n);
                const size_t plane = (size_t)n * dist_row_bytes(n, esize);
                d.Ab = copies;
                d.Atb = copies + plane;
                d.Btb = copies + 2 * plane;
            }
            return launch_chain_dist(d, sym, esize, G, 512, stream);
        }
    }
    // byte-valued chains beyond the multi-workgroup kernel's LDS budget: one
    // workgroup with Delta, A and B' in device memory
    if (bytes_ok) {
        const int wp = wg_place(n, sym);
        if (wp >= 2) {
            if (!bufs->workspace) return QAP_E_INVAL;
            if (bufs->workspace_bytes < wg_scratch_bytes(n, sym, wp)) return ws_short;
            a.gscratch = bufs->workspace;
            return launch_chain_wg(a, sym, wp, stream);
        }
    }
    return QAP_E_UNSUPPORTED;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

int static_scratch(void** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return QAP_E_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return QAP_E_DEVICE;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return QAP_OK;
}

}  // namespace

extern "C" {

QAP_API int qap_sa_run(int32_t n, const int32_t* A, const int32_t* B, int32_t* Bp, int32_t* p, int32_t* delta,
                       qap_chain_state* state, const qap_schedule* sched,
                       const qap_instance_info* info, const qap_run_buffers* bufs, hipStream_t stream)
{
    if (n < 2 || n > 46340 || !A || !B || !Bp || !p || !delta || !state || !info || !bufs || !bufs->temps)
        return QAP_E_INVAL;
    return sa_run_impl(n, A, B, Bp, p, delta, state, sched, info, bufs, stream, QAP_E_INVAL);
}

QAP_API uint64_t qap_static_scratch_bytes(void) { return kStaticScratchBytes; }

QAP_API int qap_sa_run_static(int32_t n, const int32_t* A, const int32_t* B, int32_t* Bp, int32_t* p,
                              int32_t* delta, qap_chain_state* state, const qap_schedule* sched,
                              const qap_instance_info* info, const qap_run_buffers* bufs, hipStream_t stream)
{
    if (n < 2 || n > 46340 || !A || !B || !Bp || !p || !delta || !state || !info || !bufs || !bufs->temps)
        return QAP_E_INVAL;
    if (bufs->workspace || bufs->workspace_bytes) return QAP_E_INVAL;
    void* ws = nullptr;
    const int rc = static_scratch(&ws);
    if (rc != QAP_OK) return rc;
    qap_run_buffers b = *bufs;
    b.workspace = ws;
    b.workspace_bytes = kStaticScratchBytes;
    return sa_run_impl(n, A, B, Bp, p, delta, state, sched, info, &b, stream, QAP_E_NOMEM);
}

QAP_API uint64_t qap_batch_workspace_bytes(void) { return sizeof(BatchWs); }

QAP_API int qap_single_workgroup(int32_t n, int32_t symmetric, int64_t a_range, int64_t b_range)
{
    if (n < 2 || a_range < 0 || b_range < 0 || a_range > 255 || b_range > 255) return 0;
    const int place = wg_place(n, symmetric != 0);
    if (place == 0 || place == 1) return 1;
    if (place >= 2) return 2;
    return 0;
}

QAP_API int qap_tabu_run(int32_t n, const int32_t* A, int32_t* Bp, int32_t* p, int32_t* delta,
                         qap_chain_state* state, const qap_tabu_schedule* sched,
                         const qap_instance_info* info, int32_t* tabu, const qap_run_buffers* bufs,
                         hipStream_t stream)
{
    if (n < 2 || n > 46340 || !A || !Bp || !p || !delta || !state || !sched || !info || !tabu || !bufs)
        return QAP_E_INVAL;
    if (sched->iters == 0 || sched->t_end > sched->iters || sched->tenure < 0 || sched->reserved != 0 ||
        sched->iters + (uint64_t)sched->tenure >= (1ull << 31))
        return QAP_E_INVAL;
    if (info->status != QAP_OK) return info->status;
    const bool sym = info->symmetric != 0;
    const bool bytes_ok = (int64_t)info->a_max - info->a_min <= 255 && (int64_t)info->b_max - info->b_min <= 255;
    const int place = bytes_ok ? wg_place(n, sym) : -1;
    if (place < 0) return QAP_E_UNSUPPORTED;
    ChainArgs a{};
    a.n = n;
    a.max_step = 16;
    a.flags = QAP_FLAG_DELTA_ONLY;
    a.switch_permille = 20;
    a.a_min = info->a_min;
    a.b_min = info->b_min;
    a.A = A; a.Bp = Bp; a.p = p; a.delta = delta; a.state = state;
    a.temps = bufs->temps;
    a.acc_log = bufs->accept_log; a.acc_cap = bufs->accept_log ? bufs->accept_cap : 0;
    a.prof = bufs->phase_cycles;
    a.iters = sched->iters;
    a.t_end = sched->t_end;
    a.T0 = 1.0;
    a.tabu = tabu;
    a.tenure = sched->tenure;
    if (place >= 2) {
        if (!bufs->workspace || bufs->workspace_bytes < wg_scratch_bytes(n, sym, place)) return QAP_E_INVAL;
        a.gscratch = bufs->workspace;
    }
    return launch_chain_wg(a, sym, place, stream, true);
}

QAP_API int qap_sa_run_batch(int32_t n_chains, const qap_chain_desc* host_descs, const qap_chain_desc* dev_descs,
                             const int32_t* order, const qap_batch_config* cfg, void* workspace,
                             hipStream_t stream)
{
    if (n_chains < 0 || (n_chains > 0 && (!host_descs || !dev_descs)) || !cfg || !workspace) return QAP_E_INVAL;
    if (n_chains == 0) return QAP_OK;
    const int threads = cfg->threads ? cfg->threads : 256;
    if (threads != 256) return QAP_E_INVAL;
    // With more chains than CUs, chains share CUs: those that would keep all
    // their state in LDS keep Delta in their device buffer instead (placement
    // 1), which takes less LDS per workgroup, so more of them run at once
    // (512-chain mix: 3.86 s instead of 4.06 s).  Results are the same.
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return QAP_E_DEVICE;
    const int min_place = n_chains > cus ? 1 : 0;
    // With more chains than CUs, the chains whose LDS fits twice in a CU run
    // in launches of their own (class 0), sized by their own largest chain,
    // so that two of them share a CU instead of each taking a CU's LDS as
    // the largest chains of the placement do (class 1).
    uint32_t lds_split = n_chains > cus ? (uint32_t)(kLdsLimit / 2 - kLdsStaticReserve) : 0u;
    size_t lds[kBatchKinds] = {}, lds1[kBatchKinds] = {};   // with the split, and with one class
    int kinds[kBatchKinds] = {}, kinds1[kBatchKinds] = {};
    for (int i = 0; i < n_chains; ++i) {
        const qap_chain_desc& d = host_descs[i];
        if (d.n < 2 || d.n > 46340 || !d.A || !d.Bp || !d.p || !d.delta || !d.state || !d.temps) return QAP_E_INVAL;
        if (d.iters == 0 || d.t_end > d.iters || !(d.T0 > 0.0)) return QAP_E_INVAL;
        if ((d.flags & ~(QAP_FLAG_DELTA_ONLY | QAP_FLAG_SCRATCH_ONLY | QAP_FLAG_RANDOM_ORDER)) != 0 ||
            d.switch_permille > 1000)
            return QAP_E_INVAL;
        if ((int64_t)d.a_max - d.a_min > 255 || (int64_t)d.b_max - d.b_min > 255) return QAP_E_UNSUPPORTED;
        int place = wg_place(d.n, d.symmetric != 0);
        if (place < 0) return QAP_E_UNSUPPORTED;
        if (place < min_place) place = min_place;
        if (place >= 2 && !d.scratch) return QAP_E_INVAL;
        const size_t b = lds_wg_bytes(d.n, d.symmetric != 0, place);
        const int kind = 2 * place + (lds_split && b > lds_split ? 1 : 0);
        if (b > lds[kind]) lds[kind] = b;
        kinds[kind] += 1;
        if (b > lds1[2 * place]) lds1[2 * place] = b;
        kinds1[2 * place] += 1;
    }
    // at most four kernels side by side (the caller's stream and three side
    // streams): else one class per placement
    int nonempty = 0;
    for (int k = 0; k < kBatchKinds; ++k) nonempty += kinds[k] > 0;
    if (nonempty > 4) {
        lds_split = 0;
        for (int k = 0; k < kBatchKinds; ++k) { lds[k] = lds1[k]; kinds[k] = kinds1[k]; }
    }
    BatchArgs b{};
    b.n_chains = n_chains;
    b.min_place = min_place;
    b.descs = dev_descs;
    b.order = order;
    b.ws = (BatchWs*)workspace;
    b.slice = cfg->slice;
    b.prof = cfg->phase_cycles;
    b.lds_split = lds_split;
    return launch_chain_batch(b, cfg->groups, kinds, threads, lds, stream);
}

}  // extern "C"
