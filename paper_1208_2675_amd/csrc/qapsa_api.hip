// qapsa_api.hip -- the extern "C" entry points of libqapsa: argument checks,
// kernel selection and launches.  No device memory is allocated here.
#include <hip/hip_runtime.h>
#include <math.h>

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
    if ((s->flags & ~(QAP_FLAG_DELTA_ONLY | QAP_FLAG_SCRATCH_ONLY)) != 0) return QAP_E_INVAL;
    if ((s->flags & QAP_FLAG_DELTA_ONLY) && (s->flags & QAP_FLAG_SCRATCH_ONLY)) return QAP_E_INVAL;
    if (s->switch_permille > 1000 || s->reserved != 0) return QAP_E_INVAL;
    return QAP_OK;
}

}  // namespace

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

QAP_API int qap_schedule_tables(uint64_t iters, double alpha, double* temps, hipStream_t stream)
{
    if (iters == 0 || !temps || !(alpha > 0.0) || alpha > 1.0) return QAP_E_INVAL;
    return launch_schedule_tables(iters, alpha, temps, stream);
}

QAP_API int qap_sa_run(int32_t n, const int32_t* A, int32_t* Bp, int32_t* p, int32_t* delta,
                       qap_chain_state* state, const qap_schedule* sched,
                       const qap_instance_info* info, const qap_run_buffers* bufs, hipStream_t stream)
{
    if (n < 2 || n > 46340 || !A || !Bp || !p || !delta || !state || !info || !bufs || !bufs->temps)
        return QAP_E_INVAL;
    const int rc = check_schedule(sched);
    if (rc != QAP_OK) return rc;
    if (info->status != QAP_OK) return info->status;
    const bool sym = info->symmetric != 0;
    const size_t budget = kLdsLimit - kLdsStaticReserve;

    ChainArgs a{};
    a.n = n;
    a.max_step = 16;
    a.flags = sched->flags;
    a.switch_permille = sched->switch_permille ? sched->switch_permille : 20;
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
    if (bytes_ok && lds_wg_bytes(n, sym) <= budget) {
        const int threads = n >= 48 ? 1024 : 256;
        return launch_chain_wg(a, sym, threads, stream);
    }
    // 16-bit kernel (Delta mode only)
    if (!fits16(info->a_min, info->a_max) || !fits16(info->b_min, info->b_max)) return QAP_E_UNSUPPORTED;
    bool a_lds;
    if (lds_chain_bytes(n, sym, true) <= budget) a_lds = true;
    else if (lds_chain_bytes(n, sym, false) <= budget) a_lds = false;
    else return QAP_E_UNSUPPORTED;
    a.pitch = n | 1;
    const int threads = n >= 64 ? 1024 : 256;
    return launch_chain_lds(a, sym, a_lds, threads, stream);
}

}  // extern "C"
