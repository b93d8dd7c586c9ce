// Allocation-free M^dag M: the fused operator of qedhmc_apply_MdagM with no
// handle.  The only device memory beyond the caller's input and output is the
// e^{i theta} phase cache the M^dag M kernels read, and here it lives in a
// file-scope device array (one copy per GPU, held until the process ends)
// instead of handle memory from hipMalloc.
#include <mutex>

#include "qedhmc_internal.h"

// The phase cache of the last call on this device.  Host code never passes
// this name to a kernel or a copy: on the host it is only a stand-in symbol;
// the device address comes from hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[QEDHMC_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t kScratchBytes = QEDHMC_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of scratch, per device

// Device address of this device's copy of scratch, looked up once per device
// with that device current.
qedhmc_status scratch_for(int device, void** out) {
    if (device < 0 || device >= kMaxDevices) {
        qh::set_error("device ordinal out of range for the allocation-free entry point");
        return QEDHMC_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return qh::hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) {
            qh::set_error("hipGetSymbolAddress(scratch) returned a null address");
            return QEDHMC_EHIP;
        }
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return QEDHMC_OK;
}

}  // namespace

extern "C" qedhmc_status qedhmc_apply_MdagM_noalloc(const qedhmc_params* params, const double* theta,
                                                    const void* in, void* out, qedhmc_precision prec,
                                                    void* stream) {
    if (!params || !theta || !in || !out) {
        qh::set_error("null pointer");
        return QEDHMC_EINVAL;
    }
    if (in == out) {
        qh::set_error("in and out alias");
        return QEDHMC_EINVAL;
    }
    QH_TRY(qh::check_params(params));
    QH_TRY(qh::check_prec(prec));
    const size_t n_phase = (size_t)2 * params->L * params->L * params->Nt;
    const size_t need =
        n_phase * (prec == QEDHMC_FP64 ? sizeof(qh::cplx<double>) : sizeof(qh::cplx<float>));
    if (need > kScratchBytes) {
        qh::set_error("qedhmc_apply_MdagM_noalloc: the phase cache needs " + std::to_string(need) +
                      " bytes, more than the " + std::to_string(kScratchBytes) +
                      " bytes of its static scratch (2 L^2 N_tau complex values of the working precision)");
        return QEDHMC_EINVAL;
    }
    // A context on the stack: geometry, limits and the stream only.  Its
    // phase-cache pointer is this device's scratch; nothing is allocated.
    qedhmc_ctx h{};
    QH_TRY(qh::ctx_geometry(&h, *params, stream));
    void* ptr = nullptr;
    QH_TRY(scratch_for(h.device, &ptr));
    if (prec == QEDHMC_FP64)
        h.gauge64 = static_cast<qh::cplx<double>*>(ptr);
    else
        h.gauge32 = static_cast<qh::cplx<float>*>(ptr);
    QH_TRY(qh::ensure_gauge(&h, theta, prec));
    return qh::launch_mdagm(&h, prec, in, out, nullptr);
}
