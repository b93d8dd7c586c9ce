// Shared declarations of the learned-preconditioner kernels (net.hip,
// netmfma.hip).
#pragma once
#include <cstdint>

#include "qedhmc_internal.h"

struct qedhmc_net;

namespace qh {

static constexpr int kNetLayers = 6;
static constexpr int kNetCh[kNetLayers + 1] = {6, 32, 32, 32, 32, 32, 2};
static constexpr int kWChunk = 1024;     // output sites per weight-gradient partial
static constexpr int kJudgeWindow = 10;  // flexible CG: iterations the residual judge looks back
static constexpr double kJudgeFactor = 0.5;

struct NetGeo {
    int L, Nt, Vs, N;
};

__device__ __forceinline__ void site_of(const NetGeo& g, int n, int& tau, int& y, int& x) {
    tau = n / g.Vs;
    const int s = n - tau * g.Vs;
    y = s / g.L;
    x = s - y * g.L;
}

// neighbour tau + dt; sg = -1 where it wraps (the antiperiodic sign of the
// first layer's residual channels)
__device__ __forceinline__ int wrap_tau(int t, int Nt, float& sg) {
    sg = 1.0f;
    if (t < 0) {
        t += Nt;
        sg = -1.0f;
    } else if (t >= Nt) {
        t -= Nt;
        sg = -1.0f;
    }
    return t;
}

__device__ __forceinline__ float silu_f(float a) { return a / (1.0f + expf(-a)); }
__device__ __forceinline__ float dsilu_f(float a) {
    const float s = 1.0f / (1.0f + expf(-a));
    return s * (1.0f + a * (1.0f - s));
}

// BF16 storage as the upper half of an FP32 word, rounded to nearest even
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ float to_f32(uint16_t v) { return bf16_to_f32(v); }
template <typename T>
__device__ __forceinline__ T from_f32(float v);
template <>
__device__ __forceinline__ float from_f32<float>(float v) {
    return v;
}
template <>
__device__ __forceinline__ uint16_t from_f32<uint16_t>(float v) {
    return f32_to_bf16(v);
}

// r: complex FP64, or FP32 when r32; rr: device |r|^2
qedhmc_status launch_first_bf16(const NetGeo& g, hipStream_t st, const cplx<float>* g32, const void* r, bool r32,
                                const double* rr, const float* W, const float* b, uint16_t* out);
qedhmc_status launch_last_bf16(const NetGeo& g, hipStream_t st, const uint16_t* in, const float* W, const float* b,
                               float* out);

// BF16 forward of the network (MFMA for the 32 -> 32 layers) on the
// residual r (complex FP64, or FP32 when r32) with |r|^2 at rr (device);
// leaves the two output channels in FP32 where the FP32 forward leaves them
qedhmc_status net_forward_bf16(qedhmc_net* n, const void* r, bool r32, const double* rr);
// inference in either arithmetic on a residual already on the device (the
// FP32 e^{i theta} cache of the handle built); output in n->act[kNetLayers]
qedhmc_status net_infer(qedhmc_net* n, const void* r, bool r32, const double* rr, qedhmc_net_arith a);
// number of BF16 weight elements the MFMA layers keep (fragment order)
size_t net_bf16_weight_elems();
// FP32 hidden layers of training on the matrix cores: the packed weights
// (forward and transposed, fragment order), the forward with the
// pre-activations and the data gradient of layer l (1 .. 4)
size_t net_f32_weight_elems();
qedhmc_status net_pack_f32(qedhmc_net* n);
qedhmc_status launch_fwd_mfma32(qedhmc_net* n, int l, const float* in, float* pre, float* act);
qedhmc_status launch_dgrad_mfma32(qedhmc_net* n, int l, const float* gout, const float* pre_prev, float* gin);
// QEDHMC_NET_F32=valu (read per call) keeps the FP32 hidden layers on the
// vector ALUs (tests compare both)
bool net_f32_on_vector_alus();
// mixed-precision flexible CG with the network as preconditioner (mfcg.hip):
// FP32 residual, direction and matvec, FP64 solution, reductions and
// reliable updates; the handle's FP64 and FP32 e^{i theta} caches built
qedhmc_status mfcg_solve_impl(qedhmc_net* n, const double* rhs, double* x, double tol, int maxit,
                              qedhmc_net_arith arith, qedhmc_precond fallback, int* iters, double* true_rel,
                              int* n_reliable, int* switched_at);

}  // namespace qh

// Network state bound to one lattice handle (its stream, sizes and caches).
struct qedhmc_net {
    qedhmc_ctx* h = nullptr;
    qh::NetGeo g{};
    size_t woff[qh::kNetLayers], boff[qh::kNetLayers], nparam = 0;
    float* params = nullptr;  // FP32 master, device layout
    float* grads = nullptr;
    float* adam_m = nullptr;
    float* adam_v = nullptr;
    int adam_t = 0;
    uint16_t* wbf = nullptr;   // BF16 weights of the hidden layers in MFMA fragment order
    bool wbf_ready = false;
    float* wf32 = nullptr;     // FP32 weights of the hidden layers in MFMA fragment order (forward, transposed)
    bool wf32_ready = false;
    // activations: act[l] = input of layer l (l >= 1), [N][32]; pre[l] pre-activation of layer l
    float* act[qh::kNetLayers + 1] = {};
    float* pre[qh::kNetLayers] = {};
    float* gbuf[2] = {nullptr, nullptr};
    float* wpart = nullptr;  // weight-gradient partials
    float* feat = nullptr;   // the first layer's feature map [N][8] (weight gradient on the matrix cores)
    float* wtmp = nullptr;   // group sums of the weight-gradient partials
    uint16_t* actb[2] = {nullptr, nullptr};  // BF16 ping-pong activations (inference)
    double* dscal = nullptr;  // [0] |r|^2, [1] |e|^2, [8..12) reductions
    double* dpart = nullptr;  // reduction partials
    double* hpin = nullptr;   // pinned host scalars
    bool train_ready = false;
    // flexible CG vectors (complex FP64)
    qh::cplx<double>* fr = nullptr;
    qh::cplx<double>* fp = nullptr;
    qh::cplx<double>* fs = nullptr;
    qh::cplx<double>* fz = nullptr;
};
