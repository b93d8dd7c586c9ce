// BF16 forward of the learned preconditioner: the four 32 -> 32 layers as
// MFMA products on gfx950 (v_mfma_f32_16x16x32_bf16: BF16 operands, FP32
// accumulation), the small first and last layers in FP32 on the vector ALUs.
//
// A 3x3x3 convolution with 32 input and 32 output channels is, per tap, a
// product [sites x 32] x [32 x 32]; one MFMA takes a 16-site x 32-channel
// block of the tap-shifted input (A) and a 32 x 16 block of that tap's
// weights (B), so a tap costs two MFMAs per 16 sites and a layer 54.  The
// layer's weights (27 taps x 2 column halves, 55 KB of BF16 in the MFMA B
// fragment order) are staged once per workgroup of 16 wavefronts in LDS; each
// wavefront keeps one tap's two B fragments in registers while it runs two
// 16-site tiles (the fastest of the tilings timed at L=66),
// and reads the A fragments straight from the channels-last activations
// (one 16-byte load per lane: 8 channels of one site).  Neighbour reuse
// across taps is left to L1/L2.
#include "net_internal.h"

namespace qh {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

static constexpr int kHidden = 4;             // 32 -> 32 layers (1..4, zero based)
static constexpr int kFrag = 27 * 2 * 64;     // B fragments (16 bytes each) per layer
static constexpr int kTiles = 2;              // 16-site tiles per wavefront
static constexpr int kBlock = 1024;           // threads per workgroup (16 wavefronts share the staged weights)
static constexpr int kSitesPerBlock = (kBlock / 64) * 16 * kTiles;

size_t net_bf16_weight_elems() { return (size_t)kHidden * kFrag * 8; }

// B fragment order: frag[(k * 2 + half) * 64 + lane][j] = W[k][ci][co] with
// co = 16 half + lane % 16 and ci = 8 (lane / 16) + j (device layout
// W[27][32][32] of one hidden layer)
__global__ void k_pack_bf16(const float* __restrict__ params, size_t w0, size_t stride_layer,
                            uint16_t* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kHidden * kFrag * 8) return;
    const int j = i & 7;
    const int f = (i >> 3) % kFrag;
    const int hl = (i >> 3) / kFrag;
    const int lane = f & 63, kh = f >> 6;
    const int k = kh >> 1, half = kh & 1;
    const int co = 16 * half + (lane & 15), ci = 8 * (lane >> 4) + j;
    const float* W = params + w0 + (size_t)hl * stride_layer;
    out[i] = f32_to_bf16(W[((size_t)k * 32 + ci) * 32 + co]);
}

template <bool SILU>
__global__ __launch_bounds__(kBlock) void k_conv_mfma(NetGeo g, const uint16_t* __restrict__ in,
                                                   const uint16_t* __restrict__ wfrag,
                                                   const float* __restrict__ bias, uint16_t* __restrict__ out) {
    __shared__ bf16x8 sW[kFrag];
    const bf16x8* wf = reinterpret_cast<const bf16x8*>(wfrag);
    for (int i = threadIdx.x; i < kFrag; i += blockDim.x) sW[i] = wf[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int site0 = blockIdx.x * kSitesPerBlock + wave * 16 * kTiles;
    if (site0 >= g.N) return;
    const int row = lane & 15, kq = lane >> 4;
    // this lane's A rows: site site0 + 16 t + row (clamped into range; the
    // stores below skip the clamped ones)
    int st[kTiles], sy[kTiles], sx[kTiles];
#pragma unroll
    for (int t = 0; t < kTiles; t++) {
        const int m = min(site0 + 16 * t + row, g.N - 1);
        site_of(g, m, st[t], sy[t], sx[t]);
    }
    f32x4 acc[kTiles][2];
#pragma unroll
    for (int t = 0; t < kTiles; t++)
#pragma unroll
        for (int h = 0; h < 2; h++) acc[t][h] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 1
    for (int k = 0; k < 27; k++) {
        const int dt = k / 9 - 1, dy = (k / 3) % 3 - 1, dx = k % 3 - 1;
        const bf16x8 b0 = sW[(2 * k) * 64 + lane];
        const bf16x8 b1 = sW[(2 * k + 1) * 64 + lane];
        bf16x8 a[kTiles];
#pragma unroll
        for (int t = 0; t < kTiles; t++) {
            const int m = wrap(st[t] + dt, g.Nt) * g.Vs + wrap(sy[t] + dy, g.L) * g.L + wrap(sx[t] + dx, g.L);
            a[t] = *reinterpret_cast<const bf16x8*>(in + (size_t)m * 32 + 8 * kq);
        }
#pragma unroll
        for (int t = 0; t < kTiles; t++) {
            acc[t][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t], b0, acc[t][0], 0, 0, 0);
            acc[t][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t], b1, acc[t][1], 0, 0, 0);
        }
    }
    // D fragment: lane holds rows 4 (lane / 16) + i, column lane % 16
#pragma unroll
    for (int t = 0; t < kTiles; t++)
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int co = 16 * h + row;
            const float bco = bias[co];
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int site = site0 + 16 * t + 4 * kq + i;
                if (site < g.N) {
                    const float v = acc[t][h][i] + bco;
                    out[(size_t)site * 32 + co] = f32_to_bf16(SILU ? silu_f(v) : v);
                }
            }
        }
}

qedhmc_status net_forward_bf16(qedhmc_net* n, const void* r, bool r32, const double* rr) {
    const NetGeo& g = n->g;
    hipStream_t st = n->h->stream;
    if (!n->wbf_ready) {
        const size_t stride = n->woff[2] - n->woff[1];
        const int total = kHidden * kFrag * 8;
        hipLaunchKernelGGL(k_pack_bf16, dim3((total + 255) / 256), dim3(256), 0, st, (const float*)n->params,
                           n->woff[1], stride, n->wbf);
        QH_HIP(hipGetLastError());
        n->wbf_ready = true;
    }
    QH_TRY(launch_first_bf16(g, st, n->h->gauge32, r, r32, rr, n->params + n->woff[0], n->params + n->boff[0],
                             n->actb[0]));
    int cur = 0;
    const int blocks = (g.N + kSitesPerBlock - 1) / kSitesPerBlock;
    for (int hl = 0; hl < kHidden; hl++) {
        const int l = hl + 1;
        hipEvent_t e0, e1;
        if (prof_sample(n->h, QEDHMC_K_NET_MFMA, e0, e1))
            hipExtLaunchKernelGGL((k_conv_mfma<true>), dim3(blocks), dim3(kBlock), 0, st, e0, e1, 0, g,
                                  (const uint16_t*)n->actb[cur], (const uint16_t*)(n->wbf + (size_t)hl * kFrag * 8),
                                  (const float*)(n->params + n->boff[l]), n->actb[cur ^ 1]);
        else
            hipLaunchKernelGGL((k_conv_mfma<true>), dim3(blocks), dim3(kBlock), 0, st, g, (const uint16_t*)n->actb[cur],
                               (const uint16_t*)(n->wbf + (size_t)hl * kFrag * 8),
                               (const float*)(n->params + n->boff[l]), n->actb[cur ^ 1]);
        QH_HIP(hipGetLastError());
        cur ^= 1;
    }
    return launch_last_bf16(g, st, n->actb[cur], n->params + n->woff[kNetLayers - 1],
                            n->params + n->boff[kNetLayers - 1], n->act[kNetLayers]);
}

}  // namespace qh
