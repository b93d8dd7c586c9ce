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
// across taps is left to L1/L2.  Each lane wraps its site's three
// coordinates once (three offsets per direction); a tap's site is then one
// three-way sum, and the taps are unrolled so the loads of later taps can be
// issued ahead of the products of earlier ones.
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
    // stores below skip the clamped ones), as the wrapped slice, row and
    // column offsets of its three neighbours per direction (d = 0, 1, 2 for
    // -1, 0, +1)
    int ot[kTiles][3], oy[kTiles][3], ox[kTiles][3];
#pragma unroll
    for (int t = 0; t < kTiles; t++) {
        const int m = min(site0 + 16 * t + row, g.N - 1);
        int st, sy, sx;
        site_of(g, m, st, sy, sx);
#pragma unroll
        for (int d = 0; d < 3; d++) {
            ot[t][d] = wrap(st + d - 1, g.Nt) * g.Vs;
            oy[t][d] = wrap(sy + d - 1, g.L) * g.L;
            ox[t][d] = wrap(sx + d - 1, g.L);
        }
    }
    const uint16_t* inq = in + 8 * kq;
    f32x4 acc[kTiles][2];
#pragma unroll
    for (int t = 0; t < kTiles; t++)
#pragma unroll
        for (int h = 0; h < 2; h++) acc[t][h] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < 27; k++) {
        const int dt = k / 9, dy = (k / 3) % 3, dx = k % 3;
        const bf16x8 b0 = sW[(2 * k) * 64 + lane];
        const bf16x8 b1 = sW[(2 * k + 1) * 64 + lane];
        bf16x8 a[kTiles];
#pragma unroll
        for (int t = 0; t < kTiles; t++) {
            const unsigned m = (unsigned)(ot[t][dt] + oy[t][dy] + ox[t][dx]);
            a[t] = *reinterpret_cast<const bf16x8*>(inq + (size_t)m * 32);
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

// ---------------------------------------------------------------------------
// FP32 32 -> 32 layers of training (forward with the pre-activations, and the
// data gradient) on the matrix cores: v_mfma_f32_16x16x4f32 (FP32 operands
// and accumulation, the same arithmetic as the vector kernels in another
// summation order).  Per tap the product [16 sites x 32] x [32 x 32] is
// 2 x 8 MFMAs: K = 32 channels in steps of 4, the lane of k-group q holding
// channel 8 q + kk of step kk, so each lane loads 8 consecutive channels of
// its site (two 16-byte loads) and the weights are packed in the matching
// fragment order: frag[((k 2 + ob) 8 + kk) 64 + lane] = Wt_k[8 (lane / 16) +
// kk][16 ob + lane % 16], Wt_k = W_k ([in][out], forward) or W_k^T (data
// gradient, whose tap offsets are mirrored).  The layer's 108 KB of packed
// weights are staged in LDS per workgroup of 16 wavefronts.
// ---------------------------------------------------------------------------
static constexpr int kF32Frag = 27 * 2 * 8 * 64;  // floats per layer
static constexpr int kTiles32 = 2;
static constexpr int kSitesPerBlock32 = (kBlock / 64) * 16 * kTiles32;

size_t net_f32_weight_elems() { return (size_t)2 * kHidden * kF32Frag; }

__global__ void k_pack_f32(const float* __restrict__ params, size_t w0, size_t stride_layer,
                           float* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2 * kHidden * kF32Frag) return;
    const int lane = i & 63, f = (i >> 6) % (kF32Frag / 64), hl = ((i >> 6) / (kF32Frag / 64)) % kHidden;
    const int transpose = (i >> 6) / (kF32Frag / 64) / kHidden;
    const int kk = f % 8, ob = (f / 8) % 2, k = f / 16;
    const int row = 8 * (lane >> 4) + kk, col = 16 * ob + (lane & 15);
    const float* W = params + w0 + (size_t)hl * stride_layer;
    out[i] = transpose ? W[((size_t)k * 32 + col) * 32 + row] : W[((size_t)k * 32 + row) * 32 + col];
}

// DGRAD = false: pre = conv(in) + b, out = SiLU(pre) (pre nullable);
// DGRAD = true: out = conv^T(in = the output gradient) * SiLU'(pre_prev).
template <bool DGRAD>
__global__ __launch_bounds__(kBlock) void k_conv_mfma32(NetGeo g, const float* __restrict__ in,
                                                     const float* __restrict__ wfrag,
                                                     const float* __restrict__ bias,
                                                     const float* __restrict__ pre_prev, float* __restrict__ pre,
                                                     float* __restrict__ out) {
    __shared__ float sW[kF32Frag];
    for (int i = threadIdx.x; i < kF32Frag; i += blockDim.x) sW[i] = wfrag[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int site0 = blockIdx.x * kSitesPerBlock32 + wave * 16 * kTiles32;
    if (site0 >= g.N) return;
    const int row = lane & 15, kq = lane >> 4;
    int st[kTiles32], sy[kTiles32], sx[kTiles32];
#pragma unroll
    for (int t = 0; t < kTiles32; t++) {
        const int m = min(site0 + 16 * t + row, g.N - 1);
        site_of(g, m, st[t], sy[t], sx[t]);
    }
    f32x4 acc[kTiles32][2];
#pragma unroll
    for (int t = 0; t < kTiles32; t++)
#pragma unroll
        for (int h = 0; h < 2; h++) acc[t][h] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const int sgn = DGRAD ? -1 : 1;
    // A fragments of tap k (this lane's 8 channels of its tap-shifted site)
    auto load_a = [&](int k, f32x4 (&a)[kTiles32][2]) {
        const int dt = sgn * (k / 9 - 1), dy = sgn * ((k / 3) % 3 - 1), dx = sgn * (k % 3 - 1);
#pragma unroll
        for (int t = 0; t < kTiles32; t++) {
            const int m = wrap(st[t] + dt, g.Nt) * g.Vs + wrap(sy[t] + dy, g.L) * g.L + wrap(sx[t] + dx, g.L);
            const f32x4* src = reinterpret_cast<const f32x4*>(in + (size_t)m * 32 + 8 * kq);
            a[t][0] = src[0];
            a[t][1] = src[1];
        }
    };
    f32x4 an[kTiles32][2];
    load_a(0, an);
#pragma unroll 1
    for (int k = 0; k < 27; k++) {
        f32x4 a[kTiles32][2];
#pragma unroll
        for (int t = 0; t < kTiles32; t++) {
            a[t][0] = an[t][0];
            a[t][1] = an[t][1];
        }
        if (k + 1 < 27) load_a(k + 1, an);  // the next tap's rows in flight during this tap's MFMAs
#pragma unroll
        for (int ob = 0; ob < 2; ob++)
#pragma unroll
            for (int kk = 0; kk < 8; kk++) {
                const float b = sW[((k * 2 + ob) * 8 + kk) * 64 + lane];
#pragma unroll
                for (int t = 0; t < kTiles32; t++)
                    acc[t][ob] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t][kk >> 2][kk & 3], b, acc[t][ob], 0, 0, 0);
            }
    }
    // D fragment: lane holds sites 4 (lane / 16) + i, channel 16 ob + lane % 16
#pragma unroll
    for (int t = 0; t < kTiles32; t++)
#pragma unroll
        for (int ob = 0; ob < 2; ob++) {
            const int c = 16 * ob + row;
            const float bc = DGRAD ? 0.0f : bias[c];
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int site = site0 + 16 * t + 4 * kq + i;
                if (site >= g.N) continue;
                const size_t e = (size_t)site * 32 + c;
                if constexpr (DGRAD) {
                    out[e] = acc[t][ob][i] * dsilu_f(pre_prev[e]);
                } else {
                    const float v = acc[t][ob][i] + bc;
                    if (pre) pre[e] = v;
                    out[e] = silu_f(v);
                }
            }
        }
}

qedhmc_status net_pack_f32(qedhmc_net* n) {
    if (n->wf32_ready) return QEDHMC_OK;
    const size_t stride = n->woff[2] - n->woff[1];
    const int total = 2 * kHidden * kF32Frag;
    hipLaunchKernelGGL(k_pack_f32, dim3((total + 255) / 256), dim3(256), 0, n->h->stream, (const float*)n->params,
                       n->woff[1], stride, n->wf32);
    QH_HIP(hipGetLastError());
    n->wf32_ready = true;
    return QEDHMC_OK;
}

// hidden layer l (1 .. 4) forward in FP32 on the matrix cores
qedhmc_status launch_fwd_mfma32(qedhmc_net* n, int l, const float* in, float* pre, float* act) {
    QH_TRY(net_pack_f32(n));
    const NetGeo& g = n->g;
    const int blocks = (g.N + kSitesPerBlock32 - 1) / kSitesPerBlock32;
    const float* wf = n->wf32 + (size_t)(l - 1) * kF32Frag;
    hipEvent_t e0, e1;
    if (prof_sample(n->h, QEDHMC_K_NET_FP32, e0, e1))
        hipExtLaunchKernelGGL(k_conv_mfma32<false>, dim3(blocks), dim3(kBlock), 0, n->h->stream, e0, e1, 0, g, in, wf,
                              (const float*)(n->params + n->boff[l]), (const float*)nullptr, pre, act);
    else
        hipLaunchKernelGGL(k_conv_mfma32<false>, dim3(blocks), dim3(kBlock), 0, n->h->stream, g, in, wf,
                           (const float*)(n->params + n->boff[l]), (const float*)nullptr, pre, act);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

// data gradient through hidden layer l (1 .. 4): gin = W_l^T * gout, times SiLU'(pre of layer l - 1)
qedhmc_status launch_dgrad_mfma32(qedhmc_net* n, int l, const float* gout, const float* pre_prev, float* gin) {
    QH_TRY(net_pack_f32(n));
    const NetGeo& g = n->g;
    const int blocks = (g.N + kSitesPerBlock32 - 1) / kSitesPerBlock32;
    const float* wf = n->wf32 + (size_t)(kHidden + l - 1) * kF32Frag;
    hipLaunchKernelGGL(k_conv_mfma32<true>, dim3(blocks), dim3(kBlock), 0, n->h->stream, g, gout, wf,
                       (const float*)nullptr, pre_prev, (float*)nullptr, gin);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

}  // namespace qh
