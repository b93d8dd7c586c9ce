// Learned preconditioner: a six-layer 3x3x3 convolutional network over the
// (tau, y, x) lattice, its training (loss, backward pass, Adam) and the
// flexible CG that uses it with the residual as judge and a fallback
// preconditioner.
//
// Network (channels 6 -> 32 -> 32 -> 32 -> 32 -> 32 -> 2, SiLU after every
// layer but the last).  Input channels at a site: cos, sin of the x bond and
// of the y bond leaving it, and Re, Im of rh = r / s with s = |r| / sqrt(N);
// output z = s (o_0 + i o_1).  Padding: periodic in x and y; in tau periodic,
// except that the residual channels of the first layer change sign when they
// wrap (fermion vectors are antiperiodic in tau).
//
// Activations are site-major, channels last ([N][C]).  Two arithmetics:
//   FP32   every layer in FP32 on the vector ALUs (weights FP32);
//   BF16   the four 32 -> 32 layers as MFMA products (BF16 weights and
//          activations, FP32 accumulation) -- see netmfma.hip; the small
//          first and last layers stay FP32.
// Training keeps FP32 master weights and Adam moments; gradients are
// reduced in a fixed order (per-chunk partials, then one ordered sum), so a
// training step is reproducible.
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "net_internal.h"

namespace qh {

// 1 / s with s = |r| / sqrt(N) (0 for r = 0)
__device__ __forceinline__ double inv_scale(const double* rr, int N) {
    const double s = sqrt(*rr / (double)N);
    return s > 0.0 ? 1.0 / s : 0.0;
}

// the six input channels at site m; sg multiplies the residual channels.
// The residual is complex FP64 or, inside the mixed-precision solver, FP32.
template <typename TR>
__device__ __forceinline__ void features(const NetGeo& g, const cplx<float>* __restrict__ g32,
                                         const cplx<TR>* __restrict__ r, int m, float sg, double inv_s,
                                         float (&f)[6]) {
    const cplx<float> gx = g32[m];
    const cplx<float> gy = g32[(size_t)g.N + m];
    const cplx<TR> rv = r[m];
    f[0] = gx.re;
    f[1] = gx.im;
    f[2] = gy.re;
    f[3] = gy.im;
    f[4] = sg * (float)((double)rv.re * inv_s);
    f[5] = sg * (float)((double)rv.im * inv_s);
}

// ---------------------------------------------------------------------------
// Forward convolution (FP32): one thread per output site, all COUT outputs.
// W device layout [27][CIN][COUT]; pre = W * in + b; act = SiLU(pre) or pre.
// FIRST: the input is the feature map of (theta, r).
// ---------------------------------------------------------------------------
template <int CIN, int COUT, bool FIRST, bool SILU, typename TIN, typename TOUT, typename TR = double>
__global__ __launch_bounds__(256) void k_conv_fwd(NetGeo g, const TIN* __restrict__ in,
                                                  const cplx<float>* __restrict__ g32,
                                                  const cplx<TR>* __restrict__ r, const double* __restrict__ rr,
                                                  const float* __restrict__ W, const float* __restrict__ b,
                                                  float* __restrict__ pre, TOUT* __restrict__ act) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    int tau, y, x;
    site_of(g, n, tau, y, x);
    const double inv_s = FIRST ? inv_scale(rr, g.N) : 0.0;
    float acc[COUT];
#pragma unroll
    for (int co = 0; co < COUT; co++) acc[co] = b[co];
#pragma unroll 1
    for (int dt = -1; dt <= 1; dt++) {
        float sg;
        const int tt = wrap_tau(tau + dt, g.Nt, sg);
#pragma unroll 1
        for (int dy = -1; dy <= 1; dy++) {
            const int yy = wrap(y + dy, g.L);
#pragma unroll 1
            for (int dx = -1; dx <= 1; dx++) {
                const int xx = wrap(x + dx, g.L);
                const int k = (dt + 1) * 9 + (dy + 1) * 3 + (dx + 1);
                const int m = tt * g.Vs + yy * g.L + xx;
                float v[CIN];
                if constexpr (FIRST) {
                    float f[6];
                    features(g, g32, r, m, sg, inv_s, f);
#pragma unroll
                    for (int c = 0; c < CIN; c++) v[c] = f[c];
                } else {
#pragma unroll
                    for (int c = 0; c < CIN; c++) v[c] = to_f32(in[(size_t)m * CIN + c]);
                }
                const float* Wk = W + (size_t)k * CIN * COUT;
#pragma unroll
                for (int c = 0; c < CIN; c++)
#pragma unroll
                    for (int co = 0; co < COUT; co++) acc[co] = fmaf(Wk[c * COUT + co], v[c], acc[co]);
            }
        }
    }
    if (pre)
#pragma unroll
        for (int co = 0; co < COUT; co++) pre[(size_t)n * COUT + co] = acc[co];
    if constexpr (sizeof(TOUT) == 2 && COUT % 8 == 0) {
        // BF16 out: eight channels per 16-byte store
#pragma unroll
        for (int c8 = 0; c8 < COUT; c8 += 8) {
            uint32_t w[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const float v0 = SILU ? silu_f(acc[c8 + 2 * j]) : acc[c8 + 2 * j];
                const float v1 = SILU ? silu_f(acc[c8 + 2 * j + 1]) : acc[c8 + 2 * j + 1];
                w[j] = (uint32_t)f32_to_bf16(v0) | ((uint32_t)f32_to_bf16(v1) << 16);
            }
            *reinterpret_cast<uint4*>(act + (size_t)n * COUT + c8) = make_uint4(w[0], w[1], w[2], w[3]);
        }
    } else {
#pragma unroll
        for (int co = 0; co < COUT; co++)
            act[(size_t)n * COUT + co] = from_f32<TOUT>(SILU ? silu_f(acc[co]) : acc[co]);
    }
}

// ---------------------------------------------------------------------------
// Backward data (FP32): gin[m][c] = dsilu(pre_prev[m][c]) *
//   sum_{k, co} W[k][c][co] gout[m - d_k][co]   (hidden layers: periodic)
// ---------------------------------------------------------------------------
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_conv_dgrad(NetGeo g, const float* __restrict__ gout,
                                                    const float* __restrict__ W,
                                                    const float* __restrict__ pre_prev, float* __restrict__ gin) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= g.N) return;
    int tau, y, x;
    site_of(g, m, tau, y, x);
    float acc[CIN];
#pragma unroll
    for (int c = 0; c < CIN; c++) acc[c] = 0.0f;
#pragma unroll 1
    for (int dt = -1; dt <= 1; dt++) {
        const int tt = wrap(tau - dt, g.Nt);
#pragma unroll 1
        for (int dy = -1; dy <= 1; dy++) {
            const int yy = wrap(y - dy, g.L);
#pragma unroll 1
            for (int dx = -1; dx <= 1; dx++) {
                const int xx = wrap(x - dx, g.L);
                const int k = (dt + 1) * 9 + (dy + 1) * 3 + (dx + 1);
                const int n = tt * g.Vs + yy * g.L + xx;
                float go[COUT];
#pragma unroll
                for (int co = 0; co < COUT; co++) go[co] = gout[(size_t)n * COUT + co];
                const float* Wk = W + (size_t)k * CIN * COUT;
#pragma unroll
                for (int c = 0; c < CIN; c++)
#pragma unroll
                    for (int co = 0; co < COUT; co++) acc[c] = fmaf(Wk[c * COUT + co], go[co], acc[c]);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < CIN; c++) gin[(size_t)m * CIN + c] = acc[c] * dsilu_f(pre_prev[(size_t)m * CIN + c]);
}

// ---------------------------------------------------------------------------
// Backward weights (FP32): workgroup (chunk, k) sums over its kWChunk output
// sites n
//   dW[k][c][co] = sum_n in~[n + d_k][c] gout[n][co]   (and, for the centre
//   tap, db[co] = sum_n gout[n][co])
// into part[chunk][27 CIN COUT + COUT]; thread t owns the (c, co) entries
// t, t + 256, ... of tap k (co fastest).
// ---------------------------------------------------------------------------
template <int CIN, int COUT, bool FIRST>
__global__ __launch_bounds__(256) void k_conv_wgrad(NetGeo g, const float* __restrict__ in,
                                                    const cplx<float>* __restrict__ g32,
                                                    const cplx<double>* __restrict__ r,
                                                    const double* __restrict__ rr, const float* __restrict__ gout,
                                                    float* __restrict__ part) {
    constexpr int EK = CIN * COUT;
    constexpr int PER = (EK + 255) / 256;
    constexpr int E = 27 * EK;
    const int k = blockIdx.y;
    const int dt = k / 9 - 1, dy = (k / 3) % 3 - 1, dx = k % 3 - 1;
    const int n0 = blockIdx.x * kWChunk;
    const int n1 = min(n0 + kWChunk, g.N);
    const double inv_s = FIRST ? inv_scale(rr, g.N) : 0.0;
    float acc[PER];
    int ec[PER], eo[PER];
#pragma unroll
    for (int j = 0; j < PER; j++) {
        acc[j] = 0.0f;
        const int e = threadIdx.x + 256 * j;
        const int ee = e < EK ? e : 0;
        eo[j] = ee % COUT;
        ec[j] = ee / COUT;
    }
    float accb = 0.0f;
    const bool bias = (k == 13) && threadIdx.x < COUT;
#pragma unroll 1
    for (int n = n0; n < n1; n++) {
        int tau, y, x;
        site_of(g, n, tau, y, x);
        float sg;
        const int tt = wrap_tau(tau + dt, g.Nt, sg);
        const int m = tt * g.Vs + wrap(y + dy, g.L) * g.L + wrap(x + dx, g.L);
        float f[6];
        if constexpr (FIRST) features(g, g32, r, m, sg, inv_s, f);
#pragma unroll
        for (int j = 0; j < PER; j++) {
            float v;
            if constexpr (FIRST) {
                v = f[0];
#pragma unroll
                for (int c = 1; c < 6; c++)
                    if (ec[j] == c) v = f[c];
            } else {
                v = in[(size_t)m * CIN + ec[j]];
            }
            acc[j] = fmaf(v, gout[(size_t)n * COUT + eo[j]], acc[j]);
        }
        if (bias) accb += gout[(size_t)n * COUT + threadIdx.x];
    }
    float* out = part + (size_t)blockIdx.x * (E + COUT);
#pragma unroll
    for (int j = 0; j < PER; j++) {
        const int e = threadIdx.x + 256 * j;
        if (e < EK) out[(size_t)k * EK + e] = acc[j];
    }
    if (bias) out[E + threadIdx.x] = accb;
}

// Weight gradients on the matrix cores: per tap k the product dW_k = A_k^T G
// over a chunk of sites, A_k[n][c] = in[n + tap k][c] and G[n][o] =
// gout[n][o], as v_mfma_f32_16x16x4f32 (FP32 operands, FP32 accumulation:
// the same arithmetic as the vector kernel, summed in another order), the
// channels in blocks of 16 (zero-padded: the first layer's 6 inputs, the last
// layer's 2 outputs).  A wavefront holds 7 taps (k = wave + 4 j) as
// CINB x COUTB output blocks each; the last wavefront's seventh slot is the
// bias gradient, the same product with A = 1.  Per step of 4 sites a lane
// loads one G value per output block (shared by its taps) and one input value
// per tap and input block.  The first layer reads the feature map from feat
// ([N][8], the residual channels 4, 5 sign-flipped where the tap wraps in
// tau).  Partials per chunk as the vector kernel writes them.
typedef float wg_f32x4 __attribute__((ext_vector_type(4)));
static constexpr int kWgTaps = 7;

template <int CIN, int COUT, bool FIRST>
__global__ __launch_bounds__(256) void k_wgrad_mfma(NetGeo g, int chunk, const float* __restrict__ in,
                                                    const float* __restrict__ gout, float* __restrict__ part) {
    constexpr int CINB = (CIN + 15) / 16, COUTB = (COUT + 15) / 16;
    constexpr int EK = CIN * COUT, E = 27 * EK;
    constexpr int IS = FIRST ? 8 : CIN;  // row stride of the input
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n0 = blockIdx.x * chunk, n1 = min(n0 + chunk, g.N);
    const int c16 = lane & 15, kq = lane >> 4;
    wg_f32x4 acc[kWgTaps][CINB][COUTB];
#pragma unroll
    for (int j = 0; j < kWgTaps; j++)
#pragma unroll
        for (int cb = 0; cb < CINB; cb++)
#pragma unroll
            for (int ob = 0; ob < COUTB; ob++) acc[j][cb][ob] = wg_f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 1
    for (int n = n0; n < n1; n += 4) {
        const int nn = n + kq;  // this lane's site of the 4-site step
        const bool valid = nn < n1;
        int tau, y, x;
        site_of(g, valid ? nn : n0, tau, y, x);
        float b[COUTB];
#pragma unroll
        for (int ob = 0; ob < COUTB; ob++) {
            const int o = 16 * ob + c16;
            b[ob] = (valid && o < COUT) ? gout[(size_t)nn * COUT + o] : 0.0f;
        }
#pragma unroll
        for (int j = 0; j < kWgTaps; j++) {
            const int k = wave + 4 * j;
            float a[CINB];
#pragma unroll
            for (int cb = 0; cb < CINB; cb++) a[cb] = 1.0f;  // k = 27: the bias slot
            if (k < 27) {
                const int dt = k / 9 - 1, dy = (k / 3) % 3 - 1, dx = k % 3 - 1;
                float sg = 1.0f;
                const int tt = wrap_tau(tau + dt, g.Nt, sg);
                const int m = tt * g.Vs + wrap(y + dy, g.L) * g.L + wrap(x + dx, g.L);
#pragma unroll
                for (int cb = 0; cb < CINB; cb++) {
                    const int c = 16 * cb + c16;
                    float v = c < CIN ? in[(size_t)m * IS + c] : 0.0f;
                    if (FIRST && c >= 4) v *= sg;
                    a[cb] = v;
                }
            }
#pragma unroll
            for (int cb = 0; cb < CINB; cb++)
#pragma unroll
                for (int ob = 0; ob < COUTB; ob++)
                    acc[j][cb][ob] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[cb], b[ob], acc[j][cb][ob], 0, 0, 0);
        }
    }
    // D fragment: lane holds rows 4 (lane / 16) + r (input channels), column lane % 16 (output channel)
    float* out = part + (size_t)blockIdx.x * (E + COUT);
#pragma unroll
    for (int j = 0; j < kWgTaps; j++) {
        const int k = wave + 4 * j;
#pragma unroll
        for (int cb = 0; cb < CINB; cb++)
#pragma unroll
            for (int ob = 0; ob < COUTB; ob++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int c = 16 * cb + 4 * kq + r, o = 16 * ob + c16;
                    if (o >= COUT) continue;
                    if (k < 27 && c < CIN)
                        out[(size_t)k * EK + c * COUT + o] = acc[j][cb][ob][r];
                    else if (k == 27 && c == 0)
                        out[E + o] = acc[j][cb][ob][r];
                }
    }
}

// the first layer's feature map [N][8] (channels 6, 7 zero), unsigned
template <typename TR>
__global__ void k_features(NetGeo g, const cplx<float>* __restrict__ g32, const cplx<TR>* __restrict__ r,
                           const double* __restrict__ rr, float* __restrict__ feat) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= g.N) return;
    float f[6];
    features(g, g32, r, m, 1.0f, inv_scale(rr, g.N), f);
#pragma unroll
    for (int c = 0; c < 6; c++) feat[(size_t)m * 8 + c] = f[c];
    feat[(size_t)m * 8 + 6] = 0.0f;
    feat[(size_t)m * 8 + 7] = 0.0f;
}

// sites per weight-gradient chunk on the matrix cores: about 2048 chunks,
// 256 .. 4096 sites each (a multiple of 4)
int wgrad_mfma_chunk(int N) {
    int c = (N + 2047) / 2048;
    c = ((c + 255) / 256) * 256;
    return c < 256 ? 256 : (c > 4096 ? 4096 : c);
}

// grad[e] = sum over chunks b (in order) of part[b][e]
__global__ void k_wgrad_reduce(const float* __restrict__ part, int nchunk, int E, float* __restrict__ grad) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    float s = 0.0f;
    for (int b = 0; b < nchunk; b++) s += part[(size_t)b * E + e];
    grad[e] = s;
}

// The same sum in two passes for many chunks: group g of kWgGroups adds its
// contiguous range of chunks in order, then the groups' sums are added in
// order (a fixed order either way).
static constexpr int kWgGroups = 16;

__global__ void k_wgrad_reduce_groups(const float* __restrict__ part, int nchunk, int E, float* __restrict__ tmp) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x, gidx = blockIdx.y;
    if (e >= E) return;
    const int per = (nchunk + kWgGroups - 1) / kWgGroups;
    const int b0 = gidx * per, b1 = min(nchunk, b0 + per);
    float s = 0.0f;
    for (int b = b0; b < b1; b++) s += part[(size_t)b * E + e];
    tmp[(size_t)gidx * E + e] = s;
}

// ---------------------------------------------------------------------------
// Output: z = s (o_0 + i o_1) in FP64
// ---------------------------------------------------------------------------
__global__ void k_net_out(int N, const float* __restrict__ o, const double* __restrict__ rr,
                          cplx<double>* __restrict__ z) {
    const double s = sqrt(*rr / (double)N);
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < N; n += gridDim.x * blockDim.x)
        z[n] = mk<double>(s * (double)o[2 * n], s * (double)o[2 * n + 1]);
}

// Loss |z - e|^2 / |e|^2 (partials of |z - e|^2 per block) and its gradient
// with respect to the last layer's outputs o: g = 2 s (z - e) / |e|^2.
__global__ __launch_bounds__(256) void k_net_loss(int N, const float* __restrict__ o,
                                                  const double* __restrict__ rr,
                                                  const cplx<double>* __restrict__ e,
                                                  const double* __restrict__ ee, float* __restrict__ gout,
                                                  double* __restrict__ part) {
    __shared__ double red[16];
    const double s = sqrt(*rr / (double)N);
    const double c = 2.0 * s / *ee;
    double acc = 0.0;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < N; n += gridDim.x * blockDim.x) {
        const double dre = s * (double)o[2 * n] - e[n].re;
        const double dim = s * (double)o[2 * n + 1] - e[n].im;
        acc += dre * dre + dim * dim;
        gout[2 * n] = (float)(c * dre);
        gout[2 * n + 1] = (float)(c * dim);
    }
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Residual form of the loss, |O z - r|^2 / |r|^2: the error z - e measured by
// |O (z - e)| relative to |O e| (O e = r).  It weighs the error's components
// along the eigenvectors of O by the eigenvalue, where |z - e|^2 lets the
// lowest modes of O (which a local network cannot represent) dominate.
// d = O z - r in place of O z, and per-block partials of |d|^2.
__global__ __launch_bounds__(256) void k_net_resid(int N, cplx<double>* __restrict__ d,
                                                   const cplx<double>* __restrict__ r, double* __restrict__ part) {
    __shared__ double red[16];
    double acc = 0.0;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < N; n += gridDim.x * blockDim.x) {
        const cplx<double> v = mk<double>(d[n].re - r[n].re, d[n].im - r[n].im);
        acc += v.re * v.re + v.im * v.im;
        d[n] = v;
    }
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Its gradient at the last layer's outputs o (z = s o, O Hermitian):
// g = 2 s (O d) / |r|^2.
__global__ void k_net_resgrad(int N, const cplx<double>* __restrict__ Od, const double* __restrict__ rr,
                              float* __restrict__ gout) {
    const double s = sqrt(*rr / (double)N);
    const double c = 2.0 * s / *rr;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < N; n += gridDim.x * blockDim.x) {
        gout[2 * n] = (float)(c * Od[n].re);
        gout[2 * n + 1] = (float)(c * Od[n].im);
    }
}

// Adam (Kingma and Ba 2015): m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2;
// p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
__global__ void k_adam(int n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// ---------------------------------------------------------------------------
// Complex inner products for flexible CG: per block partials of
// <a, b> = sum conj(a) b and <c, d> (FP64), then one ordered sum.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_cdot2(int N, const cplx<double>* __restrict__ a,
                                               const cplx<double>* __restrict__ b,
                                               const cplx<double>* __restrict__ c,
                                               const cplx<double>* __restrict__ d, double* __restrict__ part) {
    __shared__ double red[16];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < N; n += gridDim.x * blockDim.x) {
        const cplx<double> x = a[n], y = b[n];
        v[0] += x.re * y.re + x.im * y.im;
        v[1] += x.re * y.im - x.im * y.re;
        if (c) {
            const cplx<double> u = c[n], w = d[n];
            v[2] += u.re * w.re + u.im * w.im;
            v[3] += u.re * w.im - u.im * w.re;
        }
    }
    for (int k = 0; k < 4; k++) {
        const double t = block_sum(v[k], red);
        if (threadIdx.x == 0) part[4 * blockIdx.x + k] = t;
        __syncthreads();
    }
}

__global__ void k_sum1(const double* __restrict__ part, int nb, double* __restrict__ out) {
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int b = 0; b < nb; b++) s += part[b];
        *out = s;
    }
}

__global__ void k_sum4(const double* __restrict__ part, int nb, double* __restrict__ out) {
    if (threadIdx.x < 4) {
        double s = 0.0;
        for (int b = 0; b < nb; b++) s += part[4 * b + threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// x += alpha p; r -= alpha s (complex alpha); partials of |r|^2
__global__ __launch_bounds__(256) void k_fcg_update(int N, double are, double aim, const cplx<double>* __restrict__ p,
                                                    const cplx<double>* __restrict__ s, cplx<double>* __restrict__ x,
                                                    cplx<double>* __restrict__ r, double* __restrict__ part) {
    __shared__ double red[16];
    double acc = 0.0;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < N; n += gridDim.x * blockDim.x) {
        const cplx<double> pv = p[n], sv = s[n];
        cplx<double> xv = x[n], rv = r[n];
        xv.re += are * pv.re - aim * pv.im;
        xv.im += are * pv.im + aim * pv.re;
        rv.re -= are * sv.re - aim * sv.im;
        rv.im -= are * sv.im + aim * sv.re;
        x[n] = xv;
        r[n] = rv;
        acc += rv.re * rv.re + rv.im * rv.im;
    }
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) part[4 * blockIdx.x] = t;
    if (threadIdx.x == 1) {
        part[4 * blockIdx.x + 1] = 0.0;
        part[4 * blockIdx.x + 2] = 0.0;
        part[4 * blockIdx.x + 3] = 0.0;
    }
}

// p = z + beta p (complex beta)
__global__ void k_fcg_dir(int N, double bre, double bim, const cplx<double>* __restrict__ z,
                          cplx<double>* __restrict__ p) {
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < N; n += gridDim.x * blockDim.x) {
        const cplx<double> zv = z[n], pv = p[n];
        p[n] = mk<double>(zv.re + bre * pv.re - bim * pv.im, zv.im + bre * pv.im + bim * pv.re);
    }
}

__global__ void k_residual(int N, const cplx<double>* __restrict__ rhs, const cplx<double>* __restrict__ Ox,
                           cplx<double>* __restrict__ r) {
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < N; n += gridDim.x * blockDim.x)
        r[n] = mk<double>(rhs[n].re - Ox[n].re, rhs[n].im - Ox[n].im);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static int blocks_for(int N, int bs) { return (N + bs - 1) / bs; }

// parameter offsets (floats) of each layer's W and b; device W layout
// [27][Cin][Cout], host layout [Cout][Cin][27] (the oracle's)
static void param_offsets(size_t (&w)[kNetLayers], size_t (&b)[kNetLayers], size_t& total) {
    size_t o = 0;
    for (int l = 0; l < kNetLayers; l++) {
        w[l] = o;
        o += (size_t)27 * kNetCh[l] * kNetCh[l + 1];
        b[l] = o;
        o += kNetCh[l + 1];
    }
    total = o;
}

qedhmc_status net_alloc_train(qedhmc_net* n);

// first layer (FP32 arithmetic) writing BF16 activations, last layer
// reading BF16 activations: the ends of the BF16 forward
qedhmc_status launch_first_bf16(const NetGeo& g, hipStream_t st, const cplx<float>* g32, const void* r, bool r32,
                                const double* rr, const float* W, const float* b, uint16_t* out) {
    if (r32)
        hipLaunchKernelGGL((k_conv_fwd<6, 32, true, true, float, uint16_t, float>), dim3(blocks_for(g.N, 256)),
                           dim3(256), 0, st, g, (const float*)nullptr, g32, static_cast<const cplx<float>*>(r), rr,
                           W, b, (float*)nullptr, out);
    else
        hipLaunchKernelGGL((k_conv_fwd<6, 32, true, true, float, uint16_t>), dim3(blocks_for(g.N, 256)), dim3(256),
                           0, st, g, (const float*)nullptr, g32, static_cast<const cplx<double>*>(r), rr, W, b,
                           (float*)nullptr, out);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

qedhmc_status launch_last_bf16(const NetGeo& g, hipStream_t st, const uint16_t* in, const float* W, const float* b,
                               float* out) {
    hipLaunchKernelGGL((k_conv_fwd<32, 2, false, false, uint16_t, float>), dim3(blocks_for(g.N, 256)), dim3(256), 0,
                       st, g, in, (const cplx<float>*)nullptr, (const cplx<double>*)nullptr, (const double*)nullptr,
                       W, b, (float*)nullptr, out);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

}  // namespace qh

using namespace qh;


namespace qh {

static constexpr int kRedBlocks = 256;

static qedhmc_status net_fail(qedhmc_net* n, const char* msg, qedhmc_status st) {
    set_error(msg);
    (void)n;
    return st;
}

qedhmc_status net_alloc_train(qedhmc_net* n) {
    if (n->train_ready) return QEDHMC_OK;
    const size_t N = n->g.N;
    bool ok = true;
    for (int l = 1; l < kNetLayers; l++)
        ok = ok && hipMalloc(&n->pre[l - 1], N * 32 * sizeof(float)) == hipSuccess;
    ok = ok && hipMalloc(&n->pre[kNetLayers - 1], N * 2 * sizeof(float)) == hipSuccess;
    // act[kNetLayers] (the output channels) and gbuf exist from creation
    for (int l = 1; l < kNetLayers; l++) ok = ok && hipMalloc(&n->act[l], N * 32 * sizeof(float)) == hipSuccess;
    const size_t nchunk = std::max((N + kWChunk - 1) / kWChunk,
                                   (N + wgrad_mfma_chunk((int)N) - 1) / (size_t)wgrad_mfma_chunk((int)N));
    ok = ok && hipMalloc(&n->wpart, nchunk * (27 * 32 * 32 + 32) * sizeof(float)) == hipSuccess;
    ok = ok && hipMalloc(&n->feat, N * 8 * sizeof(float)) == hipSuccess;
    ok = ok && hipMalloc(&n->wtmp, (size_t)kWgGroups * (27 * 32 * 32 + 32) * sizeof(float)) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        return net_fail(n, "net: training buffers: device allocation failed", QEDHMC_ENOMEM);
    }
    n->train_ready = true;
    return QEDHMC_OK;
}

static qedhmc_status sumsq_to(qedhmc_net* n, const double* v, size_t count, double* dst) {
    return launch_sumsq(n->h, v, count, dst);
}

// layer l forward in FP32: input act[l] (or the features for l = 0, from
// the residual r: complex FP64, or FP32 when r32; rr: device |r|^2)
static qedhmc_status fwd_layer_f32(qedhmc_net* n, int l, const void* r, bool r32, const double* rr, const float* in,
                                   float* pre, float* act) {
    const NetGeo& g = n->g;
    const float* W = n->params + n->woff[l];
    const float* b = n->params + n->boff[l];
    const dim3 grid(blocks_for(g.N, 256)), blk(256);
    hipStream_t st = n->h->stream;
    const cplx<float>* g32 = n->h->gauge32;
    const cplx<double>* rc = static_cast<const cplx<double>*>(r);
    if (l == 0 && r32)
        hipLaunchKernelGGL((k_conv_fwd<6, 32, true, true, float, float, float>), grid, blk, 0, st, g, in, g32,
                           static_cast<const cplx<float>*>(r), rr, W, b, pre, act);
    else if (l == 0)
        hipLaunchKernelGGL((k_conv_fwd<6, 32, true, true, float, float>), grid, blk, 0, st, g, in, g32, rc, rr, W, b, pre, act);
    else if (l < kNetLayers - 1 && !net_f32_on_vector_alus())
        return launch_fwd_mfma32(n, l, in, pre, act);
    else if (l < kNetLayers - 1) {
        hipEvent_t e0, e1;
        if (prof_sample(n->h, QEDHMC_K_NET_FP32, e0, e1))
            hipExtLaunchKernelGGL((k_conv_fwd<32, 32, false, true, float, float>), grid, blk, 0, st, e0, e1, 0, g, in,
                                  g32, rc, rr, W, b, pre, act);
        else
            hipLaunchKernelGGL((k_conv_fwd<32, 32, false, true, float, float>), grid, blk, 0, st, g, in, g32, rc, rr,
                               W, b, pre, act);
    }
    else
        hipLaunchKernelGGL((k_conv_fwd<32, 2, false, false, float, float>), grid, blk, 0, st, g, in, g32, rc, rr, W, b, pre, act);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

// forward pass; keep = store every layer's input and pre-activation
// (training), else ping-pong through two buffers.  Output channels in
// n->act[kNetLayers] ([N][2] FP32).
static qedhmc_status net_forward(qedhmc_net* n, const double* theta, const double* r, qedhmc_net_arith a, bool keep,
                                 bool build_gauge = true) {
    if (build_gauge) QH_TRY(ensure_gauge(n->h, theta, QEDHMC_FP32));
    QH_TRY(sumsq_to(n, r, 2 * (size_t)n->g.N, n->dscal + 0));
    if (a == QEDHMC_NET_BF16 && !keep) return net_forward_bf16(n, r, false, n->dscal);
    const float* in = nullptr;
    for (int l = 0; l < kNetLayers; l++) {
        float* out;
        float* pre = nullptr;
        if (keep) {
            out = n->act[l + 1];
            pre = n->pre[l];
        } else {
            out = (l == kNetLayers - 1) ? n->act[kNetLayers] : n->gbuf[l & 1];
        }
        QH_TRY(fwd_layer_f32(n, l, r, false, n->dscal, in, pre, out));
        in = out;
    }
    return QEDHMC_OK;
}

}  // namespace qh

namespace qh {

// Inference on a residual already in device memory, FP64 or (r32) FP32, with
// |r|^2 at rr (device) and the FP32 e^{i theta} cache of the handle already
// built; output channels in n->act[kNetLayers].
qedhmc_status net_infer(qedhmc_net* n, const void* r, bool r32, const double* rr, qedhmc_net_arith a) {
    if (a == QEDHMC_NET_BF16) return net_forward_bf16(n, r, r32, rr);
    const float* in = nullptr;
    for (int l = 0; l < kNetLayers; l++) {
        float* out = (l == kNetLayers - 1) ? n->act[kNetLayers] : n->gbuf[l & 1];
        QH_TRY(fwd_layer_f32(n, l, r, r32, rr, in, nullptr, out));
        in = out;
    }
    return QEDHMC_OK;
}

// QEDHMC_NET_WGRAD=valu (read per call) keeps the hidden layers' weight
// gradients on the vector ALUs (tests compare the two kernels)
static bool wgrad_on_vector_alus() {
    const char* e = std::getenv("QEDHMC_NET_WGRAD");
    return e && std::strcmp(e, "valu") == 0;
}

static qedhmc_status launch_wgrad(qedhmc_net* n, int l, const double* r, const float* gout) {
    const NetGeo& g = n->g;
    int nchunk = blocks_for(g.N, kWChunk);
    hipStream_t st = n->h->stream;
    const cplx<float>* g32 = n->h->gauge32;
    const cplx<double>* rc = reinterpret_cast<const cplx<double>*>(r);
    const int cin = kNetCh[l], cout = kNetCh[l + 1];
    const int E = 27 * cin * cout + cout;
    const dim3 grid(nchunk, 27);
    if (wgrad_on_vector_alus()) {
        if (l == 0)
            hipLaunchKernelGGL((k_conv_wgrad<6, 32, true>), grid, dim3(256), 0, st, g, (const float*)nullptr, g32,
                               rc, n->dscal, gout, n->wpart);
        else if (l < kNetLayers - 1)
            hipLaunchKernelGGL((k_conv_wgrad<32, 32, false>), grid, dim3(256), 0, st, g, n->act[l], g32, rc,
                               n->dscal, gout, n->wpart);
        else
            hipLaunchKernelGGL((k_conv_wgrad<32, 2, false>), grid, dim3(256), 0, st, g, n->act[l], g32, rc,
                               n->dscal, gout, n->wpart);
    } else {
        const int chunk = wgrad_mfma_chunk(g.N);
        nchunk = blocks_for(g.N, chunk);
        if (l == 0) {
            hipLaunchKernelGGL(k_features<double>, dim3(blocks_for(g.N, 256)), dim3(256), 0, st, g, g32, rc,
                               (const double*)n->dscal, n->feat);
            hipLaunchKernelGGL((k_wgrad_mfma<6, 32, true>), dim3(nchunk), dim3(256), 0, st, g, chunk,
                               (const float*)n->feat, gout, n->wpart);
        } else if (l < kNetLayers - 1) {
            hipLaunchKernelGGL((k_wgrad_mfma<32, 32, false>), dim3(nchunk), dim3(256), 0, st, g, chunk,
                               (const float*)n->act[l], gout, n->wpart);
        } else {
            hipLaunchKernelGGL((k_wgrad_mfma<32, 2, false>), dim3(nchunk), dim3(256), 0, st, g, chunk,
                               (const float*)n->act[l], gout, n->wpart);
        }
    }
    // W and b are contiguous in the parameter vector (b follows W)
    if (nchunk > 4 * kWgGroups) {
        hipLaunchKernelGGL(k_wgrad_reduce_groups, dim3(blocks_for(E, 256), kWgGroups), dim3(256), 0, st,
                           (const float*)n->wpart, nchunk, E, n->wtmp);
        hipLaunchKernelGGL(k_wgrad_reduce, dim3(blocks_for(E, 256)), dim3(256), 0, st, (const float*)n->wtmp,
                           kWgGroups, E, n->grads + n->woff[l]);
        QH_HIP(hipGetLastError());
        return QEDHMC_OK;
    }
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(blocks_for(E, 256)), dim3(256), 0, st, (const float*)n->wpart, nchunk, E,
                       n->grads + n->woff[l]);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

bool net_f32_on_vector_alus() {
    const char* e = std::getenv("QEDHMC_NET_F32");
    return e && std::strcmp(e, "valu") == 0;
}

static qedhmc_status launch_dgrad(qedhmc_net* n, int l, const float* gout, float* gin) {
    if (l < kNetLayers - 1 && !net_f32_on_vector_alus())
        return launch_dgrad_mfma32(n, l, gout, (const float*)n->pre[l - 1], gin);
    const NetGeo& g = n->g;
    hipStream_t st = n->h->stream;
    const float* W = n->params + n->woff[l];
    if (l < kNetLayers - 1)
        hipLaunchKernelGGL((k_conv_dgrad<32, 32>), dim3(blocks_for(g.N, 256)), dim3(256), 0, st, g, gout, W,
                           (const float*)n->pre[l - 1], gin);
    else
        hipLaunchKernelGGL((k_conv_dgrad<32, 2>), dim3(blocks_for(g.N, 256)), dim3(256), 0, st, g, gout, W,
                           (const float*)n->pre[l - 1], gin);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

qedhmc_status net_backward_adam(qedhmc_net* n, const double* r, double lr, float* grad_host);

}  // namespace qh

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

qedhmc_status qedhmc_net_create(qedhmc_t h, qedhmc_net_t* out) {
    if (!h || !out) {
        set_error("net: null argument");
        return QEDHMC_EINVAL;
    }
    *out = nullptr;
    qedhmc_net* n = new (std::nothrow) qedhmc_net{};
    if (!n) {
        set_error("net: out of host memory");
        return QEDHMC_ENOMEM;
    }
    n->h = h;
    n->g = NetGeo{h->lat.L, h->lat.Nt, h->lat.Vs, (int)((size_t)h->lat.Nt * h->lat.Vs)};
    size_t total = 0;
    param_offsets(n->woff, n->boff, total);
    n->nparam = total;
    const size_t N = n->g.N;
    bool ok = true;
    ok = ok && hipMalloc(&n->params, total * sizeof(float)) == hipSuccess;
    ok = ok && hipMalloc(&n->grads, total * sizeof(float)) == hipSuccess;
    ok = ok && hipMalloc(&n->adam_m, total * sizeof(float)) == hipSuccess;
    ok = ok && hipMalloc(&n->adam_v, total * sizeof(float)) == hipSuccess;
    ok = ok && hipMalloc(&n->wbf, net_bf16_weight_elems() * sizeof(uint16_t)) == hipSuccess;
    ok = ok && hipMalloc(&n->wf32, net_f32_weight_elems() * sizeof(float)) == hipSuccess;
    for (int k = 0; k < 2; k++) ok = ok && hipMalloc(&n->gbuf[k], N * 32 * sizeof(float)) == hipSuccess;
    ok = ok && hipMalloc(&n->act[kNetLayers], N * 2 * sizeof(float)) == hipSuccess;
    for (int k = 0; k < 2; k++) ok = ok && hipMalloc(&n->actb[k], N * 32 * sizeof(uint16_t)) == hipSuccess;
    ok = ok && hipMalloc(&n->dscal, 32 * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc(&n->dpart, (size_t)4 * kRedBlocks * sizeof(double)) == hipSuccess;
    ok = ok && hipHostMalloc(&n->hpin, 16 * sizeof(double), hipHostMallocDefault) == hipSuccess;
    ok = ok && hipMalloc(&n->fr, N * sizeof(cplx<double>)) == hipSuccess;
    ok = ok && hipMalloc(&n->fp, N * sizeof(cplx<double>)) == hipSuccess;
    ok = ok && hipMalloc(&n->fs, N * sizeof(cplx<double>)) == hipSuccess;
    ok = ok && hipMalloc(&n->fz, N * sizeof(cplx<double>)) == hipSuccess;
    if (ok) ok = hipMemsetAsync(n->params, 0, total * sizeof(float), h->stream) == hipSuccess;
    if (ok) ok = hipMemsetAsync(n->adam_m, 0, total * sizeof(float), h->stream) == hipSuccess;
    if (ok) ok = hipMemsetAsync(n->adam_v, 0, total * sizeof(float), h->stream) == hipSuccess;
    if (ok) ok = hipStreamSynchronize(h->stream) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        qedhmc_net_destroy(n);
        set_error("net: device allocation failed");
        return QEDHMC_ENOMEM;
    }
    *out = n;
    return QEDHMC_OK;
}

qedhmc_status qedhmc_net_destroy(qedhmc_net_t n) {
    if (!n) return QEDHMC_OK;
    if (n->h) (void)hipStreamSynchronize(n->h->stream);
    if (n->h && n->h->pc_net == n) n->h->pc_net = nullptr;  // no longer the handle's learned preconditioner
    (void)hipFree(n->params);
    (void)hipFree(n->grads);
    (void)hipFree(n->adam_m);
    (void)hipFree(n->adam_v);
    (void)hipFree(n->wbf);
    (void)hipFree(n->wf32);
    for (int l = 0; l <= kNetLayers; l++) (void)hipFree(n->act[l]);
    for (int l = 0; l < kNetLayers; l++) (void)hipFree(n->pre[l]);
    for (int k = 0; k < 2; k++) {
        (void)hipFree(n->gbuf[k]);
        (void)hipFree(n->actb[k]);
    }
    (void)hipFree(n->wpart);
    (void)hipFree(n->feat);
    (void)hipFree(n->wtmp);
    (void)hipFree(n->dscal);
    (void)hipFree(n->dpart);
    if (n->hpin) (void)hipHostFree(n->hpin);
    (void)hipFree(n->fr);
    (void)hipFree(n->fp);
    (void)hipFree(n->fs);
    (void)hipFree(n->fz);
    delete n;
    return QEDHMC_OK;
}

int64_t qedhmc_net_param_count(void) {
    size_t w[kNetLayers], b[kNetLayers], total = 0;
    param_offsets(w, b, total);
    return (int64_t)total;
}

// host layout per layer: W[co][ci][27], then b[co]; device: W[27][ci][co]
qedhmc_status qedhmc_net_set_params(qedhmc_net_t n, const float* host, int64_t count) {
    if (!n || !host || count != (int64_t)n->nparam) {
        set_error("net: null argument or wrong parameter count");
        return QEDHMC_EINVAL;
    }
    std::vector<float> dev(n->nparam);
    for (int l = 0; l < kNetLayers; l++) {
        const int ci_n = kNetCh[l], co_n = kNetCh[l + 1];
        const float* hw = host + n->woff[l];
        float* dw = dev.data() + n->woff[l];
        for (int co = 0; co < co_n; co++)
            for (int ci = 0; ci < ci_n; ci++)
                for (int k = 0; k < 27; k++) dw[((size_t)k * ci_n + ci) * co_n + co] = hw[((size_t)co * ci_n + ci) * 27 + k];
        for (int co = 0; co < co_n; co++) dev[n->boff[l] + co] = host[n->boff[l] + co];
    }
    QH_HIP(hipMemcpyAsync(n->params, dev.data(), n->nparam * sizeof(float), hipMemcpyHostToDevice, n->h->stream));
    QH_HIP(hipStreamSynchronize(n->h->stream));
    n->wbf_ready = false;
    n->wf32_ready = false;
    return QEDHMC_OK;
}

static qedhmc_status to_host_layout(qedhmc_net* n, const float* dptr, float* host) {
    std::vector<float> dev(n->nparam);
    QH_HIP(hipMemcpyAsync(dev.data(), dptr, n->nparam * sizeof(float), hipMemcpyDeviceToHost, n->h->stream));
    QH_HIP(hipStreamSynchronize(n->h->stream));
    for (int l = 0; l < kNetLayers; l++) {
        const int ci_n = kNetCh[l], co_n = kNetCh[l + 1];
        const float* dw = dev.data() + n->woff[l];
        float* hw = host + n->woff[l];
        for (int co = 0; co < co_n; co++)
            for (int ci = 0; ci < ci_n; ci++)
                for (int k = 0; k < 27; k++) hw[((size_t)co * ci_n + ci) * 27 + k] = dw[((size_t)k * ci_n + ci) * co_n + co];
        for (int co = 0; co < co_n; co++) host[n->boff[l] + co] = dev[n->boff[l] + co];
    }
    return QEDHMC_OK;
}

qedhmc_status qedhmc_net_get_params(qedhmc_net_t n, float* host, int64_t count) {
    if (!n || !host || count != (int64_t)n->nparam) {
        set_error("net: null argument or wrong parameter count");
        return QEDHMC_EINVAL;
    }
    return to_host_layout(n, n->params, host);
}

qedhmc_status qedhmc_net_reset_optimizer(qedhmc_net_t n) {
    if (!n) {
        set_error("net: null argument");
        return QEDHMC_EINVAL;
    }
    QH_HIP(hipMemsetAsync(n->adam_m, 0, n->nparam * sizeof(float), n->h->stream));
    QH_HIP(hipMemsetAsync(n->adam_v, 0, n->nparam * sizeof(float), n->h->stream));
    QH_HIP(hipStreamSynchronize(n->h->stream));
    n->adam_t = 0;
    return QEDHMC_OK;
}

static qedhmc_status net_args(qedhmc_net* n, const void* a, const void* b, qedhmc_net_arith ar) {
    if (!n || !a || !b) {
        set_error("net: null argument");
        return QEDHMC_EINVAL;
    }
    if (ar != QEDHMC_NET_FP32 && ar != QEDHMC_NET_BF16) {
        set_error("net: bad arithmetic");
        return QEDHMC_EINVAL;
    }
    return QEDHMC_OK;
}

qedhmc_status qedhmc_net_apply(qedhmc_net_t n, const double* theta, const double* r, double* z,
                               qedhmc_net_arith a) {
    QH_TRY(net_args(n, theta, r, a));
    if (!z) {
        set_error("net: null output");
        return QEDHMC_EINVAL;
    }
    QH_TRY(net_forward(n, theta, r, a, false));
    hipLaunchKernelGGL(k_net_out, dim3(blocks_for(n->g.N, 256)), dim3(256), 0, n->h->stream, n->g.N,
                       (const float*)n->act[kNetLayers], (const double*)n->dscal, (cplx<double>*)z);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

qedhmc_status qedhmc_net_train_step(qedhmc_net_t n, const double* theta, const double* r, const double* e,
                                    double lr, qedhmc_net_arith a, double* loss, float* grad_host) {
    QH_TRY(net_args(n, theta, r, a));
    if (!e || !loss || !(lr >= 0.0)) {
        set_error("net: bad training arguments");
        return QEDHMC_EINVAL;
    }
    if (a != QEDHMC_NET_FP32) {
        set_error("net: training runs in FP32 arithmetic");
        return QEDHMC_EUNSUPPORTED;
    }
    QH_TRY(net_alloc_train(n));
    const NetGeo& g = n->g;
    hipStream_t st = n->h->stream;
    QH_TRY(net_forward(n, theta, r, a, true));
    QH_TRY(sumsq_to(n, e, 2 * (size_t)g.N, n->dscal + 1));
    // loss and its gradient at the outputs
    hipLaunchKernelGGL(k_net_loss, dim3(kRedBlocks), dim3(256), 0, st, g.N, (const float*)n->act[kNetLayers],
                       (const double*)n->dscal, (const cplx<double>*)e, (const double*)(n->dscal + 1), n->gbuf[0],
                       n->dpart);
    hipLaunchKernelGGL(k_sum1, dim3(1), dim3(64), 0, st, (const double*)n->dpart, kRedBlocks, n->dscal + 2);
    QH_HIP(hipGetLastError());
    QH_TRY(net_backward_adam(n, r, lr, grad_host));
    QH_HIP(hipMemcpyAsync(n->hpin, n->dscal, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
    QH_HIP(hipStreamSynchronize(st));
    *loss = n->hpin[1] > 0.0 ? n->hpin[2] / n->hpin[1] : 0.0;
    return QEDHMC_OK;
}

qedhmc_status qedhmc_net_train_step_residual(qedhmc_net_t n, const double* theta, const double* r, double lr,
                                             qedhmc_net_arith a, double* loss, float* grad_host) {
    QH_TRY(net_args(n, theta, r, a));
    if (!loss || !(lr >= 0.0)) {
        set_error("net: bad training arguments");
        return QEDHMC_EINVAL;
    }
    if (a != QEDHMC_NET_FP32) {
        set_error("net: training runs in FP32 arithmetic");
        return QEDHMC_EUNSUPPORTED;
    }
    QH_TRY(net_alloc_train(n));
    const NetGeo& g = n->g;
    hipStream_t st = n->h->stream;
    QH_TRY(ensure_gauge(n->h, theta, QEDHMC_FP64));
    QH_TRY(net_forward(n, theta, r, a, true));
    // z = s o (FP64), O z, d = O z - r, |d|^2, O d: the FP64 fused M^dag M
    hipLaunchKernelGGL(k_net_out, dim3(blocks_for(g.N, 256)), dim3(256), 0, st, g.N,
                       (const float*)n->act[kNetLayers], (const double*)n->dscal, n->fz);
    QH_HIP(hipGetLastError());
    QH_TRY(launch_mdagm(n->h, QEDHMC_FP64, n->fz, n->fs));
    hipLaunchKernelGGL(k_net_resid, dim3(kRedBlocks), dim3(256), 0, st, g.N, n->fs,
                       reinterpret_cast<const cplx<double>*>(r), n->dpart);
    hipLaunchKernelGGL(k_sum1, dim3(1), dim3(64), 0, st, (const double*)n->dpart, kRedBlocks, n->dscal + 2);
    QH_HIP(hipGetLastError());
    QH_TRY(launch_mdagm(n->h, QEDHMC_FP64, n->fs, n->fp));
    hipLaunchKernelGGL(k_net_resgrad, dim3(blocks_for(g.N, 256)), dim3(256), 0, st, g.N,
                       (const cplx<double>*)n->fp, (const double*)n->dscal, n->gbuf[0]);
    QH_HIP(hipGetLastError());
    QH_TRY(net_backward_adam(n, r, lr, grad_host));
    QH_HIP(hipMemcpyAsync(n->hpin, n->dscal, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
    QH_HIP(hipStreamSynchronize(st));
    *loss = n->hpin[0] > 0.0 ? n->hpin[2] / n->hpin[0] : 0.0;
    return QEDHMC_OK;
}

}  // extern "C"

namespace qh {

// Backward pass from d(loss)/d(outputs) in gbuf[0], then one Adam step.
qedhmc_status net_backward_adam(qedhmc_net* n, const double* r, double lr, float* grad_host) {
    hipStream_t st = n->h->stream;
    // backward through the layers: gbuf alternates between d(loss)/d(pre) of
    // consecutive layers
    int cur = 0;
    for (int l = kNetLayers - 1; l >= 0; l--) {
        const float* gout = n->gbuf[cur];
        QH_TRY(launch_wgrad(n, l, r, gout));
        if (l > 0) {
            QH_TRY(launch_dgrad(n, l, gout, n->gbuf[cur ^ 1]));
            cur ^= 1;
        }
    }
    if (grad_host) QH_TRY(to_host_layout(n, n->grads, grad_host));
    // Adam
    n->adam_t++;
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 - std::pow(b1, n->adam_t)), c2 = (float)(1.0 - std::pow(b2, n->adam_t));
    hipLaunchKernelGGL(k_adam, dim3(blocks_for((int)n->nparam, 256)), dim3(256), 0, st, (int)n->nparam, n->params,
                       (const float*)n->grads, n->adam_m, n->adam_v, (float)lr, (float)b1, (float)b2, 1e-8f, c1, c2);
    QH_HIP(hipGetLastError());
    n->wbf_ready = false;
    n->wf32_ready = false;
    return QEDHMC_OK;
}

}  // namespace qh

extern "C" {

// Flexible CG with the network as preconditioner (see net.hip's header and
// the FCG description): alpha = <p, r> / <p, O p>, beta = -<O p, z'> / <p, O p>;
// the residual judges the network and hands over to the fallback when |r|
// has not at least halved over the last 10 iterations.
qedhmc_status qedhmc_fcg_solve(qedhmc_net_t n, const double* theta, const double* rhs, double* x, double tol,
                               int32_t maxit, qedhmc_net_arith a, qedhmc_precond fallback, int32_t* iters,
                               double* true_rel, int32_t* switched_at) {
    QH_TRY(net_args(n, theta, rhs, a));
    if (!x || !(tol > 0.0) || maxit < 1 || (fallback != QEDHMC_PC_NONE && fallback != QEDHMC_PC_PAPER)) {
        set_error("fcg: bad arguments");
        return QEDHMC_EINVAL;
    }
    qedhmc_ctx* h = n->h;
    hipStream_t st = h->stream;
    const int N = n->g.N;
    const int nb = kRedBlocks;
    cplx<double>* X = reinterpret_cast<cplx<double>*>(x);
    const cplx<double>* B = reinterpret_cast<const cplx<double>*>(rhs);
    if (fallback == QEDHMC_PC_PAPER) QH_TRY(ensure_paper_precond(h));
    // |rhs|
    QH_TRY(launch_sumsq(h, rhs, 2 * (size_t)N, n->dscal + 4));
    QH_HIP(hipMemcpyAsync(n->hpin, n->dscal + 4, sizeof(double), hipMemcpyDeviceToHost, st));
    QH_HIP(hipMemsetAsync(x, 0, (size_t)N * sizeof(cplx<double>), st));
    QH_HIP(hipStreamSynchronize(st));
    const double nb2 = n->hpin[0];
    int it = 0, switched = -1, stalls = 0, last = -1;
    double rel = 0.0;
    if (iters) *iters = 0;
    if (switched_at) *switched_at = -1;
    if (true_rel) *true_rel = 0.0;
    if (nb2 == 0.0) return QEDHMC_OK;
    const double target2 = tol * tol * nb2;
    QH_HIP(hipMemcpyAsync(n->fr, rhs, (size_t)N * sizeof(cplx<double>), hipMemcpyDeviceToDevice, st));
    std::vector<double> hist;
    auto precond = [&](cplx<double>* out) -> qedhmc_status {
        if (switched < 0) {
            QH_TRY(net_forward(n, theta, (const double*)n->fr, a, false, false));
            hipLaunchKernelGGL(k_net_out, dim3(blocks_for(N, 256)), dim3(256), 0, st, N,
                               (const float*)n->act[kNetLayers], (const double*)n->dscal, out);
            QH_HIP(hipGetLastError());
            return QEDHMC_OK;
        }
        if (fallback == QEDHMC_PC_PAPER) return launch_apply_precond_fp32(h, (const double*)n->fr, (double*)out);
        QH_HIP(hipMemcpyAsync(out, n->fr, (size_t)N * sizeof(cplx<double>), hipMemcpyDeviceToDevice, st));
        return QEDHMC_OK;
    };
    auto dots = [&](const cplx<double>* a1, const cplx<double>* b1, const cplx<double>* a2,
                    const cplx<double>* b2) -> qedhmc_status {
        hipLaunchKernelGGL(k_cdot2, dim3(nb), dim3(256), 0, st, N, a1, b1, a2, b2, n->dpart);
        hipLaunchKernelGGL(k_sum4, dim3(1), dim3(64), 0, st, (const double*)n->dpart, nb, n->dscal + 8);
        QH_HIP(hipGetLastError());
        QH_HIP(hipMemcpyAsync(n->hpin, n->dscal + 8, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
        QH_HIP(hipStreamSynchronize(st));
        return QEDHMC_OK;
    };
    // both e^{i theta} caches once: FP64 for O, FP32 for the network's input
    QH_TRY(ensure_gauge(h, theta, QEDHMC_FP64));
    QH_TRY(ensure_gauge(h, theta, QEDHMC_FP32));
    while (true) {
        QH_TRY(precond(n->fp));
        bool broke_for_switch = false;
        while (it < maxit) {
            QH_TRY(launch_mdagm(h, QEDHMC_FP64, n->fp, n->fs, nullptr));
            QH_TRY(dots(n->fp, n->fs, n->fp, n->fr));  // <p, Op>, <p, r>
            const double ps = n->hpin[0];
            if (!(ps > 0.0)) {
                // a direction without descent: the network is not a usable preconditioner here
                if (switched < 0) {
                    switched = it;
                    broke_for_switch = true;
                }
                break;
            }
            const double are = n->hpin[2] / ps, aim = n->hpin[3] / ps;
            hipLaunchKernelGGL(k_fcg_update, dim3(nb), dim3(256), 0, st, N, are, aim, (const cplx<double>*)n->fp,
                               (const cplx<double>*)n->fs, X, n->fr, n->dpart);
            hipLaunchKernelGGL(k_sum4, dim3(1), dim3(64), 0, st, (const double*)n->dpart, nb, n->dscal + 8);
            QH_HIP(hipGetLastError());
            QH_HIP(hipMemcpyAsync(n->hpin, n->dscal + 8, sizeof(double), hipMemcpyDeviceToHost, st));
            QH_HIP(hipStreamSynchronize(st));
            const double rr = n->hpin[0];
            it++;
            hist.push_back(std::sqrt(rr));
            if (!std::isfinite(rr)) break;
            if (switched < 0 && (int)hist.size() > kJudgeWindow &&
                hist.back() > kJudgeFactor * hist[hist.size() - 1 - kJudgeWindow]) {
                switched = it;
                broke_for_switch = true;
                break;
            }
            if (rr <= target2) break;
            QH_TRY(precond(n->fz));
            QH_TRY(dots(n->fs, n->fz, nullptr, nullptr));  // <Op, z'>
            hipLaunchKernelGGL(k_fcg_dir, dim3(nb), dim3(256), 0, st, N, -n->hpin[0] / ps, -n->hpin[1] / ps,
                               (const cplx<double>*)n->fz, n->fp);
            QH_HIP(hipGetLastError());
        }
        if (broke_for_switch) continue;
        // true residual r = rhs - O x (FP64); a restart continues from it
        QH_TRY(launch_mdagm(h, QEDHMC_FP64, x, n->fs, nullptr));
        hipLaunchKernelGGL(k_residual, dim3(nb), dim3(256), 0, st, N, B, (const cplx<double>*)n->fs, n->fr);
        QH_HIP(hipGetLastError());
        QH_TRY(launch_sumsq(h, (const double*)n->fr, 2 * (size_t)N, n->dscal + 5));
        QH_HIP(hipMemcpyAsync(n->hpin, n->dscal + 5, sizeof(double), hipMemcpyDeviceToHost, st));
        QH_HIP(hipStreamSynchronize(st));
        const double t2 = n->hpin[0];
        rel = std::sqrt(t2 / nb2);
        stalls = (it == last) ? stalls + 1 : 0;
        last = it;
        if (!std::isfinite(rel) || t2 <= target2 || it >= maxit || stalls >= 3) break;
    }
    if (iters) *iters = it;
    if (true_rel) *true_rel = rel;
    if (switched_at) *switched_at = switched;
    if (std::isfinite(rel) && rel <= tol) return QEDHMC_OK;
    set_error("fcg: no convergence after " + std::to_string(it) + " iterations (true residual " +
              std::to_string(rel) + ")");
    return QEDHMC_ENOCONV;
}

}  // extern "C"
