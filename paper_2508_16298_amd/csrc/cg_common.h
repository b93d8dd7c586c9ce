// Device and host helpers shared by the CG solvers (cg.hip, pcg.hip).
#pragma once
#include <cmath>
#include <cstdlib>

#include "qedhmc_internal.h"

namespace qh {

// Scalar slot layout (two slots of 16 doubles, by launch parity)
enum {
    S_GPREV = 0,   // gamma_{i-1}
    S_APREV = 1,   // alpha_{i-1}
    S_ITERS = 2,   // completed iterations i
    S_DONE = 3,    // 0 running, 1 stop (target reached / converged), 2 pause for a reliable update,
                   // 3 pause with restart (non-positive <p, O p>), 4 breakdown (non-finite);
                   // the batched driver adds 4 final failure, 5 verified convergence,
                   // 6 iteration budget used (true residual pending)
    S_FIRST = 4,   // 1: next iteration starts a new direction sequence (beta = 0)
    S_B2 = 5,      // |rhs|^2 (FP64); < 0 until the first iteration sets it
    S_TARGET = 6,  // tol^2 |rhs|^2
    S_RRUPD = 7,   // gamma at the last reliable update
    S_ITUPD = 8,   // iteration of the last reliable update
    S_TRUE = 9,    // last FP64 true |r|^2
    S_GCUR = 10,   // gamma_i of the current state
    S_STALL = 11,  // batched driver: consecutive updates without progress
    S_LASTUP = 12, // batched driver: 1 + iteration of the last update (0: none)
    S_NREL = 13,   // batched driver: updates so far
    S_NSLOT = 16,
};
// Record of a solve kept on the device (pipelined drivers of cg.hip and
// pcg.hip): iterations, |rhs|^2 and the latest |r|^2 estimate (the FP64 true
// residual after an update, else the recursion's gamma) after every round;
// from the latest decision the FP64 true |r|^2, the reliable updates so far,
// the state (0 resumed, 4 failed, 5 converged) and, for a failure, its cause.
// Kept at scal + kRecOff, mirrored to pinned host memory at h_pinned + 32
// (two records by round parity).
enum { CR_ITERS = 0, CR_TRUE = 1, CR_B2 = 2, CR_NREL = 3, CR_DONE = 4, CR_WHY = 5, CR_EST = 6, CR_N = 8 };
enum { WHY_BREAKDOWN = 1, WHY_NONFINITE = 2, WHY_BUDGET = 3, WHY_STALL = 4 };
static constexpr int kRecOff = 40;

// Per-slice partials of one parity: <r,r>, <w,r>, <r,s>, <p,w>, <p,s>, aux
// (aux: |rhs|^2 from the start kernel, the FP64 true |r|^2 from a reliable update)
static constexpr int kNP = 6;
static constexpr double kDecade2 = 0.01;  // pause when gamma fell by 10^2 (|r| by 10)
static constexpr int kCap = 50;           // ... or after 50 iterations

template <typename R>
struct CgBufs {
    cplx<R>* r[2];
    cplx<R>* s[2];
    cplx<R>* w[2];
    cplx<R>* p;
    cplx<double>* x;
    const cplx<double>* rhs;
    const cplx<double>* Ox;  // FP64 O x for the true residual
    double* part;            // [2][Nt][kNP] per-slice partials, see kNP
};

// Block reduction of K doubles in a fixed order; result valid in thread 0.
// red: LDS scratch of at least K * 16 doubles.
template <int K>
__device__ __forceinline__ void block_sumk(double (&v)[K], double* red) {
#pragma unroll
    for (int k = 0; k < K; k++) v[k] = wave_sum_f64(v[k]);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 63)
#pragma unroll
        for (int k = 0; k < K; k++) red[K * wv + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
        for (int k = 0; k < K; k++) v[k] = 0.0;
        for (int w = 0; w < nw; w++)
#pragma unroll
            for (int k = 0; k < K; k++) v[k] += red[K * w + k];
    }
}

// The threads of one time slice inside a workgroup.  Single-lattice kernels
// give the whole workgroup to one slice; the batched kernels may pack several
// slices of one chain into a workgroup, each handled by G consecutive threads
// (G = 16, 32 or a multiple of 64) with LDS exchange buffers of its own.
struct Tile {
    int ltid;            // thread index within the group
    int G;               // threads of the group
    bool valid;          // false for a padding group past the chain's last slice
    unsigned char* buf;  // this group's LDS exchange buffers
    double* red;         // LDS scratch shared by the workgroup: kNP * 16 + 16 doubles
};

__device__ __forceinline__ Tile whole_block_tile(unsigned char* buf, double* red) {
    return Tile{(int)threadIdx.x, (int)blockDim.x, true, buf, red};
}

// Sum of K doubles over the threads of a group; the total is valid in the
// group's last thread.  Every thread of the workgroup calls it (groups of 64
// and more meet at workgroup barriers; smaller groups reduce within their
// 16- or 32-lane rows through DPP alone).  Fixed order.
template <int K>
__device__ __forceinline__ void group_sumk(double (&v)[K], const Tile& tl) {
    if (tl.G < 64) {
#pragma unroll
        for (int k = 0; k < K; k++) {
            double x = v[k];
            x += dpp_f64<0xB1, 0xF>(x);
            x += dpp_f64<0x4E, 0xF>(x);
            x += dpp_f64<0x141, 0xF>(x);
            x += dpp_f64<0x140, 0xF>(x);
            if (tl.G == 32) x += dpp_f64<0x142, 0xA>(x);
            v[k] = x;
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < K; k++) v[k] = wave_sum_f64(v[k]);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 63)
#pragma unroll
        for (int k = 0; k < K; k++) tl.red[K * wv + k] = v[k];
    __syncthreads();
    if (tl.ltid == tl.G - 1) {
        const int w0 = (threadIdx.x - tl.ltid) >> 6, nw = tl.G >> 6;
#pragma unroll
        for (int k = 0; k < K; k++) v[k] = 0.0;
        for (int w = 0; w < nw; w++)
#pragma unroll
            for (int k = 0; k < K; k++) v[k] += tl.red[K * (w0 + w) + k];
    }
}

// Sum of the Nt partial tuples of one parity (a chain's: every group of the
// workgroup belongs to it), broadcast to every thread of the workgroup.
__device__ __forceinline__ void reduce_partials(const double* __restrict__ part, int Nt, const Tile& tl,
                                                double (&out)[kNP]) {
    double v[kNP];
#pragma unroll
    for (int k = 0; k < kNP; k++) v[k] = 0.0;
    // tuples t, t + blockDim, ... in that order; up to four of them are
    // loaded before any is added, so a workgroup smaller than Nt waits for
    // memory once rather than once per tuple
    constexpr int U = 4;
    for (int t0 = threadIdx.x; t0 < Nt; t0 += U * blockDim.x) {
        double a[U][kNP];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int t = t0 + u * (int)blockDim.x;
#pragma unroll
            for (int k = 0; k < kNP; k++) a[u][k] = t < Nt ? part[kNP * t + k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; u++)
#pragma unroll
            for (int k = 0; k < kNP; k++) v[k] += a[u][k];
    }
    block_sumk<kNP>(v, tl.red);
    double* bc = tl.red + kNP * 16;
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < kNP; k++) bc[k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kNP; k++) out[k] = bc[k];
}

// The group's partial tuple into pt (skipped for padding groups).
__device__ __forceinline__ void write_partials(double* __restrict__ pt, double (&v)[kNP], const Tile& tl) {
    group_sumk<kNP>(v, tl);
    if (tl.valid && tl.ltid == tl.G - 1)
#pragma unroll
        for (int k = 0; k < kNP; k++) pt[k] = v[k];
}

template <typename R, int MC>
__device__ __forceinline__ double dot_cells(const Cells<R, MC>& a, const Cells<R, MC>& b, const bool (&own)[MC]) {
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < MC; m++)
        if (own[m])
#pragma unroll
            for (int q = 0; q < 4; q++)
                s += (double)a.v[m][q].re * (double)b.v[m][q].re + (double)a.v[m][q].im * (double)b.v[m][q].im;
    return s;
}

// Common per-block setup for the slice kernels.
template <int MC>
struct SliceCtx {
    int tau, tm, tp;
    CellGeo g[MC];
    bool own[MC];
    int idx[MC][12];
};

template <int MC>
__device__ __forceinline__ void slice_ctx(const Lat& lt, SliceCtx<MC>& c, int tau, const Tile& tl) {
    c.tau = tau;
    c.tm = c.tau == 0 ? lt.Nt - 1 : c.tau - 1;
    c.tp = c.tau == lt.Nt - 1 ? 0 : c.tau + 1;
#pragma unroll
    for (int m = 0; m < MC; m++) {
        const int cell = tl.ltid + m * tl.G;
        c.own[m] = tl.valid && cell < lt.ncell;
        c.g[m] = cell_geo(c.own[m] ? cell : 0, lt);
        phase_index(c.g[m], lt.Vs, c.idx[m]);
    }
}

// normalised (tanh-scaled) hops of slice tau, as mdagm_cells takes them
template <typename R, int MC>
__device__ __forceinline__ void hops_of(const cplx<R>* __restrict__ gauge, const Lat& lt, int tau,
                                        const int (&idx)[MC][12], const Coef<R>& co, cplx<R> (&h)[MC][12]) {
#pragma unroll
    for (int m = 0; m < MC; m++) load_hops<R, true>(gauge, lt, tau, idx[m], co, h[m]);
}

// c = (R)(a - b) (b may be null); sq += |a - b|^2 in FP64 over owned cells
template <typename R, int MC>
__device__ __forceinline__ void load_cvt(Cells<R, MC>& c, const cplx<double>* __restrict__ a,
                                         const cplx<double>* __restrict__ b, const CellGeo (&g)[MC],
                                         const bool (&own)[MC], double& sq) {
#pragma unroll
    for (int m = 0; m < MC; m++)
#pragma unroll
        for (int q = 0; q < 4; q++) {
            double re = 0, im = 0;
            if (own[m]) {
                const cplx<double> x = a[g[m].s[q]];
                re = x.re;
                im = x.im;
                if (b) {
                    const cplx<double> y = b[g[m].s[q]];
                    re -= y.re;
                    im -= y.im;
                }
            }
            sq += re * re + im * im;
            c.v[m][q] = mk<R>((R)re, (R)im);
        }
}


template <typename R>
inline const cplx<R>* gauge_for(qedhmc_ctx* h) {
    if constexpr (sizeof(R) == 8)
        return h->gauge64;
    else
        return h->gauge32;
}

template <typename R, typename F>
inline qedhmc_status with_shape(qedhmc_ctx* h, F&& f) {
    const Lat& lt = h->lat;
    const int mc = lt.ncell <= 1024 ? 1 : 2;
    int nt = ((((lt.ncell + mc - 1) / mc) + 63) / 64) * 64;
    if (nt < 64) nt = 64;
    const size_t red = (kNP * 16 + 16) * sizeof(double);
    const bool two = 4 * (size_t)lt.Vs * sizeof(cplx<R>) + red <= h->max_lds;
    if (nt > (mc == 2 ? 576 : 1024)) {
        set_error("the one-slice-per-workgroup kernels hold at most 1152 cells (L <= 66)");
        return QEDHMC_EUNSUPPORTED;
    }
    auto go = [&]<int MC, int BS>() -> qedhmc_status {
        if (two) return f.template operator()<MC, 2, BS>(nt, 4 * (size_t)lt.Vs * sizeof(cplx<R>) + red);
        return f.template operator()<MC, 1, BS>(nt, 2 * (size_t)lt.Vs * sizeof(cplx<R>) + red);
    };
    if (mc == 2) return go.template operator()<2, 576>();
    if (nt <= 256) return go.template operator()<1, 256>();
    if (nt <= 512) return go.template operator()<1, 512>();
    return go.template operator()<1, 1024>();
}

template <typename K>
inline qedhmc_status lds_attr(qedhmc_ctx* h, K kern, size_t bytes) {
    if (bytes > h->max_lds) {
        set_error("lattice too large for LDS on this device");
        return QEDHMC_EUNSUPPORTED;
    }
    if (bytes > 65536) return allow_lds((const void*)kern, h->max_lds);
    return QEDHMC_OK;
}


inline qedhmc_status read_slot(qedhmc_ctx* h, int kpar) {
    QH_HIP(hipMemcpyAsync(h->h_pinned, h->scal + S_NSLOT * kpar, S_NSLOT * sizeof(double), hipMemcpyDeviceToHost,
                          h->stream));
    QH_HIP(hipStreamSynchronize(h->stream));
    return QEDHMC_OK;
}


}  // namespace qh
