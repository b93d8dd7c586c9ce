// Lattice kernels: e^{i theta} caches, bond tables, B_tau, M, M^dag, the
// fused M^dag M and the fermion force.
//
// One workgroup owns one time slice.  Each thread keeps the four site values
// of its 2x2 cells in registers, applies the in-cell families f0 and f2 there
// and exchanges values through LDS only for the cross-cell families f1 and f3
// (four exchanges per B_tau instead of seven full sweeps through memory).
#include <cstdlib>
#include <cstring>

#include "qedhmc_internal.h"

namespace qh {

// computed in FP64, rounded once to the working precision
template <typename R>
static Coef<R> coef_rounded(const qedhmc_params& p) {
    const double h = 0.5 * p.t * p.dtau, c1 = std::cosh(h);
    const double C = c1 * c1 * c1 * c1 * c1 * c1 * std::cosh(2 * h);
    return {(R)c1, (R)std::sinh(h), (R)std::cosh(2 * h), (R)std::sinh(2 * h),
            (R)std::tanh(h), (R)std::tanh(2 * h), (R)C};
}
template <>
Coef<double> coef_of<double>(const qedhmc_params& p) {
    return coef_rounded<double>(p);
}
template <>
Coef<float> coef_of<float>(const qedhmc_params& p) {
    return coef_rounded<float>(p);
}

// ---------------------------------------------------------------------------
// e^{i theta} in the working precision, computed in FP64 and rounded once.
// ---------------------------------------------------------------------------
template <typename R>
__global__ void k_gauge(const double* __restrict__ theta, cplx<R>* __restrict__ g, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        double s, c;
        sincos(theta[i], &s, &c);
        g[i] = mk<R>((R)c, (R)s);
    }
}

static int grid_for(size_t n, int bs) {
    size_t g = (n + bs - 1) / bs;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (int)g;
}

qedhmc_status ensure_gauge(qedhmc_ctx* h, const double* theta, qedhmc_precision prec) {
    const size_t n = (size_t)2 * h->lat.Nt * h->lat.Vs;
    if (prec == QEDHMC_FP64) {
        hipLaunchKernelGGL(k_gauge<double>, dim3(grid_for(n, 256)), dim3(256), 0, h->stream, theta, h->gauge64, n);
        h->gauge_src64 = theta;
    } else {
        hipLaunchKernelGGL(k_gauge<float>, dim3(grid_for(n, 256)), dim3(256), 0, h->stream, theta, h->gauge32, n);
        h->gauge_src32 = theta;
    }
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

// ---------------------------------------------------------------------------
// Bond tables written from the same cell geometry the compute kernels use.
// Row of bond (family f, origin x, y) sits at its rank among the family's
// origins in increasing site order.
// ---------------------------------------------------------------------------
__global__ void k_bond_tables(Lat lt, int32_t* __restrict__ tab) {
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= lt.ncell) return;
    const CellGeo g = cell_geo(cell, lt);
    int idx[12];
    phase_index(g, lt.Vs, idx);
    const int half = lt.Vs / 2;
    const int fam[8] = {0, 0, 1, 1, 2, 2, 3, 3};
    const int org[8] = {g.s[0], g.s[2], g.s[1], g.s[3], g.s[0], g.s[1], g.s[2], g.s[3]};
    const int tgt[8] = {g.s[1], g.s[3], g.r0, g.r2, g.s[2], g.s[3], g.u0, g.u1};
    for (int k = 0; k < 8; k++) {
        const int f = fam[k], i = org[k];
        const int x = i % lt.L, y = i / lt.L;
        const int rank = (f < 2) ? (y * lt.hL + (x >> 1)) : ((y >> 1) * lt.L + x);
        int32_t* row = tab + 3 * ((size_t)f * half + rank);
        row[0] = i;
        row[1] = tgt[k];
        row[2] = idx[k];
    }
}

qedhmc_status launch_bond_tables(qedhmc_ctx* h) {
    const int bs = 256;
    hipLaunchKernelGGL(k_bond_tables, dim3((h->lat.ncell + bs - 1) / bs), dim3(bs), 0, h->stream, h->lat,
                       h->d_tables);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

// ---------------------------------------------------------------------------
// Per-thread cell set setup
// ---------------------------------------------------------------------------
template <int MC>
__device__ __forceinline__ void my_cells(const Lat& lt, CellGeo (&g)[MC], bool (&own)[MC], int (&idx)[MC][12]) {
#pragma unroll
    for (int m = 0; m < MC; m++) {
        const int cell = threadIdx.x + m * blockDim.x;
        own[m] = cell < lt.ncell;
        g[m] = cell_geo(own[m] ? cell : 0, lt);
        phase_index(g[m], lt.Vs, idx[m]);
    }
}

template <typename R, int MC, bool TN = false>
__device__ __forceinline__ void load_hops_all(const cplx<R>* __restrict__ gauge, const Lat& lt, int tau,
                                              const int (&idx)[MC][12], const Coef<R>& co, cplx<R> (&h)[MC][12]) {
#pragma unroll
    for (int m = 0; m < MC; m++) load_hops<R, TN>(gauge, lt, tau, idx[m], co, h[m]);
}

// ---------------------------------------------------------------------------
// out = B_tau in (one slice)
// ---------------------------------------------------------------------------
template <typename R, int MC, int NB, int BS>
__global__ __launch_bounds__(BS) void k_apply_B(Lat lt, int tau, const cplx<R>* __restrict__ in,
                                                  cplx<R>* __restrict__ out, const cplx<R>* __restrict__ gauge,
                                                  Coef<R> co) {
    extern __shared__ __align__(16) unsigned char smem[];
    Xchg<R, NB> xb{reinterpret_cast<cplx<R>*>(smem), lt.Vs, 0};
    CellGeo g[MC];
    bool own[MC];
    int idx[MC][12];
    my_cells<MC>(lt, g, own, idx);
    cplx<R> hp[MC][12];
    load_hops_all<R, MC>(gauge, lt, tau, idx, co, hp);
    Cells<R, MC> c;
    load_cells<R, MC>(c, in, g, own);
    apply_B_cells<R, MC, NB>(c, hp, g, own, co, xb);
    store_cells<R, MC>(c, out, g, own);
}

// ---------------------------------------------------------------------------
// out = M in or M^dag in
//   M:     out_tau = in_tau - eps_{tau-1} B_{tau-1} in_{tau-1}
//   M^dag: out_tau = in_tau - eps_tau     B_tau     in_{tau+1}
// eps_{Nt-1} = -1 (antiperiodic corner), every other eps = +1.
// ---------------------------------------------------------------------------
template <typename R, int MC, int NB, int BS>
__global__ __launch_bounds__(BS) void k_apply_M(Lat lt, int dagger, const cplx<R>* __restrict__ in,
                                                  cplx<R>* __restrict__ out, const cplx<R>* __restrict__ gauge,
                                                  Coef<R> co) {
    extern __shared__ __align__(16) unsigned char smem[];
    Xchg<R, NB> xb{reinterpret_cast<cplx<R>*>(smem), lt.Vs, 0};
    const int tau = slice_of_block(blockIdx.x, lt.Nt), Nt = lt.Nt;
    if (tau < 0) return;
    int src, bsl;
    R sgn;
    if (!dagger) {
        src = tau == 0 ? Nt - 1 : tau - 1;
        bsl = src;
        sgn = tau == 0 ? R(1) : R(-1);
    } else {
        src = tau == Nt - 1 ? 0 : tau + 1;
        bsl = tau;
        sgn = tau == Nt - 1 ? R(1) : R(-1);
    }
    CellGeo g[MC];
    bool own[MC];
    int idx[MC][12];
    my_cells<MC>(lt, g, own, idx);
    cplx<R> hp[MC][12];
    load_hops_all<R, MC>(gauge, lt, bsl, idx, co, hp);
    Cells<R, MC> c, d;
    load_cells<R, MC>(c, in + (size_t)src * lt.Vs, g, own);
    load_cells<R, MC>(d, in + (size_t)tau * lt.Vs, g, own);
    apply_B_cells<R, MC, NB>(c, hp, g, own, co, xb);
#pragma unroll
    for (int m = 0; m < MC; m++)
#pragma unroll
        for (int q = 0; q < 4; q++) d.v[m][q] = cfma(sgn, c.v[m][q], d.v[m][q]);
    store_cells<R, MC>(d, out + (size_t)tau * lt.Vs, g, own);
}

// ---------------------------------------------------------------------------
// Fused out = M^dag M in, slice by slice (mdagm_cells: three B applications,
// the first two together).  gate (nullable): a CG slot's stop flag; the
// launch runs only when it asks for a reliable update.
// ---------------------------------------------------------------------------
template <typename R, int MC, int NB, int BS>
__global__ __launch_bounds__(BS) void k_mdagm(Lat lt, const cplx<R>* __restrict__ in, cplx<R>* __restrict__ out,
                                              const cplx<R>* __restrict__ gauge, Coef<R> co,
                                              const double* __restrict__ gate) {
    if (gate && !gate_open(*gate)) return;
    extern __shared__ __align__(16) unsigned char smem[];
    cplx<R>* buf2 = reinterpret_cast<cplx<R>*>(smem);
    const int tau = slice_of_block(blockIdx.x, lt.Nt), Nt = lt.Nt;
    if (tau < 0) return;
    const int tm = tau == 0 ? Nt - 1 : tau - 1, tp = tau == Nt - 1 ? 0 : tau + 1;
    const R eps_m = tau == 0 ? R(-1) : R(1);
    const R eps_t = tau == Nt - 1 ? R(-1) : R(1);

    CellGeo g[MC];
    bool own[MC];
    int idx[MC][12];
    my_cells<MC>(lt, g, own, idx);
    cplx<R> hm[MC][12], ht[MC][12];
    Cells<R, MC> vm, vt, vn, o;
    load_hops_all<R, MC, true>(gauge, lt, tm, idx, co, hm);
    load_hops_all<R, MC, true>(gauge, lt, tau, idx, co, ht);
    load_cells<R, MC>(vm, in + (size_t)tm * lt.Vs, g, own);
    load_cells<R, MC>(vt, in + (size_t)tau * lt.Vs, g, own);
    load_cells<R, MC>(vn, in + (size_t)tp * lt.Vs, g, own);
    mdagm_cells<R, MC, NB>(vm, vt, vn, hm, ht, g, own, co, eps_m, eps_t, buf2, lt.Vs, o);
    store_cells<R, MC>(o, out + (size_t)tau * lt.Vs, g, own);
}

// ---------------------------------------------------------------------------
// Fermion force (SM SI), one slice per workgroup:
//   F_{b,tau} = 2 Re[ Yt_tau^dag (dB_tau/dtheta_b) X_tau ]
// B_tau = L_m E_m R_m over the seven factors m (E3 E2 E1 E0 E1 E2 E3, m=0..6
// left to right).  u_m = R_m X and w_m = L_m^dag Yt are walked together:
// u_0 = E_1 ... E_6 X is built first, then for m = 0..6 the bonds of factor
// m receive 2 Re[conj(w_i) (i h) u_j + conj(w_j) conj(i h) u_i] with
// h = sinh(a) e^{i theta}, and w_{m+1} = E_m w_m, u_{m+1} = E_{m+1}^{-1} u_m
// (the inverse of a bond block is the block with sinh(a) -> -sinh(a)).
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ R force_term(cplx<R> wi, cplx<R> wj, cplx<R> ui, cplx<R> uj, cplx<R> h) {
    // i h
    const cplx<R> ih = mk<R>(-h.im, h.re);
    // conj(wi) * (ih * uj)
    const cplx<R> a = mk<R>(ih.re * uj.re - ih.im * uj.im, ih.re * uj.im + ih.im * uj.re);
    const R t1 = wi.re * a.re + wi.im * a.im;
    // conj(wj) * (conj(ih) * ui)
    const cplx<R> b = mk<R>(ih.re * ui.re + ih.im * ui.im, ih.re * ui.im - ih.im * ui.re);
    const R t2 = wj.re * b.re + wj.im * b.im;
    return R(2) * (t1 + t2);
}

template <typename R, int MC>
__device__ __forceinline__ void publish(const Cells<R, MC>& c, cplx<R>* b, const CellGeo (&g)[MC],
                                        const bool (&own)[MC]) {
#pragma unroll
    for (int m = 0; m < MC; m++)
        if (own[m]) {
#pragma unroll
            for (int q = 0; q < 4; q++) b[g[m].s[q]] = c.v[m][q];
        }
}

// One force step for factor position m (family f) followed by the w / u moves.
template <typename R, int MC>
__device__ __forceinline__ void force_step(int f, bool last, int fnext, Cells<R, MC>& u, Cells<R, MC>& w,
                                           const cplx<R> (&hp)[MC][12], const cplx<R> (&hn)[MC][12],
                                           const CellGeo (&g)[MC], const bool (&own)[MC], const Coef<R>& co,
                                           cplx<R>* bu, cplx<R>* bw, R (&Fa)[MC][8]) {
    const R cc = f == 0 ? co.c2 : co.c1;
    if (f == 0 || f == 2) {
#pragma unroll
        for (int m = 0; m < MC; m++) {
            const cplx<R>* v = u.v[m];
            const cplx<R>* x = w.v[m];
            if (f == 0) {
                Fa[m][0] += force_term(x[0], x[1], v[0], v[1], hp[m][0]);
                Fa[m][1] += force_term(x[2], x[3], v[2], v[3], hp[m][1]);
                if (!last) sweep_f0(w.v[m], hp[m], cc);
            } else {
                Fa[m][4] += force_term(x[0], x[2], v[0], v[2], hp[m][4]);
                Fa[m][5] += force_term(x[1], x[3], v[1], v[3], hp[m][5]);
                if (!last) sweep_f2(w.v[m], hp[m], cc);
            }
        }
    } else {
        publish<R, MC>(u, bu, g, own);
        publish<R, MC>(w, bw, g, own);
        __syncthreads();
#pragma unroll
        for (int m = 0; m < MC; m++)
            if (own[m]) {
                const cplx<R>* v = u.v[m];
                const cplx<R>* x = w.v[m];
                if (f == 1) {
                    Fa[m][2] += force_term(x[1], bw[g[m].r0], v[1], bu[g[m].r0], hp[m][2]);
                    Fa[m][3] += force_term(x[3], bw[g[m].r2], v[3], bu[g[m].r2], hp[m][3]);
                    if (!last) sweep_f1(w.v[m], hp[m], cc, bw[g[m].r0], bw[g[m].r2], bw[g[m].l1], bw[g[m].l3]);
                } else {
                    Fa[m][6] += force_term(x[2], bw[g[m].u0], v[2], bu[g[m].u0], hp[m][6]);
                    Fa[m][7] += force_term(x[3], bw[g[m].u1], v[3], bu[g[m].u1], hp[m][7]);
                    if (!last) sweep_f3(w.v[m], hp[m], cc, bw[g[m].u0], bw[g[m].u1], bw[g[m].d2], bw[g[m].d3]);
                }
            }
        __syncthreads();
    }
    if (last) return;
    // u <- E_{m+1}^{-1} u
    const R cn = fnext == 0 ? co.c2 : co.c1;
    if (fnext == 0) {
#pragma unroll
        for (int m = 0; m < MC; m++) sweep_f0(u.v[m], hn[m], cn);
    } else if (fnext == 2) {
#pragma unroll
        for (int m = 0; m < MC; m++) sweep_f2(u.v[m], hn[m], cn);
    } else {
        publish<R, MC>(u, bu, g, own);
        __syncthreads();
#pragma unroll
        for (int m = 0; m < MC; m++)
            if (own[m]) {
                if (fnext == 1)
                    sweep_f1(u.v[m], hn[m], cn, bu[g[m].r0], bu[g[m].r2], bu[g[m].l1], bu[g[m].l3]);
                else
                    sweep_f3(u.v[m], hn[m], cn, bu[g[m].u0], bu[g[m].u1], bu[g[m].d2], bu[g[m].d3]);
            }
        __syncthreads();
    }
}

template <typename R, int MC, int BS>
__global__ __launch_bounds__(BS) void k_force(Lat lt, const cplx<R>* __restrict__ X, const cplx<R>* __restrict__ Y,
                                                const cplx<R>* __restrict__ gauge, Coef<R> co,
                                                double* __restrict__ F) {
    extern __shared__ __align__(16) unsigned char smem[];
    cplx<R>* bu = reinterpret_cast<cplx<R>*>(smem);
    cplx<R>* bw = bu + lt.Vs;
    const int tau = slice_of_block(blockIdx.x, lt.Nt), Nt = lt.Nt;
    if (tau < 0) return;
    const int tn = tau == Nt - 1 ? 0 : tau + 1;
    const R sg = tau == Nt - 1 ? R(1) : R(-1);

    CellGeo g[MC];
    bool own[MC];
    int idx[MC][12];
    my_cells<MC>(lt, g, own, idx);
    cplx<R> hp[MC][12], hn[MC][12];
    load_hops_all<R, MC>(gauge, lt, tau, idx, co, hp);
#pragma unroll
    for (int m = 0; m < MC; m++)
#pragma unroll
        for (int k = 0; k < 12; k++) hn[m][k] = mk<R>(-hp[m][k].re, -hp[m][k].im);
    Cells<R, MC> u, w;
    load_cells<R, MC>(u, X + (size_t)tau * lt.Vs, g, own);
    load_cells<R, MC>(w, Y + (size_t)tn * lt.Vs, g, own);
#pragma unroll
    for (int m = 0; m < MC; m++)
#pragma unroll
        for (int q = 0; q < 4; q++) w.v[m][q] = cscale(sg, w.v[m][q]);

    // u_0 = E_1 E_2 E_3 E_4 E_5 E_6 X : apply m = 6 (f3), 5 (f2), 4 (f1), 3 (f0), 2 (f1), 1 (f2)
    Xchg<R, 1> xb{bu, lt.Vs, 0};
    cross_sweep<R, MC, 1, false>(u, hp, g, own, co.c1, xb);
#pragma unroll
    for (int m = 0; m < MC; m++) sweep_f2(u.v[m], hp[m], co.c1);
    cross_sweep<R, MC, 1, true>(u, hp, g, own, co.c1, xb);
#pragma unroll
    for (int m = 0; m < MC; m++) sweep_f0(u.v[m], hp[m], co.c2);
    cross_sweep<R, MC, 1, true>(u, hp, g, own, co.c1, xb);
#pragma unroll
    for (int m = 0; m < MC; m++) sweep_f2(u.v[m], hp[m], co.c1);

    R Fa[MC][8];
#pragma unroll
    for (int m = 0; m < MC; m++)
#pragma unroll
        for (int k = 0; k < 8; k++) Fa[m][k] = R(0);
    const int fam[7] = {3, 2, 1, 0, 1, 2, 3};
#pragma unroll
    for (int p = 0; p < 7; p++)
        force_step<R, MC>(fam[p], p == 6, p < 6 ? fam[p + 1] : 0, u, w, hp, hn, g, own, co, bu, bw, Fa);

#pragma unroll
    for (int m = 0; m < MC; m++)
        if (own[m]) {
#pragma unroll
            for (int k = 0; k < 8; k++) {
                const int id = idx[m][k];
                const int d = id >= lt.Vs ? 1 : 0;
                const int s = id - d * lt.Vs;
                F[((size_t)d * Nt + tau) * lt.Vs + s] = (double)Fa[m][k];
            }
        }
}

// ---------------------------------------------------------------------------
// Launch configuration: one workgroup per slice; MC cells per thread and a
// block-size bound BS chosen so that small lattices get the full register
// file per thread (BS = 256) and L = 66 still fits (MC = 2, BS = 576).
// ---------------------------------------------------------------------------
struct Shape {
    int mc, nt, bs;
};

static Shape shape_of(const Lat& lt) {
    Shape s;
    s.mc = lt.ncell <= 1024 ? 1 : 2;
    const int per = (lt.ncell + s.mc - 1) / s.mc;
    s.nt = ((per + 63) / 64) * 64;
    if (s.nt < 64) s.nt = 64;
    s.bs = s.mc == 2 ? 576 : (s.nt <= 256 ? 256 : (s.nt <= 512 ? 512 : 1024));
    return s;
}

template <typename K>
static qedhmc_status allow_lds(qedhmc_ctx* h, K kern, size_t bytes) {
    if (bytes > h->max_lds) {
        set_error("lattice too large for LDS on this device (" + std::to_string(bytes) + " B needed)");
        return QEDHMC_EUNSUPPORTED;
    }
    if (bytes > 65536) QH_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                  (int)bytes));
    return QEDHMC_OK;
}

template <typename R>
static const cplx<R>* gauge_of(qedhmc_ctx* h);
template <>
const cplx<double>* gauge_of<double>(qedhmc_ctx* h) {
    return h->gauge64;
}
template <>
const cplx<float>* gauge_of<float>(qedhmc_ctx* h) {
    return h->gauge32;
}

// Calls f.template operator()<MC, BS>() for the shape of this lattice.
template <typename F>
static qedhmc_status dispatch_shape(const Shape& s, F&& f) {
    if (s.nt > (s.mc == 2 ? 576 : 1024)) {
        set_error("the one-slice-per-workgroup kernels hold at most 1152 cells (L <= 66)");
        return QEDHMC_EUNSUPPORTED;
    }
    if (s.mc == 2) return f.template operator()<2, 576>();
    if (s.bs == 256) return f.template operator()<1, 256>();
    if (s.bs == 512) return f.template operator()<1, 512>();
    return f.template operator()<1, 1024>();
}

template <typename R>
static qedhmc_status mdagm_t(qedhmc_ctx* h, const void* in, void* out, const double* gate) {
    const Shape s = shape_of(h->lat);
    const size_t red = 32 * sizeof(double);
    const bool two = 4 * h->lat.Vs * sizeof(cplx<R>) + red <= h->max_lds;
    return dispatch_shape(s, [&]<int MC, int BS>() -> qedhmc_status {
        auto run = [&]<int NB>() -> qedhmc_status {
            const size_t lds = (size_t)NB * 2 * h->lat.Vs * sizeof(cplx<R>) + red;
            QH_TRY(allow_lds(h, k_mdagm<R, MC, NB, BS>, lds));
            hipEvent_t e0, e1;
            if (prof_sample(h, sizeof(R) == 4 ? QEDHMC_K_MDAGM_FP32 : QEDHMC_K_MDAGM_FP64, e0, e1))
                hipExtLaunchKernelGGL((k_mdagm<R, MC, NB, BS>), dim3(slice_grid(h->lat.Nt)), dim3(s.nt), lds, h->stream, e0, e1,
                                      0, h->lat, (const cplx<R>*)in, (cplx<R>*)out, gauge_of<R>(h),
                                      coef_of<R>(h->p), gate);
            else
                hipLaunchKernelGGL((k_mdagm<R, MC, NB, BS>), dim3(slice_grid(h->lat.Nt)), dim3(s.nt), lds, h->stream, h->lat,
                                   (const cplx<R>*)in, (cplx<R>*)out, gauge_of<R>(h), coef_of<R>(h->p), gate);
            QH_HIP(hipGetLastError());
            return QEDHMC_OK;
        };
        return two ? run.template operator()<2>() : run.template operator()<1>();
    });
}

// The tiled streaming kernel serves slices past the whole-slice kernels'
// reach and every slice of more than kTiledFrom cells; QEDHMC_MDAGM=slice or
// =tiled (read per call) forces one form where it can run.
static constexpr int kTiledFrom = 1024;

static bool use_tiled(const qedhmc_ctx* h, const double* gate) {
    if (gate) return false;
    const bool fits = h->lat.ncell <= 1152;
    const char* e = std::getenv("QEDHMC_MDAGM");
    if (e && std::strcmp(e, "slice") == 0 && fits) return false;
    if (e && std::strcmp(e, "tiled") == 0) return true;
    return !fits || h->lat.ncell > kTiledFrom;
}

qedhmc_status launch_mdagm(qedhmc_ctx* h, qedhmc_precision prec, const void* in, void* out, const double* gate) {
    if (use_tiled(h, gate)) return launch_mdagm_tiled(h, prec, in, out);
    return prec == QEDHMC_FP64 ? mdagm_t<double>(h, in, out, gate) : mdagm_t<float>(h, in, out, gate);
}

template <typename R>
static qedhmc_status M_t(qedhmc_ctx* h, const void* in, void* out, int dagger) {
    const Shape s = shape_of(h->lat);
    const bool two = 2 * h->lat.Vs * sizeof(cplx<R>) <= h->max_lds;
    return dispatch_shape(s, [&]<int MC, int BS>() -> qedhmc_status {
        auto run = [&]<int NB>() -> qedhmc_status {
            const size_t lds = (size_t)NB * h->lat.Vs * sizeof(cplx<R>);
            QH_TRY(allow_lds(h, k_apply_M<R, MC, NB, BS>, lds));
            hipLaunchKernelGGL((k_apply_M<R, MC, NB, BS>), dim3(slice_grid(h->lat.Nt)), dim3(s.nt), lds, h->stream, h->lat,
                               dagger, (const cplx<R>*)in, (cplx<R>*)out, gauge_of<R>(h), coef_of<R>(h->p));
            QH_HIP(hipGetLastError());
            return QEDHMC_OK;
        };
        return two ? run.template operator()<2>() : run.template operator()<1>();
    });
}

qedhmc_status launch_apply_M(qedhmc_ctx* h, qedhmc_precision prec, const void* in, void* out, int dagger) {
    return prec == QEDHMC_FP64 ? M_t<double>(h, in, out, dagger) : M_t<float>(h, in, out, dagger);
}

template <typename R>
static qedhmc_status B_t(qedhmc_ctx* h, int tau, const void* in, void* out) {
    const Shape s = shape_of(h->lat);
    return dispatch_shape(s, [&]<int MC, int BS>() -> qedhmc_status {
        const size_t lds = (size_t)h->lat.Vs * sizeof(cplx<R>);
        QH_TRY(allow_lds(h, k_apply_B<R, MC, 1, BS>, lds));
        hipLaunchKernelGGL((k_apply_B<R, MC, 1, BS>), dim3(1), dim3(s.nt), lds, h->stream, h->lat, tau,
                           (const cplx<R>*)in, (cplx<R>*)out, gauge_of<R>(h), coef_of<R>(h->p));
        QH_HIP(hipGetLastError());
        return QEDHMC_OK;
    });
}

qedhmc_status launch_apply_B(qedhmc_ctx* h, qedhmc_precision prec, int tau, const void* in, void* out) {
    return prec == QEDHMC_FP64 ? B_t<double>(h, tau, in, out) : B_t<float>(h, tau, in, out);
}

// X (FP64 complex) -> working precision, Y = M X, then the force kernel.
template <typename R>
__global__ void k_to_prec(const cplx<double>* __restrict__ a, cplx<R>* __restrict__ b, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b[i] = mk<R>((R)a[i].re, (R)a[i].im);
}

template <typename R>
static qedhmc_status force_t(qedhmc_ctx* h, const void* X, const void* Y, double* F) {
    const Shape s = shape_of(h->lat);
    return dispatch_shape(s, [&]<int MC, int BS>() -> qedhmc_status {
        const size_t lds = (size_t)2 * h->lat.Vs * sizeof(cplx<R>);
        QH_TRY(allow_lds(h, k_force<R, MC, BS>, lds));
        hipEvent_t e0, e1;
        if (prof_sample(h, QEDHMC_K_FORCE, e0, e1))
            hipExtLaunchKernelGGL((k_force<R, MC, BS>), dim3(slice_grid(h->lat.Nt)), dim3(s.nt), lds, h->stream, e0, e1, 0,
                                  h->lat, (const cplx<R>*)X, (const cplx<R>*)Y, gauge_of<R>(h), coef_of<R>(h->p), F);
        else
            hipLaunchKernelGGL((k_force<R, MC, BS>), dim3(slice_grid(h->lat.Nt)), dim3(s.nt), lds, h->stream, h->lat,
                               (const cplx<R>*)X, (const cplx<R>*)Y, gauge_of<R>(h), coef_of<R>(h->p), F);
        QH_HIP(hipGetLastError());
        return QEDHMC_OK;
    });
}

qedhmc_status launch_force(qedhmc_ctx* h, qedhmc_precision prec, const double* X, double* F) {
    const size_t N = (size_t)h->lat.Nt * h->lat.Vs;
    if (prec == QEDHMC_FP64) {
        void* Y = h->ws[10];
        QH_TRY(launch_apply_M(h, prec, X, Y, 0));
        return force_t<double>(h, X, Y, F);
    }
    void* Xs = h->ws[10];
    void* Y = h->ws[11];
    hipLaunchKernelGGL(k_to_prec<float>, dim3(grid_for(N, 256)), dim3(256), 0, h->stream, (const cplx<double>*)X,
                       (cplx<float>*)Xs, N);
    QH_HIP(hipGetLastError());
    QH_TRY(launch_apply_M(h, prec, Xs, Y, 0));
    return force_t<float>(h, Xs, Y, F);
}

}  // namespace qh
