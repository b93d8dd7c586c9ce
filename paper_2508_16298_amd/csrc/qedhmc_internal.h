// Internal declarations shared by the HIP translation units of libqedhmc.
//
// Device data layouts
//   theta    double [2][Nt][Vs]                 (caller's buffer)
//   gauge    cplx<R> [2][Nt][Vs] = e^{i theta}  (handle workspace, one per
//            working precision, rebuilt whenever theta changes)
//   vectors  cplx<R> [Nt][Vs]
//
// Cell decomposition used by every lattice kernel: the L x L slice is tiled
// by 2x2 cells (a, b) holding sites
//   0: (2a, 2b)   1: (2a+1, 2b)   2: (2a, 2b+1)   3: (2a+1, 2b+1).
// Bond families f0 (x-bonds leaving even x) and f2 (y-bonds leaving even y)
// then lie inside a cell, and f1 / f3 join a cell to its +x / +y neighbour.
// A thread keeps the four site values of its cells in registers; only the
// f1 / f3 sweeps exchange values, through LDS.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "qedhmc.h"

namespace qh {

template <typename R>
struct alignas(2 * sizeof(R)) cplx {
    R re, im;
};

template <typename R>
__host__ __device__ __forceinline__ cplx<R> mk(R a, R b) {
    cplx<R> z;
    z.re = a;
    z.im = b;
    return z;
}

// c v + h w
template <typename R>
__device__ __forceinline__ cplx<R> rv_plus_hw(R c, cplx<R> v, cplx<R> h, cplx<R> w) {
    return mk<R>(c * v.re + (h.re * w.re - h.im * w.im), c * v.im + (h.re * w.im + h.im * w.re));
}
// c v + conj(h) w
template <typename R>
__device__ __forceinline__ cplx<R> rv_plus_hcw(R c, cplx<R> v, cplx<R> h, cplx<R> w) {
    return mk<R>(c * v.re + (h.re * w.re + h.im * w.im), c * v.im + (h.re * w.im - h.im * w.re));
}
template <typename R>
__device__ __forceinline__ cplx<R> cadd(cplx<R> a, cplx<R> b) { return mk<R>(a.re + b.re, a.im + b.im); }
template <typename R>
__device__ __forceinline__ cplx<R> csub(cplx<R> a, cplx<R> b) { return mk<R>(a.re - b.re, a.im - b.im); }
template <typename R>
__device__ __forceinline__ cplx<R> cscale(R s, cplx<R> a) { return mk<R>(s * a.re, s * a.im); }
template <typename R>
__device__ __forceinline__ cplx<R> cfma(R s, cplx<R> a, cplx<R> b) { return mk<R>(s * a.re + b.re, s * a.im + b.im); }

// Lattice constants passed by value to every kernel.
struct Lat {
    int L, Nt, Vs, hL, ncell;  // hL = L/2, ncell = hL*hL
};

// Slice of a workgroup in the one-slice-per-workgroup kernels.  Workgroups
// are dealt to the eight XCDs round robin (workgroup i runs on XCD i mod 8),
// and every stencil kernel reads the tau -+ 1 neighbours of its slice; dealing
// the slices out in eight contiguous ranges keeps a slice and its neighbours
// on one XCD, so the neighbour reads hit that XCD's L2.  Grids have
// slice_grid(Nt) workgroups; the surplus ones get -1 and exit at once.
__host__ __device__ __forceinline__ int slice_grid(int Nt) { return 8 * ((Nt + 7) / 8); }
__device__ __forceinline__ int slice_of_block(int b, int Nt) {
    const int per = (Nt + 7) >> 3;
    const int tau = (b & 7) * per + (b >> 3);
    return tau < Nt ? tau : -1;
}

// Hopping coefficients of one bond factor: cosh/sinh of the half step h and
// of the merged central step 2h (Eq. 24); and the normalised form used by the
// fused M^dag M: every site lies on exactly one bond of each family, so each
// factor is cosh(a) times (v_i, v_j) -> (v_i + tanh(a) e^{i theta} v_j,
// v_j + tanh(a) e^{-i theta} v_i), and B_tau = C B'_tau with
// C = cosh(h)^6 cosh(2h).
template <typename R>
struct Coef {
    R c1, s1, c2, s2;
    R t1, t2, C;  // tanh(h), tanh(2h), cosh(h)^6 cosh(2h)
};

// Static geometry of one 2x2 cell (site indices inside a slice).
struct CellGeo {
    int s[4];                // own sites 0..3
    int r0, r2;              // +x neighbour's sites 0 and 2
    int l1, l3;              // -x neighbour's sites 1 and 3
    int u0, u1;              // +y neighbour's sites 0 and 1
    int d2, d3;              // -y neighbour's sites 2 and 3
    int c;                   // own cell index (cy * L/2 + cx)
    int xp, xm, yp, ym;      // cell indices of the four neighbour cells
};

__device__ __forceinline__ int wrap(int x, int L) { return x < 0 ? x + L : (x >= L ? x - L : x); }

__device__ __forceinline__ CellGeo cell_geo(int cell, const Lat& lt) {
    const int a = cell % lt.hL, b = cell / lt.hL, L = lt.L;
    const int x0 = 2 * a, y0 = 2 * b;
    CellGeo g;
    g.s[0] = y0 * L + x0;
    g.s[1] = g.s[0] + 1;
    g.s[2] = g.s[0] + L;
    g.s[3] = g.s[2] + 1;
    const int xr = wrap(x0 + 2, L), xl = wrap(x0 - 1, L);
    const int yu = wrap(y0 + 2, L), yd = wrap(y0 - 1, L);
    g.r0 = y0 * L + xr;
    g.r2 = (y0 + 1) * L + xr;
    g.l1 = y0 * L + xl;
    g.l3 = (y0 + 1) * L + xl;
    g.u0 = yu * L + x0;
    g.u1 = yu * L + x0 + 1;
    g.d2 = yd * L + x0;
    g.d3 = yd * L + x0 + 1;
    const int h = lt.hL;
    g.c = cell;
    g.xp = b * h + (a + 1 == h ? 0 : a + 1);
    g.xm = b * h + (a == 0 ? h - 1 : a - 1);
    g.yp = (b + 1 == h ? 0 : b + 1) * h + a;
    g.ym = (b == 0 ? h - 1 : b - 1) * h + a;
    return g;
}

// The twelve bond phases a cell needs for one slice, index -> (d, site):
//   0,1  f0 bonds from sites 0, 2 (d=0)       pairs (0,1), (2,3)
//   2,3  f1 bonds from sites 1, 3 (d=0)       pairs (1, r0), (3, r2)
//   4,5  f2 bonds from sites 0, 1 (d=1)       pairs (0,2), (1,3)
//   6,7  f3 bonds from sites 2, 3 (d=1)       pairs (2, u0), (3, u1)
//   8,9  f1 bonds from l1, l3 (d=0)           pairs (l1, 0), (l3, 2)
//   10,11 f3 bonds from d2, d3 (d=1)          pairs (d2, 0), (d3, 1)
__device__ __forceinline__ void phase_index(const CellGeo& g, int Vs, int (&idx)[12]) {
    idx[0] = g.s[0];
    idx[1] = g.s[2];
    idx[2] = g.s[1];
    idx[3] = g.s[3];
    idx[4] = Vs + g.s[0];
    idx[5] = Vs + g.s[1];
    idx[6] = Vs + g.s[2];
    idx[7] = Vs + g.s[3];
    idx[8] = g.l1;
    idx[9] = g.l3;
    idx[10] = Vs + g.d2;
    idx[11] = Vs + g.d3;
}

// Load the scaled hopping terms h_k = sinh(a_k) e^{i theta_k} of one slice
// (TN: tanh(a_k) e^{i theta_k}, the normalised factors): gauge is
// [2][Nt][Vs]; idx (from phase_index) packs d*Vs + s.
template <typename R, bool TN = false>
__device__ __forceinline__ void load_hops(const cplx<R>* __restrict__ gauge, const Lat& lt, int tau,
                                          const int (&idx)[12], const Coef<R>& co, cplx<R> (&h)[12]) {
#pragma unroll
    for (int k = 0; k < 12; k++) {
        const int id = idx[k];
        const int d = id >= lt.Vs ? 1 : 0;
        const int s = id - d * lt.Vs;
        const cplx<R> e = gauge[((size_t)d * lt.Nt + tau) * lt.Vs + s];
        const R sc = TN ? ((k < 2) ? co.t2 : co.t1) : ((k < 2) ? co.s2 : co.s1);
        h[k] = mk<R>(sc * e.re, sc * e.im);
    }
}

// In-cell factor of family f0 (merged central step, coefficients c2/h[0..1]).
template <typename R>
__device__ __forceinline__ void sweep_f0(cplx<R> (&v)[4], const cplx<R> (&h)[12], R c) {
    const cplx<R> a0 = v[0], a1 = v[1], a2 = v[2], a3 = v[3];
    v[0] = rv_plus_hw(c, a0, h[0], a1);
    v[1] = rv_plus_hcw(c, a1, h[0], a0);
    v[2] = rv_plus_hw(c, a2, h[1], a3);
    v[3] = rv_plus_hcw(c, a3, h[1], a2);
}
// In-cell factor of family f2.
template <typename R>
__device__ __forceinline__ void sweep_f2(cplx<R> (&v)[4], const cplx<R> (&h)[12], R c) {
    const cplx<R> a0 = v[0], a1 = v[1], a2 = v[2], a3 = v[3];
    v[0] = rv_plus_hw(c, a0, h[4], a2);
    v[2] = rv_plus_hcw(c, a2, h[4], a0);
    v[1] = rv_plus_hw(c, a1, h[5], a3);
    v[3] = rv_plus_hcw(c, a3, h[5], a1);
}
// Cross-cell factor of family f1 given the neighbours' (pre-sweep) values.
template <typename R>
__device__ __forceinline__ void sweep_f1(cplx<R> (&v)[4], const cplx<R> (&h)[12], R c, cplx<R> R0,
                                         cplx<R> R2, cplx<R> L1, cplx<R> L3) {
    const cplx<R> a0 = v[0], a1 = v[1], a2 = v[2], a3 = v[3];
    v[1] = rv_plus_hw(c, a1, h[2], R0);
    v[3] = rv_plus_hw(c, a3, h[3], R2);
    v[0] = rv_plus_hcw(c, a0, h[8], L1);
    v[2] = rv_plus_hcw(c, a2, h[9], L3);
}
// Cross-cell factor of family f3.
template <typename R>
__device__ __forceinline__ void sweep_f3(cplx<R> (&v)[4], const cplx<R> (&h)[12], R c, cplx<R> U0,
                                         cplx<R> U1, cplx<R> D2, cplx<R> D3) {
    const cplx<R> a0 = v[0], a1 = v[1], a2 = v[2], a3 = v[3];
    v[2] = rv_plus_hw(c, a2, h[6], U0);
    v[3] = rv_plus_hw(c, a3, h[7], U1);
    v[0] = rv_plus_hcw(c, a0, h[10], D2);
    v[1] = rv_plus_hcw(c, a1, h[11], D3);
}

// Per-thread cell set: thread t owns cells t, t + blockDim, ... (at most MC).
template <typename R, int MC>
struct Cells {
    cplx<R> v[MC][4];
};

// LDS exchange buffers: NB buffers of Vs complex values each.  With NB = 2
// consecutive cross sweeps alternate buffers, so one barrier per sweep is
// enough (a buffer is rewritten only after a barrier that follows every read
// of its previous contents).  With NB = 1 a second barrier closes each sweep.
template <typename R, int NB>
struct Xchg {
    cplx<R>* buf;
    int Vs;
    int k;  // next buffer
    __device__ cplx<R>* next() {
        cplx<R>* b = buf + (size_t)(NB == 2 ? k : 0) * Vs;
        k ^= 1;
        return b;
    }
};

template <int NB>
__device__ __forceinline__ void xchg_close() {
    if (NB == 1) __syncthreads();
}

// Apply one cross family (f1 if X, else f3) to all cells of this thread.
template <typename R, int MC, int NB, bool X>
__device__ __forceinline__ void cross_sweep(Cells<R, MC>& c, const cplx<R> (&h)[MC][12], const CellGeo (&g)[MC],
                                            const bool (&own)[MC], R cc, Xchg<R, NB>& xb) {
    cplx<R>* b = xb.next();
#pragma unroll
    for (int m = 0; m < MC; m++)
        if (own[m]) {
#pragma unroll
            for (int q = 0; q < 4; q++) b[g[m].s[q]] = c.v[m][q];
        }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < MC; m++)
        if (own[m]) {
            if (X)
                sweep_f1(c.v[m], h[m], cc, b[g[m].r0], b[g[m].r2], b[g[m].l1], b[g[m].l3]);
            else
                sweep_f3(c.v[m], h[m], cc, b[g[m].u0], b[g[m].u1], b[g[m].d2], b[g[m].d3]);
        }
    xchg_close<NB>();
}

// B_tau on the cells of this thread: factors applied in the order
// E3, E2, E1, E0(2h), E1, E2, E3 (the product is a palindrome).
template <typename R, int MC, int NB>
__device__ __forceinline__ void apply_B_cells(Cells<R, MC>& c, const cplx<R> (&h)[MC][12], const CellGeo (&g)[MC],
                                              const bool (&own)[MC], const Coef<R>& co, Xchg<R, NB>& xb) {
    cross_sweep<R, MC, NB, false>(c, h, g, own, co.c1, xb);
#pragma unroll
    for (int m = 0; m < MC; m++) sweep_f2(c.v[m], h[m], co.c1);
    cross_sweep<R, MC, NB, true>(c, h, g, own, co.c1, xb);
#pragma unroll
    for (int m = 0; m < MC; m++) sweep_f0(c.v[m], h[m], co.c2);
    cross_sweep<R, MC, NB, true>(c, h, g, own, co.c1, xb);
#pragma unroll
    for (int m = 0; m < MC; m++) sweep_f2(c.v[m], h[m], co.c1);
    cross_sweep<R, MC, NB, false>(c, h, g, own, co.c1, xb);
}

// ---------------------------------------------------------------------------
// The fused M^dag M in normalised factors (tanh-scaled hops from
// load_hops<R, true>): four FMAs per site and sweep, C folded into the
// combinations.  Exchange buffers hold the four sites of every cell as four
// planes (site q of cell c at q * ncell + c), so a wavefront's writes and each
// of its neighbour reads are contiguous.
// ---------------------------------------------------------------------------
// v + h w and v + conj(h) w
template <typename R>
__device__ __forceinline__ cplx<R> add_hw(cplx<R> v, cplx<R> h, cplx<R> w) {
    return mk<R>(v.re + h.re * w.re - h.im * w.im, v.im + h.re * w.im + h.im * w.re);
}
template <typename R>
__device__ __forceinline__ cplx<R> add_hcw(cplx<R> v, cplx<R> h, cplx<R> w) {
    return mk<R>(v.re + h.re * w.re + h.im * w.im, v.im + h.re * w.im - h.im * w.re);
}

// In-cell normalised factor: f0 (F = 0, pairs (0,1), (2,3)) or f2 (F = 2,
// pairs (0,2), (1,3)).
template <typename R, int F>
__device__ __forceinline__ void sweep_in_n(cplx<R> (&v)[4], const cplx<R> (&h)[12]) {
    const cplx<R> a0 = v[0], a1 = v[1], a2 = v[2], a3 = v[3];
    if constexpr (F == 0) {
        v[0] = add_hw(a0, h[0], a1);
        v[1] = add_hcw(a1, h[0], a0);
        v[2] = add_hw(a2, h[1], a3);
        v[3] = add_hcw(a3, h[1], a2);
    } else {
        v[0] = add_hw(a0, h[4], a2);
        v[2] = add_hcw(a2, h[4], a0);
        v[1] = add_hw(a1, h[5], a3);
        v[3] = add_hcw(a3, h[5], a1);
    }
}

// Cross-cell normalised factor f1 (X) or f3 of one cell, the neighbours'
// pre-sweep values read from the plane buffer b.
template <typename R, bool X>
__device__ __forceinline__ void sweep_cross_n(cplx<R> (&v)[4], const cplx<R> (&h)[12], const cplx<R>* b, int nc,
                                              const CellGeo& g) {
    const cplx<R> a0 = v[0], a1 = v[1], a2 = v[2], a3 = v[3];
    if constexpr (X) {
        const cplx<R> R0 = b[g.xp], R2 = b[2 * nc + g.xp], L1 = b[nc + g.xm], L3 = b[3 * nc + g.xm];
        v[1] = add_hw(a1, h[2], R0);
        v[3] = add_hw(a3, h[3], R2);
        v[0] = add_hcw(a0, h[8], L1);
        v[2] = add_hcw(a2, h[9], L3);
    } else {
        const cplx<R> U0 = b[g.yp], U1 = b[nc + g.yp], D2 = b[2 * nc + g.ym], D3 = b[3 * nc + g.ym];
        v[2] = add_hw(a2, h[6], U0);
        v[3] = add_hw(a3, h[7], U1);
        v[0] = add_hcw(a0, h[10], D2);
        v[1] = add_hcw(a1, h[11], D3);
    }
}

// One cross family on NV vectors (1 or 2) sharing one LDS round trip.
// Buffers of 8 * nc values (2 * Vs) alternate with k (NB = 2, one barrier per
// sweep) or are closed by a second barrier (NB = 1).
template <typename R, int MC, int NB, bool X, int NV>
__device__ __forceinline__ void cross_n(Cells<R, MC>* const (&v)[NV], const cplx<R> (*const (&h)[NV])[MC][12],
                                        const CellGeo (&g)[MC], const bool (&own)[MC], int nc, cplx<R>* buf,
                                        int& k) {
    cplx<R>* b = buf + (size_t)(NB == 2 ? k : 0) * 8 * nc;
    k ^= 1;
#pragma unroll
    for (int j = 0; j < NV; j++)
#pragma unroll
        for (int m = 0; m < MC; m++)
            if (own[m])
#pragma unroll
                for (int q = 0; q < 4; q++) b[(4 * j + q) * nc + g[m].c] = v[j]->v[m][q];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; j++)
#pragma unroll
        for (int m = 0; m < MC; m++)
            if (own[m]) sweep_cross_n<R, X>(v[j]->v[m], (*h[j])[m], b + 4 * j * nc, nc, g[m]);
    if (NB == 1) __syncthreads();
}

// B'_tau on NV vectors at once (factor order of Eq. 24: E3 E2 E1 E0(2h) E1 E2 E3).
template <typename R, int MC, int NB, int NV>
__device__ __forceinline__ void apply_Bn(Cells<R, MC>* const (&v)[NV], const cplx<R> (*const (&h)[NV])[MC][12],
                                         const CellGeo (&g)[MC], const bool (&own)[MC], int nc, cplx<R>* buf,
                                         int& k) {
    cross_n<R, MC, NB, false, NV>(v, h, g, own, nc, buf, k);
#pragma unroll
    for (int j = 0; j < NV; j++)
#pragma unroll
        for (int m = 0; m < MC; m++) sweep_in_n<R, 2>(v[j]->v[m], (*h[j])[m]);
    cross_n<R, MC, NB, true, NV>(v, h, g, own, nc, buf, k);
#pragma unroll
    for (int j = 0; j < NV; j++)
#pragma unroll
        for (int m = 0; m < MC; m++) sweep_in_n<R, 0>(v[j]->v[m], (*h[j])[m]);
    cross_n<R, MC, NB, true, NV>(v, h, g, own, nc, buf, k);
#pragma unroll
    for (int j = 0; j < NV; j++)
#pragma unroll
        for (int m = 0; m < MC; m++) sweep_in_n<R, 2>(v[j]->v[m], (*h[j])[m]);
    cross_n<R, MC, NB, false, NV>(v, h, g, own, nc, buf, k);
}

// Fused M^dag M on the cells of slice tau given the cells of the input at
// tau-1 (vm), tau (vt), tau+1 (vn) and the normalised hops of slices tau-1
// (hm) and tau (ht):
//   out = vt - eps_{tau-1} C B'_{tau-1} vm + C B'_tau (C B'_tau vt - eps_tau vn),
// the definition M^dag (M v) expanded with eps^2 = 1 (eps_{Nt-1} = -1 at the
// antiperiodic corner, +1 elsewhere).  B'_{tau-1} vm and B'_tau vt run
// together.  vm is consumed.  buf2: LDS of NB * 2 * Vs values.
template <typename R, int MC, int NB>
__device__ __forceinline__ void mdagm_cells(Cells<R, MC>& vm, const Cells<R, MC>& vt, const Cells<R, MC>& vn,
                                            const cplx<R> (&hm)[MC][12], const cplx<R> (&ht)[MC][12],
                                            const CellGeo (&g)[MC], const bool (&own)[MC], const Coef<R>& co,
                                            R eps_m, R eps_t, cplx<R>* buf2, int Vs, Cells<R, MC>& out) {
    const int nc = Vs >> 2;
    const R C = co.C;
    int k = 0;
    Cells<R, MC> t = vt;
    {
        Cells<R, MC>* const v[2] = {&vm, &t};
        const cplx<R>(*const h[2])[MC][12] = {&hm, &ht};
        apply_Bn<R, MC, NB, 2>(v, h, g, own, nc, buf2, k);
    }
#pragma unroll
    for (int m = 0; m < MC; m++)
#pragma unroll
        for (int q = 0; q < 4; q++) {
            out.v[m][q] = cfma(-eps_m * C, vm.v[m][q], vt.v[m][q]);
            t.v[m][q] = mk<R>(C * t.v[m][q].re - eps_t * vn.v[m][q].re, C * t.v[m][q].im - eps_t * vn.v[m][q].im);
        }
    {
        Cells<R, MC>* const v[1] = {&t};
        const cplx<R>(*const h[1])[MC][12] = {&ht};
        apply_Bn<R, MC, NB, 1>(v, h, g, own, nc, buf2, k);
    }
#pragma unroll
    for (int m = 0; m < MC; m++)
#pragma unroll
        for (int q = 0; q < 4; q++) out.v[m][q] = cfma(C, t.v[m][q], out.v[m][q]);
}

template <typename R, int MC>
__device__ __forceinline__ void load_cells(Cells<R, MC>& c, const cplx<R>* __restrict__ slice, const CellGeo (&g)[MC],
                                           const bool (&own)[MC]) {
#pragma unroll
    for (int m = 0; m < MC; m++) {
        if (own[m]) {
#pragma unroll
            for (int q = 0; q < 4; q++) c.v[m][q] = slice[g[m].s[q]];
        } else {
#pragma unroll
            for (int q = 0; q < 4; q++) c.v[m][q] = mk<R>(0, 0);
        }
    }
}

template <typename R, int MC>
__device__ __forceinline__ void store_cells(const Cells<R, MC>& c, cplx<R>* __restrict__ slice, const CellGeo (&g)[MC],
                                            const bool (&own)[MC]) {
#pragma unroll
    for (int m = 0; m < MC; m++)
        if (own[m]) {
#pragma unroll
            for (int q = 0; q < 4; q++) slice[g[m].s[q]] = c.v[m][q];
        }
}

// Wavefront sum of one double through DPP lane moves (no LDS round trips):
// pairs, quads, half rows, rows, then rows 0+1 into row 1 and rows 0..3 into
// row 3.  Fixed order; the total is valid in lane 63.  Every lane of the
// wavefront must take part.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum_f64(double v) {
    v += dpp_f64<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
    v += dpp_f64<0x141, 0xF>(v);  // row_half_mirror
    v += dpp_f64<0x140, 0xF>(v);  // row_mirror
    v += dpp_f64<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_f64<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

// A CG slot's stop flag asks for a reliable update: stop (1), pause (2),
// pause with restart (3) or iteration budget used (6).
__host__ __device__ __forceinline__ bool gate_open(double flag) {
    return flag == 1.0 || flag == 2.0 || flag == 3.0 || flag == 6.0;
}

// Fixed-order block reduction of one double per thread (deterministic for a
// fixed block size).  red: LDS scratch of at least blockDim/64 doubles.
__device__ __forceinline__ double block_sum(double x, double* red) {
    x = wave_sum_f64(x);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 63) red[w] = x;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int k = 0; k < nw; k++) s += red[k];
    }
    return s;  // valid in thread 0
}

}  // namespace qh

// ---------------------------------------------------------------------------
// Handle and host-side helpers
// ---------------------------------------------------------------------------
// One tap of the paper's preconditioner stencil (host copy, FP64).
struct HostTap {
    int dt, dx, dy;
    double gre, gim;
};

// One pass of the preconditioner (G, then G^dag) as a gather: reach of its
// taps and where each parity's list starts in the device arrays.
struct PcPass {
    int amin, amax, bmin, bmax, cmin, cmax;
    int first[2], count[2];
    int gstart[2][17];  // per parity: start of the taps of tau offset amin + k, k = 0 .. 16
    // the same taps grouped by spatial offset (the tau-rolling kernel): where
    // each parity's offset list starts and its length (0: not built)
    int rfirst[2], rcount[2];
};

namespace qh {
// tau offsets of a pass the tau-rolling stencil kernel holds in registers
constexpr int kRollNS = 7;
// One spatial offset of a stencil pass with the taps of all its tau offsets:
// off and plane locate the source relative to the output in the LDS window
// (as for the per-tap lists), g[k] is the tap of tau offset amin + k (zero
// when the stencil has none there).
template <typename R>
struct RTap {
    int off, plane, pad0, pad1;
    cplx<R> g[kRollNS];
};
}  // namespace qh

struct qedhmc_net;

struct qedhmc_ctx {
    qedhmc_params p;
    qh::Lat lat;
    hipStream_t stream;
    int device;
    size_t max_lds;
    int n_cu;  // compute units of the device
    int32_t* d_tables;          // [4][Vs/2][3]
    // working-precision gauge caches e^{i theta}
    qh::cplx<double>* gauge64;
    qh::cplx<float>* gauge32;
    const double* gauge_src64;  // theta the caches were last built from (nullptr: stale)
    const double* gauge_src32;
    // workspace vectors
    void* ws[12];               // general complex FP64-sized vectors
    void* cg_arena;             // 7 complex FP64-sized vectors of the fused CG (r, s, w ping-pong, p)
    double* theta0;             // saved theta for Metropolis
    double* mom;                // momenta
    double* force;              // total force
    double* force_b;            // bosonic force
    double* partial;            // per-block partial sums: [2][Nt][6] for CG, then 4096 more
    double* tpart;              // slices of more than 1024 cells: CG partials per (slice, tile), then Nt more
    int tpart_tiles;            // tiles per slice the buffer holds
    double* scal;               // device scalars: [0,32) CG slots, [64,80) trajectory, [80,82) warm-start
                                // norms, [100] action
    double* h_pinned;           // pinned host mirror of a few scalars
    // sampled kernel timing (qedhmc_profile)
    int prof_every;
    int64_t prof_seen[QEDHMC_K_COUNT];
    int64_t prof_count[QEDHMC_K_COUNT];
    double prof_ms[QEDHMC_K_COUNT];
    hipEvent_t prof_ev[64][2];
    int prof_cls[64];
    int prof_weight[64];  // launches covered by the event pair
    bool prof_used[64];
    int prof_pending;
    bool prof_ready;
    // CG chunks captured into graphs: [R is double][launch parity][buffer
    // parity]; captured on a private stream (capture needs a non-null
    // stream) and launched on the handle's stream
    struct CgGraph {
        hipGraphExec_t exec;
        const void* x;
        const void* rhs;
        double tol2;
        int mixed, count, maxit;
    } cg_graph[2][2][2];
    hipStream_t cap_stream;
    hipEvent_t cg_ev[2];  // the pipelined mixed CG: one per round in flight
    // chunks of the two-launch (P)CG captured the same way: [R is
    // double][identity preconditioner][launch parity]
    struct PcgGraph {
        hipGraphExec_t exec;
        const void* x;
        const void* rhs;
        int mixed, count;
        int plan;  // the preconditioner's launch plan the graph holds
        int maxit;
        int kp;    // launch parity at the start (whole rounds)
    } pcg_graph[2][2][2];
    // whole pipelined PCG rounds (chunk, gated update, decision) by
    // precision and round parity
    PcgGraph pcg_round[2][2];
    // the paper's preconditioner (built on first use)
    bool pc_ready;
    double pc_shift;
    int pc_cap;  // tau reach of G's taps
    std::vector<HostTap> pc_taps[2];  // per x parity
    PcPass pc_pass[2];                // G and G^dag
    void* pc_dev64;                   // device taps, FP64 and FP32
    void* pc_dev32;
    void* pc_roll64;                  // device taps grouped by spatial offset (RTap), FP64 and FP32
    void* pc_roll32;
    // the same P as 2x2 blocks per spatial momentum of the two-site cell
    // (spectral application): H[a][entry][k] and the DFT twiddles, FP64 and
    // FP32; pc_spec_na = 0 when not built
    void* pc_spec64;
    void* pc_spec32;
    void* pc_tw64;
    void* pc_tw32;
    int pc_spec_a0, pc_spec_na;
    // the learned preconditioner (QEDHMC_PC_LEARNED): a network bound to this
    // handle, its arithmetic and the fallback its residual judge hands over to
    qedhmc_net* pc_net;
    qedhmc_net_arith pc_arith;
    qedhmc_precond pc_fallback;
};

namespace qh {

void set_error(const std::string& msg);
qedhmc_status hip_fail(hipError_t e, const char* what);

#define QH_HIP(call)                                                  \
    do {                                                              \
        hipError_t _e = (call);                                       \
        if (_e != hipSuccess) return ::qh::hip_fail(_e, #call);       \
    } while (0)

#define QH_TRY(call)                                                  \
    do {                                                              \
        qedhmc_status _s = (call);                                    \
        if (_s != QEDHMC_OK) return _s;                               \
    } while (0)

template <typename R>
Coef<R> coef_of(const qedhmc_params& p);

// Sampled kernel timing (api.hip).  prof_sample returns true when this launch
// of class cls is to be timed and hands out the start/stop events to pass to
// hipExtLaunchKernelGGL, which records them around the dispatch itself.
bool prof_sample(qedhmc_ctx* h, int cls, hipEvent_t& e0, hipEvent_t& e1);
// the same for an event pair around n launches of the class (a graph replay)
bool prof_sample_n(qedhmc_ctx* h, int cls, int n, hipEvent_t& e0, hipEvent_t& e1);
qedhmc_status prof_drain(qedhmc_ctx* h);

// Launch helpers implemented in lattice.hip
qedhmc_status ensure_gauge(qedhmc_ctx* h, const double* theta, qedhmc_precision prec);
// argument checks shared by the handle and the allocation-free entry point
qedhmc_status check_prec(qedhmc_precision p);
qedhmc_status check_params(const qedhmc_params* params);
// lattice geometry, stream and device limits of a context (allocates nothing)
qedhmc_status ctx_geometry(qedhmc_ctx* h, const qedhmc_params& p, void* stream);
qedhmc_status launch_apply_M(qedhmc_ctx* h, qedhmc_precision prec, const void* in, void* out, int dagger);
qedhmc_status launch_apply_B(qedhmc_ctx* h, qedhmc_precision prec, int tau, const void* in, void* out);
// out = M^dag M in; gate (nullable): a CG slot's stop flag, the launch runs
// only when the flag asks for a reliable update (1, 2 or 3; see gate_open)
qedhmc_status launch_mdagm(qedhmc_ctx* h, qedhmc_precision prec, const void* in, void* out,
                           const double* gate = nullptr);
qedhmc_status launch_force(qedhmc_ctx* h, qedhmc_precision prec, const double* X, double* F);
// Per-launch host work done once per kernel (api.hip): allow_lds lets kernel
// k take up to max_lds bytes of LDS, its static LDS included (every caller
// sets the same value); blocks_per_cu returns the workgroups of `threads` threads and
// `lds` bytes one compute unit holds, cached per (kernel, shape).
qedhmc_status allow_lds(const void* k, size_t max_lds);
qedhmc_status blocks_per_cu(const void* k, int threads, size_t lds, int* out);
// out = M^dag M in by spatial tiles streamed along tau (mdagm_tiled.hip)
qedhmc_status launch_mdagm_tiled(qedhmc_ctx* h, qedhmc_precision prec, const void* in, void* out);
// the same as the matvec of the two-launch CG: w = O u and the partial sums
// <r,r>, <r,u>, <w,u>, <u,s>, <p,w>, <p,s> (and a zero) of every (slice,
// tile) into part[7 * (tau * tiles + tile)]; stop: nullable slot flag
template <typename R>
qedhmc_status launch_mdagm_tiled_parts(qedhmc_ctx* h, const cplx<R>* u, cplx<R>* w, const cplx<R>* r,
                                       const cplx<R>* p, const cplx<R>* s, double* part, const double* stop);
// tiles per slice of the default plan (the CG form's) in FP32 or FP64
int mdagm_tiled_tiles(const Lat& lt, bool fp64);
qedhmc_status launch_bond_tables(qedhmc_ctx* h);

// CG (cg.hip) and preconditioned CG (pcg.hip)
qedhmc_status cg_solve_impl(qedhmc_ctx* h, const double* rhs, double* x, double tol, int maxit,
                            qedhmc_precision prec, int* iters, double* true_rel, int* n_reliable);
qedhmc_status pcg_solve_impl(qedhmc_ctx* h, const double* rhs, double* x, double tol, int maxit,
                             qedhmc_precision prec, int* iters, double* true_rel, int* n_reliable);
// plain CG as two launches per iteration (update; M^dag M with partials), for
// lattices with more than 1024 cells per slice
qedhmc_status cg2_solve_impl(qedhmc_ctx* h, const double* rhs, double* x, double tol, int maxit,
                             qedhmc_precision prec, int* iters, double* true_rel, int* n_reliable);
qedhmc_status ensure_paper_precond(qedhmc_ctx* h);
qedhmc_status launch_apply_precond(qedhmc_ctx* h, qedhmc_precision prec, const void* in, void* out);
// FP64 in and out, stencil passes in FP32 (scratch ws[8], ws[9])
qedhmc_status launch_apply_precond_fp32(qedhmc_ctx* h, const double* in, double* out);

// Gauge-field and trajectory kernels (boson.hip)
qedhmc_status launch_bosonic(qedhmc_ctx* h, const double* theta, double* F_B, double* S_dev);
qedhmc_status launch_heatbath(qedhmc_ctx* h, uint64_t traj, double* mom, double* R);
// production-loop observables: (S_tau, S_plaq) into out_dev[0..1]; C_flux(dtau)
// into (or added to) out_dev[0..Nt); out_dev[0..n) *= c
qedhmc_status launch_gauge_parts(qedhmc_ctx* h, const double* theta, double* out_dev);
qedhmc_status launch_flux_corr(qedhmc_ctx* h, const double* theta, bool accumulate, double* out_dev);
qedhmc_status launch_scale(qedhmc_ctx* h, double* a, int n, double c);
// batches of right-hand sides on one lattice and one gauge field (every chain
// reads chain 0's phase caches): the multi-RHS CG
qedhmc_status batch_create_shared(const qedhmc_params& params, int n, void* stream, qedhmc_batch** out);
qedhmc_ctx* batch_ctx0(qedhmc_batch* b);
qedhmc_status batch_enter(qedhmc_batch* b);
qedhmc_status batch_solve_shared(qedhmc_batch* b, const double* theta, const double* rhs_all, double* x_all,
                                 double tol, int maxit, qedhmc_precision prec, int32_t* iters, double* true_rel);
qedhmc_status launch_dot_re(qedhmc_ctx* h, const double* a, const double* b, size_t n, double* out_dev);
qedhmc_status launch_sumsq(qedhmc_ctx* h, const double* a, size_t n, double* out_dev);
qedhmc_status launch_kick(qedhmc_ctx* h, double* mom, const double* F, const double* Fb, double c, size_t n);
qedhmc_status launch_drift(qedhmc_ctx* h, double* theta, const double* mom, double c, size_t n);
qedhmc_status launch_lincomb(qedhmc_ctx* h, double* out, double a, const double* x, double b, const double* y,
                             size_t n);
// Metropolis test of the trajectory (dH, u, decision into scal_dev[6..8]);
// reject = true refuses the proposal whatever dH is (an unconverged solve)
qedhmc_status launch_metropolis(qedhmc_ctx* h, uint64_t traj, bool reject, double* scal_dev);
qedhmc_status launch_restore(qedhmc_ctx* h, double* theta, const double* theta0, const double* scal_dev, size_t n);

}  // namespace qh
