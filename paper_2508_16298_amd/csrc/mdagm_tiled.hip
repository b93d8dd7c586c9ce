// Fused M^dag M for large slices: spatial tiles streamed along tau.
//
// The whole-slice kernels keep one slice per workgroup; past about a thousand
// 2x2 cells a slice no longer fits one workgroup's threads and registers.
// Here a workgroup owns a tile of cells (with a halo, or a whole periodic
// ring of the slice in x and/or y) and a run of consecutive slices
// tau0 .. tau0 + Tc - 1, and walks it slice by slice with M^dag M written as
// M^dag (M v) (the matrices of the fermion-matrix definition):
//
//   y_{tau+1} = v_{tau+1} - e_tau B_tau v_tau            (M v)
//   out_tau   = y_tau     - e_tau B_tau y_{tau+1}         (M^dag y)
//
// with e_tau = -1 on the wrapping link tau = Nt - 1 and +1 otherwise.  Each
// step reads v_{tau+1} and the phases of slice tau once, applies B_tau twice
// and carries y to the next step, so a slice costs two B applications
// (three in the whole-slice kernel) plus one more per run for y_{tau0}.
//
// B_tau = E3 E2 E1 E0(2h) E1 E2 E3 (Eq. 24).  Every site lies on exactly one
// bond of each family, so each bond factor is cosh(a) times the normalised
// factor (v_i, v_j) -> (v_i + tanh(a) e^{i theta} v_j, v_j + tanh(a)
// e^{-i theta} v_i), and B_tau = C B'_tau with C = cosh(h)^6 cosh(2h): the
// sweeps use tanh-scaled phases (four FMAs per site and sweep) and C is
// folded into the e_tau scale.
//
// A B application moves information by at most two cells in x and in y (two
// f1 and two f3 sweeps).  With a halo of four cells around the output tile,
// the first application (on v_tau) is exact on the tile plus two cells and
// the second (on y_{tau+1}) on the tile; a region that covers the whole ring
// of a direction needs no halo in it.  Region cells past an edge read their
// own values in place of the missing neighbour: only halo results, which
// are never stored, are affected.
//
// Exchange buffers hold the four sites of every region cell as four planes
// (site q of cell c at q * ncell + c), so the writes and each neighbour read
// of a wavefront are contiguous; two buffer sets alternate so one barrier per
// cross sweep suffices.
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "qedhmc_internal.h"

namespace qh {

struct TiledGeo {
    int L, hL, Nt, Vs;
    int RW, RH;      // region cells in x and y
    int hx, hy;      // halo cells on each side (0: the region is the whole ring)
    int TX, TY;      // output cells of a tile in x and y
    int ntx, nty;    // tiles per direction
    int Tc, nchunk;  // slices per run, runs
    int nwork;       // ntx * nty * nchunk
    int skip;        // wavefronts of halo rows skip the sweeps whose results are unused
};

template <typename R>
struct TCoef {
    R t1, t2, C;  // tanh(h), tanh(2h), cosh(h)^6 cosh(2h)
};

// v + h w and v + conj(h) w
template <typename R>
__device__ __forceinline__ cplx<R> pl_hw(cplx<R> v, cplx<R> h, cplx<R> w) {
    return mk<R>(v.re + h.re * w.re - h.im * w.im, v.im + h.re * w.im + h.im * w.re);
}
template <typename R>
__device__ __forceinline__ cplx<R> pl_hcw(cplx<R> v, cplx<R> h, cplx<R> w) {
    return mk<R>(v.re + h.re * w.re + h.im * w.im, v.im + h.re * w.im - h.im * w.re);
}

__device__ __forceinline__ int ring(int a, int n) {
    a %= n;
    return a < 0 ? a + n : a;
}

// One region cell: lattice sites, neighbour cells inside the region, whether
// its output is stored.
struct TCell {
    int s0, l1, d2;        // site 0; site 1 of the -x neighbour; site 2 of the -y neighbour
    int xp, xm, yp, ym;    // region indices of the four neighbour cells
    int c;                 // own region index
    bool act, store;
};

template <bool FX, bool FY>
__device__ __forceinline__ TCell tcell(const TiledGeo& G, int tx, int ty) {
    TCell k;
    const int nreg = G.RW * G.RH;
    const int t = threadIdx.x;
    k.act = t < nreg;
    k.c = k.act ? t : nreg - 1;
    const int i = k.c % G.RW, j = k.c / G.RW;
    const int cx = ring(tx * G.TX - G.hx + i, G.hL), cy = ring(ty * G.TY - G.hy + j, G.hL);
    const int cxm = cx == 0 ? G.hL - 1 : cx - 1, cym = cy == 0 ? G.hL - 1 : cy - 1;
    k.s0 = 2 * cy * G.L + 2 * cx;
    k.l1 = 2 * cy * G.L + 2 * cxm + 1;
    k.d2 = (2 * cym + 1) * G.L + 2 * cx;
    k.xp = i + 1 < G.RW ? k.c + 1 : (FX ? k.c + 1 - G.RW : k.c);
    k.xm = i > 0 ? k.c - 1 : (FX ? k.c - 1 + G.RW : k.c);
    k.yp = j + 1 < G.RH ? k.c + G.RW : (FY ? k.c + G.RW - nreg : k.c);
    k.ym = j > 0 ? k.c - G.RW : (FY ? k.c - G.RW + nreg : k.c);
    const int ox = tx * G.TX + i - G.hx, oy = ty * G.TY + j - G.hy;  // unwrapped tile coordinates
    k.store = k.act && i >= G.hx && i < G.hx + G.TX && j >= G.hy && j < G.hy + G.TY && ox < G.hL && oy < G.hL;
    return k;
}

// tanh-scaled phases of the cell's twelve bonds in slice tau (same bond
// order as the whole-slice kernels: f0 from sites 0, 2; f1 from 1, 3; f2 from
// 0, 1; f3 from 2, 3; f1 into 0, 2; f3 into 0, 1).  HopSet<R, false> loads all
// twelve at the start of a slice and keeps them in registers; HopSet<R, true>
// (FP64, where twelve complex doubles would not fit beside the rest at 1024
// threads) fetches each sweep's phases just before that sweep's exchange.
template <typename R, bool LAZY>
struct HopSet;

template <typename R>
struct HopRef {
    const cplx<R>* g0;
    const cplx<R>* g1;
    int s0, l1, d2, L;
    R t1, t2;
    __device__ __forceinline__ void set(const cplx<R>* __restrict__ gauge, const TiledGeo& G, const TCell& k, int tau,
                                        const TCoef<R>& co) {
        g0 = gauge + (size_t)tau * G.Vs;
        g1 = gauge + ((size_t)G.Nt + tau) * G.Vs;
        s0 = k.s0;
        l1 = k.l1;
        d2 = k.d2;
        L = G.L;
        t1 = co.t1;
        t2 = co.t2;
    }
    template <int Q>
    __device__ __forceinline__ cplx<R> fetch() const {
        cplx<R> e;
        if constexpr (Q == 0) e = g0[s0];
        if constexpr (Q == 1) e = g0[s0 + L];
        if constexpr (Q == 2) e = g0[s0 + 1];
        if constexpr (Q == 3) e = g0[s0 + L + 1];
        if constexpr (Q == 4) e = g1[s0];
        if constexpr (Q == 5) e = g1[s0 + 1];
        if constexpr (Q == 6) e = g1[s0 + L];
        if constexpr (Q == 7) e = g1[s0 + L + 1];
        if constexpr (Q == 8) e = g0[l1];
        if constexpr (Q == 9) e = g0[l1 + L];
        if constexpr (Q == 10) e = g1[d2];
        if constexpr (Q == 11) e = g1[d2 + 1];
        const R t = Q < 2 ? t2 : t1;
        return mk<R>(t * e.re, t * e.im);
    }
};

template <typename R>
struct HopSet<R, false> {
    static constexpr bool lazy = false;
    cplx<R> h[12];
    __device__ __forceinline__ void set(const cplx<R>* __restrict__ gauge, const TiledGeo& G, const TCell& k, int tau,
                                        const TCoef<R>& co) {
        HopRef<R> r;
        r.set(gauge, G, k, tau, co);
        h[0] = r.template fetch<0>();
        h[1] = r.template fetch<1>();
        h[2] = r.template fetch<2>();
        h[3] = r.template fetch<3>();
        h[4] = r.template fetch<4>();
        h[5] = r.template fetch<5>();
        h[6] = r.template fetch<6>();
        h[7] = r.template fetch<7>();
        h[8] = r.template fetch<8>();
        h[9] = r.template fetch<9>();
        h[10] = r.template fetch<10>();
        h[11] = r.template fetch<11>();
    }
    template <int Q>
    __device__ __forceinline__ cplx<R> get() const {
        return h[Q];
    }
};

template <typename R>
struct HopSet<R, true> {
    static constexpr bool lazy = true;
    HopRef<R> r;
    __device__ __forceinline__ void set(const cplx<R>* __restrict__ gauge, const TiledGeo& G, const TCell& k, int tau,
                                        const TCoef<R>& co) {
        r.set(gauge, G, k, tau, co);
    }
    template <int Q>
    __device__ __forceinline__ cplx<R> get() const {
        return r.template fetch<Q>();
    }
};

template <typename R>
__device__ __forceinline__ void tile_load(cplx<R> (&v)[4], const cplx<R>* __restrict__ slice, const TiledGeo& G,
                                          const TCell& k) {
    v[0] = slice[k.s0];
    v[1] = slice[k.s0 + 1];
    v[2] = slice[k.s0 + G.L];
    v[3] = slice[k.s0 + G.L + 1];
}

// A value from the cell one to the right (+x, lane + 1) or left (-x, lane - 1)
// in a region whose rows are whole wavefronts and whole rings in x: the
// wavefront rotations wave_rol:1 and wave_ror:1 (DPP controls 0x134 / 0x13C;
// lane i receives lane i + 1, resp. i - 1, with 63 and 0 wrapping), per
// 32-bit word.
template <int CTRL>
__device__ __forceinline__ float dpp_word(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_word(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL, typename R>
__device__ __forceinline__ cplx<R> dpp_cplx(cplx<R> v) {
    return mk<R>(dpp_word<CTRL>(v.re), dpp_word<CTRL>(v.im));
}
static constexpr int kDppFromRight = 0x134;  // wave_rol:1
static constexpr int kDppFromLeft = 0x13C;   // wave_ror:1

// One cross sweep (f1 if X, else f3) of the cell through exchange buffer b,
// then the in-cell sweep IN (0: none, 1: f0, 2: f2).  The phases of both are
// read first, so lazily fetched ones are in flight across the barrier.  DPPX
// (x sweeps of a region whose rows are whole wavefronts and x rings): the x
// neighbours' values come by wavefront rotation, with no buffer and no
// barrier.  upd (uniform over the wavefront) false: the cell's result of
// this sweep is never used, so only its share of the exchange is done.
template <typename R, bool X, int IN, bool DPPX, typename HS>
__device__ __forceinline__ void tile_phase(cplx<R> (&v)[4], const HS& hs, cplx<R>* b, int nreg, const TCell& k,
                                           bool upd = true) {
    if (X && DPPX && !upd) return;
    // keep lazily fetched phases at their sweep (no hoisting of every fetch
    // of the slice to its start, which would undo the register saving)
    if constexpr (HS::lazy) asm volatile("" ::: "memory");
    const cplx<R> ha = hs.template get<X ? 2 : 6>(), hb = hs.template get<X ? 3 : 7>();
    const cplx<R> hc = hs.template get<X ? 8 : 10>(), hd = hs.template get<X ? 9 : 11>();
    cplx<R> he = mk<R>(0, 0), hf = mk<R>(0, 0);
    if constexpr (IN == 1) {
        he = hs.template get<0>();
        hf = hs.template get<1>();
    }
    if constexpr (IN == 2) {
        he = hs.template get<4>();
        hf = hs.template get<5>();
    }
    if (X && DPPX) {
        const cplx<R> R0 = dpp_cplx<kDppFromRight>(v[0]), R2 = dpp_cplx<kDppFromRight>(v[2]);
        const cplx<R> L1 = dpp_cplx<kDppFromLeft>(v[1]), L3 = dpp_cplx<kDppFromLeft>(v[3]);
        v[1] = pl_hw(v[1], ha, R0);
        v[3] = pl_hw(v[3], hb, R2);
        v[0] = pl_hcw(v[0], hc, L1);
        v[2] = pl_hcw(v[2], hd, L3);
    } else {
    if (k.act) {
        b[k.c] = v[0];
        b[nreg + k.c] = v[1];
        b[2 * nreg + k.c] = v[2];
        b[3 * nreg + k.c] = v[3];
    }
    __syncthreads();
    if (!upd) return;
    if (X) {
        const cplx<R> R0 = b[k.xp], R2 = b[2 * nreg + k.xp], L1 = b[nreg + k.xm], L3 = b[3 * nreg + k.xm];
        v[1] = pl_hw(v[1], ha, R0);
        v[3] = pl_hw(v[3], hb, R2);
        v[0] = pl_hcw(v[0], hc, L1);
        v[2] = pl_hcw(v[2], hd, L3);
    } else {
        const cplx<R> U0 = b[k.yp], U1 = b[nreg + k.yp], D2 = b[2 * nreg + k.ym], D3 = b[3 * nreg + k.ym];
        v[2] = pl_hw(v[2], ha, U0);
        v[3] = pl_hw(v[3], hb, U1);
        v[0] = pl_hcw(v[0], hc, D2);
        v[1] = pl_hcw(v[1], hd, D3);
    }
    }
    const cplx<R> a0 = v[0], a1 = v[1], a2 = v[2], a3 = v[3];
    if constexpr (IN == 1) {  // f0: pairs (0, 1) and (2, 3)
        v[0] = pl_hw(a0, he, a1);
        v[1] = pl_hcw(a1, he, a0);
        v[2] = pl_hw(a2, hf, a3);
        v[3] = pl_hcw(a3, hf, a2);
    }
    if constexpr (IN == 2) {  // f2: pairs (0, 2) and (1, 3)
        v[0] = pl_hw(a0, he, a2);
        v[2] = pl_hcw(a2, he, a0);
        v[1] = pl_hw(a1, hf, a3);
        v[3] = pl_hcw(a3, hf, a1);
    }
}

// v <- B'_tau v (normalised factors, rightmost first: f3 f2 f1 f0 f1 f2 f3).
// The exchange buffers alternate over the sweeps that use them (with DPPX
// only the y sweeps), so one barrier per such sweep suffices.  Where the
// result is needed only on region rows lo .. hi, the last y sweep updates
// rows lo .. hi and the sweeps before it rows lo - 1 .. hi + 1 (the last one
// reads them); the first y sweep reads rows lo - 2 .. hi + 2, which must hold
// valid input.  A wavefront (region rows r0 .. r1, uniform) skips a sweep
// when none of its rows is updated in it.
template <typename R, bool DPPX, typename HS>
__device__ __forceinline__ void tile_B(cplx<R> (&v)[4], const HS& hs, cplx<R>* xb, int nreg, const TCell& k,
                                       int& kb, int r0 = 0, int r1 = 0, int lo = -(1 << 20), int hi = 1 << 20) {
    const bool u3 = r1 >= lo - 1 && r0 <= hi + 1, u4 = r1 >= lo && r0 <= hi;
    tile_phase<R, false, 2, DPPX>(v, hs, xb + (size_t)kb * 4 * nreg, nreg, k, u3);
    kb ^= 1;
    tile_phase<R, true, 1, DPPX>(v, hs, xb + (size_t)kb * 4 * nreg, nreg, k, u3);
    if (!DPPX) kb ^= 1;
    tile_phase<R, true, 2, DPPX>(v, hs, xb + (size_t)kb * 4 * nreg, nreg, k, u3);
    if (!DPPX) kb ^= 1;
    tile_phase<R, false, 0, DPPX>(v, hs, xb + (size_t)kb * 4 * nreg, nreg, k, u4);
    kb ^= 1;
}

// Threads per workgroup at most: 1024 in FP32 (108 registers); 512 in FP64,
// whose 162 registers a 1024-thread workgroup cannot hold without spilling.
template <typename R>
static constexpr int kTileMaxThreads = sizeof(R) == 8 ? 512 : 1024;

// Extra operands of the CG form (PART): with w = out = O u, the partial sums
// <r,r>, <r,u>, <w,u>, <u,s>, <p,w>, <p,s> of every (slice, tile) over the
// tile's output cells go to part[kTileParts * (tau * ntile + tile)]; a
// non-zero *stop makes the launch a no-op.
static constexpr int kTileParts = 7;

template <typename R>
struct TPart {
    const cplx<R>* r;
    const cplx<R>* p;
    const cplx<R>* s;
    double* part;
    const double* stop;
};

template <typename R>
__device__ __forceinline__ double tdot(const cplx<R> (&a)[4], const cplx<R> (&b)[4]) {
    double d = 0.0;
#pragma unroll
    for (int q = 0; q < 4; q++) d += (double)a[q].re * (double)b[q].re + (double)a[q].im * (double)b[q].im;
    return d;
}

template <typename R, bool FX, bool FY, bool PART, bool DPPX = false>
__global__ __launch_bounds__(kTileMaxThreads<R>) void k_mdagm_tiled(TiledGeo G, const cplx<R>* __restrict__ in,
                                                      cplx<R>* __restrict__ out, const cplx<R>* __restrict__ gauge,
                                                      TCoef<R> co, TPart<R> ops) {
    if (PART && ops.stop && *ops.stop != 0.0) return;
    extern __shared__ __align__(16) unsigned char smem[];
    cplx<R>* xb = reinterpret_cast<cplx<R>*>(smem);
    const int nreg = G.RW * G.RH;
    double* red = reinterpret_cast<double*>(xb + (size_t)8 * nreg);  // PART: per-wavefront sums
    // work items dealt to the eight XCDs in contiguous ranges: the tiles of
    // one run and neighbouring runs share an XCD's L2 (halo and tau + 1 reads)
    const int per = (G.nwork + 7) >> 3;
    const int w = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (w >= G.nwork) return;
    const int ntile = G.ntx * G.nty;
    const int tile = w % ntile, run = w / ntile;
    const TCell k = tcell<FX, FY>(G, tile % G.ntx, tile / G.ntx);
    const int Nt = G.Nt, Vs = G.Vs;
    const int tau0 = run * G.Tc, tau1 = min(Nt, tau0 + G.Tc);
    int kb = 0;
    HopSet<R, sizeof(R) == 8> hs;
    cplx<R> y[4], u[4];
    // Rows whose results are used (regions with a y halo of hy rows each
    // side): B_tau v_tau feeds y_{tau+1}, which the second application reads
    // two rows past the tile, so the first is needed on the tile and two rows
    // either side; the second, and the one forming y_{tau0} (used only in
    // out_{tau0}), on the tile.  r0 .. r1: the region rows of this wavefront
    // (inactive threads take the last row).
    int r0 = 0, r1 = 0, lo1 = -(1 << 20), hi1 = 1 << 20, lo2 = -(1 << 20), hi2 = 1 << 20;
    if (!FY && G.skip) {
        const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
        if constexpr (DPPX) {  // a wavefront per row
            r0 = r1 = wv;
        } else {
            r0 = min(G.RH - 1, 64 * wv / G.RW);
            r1 = min(G.RH - 1, (64 * wv + 63) / G.RW);
        }
        lo1 = G.hy - 2;
        hi1 = G.hy + G.TY + 1;
        lo2 = G.hy;
        hi2 = G.hy + G.TY - 1;
    }
    // y_{tau0} = v_{tau0} - e_{tau0-1} B_{tau0-1} v_{tau0-1}
    {
        const int tm = tau0 == 0 ? Nt - 1 : tau0 - 1;
        hs.set(gauge, G, k, tm, co);
        tile_load<R>(u, in + (size_t)tm * Vs, G, k);
        tile_B<R, DPPX>(u, hs, xb, nreg, k, kb, r0, r1, lo2, hi2);
        tile_load<R>(y, in + (size_t)tau0 * Vs, G, k);
        const R e = tm == Nt - 1 ? -co.C : co.C;
#pragma unroll
        for (int q = 0; q < 4; q++) y[q] = mk<R>(y[q].re - e * u[q].re, y[q].im - e * u[q].im);
    }
    // v_tau is read again each step (it was read as v_{tau+1} one step
    // earlier and is still in L2) rather than kept in registers across both
    // B applications
    for (int tau = tau0; tau < tau1; tau++) {
        const int tp = tau == Nt - 1 ? 0 : tau + 1;
        cplx<R> vn[4];
        hs.set(gauge, G, k, tau, co);
        tile_load<R>(u, in + (size_t)tau * Vs, G, k);
        // FP32 issues the read of v_{tau+1} before the first B application;
        // FP64 after it, where its registers are free
        if constexpr (sizeof(R) == 4) tile_load<R>(vn, in + (size_t)tp * Vs, G, k);
        const R e = tau == Nt - 1 ? -co.C : co.C;
        tile_B<R, DPPX>(u, hs, xb, nreg, k, kb, r0, r1, lo1, hi1);  // B'_tau v_tau
        if constexpr (sizeof(R) == 8) tile_load<R>(vn, in + (size_t)tp * Vs, G, k);
        cplx<R> yn[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            yn[q] = mk<R>(vn[q].re - e * u[q].re, vn[q].im - e * u[q].im);
            u[q] = yn[q];
        }
        tile_B<R, DPPX>(u, hs, xb, nreg, k, kb, r0, r1, lo2, hi2);  // B'_tau y_{tau+1}
        cplx<R> w[4];
#pragma unroll
        for (int q = 0; q < 4; q++) w[q] = mk<R>(y[q].re - e * u[q].re, y[q].im - e * u[q].im);
        if (k.store) {
            cplx<R>* o = out + (size_t)tau * Vs;
            o[k.s0] = w[0];
            o[k.s0 + 1] = w[1];
            o[k.s0 + G.L] = w[2];
            o[k.s0 + G.L + 1] = w[3];
        }
        if constexpr (PART) {
            double v[kTileParts] = {0, 0, 0, 0, 0, 0, 0};
            if (k.store) {
                cplx<R> rt[4], ut[4], pt[4], st[4];
                tile_load<R>(rt, ops.r + (size_t)tau * Vs, G, k);
                tile_load<R>(ut, in + (size_t)tau * Vs, G, k);
                tile_load<R>(pt, ops.p + (size_t)tau * Vs, G, k);
                tile_load<R>(st, ops.s + (size_t)tau * Vs, G, k);
                v[0] = tdot(rt, rt);
                v[1] = tdot(rt, ut);
                v[2] = tdot(w, ut);
                v[3] = tdot(ut, st);
                v[4] = tdot(pt, w);
                v[5] = tdot(pt, st);
            }
            // fixed-order workgroup sum: DPP within each wavefront, then the
            // wavefronts' sums in order (the exchange barriers separate the
            // reuse of red from one slice to the next)
            const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
            for (int q = 0; q < kTileParts - 1; q++) v[q] = wave_sum_f64(v[q]);
            if (lane == 63)
#pragma unroll
                for (int q = 0; q < kTileParts - 1; q++) red[(kTileParts - 1) * wv + q] = v[q];
            __syncthreads();
            if (threadIdx.x == 0) {
                double t[kTileParts] = {0, 0, 0, 0, 0, 0, 0};
                const int nw = (int)(blockDim.x + 63) >> 6;
                for (int i = 0; i < nw; i++)
#pragma unroll
                    for (int q = 0; q < kTileParts - 1; q++) t[q] += red[(kTileParts - 1) * i + q];
                double* dst = ops.part + (size_t)kTileParts * ((size_t)tau * ntile + tile);
#pragma unroll
                for (int q = 0; q < kTileParts; q++) dst[q] = t[q];
            }
        }
#pragma unroll
        for (int q = 0; q < 4; q++) y[q] = yn[q];
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct TiledPlan {
    TiledGeo g;
    bool fx, fy;
    int threads;
};

// Run length: each workgroup walks Tc slices (plus one B application for
// y_{tau0}), and the workgroups run in rounds of `slots` (the workgroups the
// device holds at once), so a pass costs about rounds x (Tc + 1/2) slice
// steps; the smallest such Tc is taken.  Counting rounds matters: a last
// round that is only partly filled costs as much as a full one.
static void set_run_length(TiledGeo& g, int tc, int slots) {
    const int ntile = g.ntx * g.nty;
    if (tc <= 0) {
        double best = 0.0;
        tc = 1;
        for (int c = 1; c <= std::min(g.Nt, 64); c++) {
            const long nwork = (long)ntile * ((g.Nt + c - 1) / c);
            const long rounds = (nwork + slots - 1) / slots;
            const double cost = (double)rounds * (c + 0.5);
            if (c == 1 || cost < best) {
                best = cost;
                tc = c;
            }
        }
    }
    g.Tc = std::min(tc, g.Nt);
    g.nchunk = (g.Nt + g.Tc - 1) / g.Tc;
    g.nwork = ntile * g.nchunk;
}

// Region shape for a slice of hL x hL cells and a cap of `cap` threads (one
// per region cell): the whole slice when it fits; else full x rings with a y
// halo (strips) while a strip of at least four output rows fits; else square
// tiles with halos both ways.  The run length is set later (set_run_length).
static TiledPlan plan_tiled(const Lat& lt, int cap) {
    TiledPlan p{};
    TiledGeo& g = p.g;
    g.L = lt.L;
    g.hL = lt.hL;
    g.Nt = lt.Nt;
    g.Vs = lt.Vs;
    const int hL = lt.hL;
    if (hL * hL <= cap) {
        p.fx = p.fy = true;
        g.RW = g.RH = g.TX = g.TY = hL;
        g.hx = g.hy = 0;
        g.ntx = g.nty = 1;
    } else if (cap / hL - 8 >= 4) {
        p.fx = true;
        p.fy = false;
        g.RW = g.TX = hL;
        g.hx = 0;
        g.ntx = 1;
        const int tymax = cap / hL - 8;
        g.nty = (hL + tymax - 1) / tymax;
        g.TY = (hL + g.nty - 1) / g.nty;
        g.hy = 4;
        g.RH = g.TY + 8;
    } else {
        p.fx = p.fy = false;
        int side = 1;
        while ((side + 1) * (side + 1) <= cap) side++;
        const int tmax = side - 8;
        g.ntx = g.nty = (hL + tmax - 1) / tmax;
        g.TX = g.TY = (hL + g.ntx - 1) / g.ntx;
        g.hx = g.hy = 4;
        g.RW = g.RH = g.TX + 8;
    }
    p.threads = ((g.RW * g.RH + 63) / 64) * 64;
    return p;
}

template <typename R>
static TCoef<R> tcoef_of(const qedhmc_params& prm) {
    const double h = 0.5 * prm.t * prm.dtau;
    return {(R)std::tanh(h), (R)std::tanh(2 * h), (R)(std::pow(std::cosh(h), 6) * std::cosh(2 * h))};
}

// Tuning overrides, read per call: QEDHMC_TILE_TC (slices per run, 0 =
// automatic) and QEDHMC_TILE_THREADS (thread cap of a region, 100 .. 1024,
// at most 512 in FP64).
static int env_int(const char* name, int dflt) {
    const char* s = std::getenv(name);
    return s ? std::atoi(s) : dflt;
}

// The region plan of precision R (the run length is set at launch): the
// tuning variables apply to the plain operator only; the CG form always takes
// the default plan (its partial buffer is sized for it).
template <typename R>
static TiledPlan plan_for(const Lat& lt, bool tunable, int* tc) {
    int cap = kTileMaxThreads<R>;
    *tc = 0;
    if (tunable) {
        cap = std::max(100, std::min(kTileMaxThreads<R>, env_int("QEDHMC_TILE_THREADS", 1024)));
        *tc = env_int("QEDHMC_TILE_TC", 0);
    }
    return plan_tiled(lt, cap);
}

int mdagm_tiled_tiles(const Lat& lt, bool fp64) {
    int tc;
    const TiledPlan p = fp64 ? plan_for<double>(lt, false, &tc) : plan_for<float>(lt, false, &tc);
    return p.g.ntx * p.g.nty;
}

template <typename R, bool PART>
static qedhmc_status mdagm_tiled_t(qedhmc_ctx* h, const void* in, void* out, const TPart<R>& tpart) {
    int tc;
    TiledPlan p = plan_for<R>(h->lat, !PART, &tc);
    const size_t lds = (size_t)8 * p.g.RW * p.g.RH * sizeof(cplx<R>) + (PART ? 16 * kTileParts * sizeof(double) : 0);
    if (lds > h->max_lds) {
        set_error("tiled M^dag M: exchange buffers exceed the workgroup's LDS");
        return QEDHMC_EUNSUPPORTED;
    }
    const cplx<R>* gauge = sizeof(R) == 8 ? reinterpret_cast<const cplx<R>*>(h->gauge64)
                                          : reinterpret_cast<const cplx<R>*>(h->gauge32);
    const TCoef<R> co = tcoef_of<R>(h->p);
    auto go = [&](auto kern) -> qedhmc_status {
        if (lds > 65536) QH_TRY(allow_lds((const void*)kern, h->max_lds));
        int per_cu = 0;
        QH_TRY(blocks_per_cu((const void*)kern, p.threads, lds, &per_cu));
        set_run_length(p.g, tc, std::max(1, per_cu) * std::max(1, h->n_cu));
        const int grid = 8 * ((p.g.nwork + 7) / 8);
        hipEvent_t e0, e1;
        const int cls = PART ? (sizeof(R) == 4 ? QEDHMC_K_PCG_MV_FP32 : QEDHMC_K_PCG_MV_FP64)
                             : (sizeof(R) == 4 ? QEDHMC_K_MDAGM_FP32 : QEDHMC_K_MDAGM_FP64);
        if (prof_sample(h, cls, e0, e1))
            hipExtLaunchKernelGGL(kern, dim3(grid), dim3(p.threads), lds, h->stream, e0, e1, 0, p.g,
                                  (const cplx<R>*)in, (cplx<R>*)out, gauge, co, tpart);
        else
            hipLaunchKernelGGL(kern, dim3(grid), dim3(p.threads), lds, h->stream, p.g, (const cplx<R>*)in,
                               (cplx<R>*)out, gauge, co, tpart);
        QH_HIP(hipGetLastError());
        return QEDHMC_OK;
    };
    // x exchanges by wavefront rotation when every region row is one whole
    // wavefront and a whole x ring; QEDHMC_TILE_DPP=0 (read per call) keeps
    // them in LDS
    const bool dppx = p.fx && !p.fy && p.g.RW == 64 && p.threads == p.g.RW * p.g.RH &&
                      env_int("QEDHMC_TILE_DPP", 1) != 0;
    // QEDHMC_TILE_SKIP=0 (read per call) keeps every halo row's sweeps
    p.g.skip = env_int("QEDHMC_TILE_SKIP", 1) != 0;
    if (p.fx && p.fy) return go(k_mdagm_tiled<R, true, true, PART>);
    if (dppx) return go(k_mdagm_tiled<R, true, false, PART, true>);
    if (p.fx) return go(k_mdagm_tiled<R, true, false, PART>);
    return go(k_mdagm_tiled<R, false, false, PART>);
}

qedhmc_status launch_mdagm_tiled(qedhmc_ctx* h, qedhmc_precision prec, const void* in, void* out) {
    return prec == QEDHMC_FP64 ? mdagm_tiled_t<double, false>(h, in, out, TPart<double>{})
                               : mdagm_tiled_t<float, false>(h, in, out, TPart<float>{});
}

template <typename R>
qedhmc_status launch_mdagm_tiled_parts(qedhmc_ctx* h, const cplx<R>* u, cplx<R>* w, const cplx<R>* r,
                                       const cplx<R>* p, const cplx<R>* s, double* part, const double* stop) {
    return mdagm_tiled_t<R, true>(h, u, w, TPart<R>{r, p, s, part, stop});
}
template qedhmc_status launch_mdagm_tiled_parts<float>(qedhmc_ctx*, const cplx<float>*, cplx<float>*,
                                                       const cplx<float>*, const cplx<float>*, const cplx<float>*,
                                                       double*, const double*);
template qedhmc_status launch_mdagm_tiled_parts<double>(qedhmc_ctx*, const cplx<double>*, cplx<double>*,
                                                        const cplx<double>*, const cplx<double>*,
                                                        const cplx<double>*, double*, const double*);

}  // namespace qh
