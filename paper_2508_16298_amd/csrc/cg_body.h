// Conjugate gradient on O = M^dag M (Methods, Eq. pCG), started from x = 0,
// one kernel launch per iteration.
//
// The recursion is CG with a single global reduction phase per iteration
// (the Chronopoulos-Gear arrangement: s = O p carried as a recurrence):
//   beta_i  = gamma_i / gamma_{i-1}            (0 on the first iteration)
//   p_i = r_i + beta_i p_{i-1},  s_i = w_i + beta_i s_{i-1}     (s = O p)
//   alpha_i = gamma_i / <p_i, s_i>
//   x_{i+1} = x_i + alpha_i p_i,  r_{i+1} = r_i - alpha_i s_i
//   w_{i+1} = O r_{i+1}
// mathematically the same iterates as Eq. pCG without preconditioner.  The
// denominator is expanded over vectors the previous launch already holds,
//   <p_i, s_i> = <r_i,w_i> + beta_i (<r_i,s_{i-1}> + <p_{i-1},w_i>)
//                + beta_i^2 <p_{i-1},s_{i-1}>,
// so one launch computes all five inner products of the next iteration
// together.  (The textbook Chronopoulos-Gear denominator
// delta - beta gamma / alpha_{i-1} leans on an orthogonality identity that
// FP32 rounding breaks: in emulation it needed 15-23% more iterations and
// diverged on ill-conditioned systems, while the expansion tracks the
// two-reduction form iteration for iteration.)
// A launch boundary is the only grid-wide synchronisation: every workgroup
// (one per time slice) reduces the per-slice partials of the previous launch
// in a fixed order (bitwise reproducible), recomputes the recurrences on the
// two neighbouring slices it needs for the stencil, and applies O to its
// slice.  r, s and w alternate between two buffers by iteration parity; the
// device scalars alternate between two slots by launch parity, so no launch
// reads what a concurrent workgroup writes.
//
// Stop and pause: an iteration that finds gamma_i <= tol^2 |rhs|^2 turns
// itself and all later launches into no-ops (the host reads the flag once per
// chunk).  The mixed path (complex-FP32 r, p, s, w, O; FP64 x and reductions)
// also pauses when gamma has fallen by 100 since the last reliable update or
// 50 iterations have passed (Sleijpen and van der Vorst 1996): then
// r = rhs - O x is recomputed with the FP64 operator and copied into the FP32
// recursion, w = O r and s = O p are recomputed (s is otherwise only a
// recurrence and drifts; the drift turns the denominator <p, O p> =
// delta - beta gamma / alpha negative on ill-conditioned systems) and the
// iteration resumes with p kept.  A denominator that is not positive forces
// the same update with a restart (beta = 0).  At a stop the FP64 true
// residual decides: converged, or resume (the FP64 path restarts with p = r,
// as the oracle does).
#pragma once
#include <cmath>

#include "cg_common.h"

namespace qh {

// ---------------------------------------------------------------------------
// Start: r_0 = rhs, w_0 = O r_0, x = p = s = 0, partials of iteration 0,
// slot 0 initialised.
// ---------------------------------------------------------------------------
template <typename R, int MC, int NB>
__device__ __forceinline__ void cg_start_body(const Lat& lt, const CgBufs<R>& B, const cplx<R>* __restrict__ gauge,
                                              const Coef<R>& co, double* __restrict__ scal, int tau, bool lead,
                                              const Tile& tl) {
    cplx<R>* buf2 = reinterpret_cast<cplx<R>*>(tl.buf);
    SliceCtx<MC> c;
    slice_ctx<MC>(lt, c, tau, tl);
    const size_t Vs = lt.Vs;
    cplx<R> hm[MC][12], ht[MC][12];
    hops_of<R, MC>(gauge, lt, c.tm, c.idx, co, hm);
    hops_of<R, MC>(gauge, lt, c.tau, c.idx, co, ht);
    Cells<R, MC> vm, vt, vn, w;
    double b2 = 0.0, dummy = 0.0;
    load_cvt<R, MC>(vm, B.rhs + c.tm * Vs, nullptr, c.g, c.own, dummy);
    load_cvt<R, MC>(vt, B.rhs + c.tau * Vs, nullptr, c.g, c.own, b2);
    load_cvt<R, MC>(vn, B.rhs + c.tp * Vs, nullptr, c.g, c.own, dummy);
    Cells<R, MC> zero;
    Cells<double, MC> zx;
#pragma unroll
    for (int m = 0; m < MC; m++)
#pragma unroll
        for (int q = 0; q < 4; q++) {
            zero.v[m][q] = mk<R>(0, 0);
            zx.v[m][q] = mk<double>(0, 0);
        }
    store_cells<R, MC>(vt, B.r[0] + c.tau * Vs, c.g, c.own);
    store_cells<R, MC>(zero, B.s[0] + c.tau * Vs, c.g, c.own);
    store_cells<R, MC>(zero, B.p + c.tau * Vs, c.g, c.own);
    store_cells<double, MC>(zx, B.x + c.tau * Vs, c.g, c.own);
    const Cells<R, MC> r0 = vt;
    mdagm_cells<R, MC, NB>(vm, vt, vn, hm, ht, c.g, c.own, co, c.tau == 0 ? R(-1) : R(1),
                           c.tau == lt.Nt - 1 ? R(-1) : R(1), buf2, lt.Vs, w);
    store_cells<R, MC>(w, B.w[0] + c.tau * Vs, c.g, c.own);
    double v[kNP] = {dot_cells<R, MC>(r0, r0, c.own), dot_cells<R, MC>(w, r0, c.own), 0.0, 0.0, 0.0, b2};
    write_partials(B.part + kNP * (size_t)c.tau, v, tl);  // parity 0
    if (lead && tl.ltid < S_NSLOT) {
        double v = 0.0;
        if (tl.ltid == S_FIRST) v = 1.0;
        if (tl.ltid == S_B2) v = -1.0;
        if (tl.ltid == S_GPREV || tl.ltid == S_APREV) v = 1.0;
        scal[tl.ltid] = v;
    }
}

// ---------------------------------------------------------------------------
// One CG iteration.  kpar: launch parity (slot in = kpar, slot out = kpar^1).
// ---------------------------------------------------------------------------
template <typename R, int MC, int NB>
__device__ __forceinline__ void cg_iter_body(const Lat& lt, const CgBufs<R>& B, const cplx<R>* __restrict__ gauge,
                                             const Coef<R>& co, double* __restrict__ scal, int kpar, int ipar,
                                             double tol2, int mixed, int maxit, int tau, bool lead,
                                             const Tile& tl) {
    cplx<R>* buf2 = reinterpret_cast<cplx<R>*>(tl.buf);
    const double* sin_ = scal + S_NSLOT * kpar;
    double* sout = scal + S_NSLOT * (kpar ^ 1);
    // Every load of the launch is issued before the scalars arrive: the
    // buffer parity ipar comes from the host -- the parity of the number of
    // iterations since the last reliable update (the ping-pong of r, s, w
    // restarts at buffer 0 after every update, so a chunk that starts right
    // after one has ipar = launch index & 1 whatever the iteration count; after
    // a stop or pause inside a chunk the remaining launches are no-ops, so the
    // guess is never used wrongly) -- and the stop flag is looked at only
    // after the loads.  All loads are in bounds whatever the flag says.
    const double done = sin_[S_DONE];
    const int it = (int)sin_[S_ITERS];
    const int ip = ipar, nx = ip ^ 1;
    SliceCtx<MC> c;
    slice_ctx<MC>(lt, c, tau, tl);
    const size_t Vs = lt.Vs;
    Cells<R, MC> wm, wt, wn, sm, st, sn, rm, rt, rn, pp;
    load_cells<R, MC>(wm, B.w[ip] + c.tm * Vs, c.g, c.own);
    load_cells<R, MC>(wt, B.w[ip] + c.tau * Vs, c.g, c.own);
    load_cells<R, MC>(wn, B.w[ip] + c.tp * Vs, c.g, c.own);
    load_cells<R, MC>(sm, B.s[ip] + c.tm * Vs, c.g, c.own);
    load_cells<R, MC>(st, B.s[ip] + c.tau * Vs, c.g, c.own);
    load_cells<R, MC>(sn, B.s[ip] + c.tp * Vs, c.g, c.own);
    load_cells<R, MC>(rm, B.r[ip] + c.tm * Vs, c.g, c.own);
    load_cells<R, MC>(rt, B.r[ip] + c.tau * Vs, c.g, c.own);
    load_cells<R, MC>(rn, B.r[ip] + c.tp * Vs, c.g, c.own);
    load_cells<R, MC>(pp, B.p + c.tau * Vs, c.g, c.own);
    cplx<R> hm[MC][12], ht[MC][12];
    hops_of<R, MC>(gauge, lt, c.tm, c.idx, co, hm);
    hops_of<R, MC>(gauge, lt, c.tau, c.idx, co, ht);
    // x is read here with the rest (its update comes after stores that the
    // compiler cannot tell apart from x, which would hold the read back)
    Cells<double, MC> xo;
    load_cells<double, MC>(xo, B.x + c.tau * Vs, c.g, c.own);
    if (done != 0.0 || it >= maxit) {
        // stopped or paused: carry the state over; a running solve that used
        // its iteration budget is marked for its final true residual (6)
        if (lead && tl.ltid < S_NSLOT) {
            double v = sin_[tl.ltid];
            if (tl.ltid == S_DONE && v == 0.0) v = 6.0;
            sout[tl.ltid] = v;
        }
        return;
    }

    double pr[kNP];
    reduce_partials(B.part + kNP * (size_t)lt.Nt * ip, lt.Nt, tl, pr);
    const double gam = pr[0], del = pr[1], aux = pr[5];
    double b2 = sin_[S_B2], target = sin_[S_TARGET], rrupd = sin_[S_RRUPD];
    if (b2 < 0.0) {  // first iteration of the solve: the start kernel left |rhs|^2 partials in aux
        b2 = aux;
        target = tol2 * aux;
        rrupd = gam;
    }
    int stop = 0;
    if (!isfinite(gam) || !isfinite(del) || ((it - (int)sin_[S_ITUPD]) & 1) != ipar)
        stop = 4;  // breakdown: non-finite recursion (or a host/device parity mismatch)
    else if (gam <= target)
        stop = 1;
    else if (mixed && (gam <= kDecade2 * rrupd || it - (int)sin_[S_ITUPD] >= kCap))
        stop = 2;
    if (stop) {
        if (lead && tl.ltid < S_NSLOT) {
            double v = sin_[tl.ltid];
            if (tl.ltid == S_DONE) v = (double)stop;
            if (tl.ltid == S_B2) v = b2;
            if (tl.ltid == S_TARGET) v = target;
            if (tl.ltid == S_RRUPD) v = rrupd;
            if (tl.ltid == S_GCUR) v = gam;
            sout[tl.ltid] = v;
        }
        return;
    }
    const bool first = sin_[S_FIRST] != 0.0;
    const double beta = first ? 0.0 : gam / sin_[S_GPREV];
    const double den = first ? del : del + beta * (pr[2] + pr[3]) + beta * beta * pr[4];  // <p_i, s_i>
    if (!(den > 0.0)) {
        if (lead && tl.ltid < S_NSLOT) {
            double v = sin_[tl.ltid];
            if (tl.ltid == S_DONE) v = 3.0;
            if (tl.ltid == S_B2) v = b2;
            if (tl.ltid == S_TARGET) v = target;
            if (tl.ltid == S_RRUPD) v = rrupd;
            if (tl.ltid == S_GCUR) v = gam;
            sout[tl.ltid] = v;
        }
        return;
    }
    const double alpha = gam / den;
    const R b = (R)beta, a = (R)alpha;

    // s_i = w_i + beta s_{i-1};  r_{i+1} = r_i - alpha s_i on the three slices
#pragma unroll
    for (int m = 0; m < MC; m++)
#pragma unroll
        for (int q = 0; q < 4; q++) {
            sm.v[m][q] = cfma(b, sm.v[m][q], wm.v[m][q]);
            st.v[m][q] = cfma(b, st.v[m][q], wt.v[m][q]);
            sn.v[m][q] = cfma(b, sn.v[m][q], wn.v[m][q]);
            pp.v[m][q] = cfma(b, pp.v[m][q], rt.v[m][q]);  // p_i = r_i + beta p_{i-1}
            rm.v[m][q] = cfma(-a, sm.v[m][q], rm.v[m][q]);
            rt.v[m][q] = cfma(-a, st.v[m][q], rt.v[m][q]);
            rn.v[m][q] = cfma(-a, sn.v[m][q], rn.v[m][q]);
        }
    store_cells<R, MC>(st, B.s[nx] + c.tau * Vs, c.g, c.own);
    store_cells<R, MC>(rt, B.r[nx] + c.tau * Vs, c.g, c.own);
    store_cells<R, MC>(pp, B.p + c.tau * Vs, c.g, c.own);
    // x_{i+1} = x_i + alpha p_i in FP64
#pragma unroll
    for (int m = 0; m < MC; m++)
#pragma unroll
        for (int q = 0; q < 4; q++) {
            xo.v[m][q].re += alpha * (double)pp.v[m][q].re;
            xo.v[m][q].im += alpha * (double)pp.v[m][q].im;
        }
    store_cells<double, MC>(xo, B.x + c.tau * Vs, c.g, c.own);
    const Cells<R, MC> rnew = rt;
    Cells<R, MC> w;
    mdagm_cells<R, MC, NB>(rm, rt, rn, hm, ht, c.g, c.own, co, c.tau == 0 ? R(-1) : R(1),
                           c.tau == lt.Nt - 1 ? R(-1) : R(1), buf2, lt.Vs, w);
    store_cells<R, MC>(w, B.w[nx] + c.tau * Vs, c.g, c.own);
    double v[kNP] = {dot_cells<R, MC>(rnew, rnew, c.own), dot_cells<R, MC>(w, rnew, c.own),
                     dot_cells<R, MC>(rnew, st, c.own), dot_cells<R, MC>(pp, w, c.own),
                     dot_cells<R, MC>(pp, st, c.own), 0.0};
    write_partials(B.part + kNP * ((size_t)lt.Nt * nx + c.tau), v, tl);
    if (lead && tl.ltid < S_NSLOT) {
        double v = sin_[tl.ltid];
        if (tl.ltid == S_GPREV) v = gam;
        if (tl.ltid == S_APREV) v = alpha;
        if (tl.ltid == S_ITERS) v = (double)(it + 1);
        if (tl.ltid == S_FIRST) v = 0.0;
        if (tl.ltid == S_B2) v = b2;
        if (tl.ltid == S_TARGET) v = target;
        if (tl.ltid == S_RRUPD) v = rrupd;
        if (tl.ltid == S_GCUR) v = gam;
        sout[tl.ltid] = v;
    }
}

// ---------------------------------------------------------------------------
// Reliable update / true residual: r_i = rhs - O x (FP64 O x given), w_i =
// O r_i in the working precision, partials of iteration i replaced; aux gets
// the FP64 |rhs - O x|^2.  Slot kpar is only read.
// ---------------------------------------------------------------------------
template <typename R, int MC, int NB>
__device__ __forceinline__ void cg_replace_body(const Lat& lt, const CgBufs<R>& B, const cplx<R>* __restrict__ gauge,
                                                const Coef<R>& co, const double* __restrict__ scal, int kpar,
                                                int tau, const Tile& tl) {
    cplx<R>* buf2 = reinterpret_cast<cplx<R>*>(tl.buf);
    const int ip = 0;  // the resumed recursion restarts its ping-pong at buffer 0
    SliceCtx<MC> c;
    slice_ctx<MC>(lt, c, tau, tl);
    const size_t Vs = lt.Vs;
    cplx<R> hm[MC][12], ht[MC][12];
    hops_of<R, MC>(gauge, lt, c.tm, c.idx, co, hm);
    hops_of<R, MC>(gauge, lt, c.tau, c.idx, co, ht);
    Cells<R, MC> vm, vt, vn, w;
    double t2 = 0.0, dummy = 0.0;
    load_cvt<R, MC>(vm, B.rhs + c.tm * Vs, B.Ox + c.tm * Vs, c.g, c.own, dummy);
    load_cvt<R, MC>(vt, B.rhs + c.tau * Vs, B.Ox + c.tau * Vs, c.g, c.own, t2);
    load_cvt<R, MC>(vn, B.rhs + c.tp * Vs, B.Ox + c.tp * Vs, c.g, c.own, dummy);
    store_cells<R, MC>(vt, B.r[ip] + c.tau * Vs, c.g, c.own);
    const Cells<R, MC> r0 = vt;
    const R em = c.tau == 0 ? R(-1) : R(1), et = c.tau == lt.Nt - 1 ? R(-1) : R(1);
    mdagm_cells<R, MC, NB>(vm, vt, vn, hm, ht, c.g, c.own, co, em, et, buf2, lt.Vs, w);
    store_cells<R, MC>(w, B.w[ip] + c.tau * Vs, c.g, c.own);
    // s_{i-1} = O p_{i-1}, recomputed
    Cells<R, MC> pm, pt_, pn, sp;
    load_cells<R, MC>(pm, B.p + c.tm * Vs, c.g, c.own);
    load_cells<R, MC>(pt_, B.p + c.tau * Vs, c.g, c.own);
    load_cells<R, MC>(pn, B.p + c.tp * Vs, c.g, c.own);
    __syncthreads();  // LDS exchange buffers are reused
    mdagm_cells<R, MC, NB>(pm, pt_, pn, hm, ht, c.g, c.own, co, em, et, buf2, lt.Vs, sp);
    store_cells<R, MC>(sp, B.s[ip] + c.tau * Vs, c.g, c.own);
    double v[kNP] = {dot_cells<R, MC>(r0, r0, c.own), dot_cells<R, MC>(w, r0, c.own),
                     dot_cells<R, MC>(r0, sp, c.own), dot_cells<R, MC>(pt_, w, c.own),
                     dot_cells<R, MC>(pt_, sp, c.own), t2};
    write_partials(B.part + kNP * ((size_t)lt.Nt * ip + c.tau), v, tl);
}


// After k_cg_replace: true |r|^2 into the slot; converged -> stop flag 1;
// otherwise clear the flag and resume (restart: beta = 0 on the next
// iteration, the FP64 path's p = r).
__device__ __forceinline__ void cg_check_body(double* __restrict__ scal, int kpar, const double* __restrict__ part,
                                              int Nt, int restart, double* red) {
    double* sl = scal + S_NSLOT * kpar;
    const int ip = 0;  // the replacement's partials
    double pr[kNP];
    reduce_partials(part + kNP * (size_t)Nt * ip, Nt, whole_block_tile(nullptr, red), pr);
    const double a = pr[0], c = pr[5];
    if (threadIdx.x == 0) {
        sl[S_TRUE] = c;
        if (c <= sl[S_TARGET]) {
            sl[S_DONE] = 1.0;
        } else {
            sl[S_DONE] = 0.0;
            if (restart) sl[S_FIRST] = 1.0;
            sl[S_ITUPD] = sl[S_ITERS];
            sl[S_RRUPD] = a;
        }
    }
}

}  // namespace qh
