// Conjugate gradient on O = M^dag M (Methods, Eq. pCG), started from x = 0.
//
// Every scalar of the recursion (alpha, beta, |r|^2) lives on the device and
// is reduced in FP64 in a fixed order, so a solve is bitwise reproducible for
// a given launch shape.  A device stop flag turns the remaining iterations of
// a launched chunk into no-ops once |r| <= tol |rhs|, so the host only reads
// the flag once per chunk.
//
// Mixed precision (QEDHMC_FP32): r, p and O p are complex FP32 and the matvec
// runs in FP32; x accumulates in FP64.  The residual is recomputed in FP64 as
// r = rhs - O x and copied into the FP32 r, with p kept (a reliable update,
// Sleijpen and van der Vorst 1996), whenever the recursive residual has
// dropped by a factor 10 since the last update, at least every 50
// iterations, and when it reaches the target.  The solve ends when that FP64
// true residual meets tol.  Updating once per decade keeps the gap between
// the FP32 recursion and the true residual far below the residual itself, so
// replacing r does not disturb the conjugacy of the directions.
#include "qedhmc_internal.h"

namespace qh {

// Device scalar slots (h->scal)
enum {
    S_RR = 0,      // current |r|^2 of the recursion
    S_ALPHA = 1,
    S_BETA = 2,
    S_B2 = 3,      // |rhs|^2
    S_DONE = 4,    // 1: recursive residual reached the target
    S_TARGET = 5,  // tol^2 |rhs|^2
    S_ITERS = 6,   // iterations performed
    S_TRUE = 7,    // last true |r|^2
    S_RRUPD = 8,   // |r|^2 at the last reliable update (mixed path)
    S_RRPREV = 9,  // |r|^2 before the last recursive update (for beta after a replacement)
    S_ITUPD = 10,  // iteration count at the last reliable update
};
// S_DONE values: 0 running, 1 target reached, 2 paused for a reliable update
static constexpr double kDelta2 = 0.01;  // (factor 10)^-2

static constexpr int kGridV = 512;   // blocks of the vector kernels (fixed: deterministic sums)
static constexpr int kBlockV = 256;

// partial slots in h->partial: [0, Nt) per-slice partials of <p, Op>, then
// kGridV partials of the vector kernels (see part_vec)
static double* part_dot(qedhmc_ctx* h) { return h->partial; }
static double* part_vec(qedhmc_ctx* h) { return h->partial + h->lat.Nt; }

__global__ void k_finish_sum(const double* __restrict__ part, int n, double* __restrict__ out) {
    __shared__ double red[16];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) *out = s;
}

// r = rhs (in working precision), p = r, x = 0; partial |rhs|^2
template <typename R>
__global__ void k_cg_init(const cplx<double>* __restrict__ rhs, cplx<R>* __restrict__ r, cplx<R>* __restrict__ p,
                          cplx<double>* __restrict__ x, size_t n, double* __restrict__ part) {
    __shared__ double red[16];
    double s = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const cplx<double> b = rhs[i];
        const cplx<R> br = mk<R>((R)b.re, (R)b.im);
        r[i] = br;
        p[i] = br;
        x[i] = mk<double>(0.0, 0.0);
        s += b.re * b.re + b.im * b.im;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_cg_setup(double* __restrict__ sc, const double* __restrict__ part, int n, double tol2) {
    __shared__ double red[16];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
        sc[S_B2] = s;
        sc[S_RR] = s;
        sc[S_TARGET] = tol2 * s;
        sc[S_DONE] = (s <= tol2 * s) ? 1.0 : 0.0;
        sc[S_ITERS] = 0.0;
        sc[S_RRUPD] = s;
        sc[S_RRPREV] = s;
        sc[S_ITUPD] = 0.0;
    }
}

// alpha = |r|^2 / <p, Op> (0 once the stop flag is up)
__global__ void k_cg_alpha(double* __restrict__ sc, const double* __restrict__ part, int n) {
    __shared__ double red[16];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) sc[S_ALPHA] = sc[S_DONE] != 0.0 ? 0.0 : sc[S_RR] / s;
}

// x += alpha p; r -= alpha Op; partial |r|^2
template <typename R>
__global__ void k_cg_update(double* __restrict__ sc, cplx<double>* __restrict__ x, cplx<R>* __restrict__ r,
                            const cplx<R>* __restrict__ p, const cplx<R>* __restrict__ q, size_t n,
                            double* __restrict__ part) {
    __shared__ double red[16];
    const double alpha = sc[S_ALPHA];
    const bool live = sc[S_DONE] == 0.0;
    const R ar = (R)alpha;
    double s = 0.0;
    if (live) {
        for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
            const cplx<R> pi = p[i];
            cplx<double> xi = x[i];
            xi.re += alpha * (double)pi.re;
            xi.im += alpha * (double)pi.im;
            x[i] = xi;
            cplx<R> ri = r[i];
            const cplx<R> qi = q[i];
            ri.re -= ar * qi.re;
            ri.im -= ar * qi.im;
            r[i] = ri;
            s += (double)ri.re * (double)ri.re + (double)ri.im * (double)ri.im;
        }
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// beta = |r_new|^2 / |r|^2; stop flag when |r_new|^2 <= target.  Mixed path:
// pause flag (before p is updated) when |r| fell by 10 since the last reliable
// update or 50 iterations have passed since it.
__global__ void k_cg_beta(double* __restrict__ sc, const double* __restrict__ part, int n, int mixed) {
    __shared__ double red[16];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
        if (sc[S_DONE] == 0.0) {
            const double prev = sc[S_RR];
            sc[S_RRPREV] = prev;
            sc[S_BETA] = s / prev;
            sc[S_RR] = s;
            sc[S_ITERS] += 1.0;
            if (s <= sc[S_TARGET])
                sc[S_DONE] = 1.0;
            else if (mixed && (s <= kDelta2 * sc[S_RRUPD] || sc[S_ITERS] - sc[S_ITUPD] >= 50.0))
                sc[S_DONE] = 2.0;
        }
    }
}

// p = r + beta p
template <typename R>
__global__ void k_cg_p(const double* __restrict__ sc, const cplx<R>* __restrict__ r, cplx<R>* __restrict__ p,
                       size_t n) {
    if (sc[S_DONE] != 0.0) return;
    const R b = (R)sc[S_BETA];
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const cplx<R> ri = r[i], pi = p[i];
        p[i] = mk<R>(ri.re + b * pi.re, ri.im + b * pi.im);
    }
}

// True residual in FP64: r64 = rhs - Ox; r (working precision) = r64; partial |r64|^2.
// restart != 0 also sets p = r (used when the recursion stopped but the true
// residual is still above tol).
template <typename R>
__global__ void k_cg_true(const cplx<double>* __restrict__ rhs, const cplx<double>* __restrict__ Ox,
                          cplx<R>* __restrict__ r, cplx<R>* __restrict__ p, int restart, size_t n,
                          double* __restrict__ part) {
    __shared__ double red[16];
    double s = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const cplx<double> b = rhs[i], o = Ox[i];
        const double re = b.re - o.re, im = b.im - o.im;
        const cplx<R> rr = mk<R>((R)re, (R)im);
        r[i] = rr;
        if (restart) p[i] = rr;
        s += re * re + im * im;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// After a true-residual recomputation: |r|^2 <- true value and the stop flag
// is cleared.  complete != 0 finishes the interrupted iteration: beta is
// recomputed against the replaced residual, beta = |r_true|^2 / |r_prev|^2,
// for the p update that follows.
__global__ void k_cg_after_true(double* __restrict__ sc, const double* __restrict__ part, int n, int complete) {
    __shared__ double red[16];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
        sc[S_TRUE] = s;
        sc[S_RR] = s;
        sc[S_RRUPD] = s;
        sc[S_ITUPD] = sc[S_ITERS];
        if (complete) sc[S_BETA] = s / sc[S_RRPREV];
        sc[S_DONE] = 0.0;
    }
}

__global__ void k_cg_fix_beta(double* __restrict__ sc) {
    if (threadIdx.x == 0) sc[S_BETA] = sc[S_TRUE] / sc[S_RRPREV];
}

template <typename R>
__global__ void k_cg_copy(const cplx<R>* __restrict__ a, cplx<R>* __restrict__ b, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

template <typename R>
static qedhmc_status cg_iterations(qedhmc_ctx* h, qedhmc_precision prec, double* x, cplx<R>* r, cplx<R>* p,
                                   cplx<R>* q, int count) {
    const size_t N = (size_t)h->lat.Nt * h->lat.Vs;
    double* sc = h->scal;
    double* pd = part_dot(h);
    double* pv = part_vec(h);
    for (int k = 0; k < count; k++) {
        QH_TRY(launch_mdagm(h, prec, p, q, pd));
        hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(256), 0, h->stream, sc, pd, h->lat.Nt);
        hipLaunchKernelGGL(k_cg_update<R>, dim3(kGridV), dim3(kBlockV), 0, h->stream, sc, (cplx<double>*)x, r,
                           (const cplx<R>*)p, (const cplx<R>*)q, N, pv);
        hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(256), 0, h->stream, sc, pv, kGridV, prec != QEDHMC_FP64 ? 1 : 0);
        hipLaunchKernelGGL(k_cg_p<R>, dim3(kGridV), dim3(kBlockV), 0, h->stream, (const double*)sc,
                           (const cplx<R>*)r, p, N);
    }
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

// Recompute the true residual in FP64 into r.  mode 0: only replace r;
// mode 1: restart (p = r); mode 2: replace r and finish the interrupted
// iteration with p = r + beta p.
template <typename R>
static qedhmc_status cg_true_resid(qedhmc_ctx* h, const double* rhs, const double* x, cplx<R>* r, cplx<R>* p,
                                   int mode) {
    const size_t N = (size_t)h->lat.Nt * h->lat.Vs;
    double* Ox = (double*)h->ws[3];
    double* pv = part_vec(h);
    QH_TRY(launch_mdagm(h, QEDHMC_FP64, x, Ox, nullptr));
    hipLaunchKernelGGL(k_cg_true<R>, dim3(kGridV), dim3(kBlockV), 0, h->stream, (const cplx<double>*)rhs,
                       (const cplx<double>*)Ox, r, p, mode == 1 ? 1 : 0, N, pv);
    hipLaunchKernelGGL(k_cg_after_true, dim3(1), dim3(256), 0, h->stream, h->scal, pv, kGridV, mode == 2 ? 1 : 0);
    if (mode == 2)
        hipLaunchKernelGGL(k_cg_p<R>, dim3(kGridV), dim3(kBlockV), 0, h->stream, (const double*)h->scal,
                           (const cplx<R>*)r, p, N);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

static qedhmc_status read_scal(qedhmc_ctx* h) {
    QH_HIP(hipMemcpyAsync(h->h_pinned, h->scal, 8 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    QH_HIP(hipStreamSynchronize(h->stream));
    return QEDHMC_OK;
}

// True residual into r (no change of p), its relative norm on the host.
template <typename R>
static qedhmc_status read_true(qedhmc_ctx* h, const double* rhs, const double* x, cplx<R>* r, cplx<R>* p, int mode,
                               double b2, double& rel) {
    QH_TRY(cg_true_resid<R>(h, rhs, x, r, p, mode));
    QH_TRY(read_scal(h));
    rel = std::sqrt(h->h_pinned[S_TRUE] / b2);
    return QEDHMC_OK;
}

// Continue after a failed convergence check whose true residual is in r:
// mixed -> finish the iteration (beta against the replaced residual, then
// p = r + beta p); FP64 -> restart with p = r.
template <typename R>
static qedhmc_status cg_continue(qedhmc_ctx* h, cplx<R>* r, cplx<R>* p, bool mixed) {
    const size_t N = (size_t)h->lat.Nt * h->lat.Vs;
    if (mixed) {
        hipLaunchKernelGGL(k_cg_fix_beta, dim3(1), dim3(64), 0, h->stream, h->scal);
        hipLaunchKernelGGL(k_cg_p<R>, dim3(kGridV), dim3(kBlockV), 0, h->stream, (const double*)h->scal,
                           (const cplx<R>*)r, p, N);
    } else {
        hipLaunchKernelGGL(k_cg_copy<R>, dim3(kGridV), dim3(kBlockV), 0, h->stream, (const cplx<R>*)r, p, N);
    }
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

template <typename R>
static qedhmc_status cg_t(qedhmc_ctx* h, const double* rhs, double* x, double tol, int maxit, qedhmc_precision prec,
                          int* iters, double* true_rel, int* n_reliable) {
    const size_t N = (size_t)h->lat.Nt * h->lat.Vs;
    cplx<R>* r = (cplx<R>*)h->ws[0];
    cplx<R>* p = (cplx<R>*)h->ws[1];
    cplx<R>* q = (cplx<R>*)h->ws[2];
    const bool mixed = prec != QEDHMC_FP64;
    const int kChunk = 50;  // host check period (the mixed path pauses itself at least every 50)
    int nrel = 0;

    // FP64 rhs -> working precision before the ensure_gauge of the caller's theta
    hipLaunchKernelGGL(k_cg_init<R>, dim3(kGridV), dim3(kBlockV), 0, h->stream, (const cplx<double>*)rhs, r, p,
                       (cplx<double>*)x, N, part_vec(h));
    hipLaunchKernelGGL(k_cg_setup, dim3(1), dim3(256), 0, h->stream, h->scal, part_vec(h), kGridV, tol * tol);
    QH_HIP(hipGetLastError());
    QH_TRY(read_scal(h));
    const double b2 = h->h_pinned[S_B2];
    if (b2 == 0.0) {
        if (iters) *iters = 0;
        if (true_rel) *true_rel = 0.0;
        if (n_reliable) *n_reliable = 0;
        return QEDHMC_OK;
    }
    int it = 0;
    double rel = 1.0;
    bool converged = false;
    while (true) {
        const int left = maxit - it;
        if (left > 0) QH_TRY(cg_iterations<R>(h, prec, x, r, p, q, left < kChunk ? left : kChunk));
        QH_TRY(read_scal(h));
        it = (int)h->h_pinned[S_ITERS];
        const double flag = h->h_pinned[S_DONE];
        if (flag == 1.0 || it >= maxit) {
            // true residual check (FP64).  Not yet converged: the FP64 path
            // restarts from it (p = r); the mixed path keeps p and finishes the
            // interrupted iteration (a reliable update).
            QH_TRY(read_true(h, rhs, x, r, p, 0, b2, rel));
            nrel++;
            if (rel <= tol) {
                converged = true;
                break;
            }
            if (it >= maxit) break;
            QH_TRY(cg_continue<R>(h, r, p, mixed));
        } else if (flag == 2.0) {
            // reliable update at the pause: replace r, keep p, finish the iteration
            QH_TRY(cg_true_resid<R>(h, rhs, x, r, p, 2));
            nrel++;
        }
    }
    if (iters) *iters = it;
    if (true_rel) *true_rel = rel;
    if (n_reliable) *n_reliable = nrel;
    return converged ? QEDHMC_OK : QEDHMC_ENOCONV;
}

qedhmc_status cg_solve_impl(qedhmc_ctx* h, const double* rhs, double* x, double tol, int maxit,
                            qedhmc_precision prec, int* iters, double* true_rel, int* n_reliable) {
    if (prec == QEDHMC_FP64) return cg_t<double>(h, rhs, x, tol, maxit, prec, iters, true_rel, n_reliable);
    return cg_t<float>(h, rhs, x, tol, maxit, prec, iters, true_rel, n_reliable);
}

}  // namespace qh
