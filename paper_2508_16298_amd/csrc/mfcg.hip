// Flexible CG on M^dag M x = eta with the learned preconditioner in mixed
// precision: the residual r, the direction p, s = O p and the preconditioned
// residual z in complex FP32 with the FP32 fused M^dag M; the solution x, every
// inner product and the coefficients in FP64; reliable updates that replace
// r by the FP64 residual eta - O x (Sleijpen and van der Vorst 1996).
//
// Iteration (Notay's flexible CG, the complex form of the method's CG of
// Methods, "CG method and preconditioner", Eq. pCG, with z = N(theta, r)):
//   s = O p;  alpha = <p, r> / <p, s>;  x += alpha p;  r -= alpha s;
//   z = N(r) (or the fallback);  beta = -<s, z> / <p, s>;  p = z + beta p,
// with <a, b> = sum conj(a) b.  The residual judges the network: it keeps the
// solve while |r| at least halves over every 10 iterations and its
// directions descend (<p, O p> > 0); otherwise the fallback finishes the
// solve from the current x: the residual system O d = eta - O x (residual in
// FP64) goes to the library's device-driven mixed CG (with the paper's
// preconditioner, or none) at the tolerance that makes x + d meet the
// original one, and x += d.
//
// alpha and beta are formed on the device from the partial sums (one small
// kernel each), so the host reads back only <p, O p> and |r|^2 once per
// iteration to take the stop, reliable-update and judge decisions.
#include <cmath>
#include <string>
#include <vector>

#include "net_internal.h"

namespace qh {

static constexpr int kMfBlocks = 256;  // partial-sum blocks of every reduction
static constexpr int kMfThreads = 256;
static constexpr int kRelEvery = 50;   // iterations between reliable updates at most
static constexpr double kRelDrop = 1e-4;  // |r|^2 fall that triggers one earlier

// device scalar slots (n->dscal): the network reads |r|^2 at 0
enum { M_RR = 0, M_PS = 16, M_ARE, M_AIM, M_BRE, M_BIM };

__device__ __forceinline__ void part_out(double v, double* red, double* part, int k) {
    const double t = block_sum(v, red);
    if (threadIdx.x == 0) part[4 * blockIdx.x + k] = t;
    __syncthreads();
}

// x = 0, r = eta rounded to FP32, partials of |eta|^2
__global__ __launch_bounds__(kMfThreads) void k_mf_start(int N, const cplx<double>* __restrict__ eta,
                                                         cplx<double>* __restrict__ x, cplx<float>* __restrict__ r,
                                                         double* __restrict__ part) {
    __shared__ double red[16];
    double acc = 0.0;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < N; n += gridDim.x * blockDim.x) {
        const cplx<double> e = eta[n];
        x[n] = mk<double>(0.0, 0.0);
        r[n] = mk<float>((float)e.re, (float)e.im);
        acc += e.re * e.re + e.im * e.im;
    }
    part_out(acc, red, part, 0);
}

// partials of <p, s> (real: O is Hermitian) and <p, r>
__global__ __launch_bounds__(kMfThreads) void k_mf_dot_pspr(int N, const cplx<float>* __restrict__ p,
                                                            const cplx<float>* __restrict__ s,
                                                            const cplx<float>* __restrict__ r,
                                                            double* __restrict__ part) {
    __shared__ double red[16];
    double ps = 0.0, prr = 0.0, pri = 0.0;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < N; n += gridDim.x * blockDim.x) {
        const cplx<float> a = p[n], b = s[n], c = r[n];
        const double ar = a.re, ai = a.im;
        ps += ar * b.re + ai * b.im;
        prr += ar * c.re + ai * c.im;
        pri += ar * c.im - ai * c.re;
    }
    part_out(ps, red, part, 0);
    part_out(prr, red, part, 1);
    part_out(pri, red, part, 2);
}

// partials of <s, z>
__global__ __launch_bounds__(kMfThreads) void k_mf_dot_sz(int N, const cplx<float>* __restrict__ s,
                                                          const cplx<float>* __restrict__ z,
                                                          double* __restrict__ part) {
    __shared__ double red[16];
    double re = 0.0, im = 0.0;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < N; n += gridDim.x * blockDim.x) {
        const cplx<float> a = s[n], b = z[n];
        const double ar = a.re, ai = a.im;
        re += ar * b.re + ai * b.im;
        im += ar * b.im - ai * b.re;
    }
    part_out(re, red, part, 0);
    part_out(im, red, part, 1);
}

// ordered sums of the partials, then the coefficient of the step:
// mode 0: |r|^2 into sc[M_RR]
// mode 1: <p, s> into sc[M_PS] and alpha = <p, r> / <p, s> (0 when <p, s> is
//         not positive: the update is then a no-op and the host switches)
// mode 2: beta = -<s, z> / <p, s>
__global__ void k_mf_coef(const double* __restrict__ part, int nb, int mode, double* __restrict__ sc) {
    if (threadIdx.x != 0) return;
    double v[3] = {0.0, 0.0, 0.0};
    for (int b = 0; b < nb; b++)
        for (int k = 0; k < 3; k++) v[k] += part[4 * b + k];
    if (mode == 0) {
        sc[M_RR] = v[0];
    } else if (mode == 1) {
        const double ps = v[0];
        sc[M_PS] = ps;
        const bool ok = ps > 0.0;
        sc[M_ARE] = ok ? v[1] / ps : 0.0;
        sc[M_AIM] = ok ? v[2] / ps : 0.0;
    } else {
        const double ps = sc[M_PS];
        sc[M_BRE] = -v[0] / ps;
        sc[M_BIM] = -v[1] / ps;
    }
}

// x += alpha p (FP64); r -= alpha s (formed in FP64, stored FP32); partials of |r|^2
__global__ __launch_bounds__(kMfThreads) void k_mf_update(int N, const double* __restrict__ sc,
                                                          const cplx<float>* __restrict__ p,
                                                          const cplx<float>* __restrict__ s,
                                                          cplx<double>* __restrict__ x, cplx<float>* __restrict__ r,
                                                          double* __restrict__ part) {
    __shared__ double red[16];
    const double are = sc[M_ARE], aim = sc[M_AIM];
    double acc = 0.0;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < N; n += gridDim.x * blockDim.x) {
        const cplx<float> pv = p[n], sv = s[n];
        cplx<double> xv = x[n];
        const cplx<float> rv = r[n];
        xv.re += are * pv.re - aim * pv.im;
        xv.im += are * pv.im + aim * pv.re;
        const double rre = (double)rv.re - (are * sv.re - aim * sv.im);
        const double rim = (double)rv.im - (are * sv.im + aim * sv.re);
        x[n] = xv;
        const cplx<float> rn = mk<float>((float)rre, (float)rim);
        r[n] = rn;
        acc += (double)rn.re * rn.re + (double)rn.im * rn.im;
    }
    part_out(acc, red, part, 0);
}

// p = z + beta p
__global__ void k_mf_dir(int N, const double* __restrict__ sc, const cplx<float>* __restrict__ z,
                         cplx<float>* __restrict__ p) {
    const double bre = sc[M_BRE], bim = sc[M_BIM];
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < N; n += gridDim.x * blockDim.x) {
        const cplx<float> zv = z[n], pv = p[n];
        p[n] = mk<float>((float)(zv.re + bre * pv.re - bim * pv.im), (float)(zv.im + bre * pv.im + bim * pv.re));
    }
}

// reliable update: r = eta - O x in FP64, stored FP32; partials of |eta - O x|^2
__global__ __launch_bounds__(kMfThreads) void k_mf_replace(int N, const cplx<double>* __restrict__ eta,
                                                           const cplx<double>* __restrict__ Ox,
                                                           cplx<float>* __restrict__ r, double* __restrict__ part) {
    __shared__ double red[16];
    double acc = 0.0;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < N; n += gridDim.x * blockDim.x) {
        const double re = eta[n].re - Ox[n].re, im = eta[n].im - Ox[n].im;
        r[n] = mk<float>((float)re, (float)im);
        acc += re * re + im * im;
    }
    part_out(acc, red, part, 0);
}

// r64 = eta - O x in FP64; partials of |r64|^2
__global__ __launch_bounds__(kMfThreads) void k_mf_resid64(int N, const cplx<double>* __restrict__ eta,
                                                           const cplx<double>* __restrict__ Ox,
                                                           cplx<double>* __restrict__ r, double* __restrict__ part) {
    __shared__ double red[16];
    double acc = 0.0;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < N; n += gridDim.x * blockDim.x) {
        const double re = eta[n].re - Ox[n].re, im = eta[n].im - Ox[n].im;
        r[n] = mk<double>(re, im);
        acc += re * re + im * im;
    }
    part_out(acc, red, part, 0);
}

// x += d
__global__ void k_mf_add64(int N, cplx<double>* __restrict__ x, const cplx<double>* __restrict__ d) {
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < N; n += gridDim.x * blockDim.x)
        x[n] = mk<double>(x[n].re + d[n].re, x[n].im + d[n].im);
}

// the network's output in FP32: z = s (o_0 + i o_1), s = |r| / sqrt(N)
__global__ void k_net_out32(int N, const float* __restrict__ o, const double* __restrict__ rr,
                            cplx<float>* __restrict__ z) {
    const double s = sqrt(*rr / (double)N);
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < N; n += gridDim.x * blockDim.x)
        z[n] = mk<float>((float)(s * (double)o[2 * n]), (float)(s * (double)o[2 * n + 1]));
}

static int mf_grid(int N) {
    const int g = (N + kMfThreads - 1) / kMfThreads;
    return g < kMfBlocks ? (g < 1 ? 1 : g) : kMfBlocks;
}

qedhmc_status mfcg_solve_impl(qedhmc_net* n, const double* rhs, double* x, double tol, int maxit,
                              qedhmc_net_arith arith, qedhmc_precond fallback, int* iters, double* true_rel,
                              int* n_reliable, int* switched_at) {
    qedhmc_ctx* h = n->h;
    hipStream_t st = h->stream;
    const int N = n->g.N;
    const int nb = mf_grid(N);
    const dim3 grid(nb), blk(kMfThreads);
    // FP32 vectors in the network's solver buffers (each sized for FP64)
    cplx<float>* r = reinterpret_cast<cplx<float>*>(n->fr);
    cplx<float>* p = reinterpret_cast<cplx<float>*>(n->fp);
    cplx<float>* s = reinterpret_cast<cplx<float>*>(n->fs);
    cplx<float>* z = reinterpret_cast<cplx<float>*>(n->fz);
    cplx<double>* X = reinterpret_cast<cplx<double>*>(x);
    const cplx<double>* eta = reinterpret_cast<const cplx<double>*>(rhs);
    double* sc = n->dscal;
    double* part = n->dpart;
    *iters = 0;
    *true_rel = 0.0;
    *n_reliable = 0;
    *switched_at = -1;
    double true_rr_out = 0.0;  // the fallback's finish: true |r|^2 of its result
    if (fallback == QEDHMC_PC_PAPER) QH_TRY(ensure_paper_precond(h));

    auto read = [&](int a, int b) -> qedhmc_status {  // host copies of sc[a], sc[b]
        QH_HIP(hipMemcpyAsync(n->hpin, sc + a, sizeof(double), hipMemcpyDeviceToHost, st));
        QH_HIP(hipMemcpyAsync(n->hpin + 1, sc + b, sizeof(double), hipMemcpyDeviceToHost, st));
        QH_HIP(hipStreamSynchronize(st));
        return QEDHMC_OK;
    };
    bool net_on = true;
    auto precond = [&]() -> qedhmc_status {  // z from r
        if (net_on) {
            QH_TRY(net_infer(n, r, true, sc + M_RR, arith));
            hipLaunchKernelGGL(k_net_out32, grid, blk, 0, st, N, (const float*)n->act[kNetLayers],
                               (const double*)(sc + M_RR), z);
            QH_HIP(hipGetLastError());
            return QEDHMC_OK;
        }
        if (fallback == QEDHMC_PC_PAPER) return launch_apply_precond(h, QEDHMC_FP32, r, z);
        QH_HIP(hipMemcpyAsync(z, r, (size_t)N * sizeof(cplx<float>), hipMemcpyDeviceToDevice, st));
        return QEDHMC_OK;
    };
    auto restart = [&]() -> qedhmc_status {  // p = z = P r
        QH_TRY(precond());
        QH_HIP(hipMemcpyAsync(p, z, (size_t)N * sizeof(cplx<float>), hipMemcpyDeviceToDevice, st));
        return QEDHMC_OK;
    };
    auto reliable = [&](double& rr) -> qedhmc_status {  // r = eta - O x in FP64; |r|^2
        QH_TRY(launch_mdagm(h, QEDHMC_FP64, x, h->ws[3], nullptr));
        hipLaunchKernelGGL(k_mf_replace, grid, blk, 0, st, N, eta, (const cplx<double>*)h->ws[3], r, part);
        hipLaunchKernelGGL(k_mf_coef, dim3(1), dim3(64), 0, st, (const double*)part, nb, 0, sc);
        QH_HIP(hipGetLastError());
        QH_TRY(read(M_RR, M_RR));
        rr = n->hpin[0];
        (*n_reliable)++;
        return QEDHMC_OK;
    };

    // the fallback's finish: O d = eta - O x by the device-driven mixed (P)CG,
    // x += d; true_rr from the FP64 residual of the sum
    auto finish = [&](double nb2_, bool& conv) -> qedhmc_status {
        cplx<double>* r64 = n->fp;  // FP64-sized buffers of the network's solver, free now
        cplx<double>* d = n->fz;
        auto resid = [&](double& rr) -> qedhmc_status {
            QH_TRY(launch_mdagm(h, QEDHMC_FP64, x, h->ws[3], nullptr));
            hipLaunchKernelGGL(k_mf_resid64, grid, blk, 0, st, N, eta, (const cplx<double>*)h->ws[3], r64, part);
            hipLaunchKernelGGL(k_mf_coef, dim3(1), dim3(64), 0, st, (const double*)part, nb, 0, sc);
            QH_HIP(hipGetLastError());
            QH_TRY(read(M_RR, M_RR));
            rr = n->hpin[0];
            return QEDHMC_OK;
        };
        double rr = 0.0;
        QH_TRY(resid(rr));
        conv = rr <= tol * tol * nb2_;
        if (conv || !std::isfinite(rr)) {
            true_rr_out = rr;
            return QEDHMC_OK;
        }
        const double tol_d = tol * std::sqrt(nb2_ / rr);
        int it_d = 0, nrel_d = 0;
        double rel_d = 0.0;
        const int budget = std::max(1, maxit - *iters);
        const qedhmc_status sd = fallback == QEDHMC_PC_PAPER
                                     ? pcg_solve_impl(h, (const double*)r64, (double*)d, tol_d, budget, QEDHMC_FP32,
                                                      &it_d, &rel_d, &nrel_d)
                                     : cg_solve_impl(h, (const double*)r64, (double*)d, tol_d, budget, QEDHMC_FP32,
                                                     &it_d, &rel_d, &nrel_d);
        if (sd != QEDHMC_OK && sd != QEDHMC_ENOCONV) return sd;
        *iters += it_d;
        *n_reliable += nrel_d;
        hipLaunchKernelGGL(k_mf_add64, grid, blk, 0, st, N, X, (const cplx<double>*)d);
        QH_HIP(hipGetLastError());
        QH_TRY(resid(rr));
        true_rr_out = rr;
        conv = rr <= tol * tol * nb2_;
        return QEDHMC_OK;
    };

    hipLaunchKernelGGL(k_mf_start, grid, blk, 0, st, N, eta, X, r, part);
    hipLaunchKernelGGL(k_mf_coef, dim3(1), dim3(64), 0, st, (const double*)part, nb, 0, sc);
    QH_HIP(hipGetLastError());
    QH_TRY(read(M_RR, M_RR));
    const double nb2 = n->hpin[0];
    if (nb2 == 0.0) return QEDHMC_OK;
    if (!std::isfinite(nb2)) {
        set_error("mixed flexible CG: non-finite right-hand side");
        return QEDHMC_ENOCONV;
    }
    const double target2 = tol * tol * nb2;
    std::vector<double> hist;  // |r| after every iteration, for the judge
    int it = 0, since = 0, stalls = 0;
    double rr_rel = nb2;      // |r|^2 at the last reliable update
    double best_true = nb2;   // smallest true |r|^2 so far
    double true_rr = nb2;
    bool converged = false, broke = false, handed_over = false;
    const char* why = "maximum iteration count reached";
    QH_TRY(restart());
    while (true) {
        QH_TRY(launch_mdagm(h, QEDHMC_FP32, p, s, nullptr));
        hipLaunchKernelGGL(k_mf_dot_pspr, grid, blk, 0, st, N, (const cplx<float>*)p, (const cplx<float>*)s,
                           (const cplx<float>*)r, part);
        hipLaunchKernelGGL(k_mf_coef, dim3(1), dim3(64), 0, st, (const double*)part, nb, 1, sc);
        hipLaunchKernelGGL(k_mf_update, grid, blk, 0, st, N, (const double*)sc, (const cplx<float>*)p,
                           (const cplx<float>*)s, X, r, part);
        hipLaunchKernelGGL(k_mf_coef, dim3(1), dim3(64), 0, st, (const double*)part, nb, 0, sc);
        QH_HIP(hipGetLastError());
        QH_TRY(read(M_PS, M_RR));
        const double ps = n->hpin[0], rr = n->hpin[1];
        if (!std::isfinite(ps) || !std::isfinite(rr)) {
            broke = true;
            why = "non-finite inner product";
            break;
        }
        if (!(ps > 0.0)) {
            // no descent direction (alpha was 0: x and r unchanged)
            if (net_on) {
                net_on = false;
                *switched_at = it;
                handed_over = true;
                break;
            }
            // the fallback lost descent in FP32: restart from the FP64 residual
            double t2;
            QH_TRY(reliable(t2));
            true_rr = t2;
            if (t2 <= target2) {
                converged = true;
                break;
            }
            if (++stalls >= 3) {
                broke = true;
                why = "no descent direction after restarts";
                break;
            }
            QH_TRY(restart());
            continue;
        }
        it++;
        since++;
        hist.push_back(std::sqrt(rr));
        bool judge_out = false;
        if (net_on && (int)hist.size() > kJudgeWindow &&
            hist.back() > kJudgeFactor * hist[hist.size() - 1 - kJudgeWindow])
            judge_out = true;
        if (rr <= target2 || since >= kRelEvery || rr <= kRelDrop * rr_rel || it >= maxit) {
            double t2;
            QH_TRY(reliable(t2));
            true_rr = t2;
            since = 0;
            rr_rel = t2;
            if (!std::isfinite(t2)) {
                broke = true;
                why = "non-finite true residual";
                break;
            }
            if (t2 <= target2) {
                converged = true;
                break;
            }
            if (t2 < best_true) {
                best_true = t2;
                stalls = 0;
            } else if (++stalls >= 3) {
                broke = true;
                why = "three reliable updates without progress";
                break;
            }
        }
        if (it >= maxit) break;
        if (judge_out) {
            net_on = false;
            *switched_at = it;
            handed_over = true;
            break;
        }
        QH_TRY(precond());
        hipLaunchKernelGGL(k_mf_dot_sz, grid, blk, 0, st, N, (const cplx<float>*)s, (const cplx<float>*)z, part);
        hipLaunchKernelGGL(k_mf_coef, dim3(1), dim3(64), 0, st, (const double*)part, nb, 2, sc);
        hipLaunchKernelGGL(k_mf_dir, grid, blk, 0, st, N, (const double*)sc, (const cplx<float>*)z, p);
        QH_HIP(hipGetLastError());
    }
    *iters = it;
    if (handed_over) {
        QH_TRY(finish(nb2, converged));
        true_rr = true_rr_out;
        broke = !converged;
        why = "the fallback did not reach the tolerance";
    }
    *true_rel = std::sqrt(true_rr / nb2);
    if (converged) return QEDHMC_OK;
    set_error(std::string("mixed flexible CG: ") + (broke ? why : "maximum iteration count reached") + " after " +
              std::to_string(it) + " iterations (true residual " + std::to_string(*true_rel) + ")");
    return QEDHMC_ENOCONV;
}

}  // namespace qh
