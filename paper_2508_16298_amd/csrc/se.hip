// Stochastic estimation of fermionic observables (Methods, "Stochastic
// estimation of fermionic observables", Eq. Cij_est and the FFT translational
// average; Supplemental Material SIV for the spin correlator).
//
//   probes   xi_p, p < n_rv: complex Gaussian, E[xi^* xi^T] = 1 (Philox
//            purpose 4, element p N + n, index = the measurement index)
//   solve    X_p = (M^dag M)^{-1} M^dag xi_p = G xi_p for all p at once: a
//            batch of n_rv right-hand sides whose workgroups all read one
//            gauge field (the multi-RHS CG)
//   spin     C_S(Delta) = delta_{Delta,0} T1 - T2(Delta) with
//            T1 = (1/(n_rv N)) sum_p sum_i X_p,i conj(xi_p,i) and
//            T2 = 1/(n_rv (n_rv-1) N^2) sum_k S_k e^{+i k.Delta},
//            S_k = sum_{p<q} A_{-k} B_k + A_k B_{-k},
//            A = DFT[X_p conj(xi_q)], B = DFT[X_q conj(xi_p)]
//
// The three-dimensional DFTs are separable: one kernel transforms both
// spatial axes of a slice in LDS (forming the pair products on the way in),
// one transforms the tau axis of a tile of spatial frequencies in LDS, one
// accumulates the pair products in k-space.  Sums run over the twiddle table
// e^{-2 pi i k / n} of each axis length (FP64, from sincospi), in a fixed
// order: the result does not depend on the launch shape.
#include <algorithm>
#include <cstdlib>
#include <new>
#include <vector>

#include "qedhmc_internal.h"
#include "rng.h"

struct qedhmc_se {
    qedhmc_params p{};
    int n_rv = 0;
    int64_t N = 0;
    int L = 0, Nt = 0, Vs = 0;
    hipStream_t stream = nullptr;
    qedhmc_batch* b = nullptr;     // n_rv right-hand sides sharing one gauge field
    qh::cplx<double>* rhs = nullptr;  // n_rv x N: M^dag xi_p
    qh::cplx<double>* ws = nullptr;   // 4 x P x N: spatial and full transforms of P pairs
    qh::cplx<double>* S = nullptr;    // N: pair products accumulated in k-space
    qh::cplx<double>* twL = nullptr;  // L twiddles
    qh::cplx<double>* twT = nullptr;  // Nt twiddles
    qh::cplx<double>* part = nullptr; // T1 partial sums
    int P = 0;                        // pairs per pass
    int n_part = 0;
};

namespace qh {

namespace {

constexpr int kBS = 256;
constexpr size_t kWorkBytes = (size_t)512 << 20;  // transform workspace cap

__device__ __forceinline__ cplx<double> cmul(cplx<double> a, cplx<double> b) {
    return mk<double>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
__device__ __forceinline__ cplx<double> cmulc(cplx<double> a, cplx<double> b) {  // a conj(b)
    return mk<double>(a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im);
}

__global__ void k_se_probes(uint64_t seed, uint64_t meas, uint32_t total, cplx<double>* __restrict__ xi) {
    const double r2 = 0.70710678118654752440;
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        uint32_t x[4];
        double g1, g2;
        draw_block(seed, meas, RNG_PROBE, e, x);
        gauss_pair(x, g1, g2);
        xi[e] = mk<double>(r2 * g1, r2 * g2);
    }
}

__global__ void k_se_twiddle(int n, cplx<double>* __restrict__ tw) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double s, c;
    sincospi(-2.0 * (double)k / (double)n, &s, &c);
    tw[k] = mk<double>(c, s);
}

// Pair number t in the order (0,1), (0,2), ..., (0,n-1), (1,2), ...
__device__ __forceinline__ void pair_of(int t, int n, int& p, int& q) {
    p = 0;
    int first = 0;  // index of (p, p + 1)
    while (t >= first + (n - 1 - p)) {
        first += n - 1 - p;
        p++;
    }
    q = p + 1 + (t - first);
}

// Spatial DFT of one slice of one vector: out(ky, kx) = sum_{y,x} in(y, x)
// w^{y ky} w^{x kx}, w = e^{-+2 pi i / L} (conj = 1: the inverse sign).
// PROD: vector v of pair t0 + v/2 is a = X_p conj(xi_q) (v even) or
// b = X_q conj(xi_p) (v odd); otherwise vector v of in.
template <bool PROD>
__global__ __launch_bounds__(kBS) void k_se_xy(int L, int Nt, int64_t N, int n_rv, int t0, const cplx<double>* __restrict__ X,
                                               const cplx<double>* __restrict__ xi, const cplx<double>* __restrict__ in,
                                               const cplx<double>* __restrict__ tw, int conj, cplx<double>* __restrict__ out) {
    extern __shared__ unsigned char smem[];
    cplx<double>* s0 = reinterpret_cast<cplx<double>*>(smem);
    cplx<double>* s1 = s0 + L * L;
    cplx<double>* w = s1 + L * L;
    const int tau = blockIdx.x, v = blockIdx.y, Vs = L * L;
    const int64_t off = (int64_t)tau * Vs;
    for (int k = threadIdx.x; k < L; k += blockDim.x) {
        const cplx<double> t = tw[k];
        w[k] = mk<double>(t.re, conj ? -t.im : t.im);
    }
    if constexpr (PROD) {
        int p, q;
        pair_of(t0 + v / 2, n_rv, p, q);
        const int u = (v & 1) ? q : p, z = (v & 1) ? p : q;
        const cplx<double>* Xu = X + (int64_t)u * N + off;
        const cplx<double>* xz = xi + (int64_t)z * N + off;
        for (int s = threadIdx.x; s < Vs; s += blockDim.x) s0[s] = cmulc(Xu[s], xz[s]);
    } else {
        const cplx<double>* src = in + (int64_t)v * N + off;
        for (int s = threadIdx.x; s < Vs; s += blockDim.x) s0[s] = src[s];
    }
    __syncthreads();
    for (int s = threadIdx.x; s < Vs; s += blockDim.x) {  // along x: s1(y, kx)
        const int y = s / L, kx = s - y * L;
        cplx<double> acc = mk<double>(0.0, 0.0);
        int e = 0;
        for (int x = 0; x < L; x++) {
            const cplx<double> a = s0[y * L + x], t = w[e];
            acc.re = fma(a.re, t.re, fma(-a.im, t.im, acc.re));
            acc.im = fma(a.re, t.im, fma(a.im, t.re, acc.im));
            e += kx;
            if (e >= L) e -= L;
        }
        s1[s] = acc;
    }
    __syncthreads();
    cplx<double>* dst = out + (int64_t)v * N + off;
    for (int s = threadIdx.x; s < Vs; s += blockDim.x) {  // along y: out(ky, kx)
        const int ky = s / L, kx = s - ky * L;
        cplx<double> acc = mk<double>(0.0, 0.0);
        int e = 0;
        for (int y = 0; y < L; y++) {
            const cplx<double> a = s1[y * L + kx], t = w[e];
            acc.re = fma(a.re, t.re, fma(-a.im, t.im, acc.re));
            acc.im = fma(a.re, t.im, fma(a.im, t.re, acc.im));
            e += ky;
            if (e >= L) e -= L;
        }
        dst[s] = acc;
    }
}

// DFT along tau of KT spatial columns of one vector, staged in LDS:
// out(kt, c) = sum_tau in(tau, c) w^{tau kt}.
__global__ __launch_bounds__(kBS) void k_se_t(int Nt, int Vs, int64_t N, int KT, const cplx<double>* __restrict__ in,
                                              const cplx<double>* __restrict__ tw, int conj,
                                              cplx<double>* __restrict__ out) {
    extern __shared__ unsigned char smem[];
    cplx<double>* col = reinterpret_cast<cplx<double>*>(smem);  // [Nt][KT]
    cplx<double>* w = col + (size_t)Nt * KT;
    const int c0 = blockIdx.x * KT, v = blockIdx.y;
    const int nc = min(KT, Vs - c0);
    const cplx<double>* src = in + (int64_t)v * N;
    for (int k = threadIdx.x; k < Nt; k += blockDim.x) {
        const cplx<double> t = tw[k];
        w[k] = mk<double>(t.re, conj ? -t.im : t.im);
    }
    for (int e = threadIdx.x; e < Nt * KT; e += blockDim.x) {
        const int tau = e / KT, c = e - tau * KT;
        col[e] = c < nc ? src[(int64_t)tau * Vs + c0 + c] : mk<double>(0.0, 0.0);
    }
    __syncthreads();
    cplx<double>* dst = out + (int64_t)v * N;
    for (int e = threadIdx.x; e < Nt * KT; e += blockDim.x) {
        const int kt = e / KT, c = e - kt * KT;
        if (c >= nc) continue;
        cplx<double> acc = mk<double>(0.0, 0.0);
        int idx = 0;
        for (int tau = 0; tau < Nt; tau++) {
            const cplx<double> a = col[tau * KT + c], t = w[idx];
            acc.re = fma(a.re, t.re, fma(-a.im, t.im, acc.re));
            acc.im = fma(a.re, t.im, fma(a.im, t.re, acc.im));
            idx += kt;
            if (idx >= Nt) idx -= Nt;
        }
        dst[(int64_t)kt * Vs + c0 + c] = acc;
    }
}

// S_k += sum over the pass's pairs j of A_j(-k) B_j(k) + A_j(k) B_j(-k);
// A_j = vector 2j, B_j = vector 2j + 1 of F.
__global__ void k_se_accum(int L, int Nt, int64_t N, int npairs, const cplx<double>* __restrict__ F,
                           cplx<double>* __restrict__ S) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= N) return;
    const int Vs = L * L;
    const int kt = (int)(k / Vs), ks = (int)(k - (int64_t)kt * Vs), ky = ks / L, kx = ks - ky * L;
    const int64_t m = (int64_t)((Nt - kt) % Nt) * Vs + ((L - ky) % L) * L + (L - kx) % L;
    cplx<double> acc = S[k];
    for (int j = 0; j < npairs; j++) {
        const cplx<double>* A = F + (int64_t)(2 * j) * N;
        const cplx<double>* B = A + N;
        const cplx<double> t1 = cmul(A[m], B[k]), t2 = cmul(A[k], B[m]);
        acc.re += t1.re + t2.re;
        acc.im += t1.im + t2.im;
    }
    S[k] = acc;
}

// Partial sums of sum_p sum_i X_p,i conj(xi_p,i): one per workgroup.
__global__ __launch_bounds__(kBS) void k_se_t1(int64_t total, const cplx<double>* __restrict__ X,
                                               const cplx<double>* __restrict__ xi, cplx<double>* __restrict__ part) {
    __shared__ double red[2][kBS];
    double sx = 0.0, sy = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)kBS + threadIdx.x; e < total; e += (int64_t)gridDim.x * kBS) {
        const cplx<double> t = cmulc(X[e], xi[e]);
        sx += t.re;
        sy += t.im;
    }
    red[0][threadIdx.x] = sx;
    red[1][threadIdx.x] = sy;
    __syncthreads();
    for (int h = kBS / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[1][threadIdx.x] += red[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = mk<double>(red[0][0], red[1][0]);
}

// C = -scale_T2 * T (T: the inverse transform of S); C(0) += T1, with T1 the
// partial sums added in order and divided by n_rv N.
__global__ void k_se_finish(int64_t N, double scale_T2, int n_part, const cplx<double>* __restrict__ part,
                            double inv_t1, const cplx<double>* __restrict__ T, cplx<double>* __restrict__ C) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= N) return;
    cplx<double> c = mk<double>(-scale_T2 * T[k].re, -scale_T2 * T[k].im);
    if (k == 0) {
        double sx = 0.0, sy = 0.0;
        for (int j = 0; j < n_part; j++) {
            sx += part[j].re;
            sy += part[j].im;
        }
        c.re += sx * inv_t1;
        c.im += sy * inv_t1;
    }
    C[k] = c;
}

__global__ void k_se_zero(int64_t n, cplx<double>* __restrict__ a) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k < n) a[k] = mk<double>(0.0, 0.0);
}

int tau_tile(int Nt) { return Nt <= 256 ? 16 : 8; }

size_t xy_lds(int L) { return (size_t)(2 * L * L + L) * sizeof(cplx<double>); }
size_t t_lds(int Nt) { return (size_t)(Nt * tau_tile(Nt) + Nt) * sizeof(cplx<double>); }

qedhmc_status set_lds_attr(const void* k, size_t bytes) {
    if (bytes > 65536) QH_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    return QEDHMC_OK;
}

// Transform nvec vectors of N: spatial pass from X/xi pairs (PROD) or from
// in, into tmp; tau pass from tmp into out.
template <bool PROD>
qedhmc_status dft3(qedhmc_se* se, int nvec, int t0, const cplx<double>* X, const cplx<double>* xi,
                   const cplx<double>* in, int conj, cplx<double>* tmp, cplx<double>* out) {
    const int L = se->L, Nt = se->Nt, Vs = se->Vs, KT = tau_tile(Nt);
    hipLaunchKernelGGL(k_se_xy<PROD>, dim3(Nt, nvec), dim3(kBS), xy_lds(L), se->stream, L, Nt, se->N, se->n_rv, t0,
                       X, xi, in, se->twL, conj, tmp);
    hipLaunchKernelGGL(k_se_t, dim3((Vs + KT - 1) / KT, nvec), dim3(kBS), t_lds(Nt), se->stream, Nt, Vs, se->N, KT,
                       tmp, se->twT, conj, out);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

qedhmc_status se_fail(qedhmc_se* se, qedhmc_status st) {
    qedhmc_se_destroy(se);
    return st;
}

}  // namespace

}  // namespace qh

using namespace qh;

extern "C" {

qedhmc_status qedhmc_se_create(const qedhmc_params* params, int32_t n_rv, void* stream, qedhmc_se_t* out) {
    if (!params || !out) {
        set_error("se: null argument");
        return QEDHMC_EINVAL;
    }
    *out = nullptr;
    QH_TRY(check_params(params));
    const int64_t N = (int64_t)params->L * params->L * params->Nt;
    if (n_rv < 2 || (int64_t)n_rv * N >= ((int64_t)1 << 32)) {
        set_error("se: need 2 <= n_rv and n_rv * L^2 * Nt < 2^32");
        return QEDHMC_EINVAL;
    }
    if (params->L > 44) {
        set_error("se: the multi-RHS CG holds a slice in one workgroup group of at most 256 threads (L <= 44)");
        return QEDHMC_EUNSUPPORTED;
    }
    qedhmc_se* se = new (std::nothrow) qedhmc_se{};
    if (!se) return QEDHMC_ENOMEM;
    se->p = *params;
    se->n_rv = n_rv;
    se->N = N;
    se->L = params->L;
    se->Nt = params->Nt;
    se->Vs = params->L * params->L;
    se->stream = (hipStream_t)stream;
    int dev = 0;
    int lds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return se_fail(se, hip_fail(hipGetLastError(), "se: device attributes"));
    if (xy_lds(se->L) > (size_t)lds || t_lds(se->Nt) > (size_t)lds) {
        set_error("se: transform tiles exceed the LDS of a workgroup");
        return se_fail(se, QEDHMC_EUNSUPPORTED);
    }
    qedhmc_status st = batch_create_shared(*params, n_rv, stream, &se->b);
    if (st != QEDHMC_OK) return se_fail(se, st);
    const int64_t npairs = (int64_t)n_rv * (n_rv - 1) / 2;
    se->P = (int)std::max<int64_t>(1, std::min<int64_t>(npairs, kWorkBytes / (4 * N * sizeof(cplx<double>))));
    // QEDHMC_SE_PAIRS (tuning and tests): at most this many pairs per pass
    if (const char* e = std::getenv("QEDHMC_SE_PAIRS"))
        if (std::atoi(e) > 0) se->P = std::min(se->P, std::atoi(e));
    se->n_part = 1024;
    bool ok = hipMalloc(&se->rhs, (size_t)n_rv * N * sizeof(cplx<double>)) == hipSuccess;
    ok = ok && hipMalloc(&se->ws, (size_t)4 * se->P * N * sizeof(cplx<double>)) == hipSuccess;
    ok = ok && hipMalloc(&se->S, (size_t)N * sizeof(cplx<double>)) == hipSuccess;
    ok = ok && hipMalloc(&se->twL, (size_t)se->L * sizeof(cplx<double>)) == hipSuccess;
    ok = ok && hipMalloc(&se->twT, (size_t)se->Nt * sizeof(cplx<double>)) == hipSuccess;
    ok = ok && hipMalloc(&se->part, (size_t)se->n_part * sizeof(cplx<double>)) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        set_error("se: device allocation failed");
        return se_fail(se, QEDHMC_ENOMEM);
    }
    st = set_lds_attr((const void*)k_se_xy<true>, xy_lds(se->L));
    if (st == QEDHMC_OK) st = set_lds_attr((const void*)k_se_xy<false>, xy_lds(se->L));
    if (st == QEDHMC_OK) st = set_lds_attr((const void*)k_se_t, t_lds(se->Nt));
    if (st != QEDHMC_OK) return se_fail(se, st);
    hipLaunchKernelGGL(k_se_twiddle, dim3((se->L + 255) / 256), dim3(256), 0, se->stream, se->L, se->twL);
    hipLaunchKernelGGL(k_se_twiddle, dim3((se->Nt + 255) / 256), dim3(256), 0, se->stream, se->Nt, se->twT);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(se->stream) != hipSuccess)
        return se_fail(se, hip_fail(hipGetLastError(), "se: twiddle tables"));
    *out = se;
    return QEDHMC_OK;
}

qedhmc_status qedhmc_se_destroy(qedhmc_se_t se) {
    if (!se) return QEDHMC_OK;
    if (se->b) qedhmc_batch_destroy(se->b);
    for (void* ptr : {(void*)se->rhs, (void*)se->ws, (void*)se->S, (void*)se->twL, (void*)se->twT, (void*)se->part})
        if (ptr) (void)hipFree(ptr);
    delete se;
    return QEDHMC_OK;
}

qedhmc_status qedhmc_se_probes(qedhmc_se_t se, uint64_t meas_index, double* xi_all) {
    if (!se || !xi_all) {
        set_error("se: null argument");
        return QEDHMC_EINVAL;
    }
    const uint32_t total = (uint32_t)((int64_t)se->n_rv * se->N);
    const int grid = (int)std::min<int64_t>(((int64_t)total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_se_probes, dim3(grid), dim3(256), 0, se->stream, se->p.seed, meas_index, total,
                       reinterpret_cast<cplx<double>*>(xi_all));
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

qedhmc_status qedhmc_se_solve(qedhmc_se_t se, const double* theta, const double* xi_all, double* X_all, double tol,
                              int32_t maxit, qedhmc_precision prec, int32_t* iters, double* true_rel) {
    if (!se || !theta || !xi_all || !X_all || !iters || !true_rel) {
        set_error("se: null argument");
        return QEDHMC_EINVAL;
    }
    if (xi_all == X_all) {
        set_error("se: xi and X alias");
        return QEDHMC_EINVAL;
    }
    if (!(tol > 0.0) || maxit < 1 || (prec != QEDHMC_FP64 && prec != QEDHMC_FP32)) {
        set_error("se: bad solver arguments");
        return QEDHMC_EINVAL;
    }
    // R_p = M^dag xi_p on the batch's stream (ordered after the caller's work)
    QH_TRY(batch_enter(se->b));
    qedhmc_ctx* h0 = batch_ctx0(se->b);
    QH_TRY(ensure_gauge(h0, theta, QEDHMC_FP64));
    for (int k = 0; k < se->n_rv; k++)
        QH_TRY(launch_apply_M(h0, QEDHMC_FP64, xi_all + 2 * se->N * k, se->rhs + se->N * k, 1));
    return batch_solve_shared(se->b, theta, reinterpret_cast<const double*>(se->rhs), X_all, tol, maxit, prec, iters,
                              true_rel);
}

qedhmc_status qedhmc_se_spin_correlator(qedhmc_se_t se, const double* xi_all, const double* X_all, double* C_out) {
    if (!se || !xi_all || !X_all || !C_out) {
        set_error("se: null argument");
        return QEDHMC_EINVAL;
    }
    const int64_t N = se->N;
    const int n = se->n_rv;
    const cplx<double>* xi = reinterpret_cast<const cplx<double>*>(xi_all);
    const cplx<double>* X = reinterpret_cast<const cplx<double>*>(X_all);
    cplx<double>* C = reinterpret_cast<cplx<double>*>(C_out);
    const int eg = (int)((N + 255) / 256);
    hipLaunchKernelGGL(k_se_zero, dim3(eg), dim3(256), 0, se->stream, N, se->S);
    hipLaunchKernelGGL(k_se_t1, dim3(se->n_part), dim3(kBS), 0, se->stream, (int64_t)n * N, X, xi, se->part);
    QH_HIP(hipGetLastError());
    cplx<double>* tmp = se->ws;
    cplx<double>* full = se->ws + (int64_t)2 * se->P * N;
    const int npairs = n * (n - 1) / 2;
    for (int t0 = 0; t0 < npairs; t0 += se->P) {
        const int np = std::min(se->P, npairs - t0);
        QH_TRY(dft3<true>(se, 2 * np, t0, X, xi, nullptr, 0, tmp, full));
        hipLaunchKernelGGL(k_se_accum, dim3(eg), dim3(256), 0, se->stream, se->L, se->Nt, N, np, full, se->S);
        QH_HIP(hipGetLastError());
    }
    // T(Delta) = sum_k S_k e^{+i k.Delta}: the transform with the conjugate twiddles
    QH_TRY(dft3<false>(se, 1, 0, nullptr, nullptr, se->S, 1, tmp, full));
    const double scale = 1.0 / ((double)n * (double)(n - 1) * (double)N * (double)N);
    hipLaunchKernelGGL(k_se_finish, dim3(eg), dim3(256), 0, se->stream, N, scale, se->n_part, se->part,
                       1.0 / ((double)n * (double)N), full, C);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

}  // extern "C"
