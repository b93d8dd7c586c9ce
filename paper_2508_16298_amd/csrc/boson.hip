// Gauge-field side of the trajectory: compact action and force, Philox heat
// bath, leapfrog kicks and drifts, FP64 reductions, Metropolis test.
#include "qedhmc_internal.h"
#include "rng.h"

namespace qh {

static constexpr int kGridR = 512;
static constexpr int kBlockR = 256;

__global__ void k_sum_partials(const double* __restrict__ part, int n, double* __restrict__ out) {
    __shared__ double red[16];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) *out = s;
}

// ---------------------------------------------------------------------------
// Gauge action (Results, L_B^c and Eq. 3 for L_B^nc, integrated as dtau sum_tau):
//   S_B = 1/(J dtau) sum_{d,tau,s} k(theta_{d,tau+1,s} - theta_{d,tau,s})
//       + K dtau sum_{tau,s} cos Phi_{tau,s},
//   k(u) = 1 - cos u (compact) or u^2 (non-compact),
//   Phi_{tau,s} = th_x(s) + th_y(s+x) - th_x(s+y) - th_y(s).
// One thread per space-time site; the force on the two bonds leaving the
// site is assembled from the two time-link terms and the two plaquettes each
// bond borders.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double plaq(const double* __restrict__ th, const Lat& lt, int tau, int x, int y) {
    const int L = lt.L, Vs = lt.Vs;
    const int xp = x + 1 == L ? 0 : x + 1, yp = y + 1 == L ? 0 : y + 1;
    const double* tx = th + (size_t)tau * Vs;
    const double* ty = th + ((size_t)lt.Nt + tau) * Vs;
    return tx[y * L + x] + ty[y * L + xp] - tx[yp * L + x] - ty[y * L + x];
}

__global__ void k_bosonic(Lat lt, double J, double K, double dtau, int noncompact, const double* __restrict__ th,
                          double* __restrict__ F, double* __restrict__ part) {
    __shared__ double red[16];
    const double cj = 1.0 / (J * dtau), kd = K * dtau;
    const size_t N = (size_t)lt.Nt * lt.Vs;
    double s_act = 0.0;
    for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < N; n += (size_t)gridDim.x * blockDim.x) {
        const int tau = (int)(n / lt.Vs), s = (int)(n - (size_t)tau * lt.Vs);
        const int x = s % lt.L, y = s / lt.L;
        const int tp = tau + 1 == lt.Nt ? 0 : tau + 1, tm = tau == 0 ? lt.Nt - 1 : tau - 1;
        const int xm = x == 0 ? lt.L - 1 : x - 1, ym = y == 0 ? lt.L - 1 : y - 1;
        const double P = plaq(th, lt, tau, x, y);
        s_act += kd * cos(P);
        double f[2];
        for (int d = 0; d < 2; d++) {
            const double* td = th + (size_t)d * N;
            const double a = td[(size_t)tau * lt.Vs + s];
            const double an = td[(size_t)tp * lt.Vs + s];
            const double ap = td[(size_t)tm * lt.Vs + s];
            if (noncompact) {
                s_act += cj * (an - a) * (an - a);
                f[d] = cj * (2.0 * (an - a) - 2.0 * (a - ap));
            } else {
                s_act += cj * (1.0 - cos(an - a));
                f[d] = cj * (sin(an - a) - sin(a - ap));
            }
        }
        if (F) {
            const double g0 = kd * sin(P);
            const double gy = kd * sin(plaq(th, lt, tau, x, ym));  // plaquette below: bond is its top edge
            const double gx = kd * sin(plaq(th, lt, tau, xm, y));  // plaquette to the left: bond is its right edge
            F[(size_t)tau * lt.Vs + s] = f[0] + g0 - gy;
            F[N + (size_t)tau * lt.Vs + s] = f[1] + gx - g0;
        }
    }
    s_act = block_sum(s_act, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s_act;
}

qedhmc_status launch_bosonic(qedhmc_ctx* h, const double* theta, double* F_B, double* S_dev) {
    double* part = (h->partial + 12 * (size_t)h->lat.Nt);
    hipLaunchKernelGGL(k_bosonic, dim3(kGridR), dim3(kBlockR), 0, h->stream, h->lat, h->p.J, h->p.K, h->p.dtau,
                       h->p.action == QEDHMC_NONCOMPACT ? 1 : 0, theta, F_B, part);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, h->stream, (const double*)part, kGridR, S_dev);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

// p ~ N(0, 1/2) per bond (pair 2k, 2k+1 from block k of purpose 1) and
// R ~ Re, Im N(0, 1/2) per site (block k of purpose 2).
__global__ void k_heatbath(uint64_t seed, uint64_t traj, size_t N, double* __restrict__ mom,
                           cplx<double>* __restrict__ R) {
    const double r2 = 0.70710678118654752440;
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < N; k += (size_t)gridDim.x * blockDim.x) {
        uint32_t x[4];
        double g1, g2;
        draw_block(seed, traj, 1u, (uint32_t)k, x);
        gauss_pair(x, g1, g2);
        mom[2 * k] = r2 * g1;
        mom[2 * k + 1] = r2 * g2;
        draw_block(seed, traj, 2u, (uint32_t)k, x);
        gauss_pair(x, g1, g2);
        R[k] = mk<double>(r2 * g1, r2 * g2);
    }
}

qedhmc_status launch_heatbath(qedhmc_ctx* h, uint64_t traj, double* mom, double* R) {
    const size_t N = (size_t)h->lat.Nt * h->lat.Vs;
    hipLaunchKernelGGL(k_heatbath, dim3(kGridR), dim3(kBlockR), 0, h->stream, h->p.seed, traj, N, mom,
                       (cplx<double>*)R);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

// ---------------------------------------------------------------------------
// FP64 reductions (fixed grid: deterministic)
// ---------------------------------------------------------------------------
__global__ void k_dot(const double* __restrict__ a, const double* __restrict__ b, size_t n,
                      double* __restrict__ part) {
    __shared__ double red[16];
    double s = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        s += a[i] * b[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Re <a, b> of complex vectors = sum over the interleaved reals of a*b (n reals)
qedhmc_status launch_dot_re(qedhmc_ctx* h, const double* a, const double* b, size_t n, double* out_dev) {
    double* part = (h->partial + 12 * (size_t)h->lat.Nt);
    hipLaunchKernelGGL(k_dot, dim3(kGridR), dim3(kBlockR), 0, h->stream, a, b, n, part);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, h->stream, (const double*)part, kGridR, out_dev);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

qedhmc_status launch_sumsq(qedhmc_ctx* h, const double* a, size_t n, double* out_dev) {
    return launch_dot_re(h, a, a, n, out_dev);
}

// ---------------------------------------------------------------------------
// Leapfrog (Eq. leapfrog): p += c (F_F + F_B);  theta += c p
// ---------------------------------------------------------------------------
__global__ void k_kick(double* __restrict__ mom, const double* __restrict__ F, const double* __restrict__ Fb,
                       double c, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        mom[i] += c * (F[i] + Fb[i]);
}

__global__ void k_drift(double* __restrict__ th, const double* __restrict__ mom, double c, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        th[i] += c * mom[i];
}

qedhmc_status launch_kick(qedhmc_ctx* h, double* mom, const double* F, const double* Fb, double c, size_t n) {
    hipLaunchKernelGGL(k_kick, dim3(kGridR), dim3(kBlockR), 0, h->stream, mom, F, Fb, c, n);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

qedhmc_status launch_drift(qedhmc_ctx* h, double* theta, const double* mom, double c, size_t n) {
    hipLaunchKernelGGL(k_drift, dim3(kGridR), dim3(kBlockR), 0, h->stream, theta, mom, c, n);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

// out = a x + b y (n doubles; out may be x or y)
__global__ void k_lincomb(double* out, double a, const double* x, double b, const double* y, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = a * x[i] + b * y[i];
}

qedhmc_status launch_lincomb(qedhmc_ctx* h, double* out, double a, const double* x, double b, const double* y,
                             size_t n) {
    hipLaunchKernelGGL(k_lincomb, dim3(kGridR), dim3(kBlockR), 0, h->stream, out, a, x, b, y, n);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

// ---------------------------------------------------------------------------
// Metropolis (step iii): scalar slots sc[0..5] = SB0, K0, SF0, SB1, K1, SF1;
// writes sc[6] = dH, sc[7] = u, sc[8] = accepted (1/0).
// ---------------------------------------------------------------------------
// reject: a solve of the trajectory did not converge, so the energy change
// is not that of the reversible leapfrog and the proposal is refused whatever
// dH and u say.
__global__ void k_metropolis(uint64_t seed, uint64_t traj, int reject, double* __restrict__ sc) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double H0 = sc[0] + sc[1] + sc[2];
    const double H1 = sc[3] + sc[4] + sc[5];
    const double dH = H1 - H0;
    uint32_t x[4];
    draw_block(seed, traj, 3u, 0u, x);
    const double u = uniform53(x[0], x[1]);
    const bool acc = !reject && ((dH <= 0.0) || (u < exp(-dH)));
    sc[6] = dH;
    sc[7] = u;
    sc[8] = acc ? 1.0 : 0.0;
}

qedhmc_status launch_metropolis(qedhmc_ctx* h, uint64_t traj, bool reject, double* scal_dev) {
    hipLaunchKernelGGL(k_metropolis, dim3(1), dim3(64), 0, h->stream, h->p.seed, traj, reject ? 1 : 0, scal_dev);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

__global__ void k_restore(double* __restrict__ th, const double* __restrict__ th0, const double* __restrict__ sc,
                          size_t n) {
    if (sc[8] != 0.0) return;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        th[i] = th0[i];
}

qedhmc_status launch_restore(qedhmc_ctx* h, double* theta, const double* theta0, const double* scal_dev, size_t n) {
    hipLaunchKernelGGL(k_restore, dim3(kGridR), dim3(kBlockR), 0, h->stream, theta, theta0, scal_dev, n);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

// ---------------------------------------------------------------------------
// Gauge observables of the production loop (Supplemental Material SV; Results,
// Eq. 33): the time-link and plaquette terms of the action separately, and
// the flux correlator C(dtau) = 1/(V_s N_tau) sum_{tau,s} sin Phi(tau + dtau, s)
// sin Phi(tau, s) with tau periodic.
// ---------------------------------------------------------------------------
__global__ void k_gauge_parts(Lat lt, double J, double K, double dtau, int noncompact, const double* __restrict__ th,
                              double* __restrict__ part) {
    __shared__ double red[16];
    const double cj = 1.0 / (J * dtau), kd = K * dtau;
    const size_t N = (size_t)lt.Nt * lt.Vs;
    double st = 0.0, sp = 0.0;
    for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < N; n += (size_t)gridDim.x * blockDim.x) {
        const int tau = (int)(n / lt.Vs), s = (int)(n - (size_t)tau * lt.Vs);
        const int tp = tau + 1 == lt.Nt ? 0 : tau + 1;
        sp += kd * cos(plaq(th, lt, tau, s % lt.L, s / lt.L));
        for (int d = 0; d < 2; d++) {
            const double u = th[(size_t)d * N + (size_t)tp * lt.Vs + s] - th[(size_t)d * N + (size_t)tau * lt.Vs + s];
            st += cj * (noncompact ? u * u : 1.0 - cos(u));
        }
    }
    st = block_sum(st, red);
    __syncthreads();
    sp = block_sum(sp, red);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = st;
        part[gridDim.x + blockIdx.x] = sp;
    }
}

qedhmc_status launch_gauge_parts(qedhmc_ctx* h, const double* theta, double* out_dev) {
    double* part = (h->partial + 12 * (size_t)h->lat.Nt);  // 2 x kGridR of the 4096 spare doubles
    hipLaunchKernelGGL(k_gauge_parts, dim3(kGridR), dim3(kBlockR), 0, h->stream, h->lat, h->p.J, h->p.K, h->p.dtau,
                       h->p.action == QEDHMC_NONCOMPACT ? 1 : 0, theta, part);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, h->stream, (const double*)part, kGridR, out_dev);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, h->stream, (const double*)(part + kGridR), kGridR,
                       out_dev + 1);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

__global__ void k_sin_plaq(Lat lt, const double* __restrict__ th, double* __restrict__ sp) {
    const size_t N = (size_t)lt.Nt * lt.Vs;
    for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < N; n += (size_t)gridDim.x * blockDim.x) {
        const int tau = (int)(n / lt.Vs), s = (int)(n - (size_t)tau * lt.Vs);
        sp[n] = sin(plaq(th, lt, tau, s % lt.L, s / lt.L));
    }
}

// one workgroup per dtau; acc: C is added to out (accumulate = 1) or written
__global__ void k_flux_corr(Lat lt, const double* __restrict__ sp, int accumulate, double* __restrict__ out) {
    __shared__ double red[16];
    const int dt = blockIdx.x;
    const size_t N = (size_t)lt.Nt * lt.Vs;
    double c = 0.0;
    for (size_t n = threadIdx.x; n < N; n += blockDim.x) {
        const int tau = (int)(n / lt.Vs), s = (int)(n - (size_t)tau * lt.Vs);
        int t2 = tau + dt;
        if (t2 >= lt.Nt) t2 -= lt.Nt;
        c += sp[n] * sp[(size_t)t2 * lt.Vs + s];
    }
    c = block_sum(c, red);
    if (threadIdx.x == 0) {
        c /= (double)N;
        out[dt] = accumulate ? out[dt] + c : c;
    }
}

qedhmc_status launch_flux_corr(qedhmc_ctx* h, const double* theta, bool accumulate, double* out_dev) {
    double* sp = static_cast<double*>(h->ws[10]);
    hipLaunchKernelGGL(k_sin_plaq, dim3(kGridR), dim3(kBlockR), 0, h->stream, h->lat, theta, sp);
    hipLaunchKernelGGL(k_flux_corr, dim3(h->lat.Nt), dim3(kBlockR), 0, h->stream, h->lat, (const double*)sp,
                       accumulate ? 1 : 0, out_dev);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

__global__ void k_scale(double* __restrict__ a, int n, double c) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] *= c;
}

qedhmc_status launch_scale(qedhmc_ctx* h, double* a, int n, double c) {
    hipLaunchKernelGGL(k_scale, dim3((n + 255) / 256), dim3(256), 0, h->stream, a, n, c);
    QH_HIP(hipGetLastError());
    return QEDHMC_OK;
}

}  // namespace qh
