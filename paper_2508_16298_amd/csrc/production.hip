// Production loop around the trajectory (Methods, "HQMC algorithm": N_leapfrog
// leapfrog steps per trajectory with the step size tuned to keep a moderate
// acceptance rate), the gauge observables it logs (Supplemental Material SV:
// S_tau and S_plaq), the flux correlator (Results, Eq. 33) and the
// autocorrelation analysis of a logged series.
//
// Step-size rule (the paper names no rule): during thermalisation, after
// each trajectory dt <- dt * exp(gain * (min(1, e^{-dH}) - target)), the
// factor clipped to [1/2, 2]; the step is then frozen for the measured
// trajectories, so those form a fixed Markov chain.
#include <algorithm>
#include <cmath>
#include <vector>

#include "qedhmc_internal.h"

using namespace qh;

namespace {

double adapted_dt(double dt, double dH, double target, double gain) {
    const double a = dH <= 0.0 ? 1.0 : std::exp(-dH);
    const double f = std::exp(gain * (a - target));
    return dt * std::min(2.0, std::max(0.5, f));
}

qedhmc_status gauge_obs(qedhmc_t h, const double* theta, double* S_tau, double* S_plaq) {
    double* dev = h->scal + 104;  // two spare device scalars
    QH_TRY(launch_gauge_parts(h, theta, dev));
    QH_HIP(hipMemcpyAsync(h->h_pinned + 20, dev, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    QH_HIP(hipStreamSynchronize(h->stream));
    *S_tau = h->h_pinned[20];
    *S_plaq = h->h_pinned[21];
    return QEDHMC_OK;
}

}  // namespace

extern "C" {

qedhmc_status qedhmc_gauge_observables(qedhmc_t h, const double* theta, double* S_tau, double* S_plaq) {
    if (!h || !theta || !S_tau || !S_plaq) {
        set_error("null argument");
        return QEDHMC_EINVAL;
    }
    return gauge_obs(h, theta, S_tau, S_plaq);
}

qedhmc_status qedhmc_flux_correlator(qedhmc_t h, const double* theta, double* C_out) {
    if (!h || !theta || !C_out) {
        set_error("null argument");
        return QEDHMC_EINVAL;
    }
    return launch_flux_corr(h, theta, false, C_out);
}

qedhmc_status qedhmc_production(qedhmc_t h, double* theta, const qedhmc_prod_params* pp, qedhmc_prod_record* records,
                                double* C_flux_mean, double* dt_final) {
    if (!h || !theta || !pp || !records) {
        set_error("null argument");
        return QEDHMC_EINVAL;
    }
    if (pp->n_therm < 0 || pp->n_meas < 0 || pp->n_steps < 1 || !(pp->dt0 > 0.0) || !(pp->target_accept > 0.0) ||
        !(pp->target_accept < 1.0) || !(pp->gain >= 0.0) || !(pp->tol > 0.0) || pp->maxit < 1) {
        set_error("production: need n_therm, n_meas >= 0, n_steps >= 1, dt0 > 0, 0 < target < 1, gain >= 0, "
                  "tol > 0, maxit >= 1");
        return QEDHMC_EINVAL;
    }
    if (C_flux_mean) QH_TRY(launch_scale(h, C_flux_mean, h->lat.Nt, 0.0));
    double dt = pp->dt0;
    qedhmc_status worst = QEDHMC_OK;
    const int total = pp->n_therm + pp->n_meas;
    for (int k = 0; k < total; k++) {
        qedhmc_traj_result r{};
        const uint64_t idx = pp->first_traj + (uint64_t)k;
        const qedhmc_status st = qedhmc_hmc_trajectory(h, theta, idx, pp->n_steps, pp->n_steps * dt, pp->tol,
                                                       pp->maxit, pp->prec, pp->pc, &r);
        if (st != QEDHMC_OK && st != QEDHMC_ENOCONV) return st;
        if (st == QEDHMC_ENOCONV) worst = QEDHMC_ENOCONV;
        qedhmc_prod_record& rec = records[k];
        rec = qedhmc_prod_record{};
        rec.traj = idx;
        rec.dt = dt;
        rec.dH = r.dH;
        rec.accepted = r.accepted;
        rec.cg_iters = r.cg_iters_total;
        rec.status = r.status;
        QH_TRY(gauge_obs(h, theta, &rec.S_tau, &rec.S_plaq));
        if (k < pp->n_therm)
            dt = adapted_dt(dt, r.dH, pp->target_accept, pp->gain);
        else if (C_flux_mean)
            QH_TRY(launch_flux_corr(h, theta, true, C_flux_mean));
    }
    if (C_flux_mean && pp->n_meas > 0) QH_TRY(launch_scale(h, C_flux_mean, h->lat.Nt, 1.0 / pp->n_meas));
    if (dt_final) *dt_final = dt;
    QH_HIP(hipStreamSynchronize(h->stream));
    if (worst != QEDHMC_OK) set_error("production: at least one trajectory had an unconverged solve (rejected)");
    return worst;
}

qedhmc_status qedhmc_autocorrelation(const double* series, int32_t n, int32_t kmax, double* rho, double* tau_int,
                                     double* tau_exp) {
    if (!series || !rho || !tau_int || !tau_exp || n < 2 || kmax < 1 || kmax >= n) {
        set_error("autocorrelation: need series, outputs, n >= 2 and 1 <= kmax < n");
        return QEDHMC_EINVAL;
    }
    double m = 0.0;
    for (int t = 0; t < n; t++) m += series[t];
    m /= n;
    std::vector<double> c(kmax + 1);
    for (int k = 0; k <= kmax; k++) {
        double s = 0.0;
        for (int t = 0; t + k < n; t++) s += (series[t] - m) * (series[t + k] - m);
        c[k] = s / (n - k);
    }
    if (!(c[0] > 0.0)) {
        set_error("autocorrelation: the series is constant");
        return QEDHMC_EINVAL;
    }
    for (int k = 0; k <= kmax; k++) rho[k] = c[k] / c[0];
    // integrated time with Sokal's window: the smallest W with W >= 5 tau(W)
    double tau = 0.5, acc = 0.0;
    for (int W = 1; W <= kmax; W++) {
        acc += rho[W];
        tau = 0.5 + acc;
        if (W >= 5.0 * tau) break;
    }
    *tau_int = tau;
    // exponential time: least squares of log rho(k) = -k / tau over the k
    // before rho first drops below 0.1
    double skk = 0.0, skl = 0.0;
    for (int k = 1; k <= kmax && rho[k] >= 0.1; k++) {
        skk += (double)k * k;
        skl += k * std::log(rho[k]);
    }
    *tau_exp = skl < 0.0 ? -skk / skl : 0.0;
    return QEDHMC_OK;
}

}  // extern "C"
