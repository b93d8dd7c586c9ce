"""Oracle of the production loop around the trajectory: the gauge observables
logged per trajectory, the flux correlator, the autocorrelation analysis and
the step-size adaptation.  TEST INFRASTRUCTURE ONLY: imported by tests/ and
bench.py's CPU baseline, never by the product library.

Passages: Methods, "HQMC algorithm" (N_leapfrog = 3, Delta t tuned to keep a
moderate acceptance rate); Results, Eq. (33) (flux correlator);
Supplemental Material SV (S_tau, S_plaq and their autocorrelation).

Readings (the paper gives no formula for these):
* S_tau and S_plaq are the two terms of the gauge action of the handle:
  S_tau = 1/(J dtau) sum f(theta_{tau+1} - theta_tau), f = (.)^2 for the
  non-compact action (SV's definition) and 1 - cos for the compact one;
  S_plaq = K dtau sum_plaquettes cos(curl theta).
* C_flux(dtau) = 1/(V_s N_tau) sum_{tau, plaquettes} sin Phi(tau + dtau)
  sin Phi(tau), tau periodic: Eq. (33) averaged over the time origin.
* Step size: during thermalisation, after each trajectory
  dt <- dt * exp(gain * (min(1, e^{-dH}) - target)), the factor clipped to
  [1/2, 2]; frozen afterwards (so the measured chain is a fixed Markov chain).
* Autocorrelation: rho(k) = C(k)/C(0), C(k) = 1/(n-k) sum_t (x_t - m)(x_{t+k} - m);
  integrated time tau_int = 1/2 + sum_{k=1}^{W} rho(k) with W the smallest
  window with W >= 5 tau_int(W) (Sokal); exponential time from a least-squares
  fit of log rho(k) = -k / tau_exp over 1 <= k < the first k with rho(k) < 0.1.
"""
import numpy as np

from . import hmc_trajectory


def _plaquettes(p, theta):
    """Phi(tau, y, x) = th_x(s) + th_y(s + x) - th_x(s + y) - th_y(s)."""
    tx, ty = theta[0], theta[1]
    return tx + np.roll(ty, -1, axis=2) - np.roll(tx, -1, axis=1) - ty


def gauge_parts(p, theta):
    """(S_tau, S_plaq) of the configuration."""
    th = np.asarray(theta, dtype=np.float64).reshape(2, p.Nt, p.L, p.L)
    d = np.roll(th, -1, axis=1) - th
    f = d * d if p.noncompact else 1.0 - np.cos(d)
    S_tau = f.sum() / (p.J * p.dtau)
    S_plaq = p.K * p.dtau * np.cos(_plaquettes(p, th)).sum()
    return float(S_tau), float(S_plaq)


def flux_correlator(p, theta):
    """C_flux(dtau), dtau = 0 .. N_tau - 1."""
    th = np.asarray(theta, dtype=np.float64).reshape(2, p.Nt, p.L, p.L)
    s = np.sin(_plaquettes(p, th)).reshape(p.Nt, -1)
    C = np.empty(p.Nt)
    for dt in range(p.Nt):
        C[dt] = np.sum(np.roll(s, -dt, axis=0) * s) / (p.Vs * p.Nt)
    return C


def autocorrelation(x, kmax):
    """(rho[0..kmax], tau_int, tau_exp) of a time series."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    m = x.mean()
    c = np.array([np.sum((x[:n - k] - m) * (x[k:] - m)) / (n - k) for k in range(kmax + 1)])
    rho = c / c[0]
    tau = 0.5
    for W in range(1, kmax + 1):
        tau = 0.5 + rho[1:W + 1].sum()
        if W >= 5 * tau:
            break
    k = 1
    while k <= kmax and rho[k] >= 0.1:
        k += 1
    ks = np.arange(1, k)
    if ks.size:
        tau_exp = -np.sum(ks * ks) / np.sum(ks * np.log(rho[1:k]))
    else:
        tau_exp = 0.0
    return rho, float(tau), float(tau_exp)


def adapt_dt(dt, dH, target, gain):
    """One step-size update from one trajectory's energy error."""
    a = 1.0 if dH <= 0 else float(np.exp(-dH))
    f = float(np.exp(gain * (a - target)))
    return dt * min(2.0, max(0.5, f))


def production(p, theta, seed, first_traj, n_therm, n_meas, dt0, target=0.7, gain=1.0, n_steps=3,
               tol=1e-10):
    """Thermalisation with step-size adaptation, then measurement at a fixed
    step; returns (theta, records, C_flux mean over the measured trajectories,
    final dt).  Trajectory k has index first_traj + k and n_steps leapfrog
    steps of dt (length n_steps dt)."""
    th = np.array(theta, dtype=np.float64, copy=True)
    dt = dt0
    rec = []
    Cf = np.zeros(p.Nt)
    for k in range(n_therm + n_meas):
        th, r, *_ = hmc_trajectory(p, th, seed=seed, traj=first_traj + k, n_steps=n_steps,
                                   traj_len=n_steps * dt, tol=tol)
        S_tau, S_plaq = gauge_parts(p, th)
        rec.append({"traj": first_traj + k, "dt": dt, "dH": r["dH"], "accepted": r["accepted"],
                    "S_tau": S_tau, "S_plaq": S_plaq, "cg_iters": r["cg_iters_total"]})
        if k < n_therm:
            dt = adapt_dt(dt, r["dH"], target, gain)
        else:
            Cf += flux_correlator(p, th)
    if n_meas:
        Cf /= n_meas
    return th, rec, Cf, dt
