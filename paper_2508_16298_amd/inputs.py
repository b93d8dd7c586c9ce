"""Seeded synthetic inputs for the HQMC workloads.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic, so the product library, the tests and the CPU oracle can
all be fed from it without sharing any computation.

Layouts
  theta  float64 (2, Nt, L, L): angle on the bond from site (x, y) to its +x
         (d=0) or +y (d=1) neighbour in slice tau, indexed [d, tau, y, x]
  vector complex128 (Nt, L, L), indexed [tau, y, x]

The paper generates its workloads itself by Monte Carlo; the stand-ins here
are its hot start (angles i.i.d. uniform on [0, 2 pi)), the pi-flux
configuration it builds its preconditioner on (Methods, CG method and
preconditioner), pi-flux plus Gaussian noise as a stand-in for thermalised
configurations, and complex Gaussian sources.
"""
from dataclasses import dataclass, field
from typing import List

import numpy as np


@dataclass(frozen=True)
class Workload:
    """One named workload: lattice, couplings, trajectory shape, precision."""
    name: str
    L: int
    Nt: int
    dtau: float = 0.1
    t: float = 1.0
    J: float = 1.0
    K: float = 1.0
    seed: int = 0
    n_steps: int = 10
    traj_len: float = 1.0
    tol: float = 1e-10
    precision: str = "fp64"
    n_traj: int = 1
    theta: str = "hot"          # "hot": uniform [0, 2 pi); "pi_noise": pi flux + N(0, sigma^2)
    sigma: float = 0.0
    theta_seed: int = 0
    chains: List[int] = field(default_factory=list)

    @property
    def N(self) -> int:
        return self.L * self.L * self.Nt

    def initial_theta(self) -> np.ndarray:
        if self.theta == "hot":
            return hot_start_theta(self.L, self.Nt, self.theta_seed or self.seed)
        if self.theta == "pi_noise":
            return noisy_pi_flux_theta(self.L, self.Nt, self.sigma, self.theta_seed or self.seed)
        raise ValueError(self.theta)


# The workloads of the hot path (lattice sizes, couplings, CG residual,
# trajectory shape).  Trajectory length is 1 everywhere.  From L = 12 up a
# hot start sits next to det M = 0: the fermion force diverges within the
# first leapfrog step and the trajectory is meaningless, so trajectories at
# those sizes start from pi flux plus Gaussian noise (sigma 0.3), the stand-in
# for a thermalised configuration; hot starts remain the first-solve workloads
# ("*_hot").
WORKLOADS = {
    "cpu_small": Workload("cpu_small", L=6, Nt=10, seed=1001, n_steps=10, tol=1e-10),
    "fp64_l12": Workload("fp64_l12", L=12, Nt=120, seed=1002, n_steps=20, tol=1e-10,
                         n_traj=20, theta="pi_noise", sigma=0.3, theta_seed=1012),
    "fp64_l12_hot": Workload("fp64_l12_hot", L=12, Nt=120, seed=1002, n_steps=20, tol=1e-10),
    "mixed_l24": Workload("mixed_l24", L=24, Nt=240, seed=1003, n_steps=20, tol=1e-8,
                          precision="mixed", theta="pi_noise", sigma=0.3, theta_seed=1013),
    "mixed_l24_hot": Workload("mixed_l24_hot", L=24, Nt=240, seed=1003, n_steps=20, tol=1e-8,
                              precision="mixed"),
    "batched_chains": Workload("batched_chains", L=0, Nt=0, seed=1004, n_steps=20,
                               tol=1e-8, precision="mixed"),
    "learned_l66": Workload("learned_l66", L=66, Nt=660, seed=1005, n_steps=20, tol=1e-8,
                            precision="mixed"),
    # stochastic estimation: the angles of mixed_l24, 40 probes per measurement (seed 1006)
    "se_l24": Workload("se_l24", L=24, Nt=240, seed=1006, n_steps=0, tol=1e-8, precision="mixed",
                       theta="pi_noise", sigma=0.3, theta_seed=1013),
}
SE_PROBES = 40


def hot_start_theta(L: int, Nt: int, seed: int) -> np.ndarray:
    """Angles i.i.d. uniform on [0, 2 pi) on every spatial bond of every slice."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 2.0 * np.pi, size=(2, Nt, L, L))


def pi_flux_theta(L: int, Nt: int) -> np.ndarray:
    """theta_x = 0, theta_y(x, y) = pi x: flux pi through every plaquette for even L."""
    th = np.zeros((2, Nt, L, L))
    th[1] = np.pi * np.arange(L)[None, None, :]
    return th


def noisy_pi_flux_theta(L: int, Nt: int, sigma: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return pi_flux_theta(L, Nt) + rng.normal(0.0, sigma, size=(2, Nt, L, L))


def gauss_cvec(L: int, Nt: int, seed: int) -> np.ndarray:
    """Complex Gaussian vector, Re and Im i.i.d. N(0, 1/2)."""
    rng = np.random.default_rng(seed)
    s = np.sqrt(0.5)
    return (rng.normal(0.0, s, size=(Nt, L, L))
            + 1j * rng.normal(0.0, s, size=(Nt, L, L)))


def gauss_real(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, size=shape)


def gauge_angles(L: int, seed: int) -> np.ndarray:
    """Random site angles alpha_s (shape (L, L)) for gauge transformations."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-np.pi, np.pi, size=(L, L))


def chain_sizes(n_chains: int = 64, seed: int = 1004, sizes=(8, 12, 16, 20)) -> List[int]:
    """Linear sizes of independent chains, drawn uniformly from ``sizes``."""
    rng = np.random.default_rng(seed)
    return [int(x) for x in rng.choice(np.asarray(sizes), size=n_chains)]


def batched_chain_inputs(n_chains: int = 64, seed: int = 1004, sigma: float = 0.3):
    """The batched-chains workload: sizes (L, 10 L) with L drawn from
    8/12/16/20, starting angles pi flux plus N(0, sigma^2) noise, and one
    heat-bath seed per chain."""
    sizes = [(L, 10 * L) for L in chain_sizes(n_chains, seed)]
    seeds = [4000 + c for c in range(n_chains)]
    thetas = [noisy_pi_flux_theta(L, Nt, sigma, s) for (L, Nt), s in zip(sizes, seeds)]
    return sizes, thetas, seeds


NET_CHANNELS = (6, 32, 32, 32, 32, 32, 2)


def net_init_weights(seed: int, ch=NET_CHANNELS):
    """Initial weights of the preconditioner network: per layer W of shape
    (Cout, Cin, 27) drawn N(0, 2 / (27 Cin)) (the last layer scaled by 0.1)
    and zero biases."""
    rng = np.random.default_rng(seed)
    params = []
    for l in range(len(ch) - 1):
        cin, cout = ch[l], ch[l + 1]
        W = rng.normal(0.0, np.sqrt(2.0 / (27 * cin)), size=(cout, cin, 27))
        if l == len(ch) - 2:
            W *= 0.1
        params.append((W, np.zeros(cout)))
    return params
