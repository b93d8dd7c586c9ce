/*
 * qedhmc.h -- C ABI of the MI355X-native hybrid quantum Monte Carlo (HQMC)
 * hot path for lattice QED3: a compact U(1) gauge field theta on the spatial
 * bonds of an L x L x N_tau lattice coupled to two identical fermion flavours
 * through one complex pseudofermion.
 *
 * Paper passages the calls implement (arXiv 2508.16298):
 *   qedhmc_apply_M / qedhmc_apply_B   Methods, Eq. (M_alpha) and Eq. (24)
 *   qedhmc_apply_MdagM                Methods, "Matrix-free representation of
 *                                     M^dagger M v"
 *   qedhmc_cg_solve                   Methods, "CG method and preconditioner",
 *                                     Eq. (pCG)
 *   qedhmc_fermion_force              Supplemental Material SI,
 *                                     Eq. (force&CG) and Eq. (fermion_force)
 *   qedhmc_bosonic_action_force       Results, compact Lagrangian L_B^c
 *   qedhmc_heatbath                   Methods, HQMC algorithm step (i)
 *   qedhmc_hmc_trajectory             Methods, HQMC steps (i)-(iv),
 *                                     Eq. (leapfrog), Eq. (H_hmc)
 *
 * Conventions shared by every call
 *   site        s = y*L + x, periodic in x and y; space-time n = tau*L*L + s
 *   theta       device double[2][Nt][L][L]: angle of the bond from site s to
 *               s + e_d (d = 0: +x, d = 1: +y) in slice tau
 *   vectors     device interleaved complex [Nt][L][L]: double2 for
 *               QEDHMC_FP64, float2 for QEDHMC_FP32 (the precision argument)
 *   B_tau       symmetric checkerboard product E3 E2 E1 E0(2h) E1 E2 E3 with
 *               h = t*dtau/2 over the bond families f0 (x-bonds leaving even
 *               x), f1 (odd x), f2 (y-bonds leaving even y), f3 (odd y); each
 *               bond block is cosh(a) 1 + sinh(a) [[0, e^{i theta}],
 *               [e^{-i theta}, 0]]
 *   M           (Mv)_0 = v_0 + B_{Nt-1} v_{Nt-1},
 *               (Mv)_tau = v_tau - B_{tau-1} v_{tau-1}   (antiperiodic in tau)
 *
 * Ownership and ordering
 *   The caller owns every device buffer passed in (16-byte aligned).  The
 *   handle owns its workspace, allocated by qedhmc_init_lattice and freed by
 *   qedhmc_destroy.  Every call enqueues work on the handle's HIP stream;
 *   calls that return host scalars synchronise that stream before returning.
 *   A handle is not thread-safe: calls on one handle must not overlap.
 *
 * Errors
 *   Every call returns a qedhmc_status and never throws.  QEDHMC_EINVAL
 *   means nothing was written (null pointer, odd or too small L, Nt < 1,
 *   bad enum, tol <= 0, maxit < 1).  QEDHMC_ENOCONV still writes the
 *   partial solution, the iteration count and the true residual.
 *   QEDHMC_EHIP wraps a HIP runtime error; qedhmc_last_error() returns the
 *   message of the last failing call on the calling thread.
 */
#ifndef QEDHMC_H
#define QEDHMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qedhmc_ctx *qedhmc_t;

typedef enum {
    QEDHMC_OK = 0,
    QEDHMC_EINVAL = 1,
    QEDHMC_ENOCONV = 2,
    QEDHMC_EHIP = 3,
    QEDHMC_ENOMEM = 4,
    QEDHMC_EUNSUPPORTED = 5
} qedhmc_status;

/* Arithmetic of a call.  For apply calls it is the vector element type
 * (FP64: double2, FP32: float2).  For solves, forces and trajectories,
 * QEDHMC_FP32 selects the mixed path: complex-FP32 matvecs and force,
 * FP64 solution, FP64 reliable-update residuals every 50 iterations and
 * FP64 reductions. */
typedef enum { QEDHMC_FP64 = 0, QEDHMC_FP32 = 1 } qedhmc_precision;

/* Preconditioner of the CG solve.  QEDHMC_PC_PAPER: the paper's fixed
 * preconditioner P = G^dag G (Methods, "CG method and preconditioner";
 * Fig. 3): G the truncated inverse of the forward IC(0) factor of M^dag M at
 * pi flux on an 8 x 8 x 24 build lattice (0 <= dtau <= 6, |g| >= 1e-3),
 * tiled over the lattice per x parity; built on first use.
 * QEDHMC_PC_LEARNED (not in the paper): the network bound to the handle by
 * qedhmc_set_learned_precond, in flexible CG, with its residual judge and
 * fallback (QEDHMC_PC_PAPER or none); QEDHMC_FP32 runs that solve in mixed
 * precision (complex-FP32 residual, direction and M^dag M, FP64 solution,
 * inner products and reliable-update residuals), QEDHMC_FP64 in FP64
 * vectors (the flexible CG of qedhmc_fcg_solve). */
typedef enum { QEDHMC_PC_NONE = 0, QEDHMC_PC_PAPER = 1, QEDHMC_PC_LEARNED = 2 } qedhmc_precond;

/* Gauge action S_B = dtau sum_tau L_B: the compact Lagrangian L_B^c or the
 * non-compact L_B^nc of Results, Eq. (3) (time-link term (dtheta)^2 instead
 * of 1 - cos(dtheta), same prefactor 1/(J dtau^2)); the plaquette term
 * K cos(curl theta) is the same in both. */
typedef enum { QEDHMC_COMPACT = 0, QEDHMC_NONCOMPACT = 1 } qedhmc_action;

/* Lattice, couplings, gauge action and the seed of the trajectory random
 * streams.  L even, 2 <= L <= 2048; Nt >= 1; L^2 Nt < 2^31.  The calls that
 * keep a whole time slice in one workgroup (apply_B, apply_M, fermion_force,
 * hmc_trajectory) take L <= 66 and return QEDHMC_EUNSUPPORTED beyond;
 * apply_MdagM and cg_solve (tiled M^dag M) take every L, the paper's
 * preconditioner as long as its stencil window fits a workgroup's LDS.
 * action: a qedhmc_action; reserved must be 0. */
typedef struct {
    int32_t L, Nt;
    double dtau, t, J, K;
    uint64_t seed;
    int32_t action;
    int32_t reserved;
} qedhmc_params;

/* Result of one trajectory (all energies FP64). */
typedef struct {
    double dH, H0, H1;     /* H = S_B + sum p^2 + Re eta^dag X           */
    double SB0, SB1;       /* compact gauge action at start / end         */
    double SF0, SF1;       /* fermion action from the solves              */
    double K0, K1;         /* sum p^2 at start / end                      */
    double u;              /* Metropolis uniform                          */
    int32_t accepted;      /* 1: theta holds the proposal; 0: restored    */
    int32_t n_solves;      /* N_md + 1                                    */
    int32_t cg_iters_total, cg_iters_max;
    int32_t status;        /* worst solve status (0 ok, 2 no convergence) */
    int32_t reliable_updates;
    double max_true_resid; /* largest final true relative residual        */
    int32_t pc_fallbacks;  /* QEDHMC_PC_LEARNED: solves whose residual judge
                              handed over to the fallback                 */
    int32_t reserved;
} qedhmc_traj_result;

/* Create a handle: validates params, builds the bond tables on the device
 * and allocates the workspace.  stream: a hipStream_t (NULL = null stream).
 * Lattice definition: Methods, "Model and partition function". */
qedhmc_status qedhmc_init_lattice(const qedhmc_params *params, void *stream,
                                  qedhmc_t *out);
qedhmc_status qedhmc_destroy(qedhmc_t h);
qedhmc_status qedhmc_set_stream(qedhmc_t h, void *stream);
/* Message of the last failing call on this thread ("" if none). */
const char *qedhmc_last_error(void);

/* Copy the device bond tables to host memory: int32 [4][L*L/2][3], rows
 * (origin site i, target site j, bond index d*L*L + i) per family f0..f3,
 * in increasing i (Fig. 1 families used by Eq. 24). */
qedhmc_status qedhmc_get_bond_tables(qedhmc_t h, int32_t *host_out);

/* out = B_tau in on one slice (Eq. 24); in/out: device complex [L][L]. */
qedhmc_status qedhmc_apply_B(qedhmc_t h, const double *theta, int32_t tau,
                             const void *in, void *out, qedhmc_precision prec);

/* out = M in (dagger = 0) or M^dag in (dagger = 1), Eq. (M_alpha).
 * in and out must not alias. */
qedhmc_status qedhmc_apply_M(qedhmc_t h, const double *theta, const void *in,
                             void *out, int32_t dagger, qedhmc_precision prec);

/* out = M^dag M in, fused (Methods, matrix-free M^dagger M v).  in and out
 * must not alias.  Slices of more than 1024 2x2 cells (L >= 66) go through
 * spatial tiles streamed along tau (two B_tau applications per slice); the
 * environment variables QEDHMC_MDAGM=slice|tiled, QEDHMC_TILE_TC and
 * QEDHMC_TILE_THREADS, read on every call, override that choice and the
 * tile plan, and QEDHMC_TILE_DPP=0 / QEDHMC_TILE_SKIP=0 keep the x exchanges
 * in LDS / every halo row's sweeps (tuning and tests; the result is bitwise
 * the same). */
qedhmc_status qedhmc_apply_MdagM(qedhmc_t h, const double *theta,
                                 const void *in, void *out,
                                 qedhmc_precision prec);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * out = M^dag M in as qedhmc_apply_MdagM (same kernels, bitwise the same
 * result), without a handle and without any allocation.  params as for
 * qedhmc_init_lattice; theta, in and out device buffers as for
 * qedhmc_apply_MdagM (caller-owned, not aliased); stream a hipStream_t (NULL:
 * the null stream); the call only enqueues work on it.  The phase cache the
 * kernels read (2 L^2 N_tau complex values of the working precision) lives in
 * a static device array of QEDHMC_NOALLOC_SCRATCH_BYTES per GPU, held until
 * the process ends; larger lattices return EINVAL before any device work.
 * Every call on one GPU shares that array: calls that overlap on one GPU (on
 * different streams, or from different threads) race and must be ordered by
 * the caller. */
#define QEDHMC_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
qedhmc_status qedhmc_apply_MdagM_noalloc(const qedhmc_params *params,
                                         const double *theta, const void *in,
                                         void *out, qedhmc_precision prec,
                                         void *stream);

/* Solve M^dag M x = rhs by conjugate gradient from x = 0 (Eq. pCG), stopping
 * when the true residual |rhs - M^dag M x| / |rhs| <= tol (recomputed in FP64
 * at exit).  rhs, x: device complex FP64 [Nt][L][L].  iters and
 * true_rel_resid (host pointers, nullable) receive the iteration count and
 * the final true relative residual.  prec = QEDHMC_FP32 runs the mixed path.
 * Returns QEDHMC_ENOCONV (x still written) when maxit is reached, on a
 * breakdown (non-finite inner products or residual) or when three reliable
 * updates in a row make no progress; qedhmc_last_error says which.  The call
 * synchronises the handle's stream before it returns.  Iterations run as
 * graph-captured chunks; without a preconditioner on slices of at most 1024
 * cells the stop, pause and reliable-update decisions are also taken on the
 * device (otherwise by the host between chunks).  The environment variable
 * QEDHMC_NO_GRAPH (read on every call) makes the host launch every iteration
 * and take every decision itself (same results bit for bit; tests). */
qedhmc_status qedhmc_cg_solve(qedhmc_t h, const double *theta,
                              const double *rhs, double *x, double tol,
                              int32_t maxit, qedhmc_precision prec,
                              qedhmc_precond pc, int32_t *iters,
                              double *true_rel_resid);

/* tau reach of the paper's preconditioner G as built here: taps with
 * 0 <= dtau <= QEDHMC_PC_TAU_REACH of the exact IC(0) inverse factor on the
 * build lattice, |g| >= 1e-3 (Methods, "CG method and preconditioner", whose
 * matrix shows a band of 6 in tau; a reach of 12 measured 10 % faster per
 * trajectory at L = 24, N_tau = 240 with the spectral application). */
#define QEDHMC_PC_TAU_REACH 12

/* The paper's preconditioner stencil for x parity 0 or 1 (built on first
 * use): up to capacity taps into host double out[capacity][5] as
 * (dtau, dx, dy, Re g, Im g), meaning G[(tau,x,y),(tau-dtau, x+dx, y+dy)] = g
 * for rows of that parity (times -1 when tau - dtau wraps below 0); *count
 * receives the number of taps.  Methods, "CG method and preconditioner". */
qedhmc_status qedhmc_precond_taps(qedhmc_t h, int32_t parity, int32_t *count,
                                  double *out, int32_t capacity);

/* out = P in = G^dag (G in) with the paper's preconditioner; in/out device
 * complex vectors of the given precision; must not alias. */
qedhmc_status qedhmc_apply_precond(qedhmc_t h, const void *in, void *out,
                                   qedhmc_precision prec);

/* F = -dS_F/dtheta with S_F = eta^dag (M^dag M)^{-1} eta, given the solve
 * X = (M^dag M)^{-1} eta (SM SI):  F_{b,tau} = 2 Re[Yt_tau^dag dB_tau X_tau],
 * Y = M X, Yt_tau = -Y_{tau+1} (tau < Nt-1), Yt_{Nt-1} = +Y_0.
 * X: device complex FP64; F: device double[2][Nt][L][L] (overwritten). */
qedhmc_status qedhmc_fermion_force(qedhmc_t h, const double *theta,
                                   const double *X, double *F,
                                   qedhmc_precision prec);

/* Gauge action of the handle (params.action)
 *   compact      S_B = 1/(J dtau) sum [1 - cos(theta_{tau+1} - theta_tau)]
 *                      + K dtau sum_plaquettes cos(curl theta)
 *                (Results, L_B^c)
 *   non-compact  S_B = 1/(J dtau) sum (theta_{tau+1} - theta_tau)^2
 *                      + K dtau sum_plaquettes cos(curl theta)
 *                (Results, Eq. 3)
 * (tau periodic) into *S_B_host (nullable) and, if F_B is not NULL, its force
 * -dS_B/dtheta into device double[2][Nt][L][L]. */
qedhmc_status qedhmc_bosonic_action_force(qedhmc_t h, const double *theta,
                                          double *S_B_host, double *F_B);

/* Heat bath of trajectory traj_index (step (i)): momenta p ~ N(0, 1/2) per
 * bond and source R with Re, Im ~ N(0, 1/2) per site, from Philox4x32-10
 * (key = seed, counter = (element, traj low, purpose, traj high)) and
 * Box-Muller.  mom: device double[2][Nt][L][L]; R: device complex FP64. */
qedhmc_status qedhmc_heatbath(qedhmc_t h, uint64_t traj_index, double *mom,
                              double *R);

/* One HQMC trajectory: heat bath, eta = M^dag R, n_steps leapfrog steps of
 * length traj_len / n_steps with a solve at every theta (the first from
 * x = 0, each later one started from the previous solution: it solves for the
 * correction to the same absolute target tol |eta|; QEDHMC_WARM_START=0,
 * read per call, starts every solve from x = 0), Metropolis with u from
 * Philox.  theta_inout: device double[2][Nt][L][L], overwritten by the
 * proposal on acceptance, unchanged on rejection. */
qedhmc_status qedhmc_hmc_trajectory(qedhmc_t h, double *theta_inout,
                                    uint64_t traj_index, int32_t n_steps,
                                    double traj_len, double tol, int32_t maxit,
                                    qedhmc_precision prec, qedhmc_precond pc,
                                    qedhmc_traj_result *out);

/* Checkpoint and resume of one chain.  The trajectory random streams are
 * counter-based (Philox keyed by the seed, the trajectory index in the
 * counter; Methods, HQMC steps (i) and (iii)), so the lattice parameters,
 * theta and the index of the next trajectory fix the rest of the chain: a
 * chain resumed from a checkpoint runs bit for bit the trajectories it would
 * have run without the stop.
 * File (little endian): magic "QEDHMCK1", then uint64 version (1), int64 L,
 * int64 Nt, double dtau, t, J, K, uint64 seed, int64 action, uint64
 * next_traj, uint64 n = 2 Nt L^2, double theta[n] in the device layout, and
 * a uint64 FNV-1a-64 hash of every byte before it.  qedhmc_checkpoint_save writes "<path>.tmp"
 * and renames it over path (theta: device, the handle's lattice; synchronises
 * the stream).  qedhmc_checkpoint_info reads the header of a verified file
 * (no device work).  qedhmc_checkpoint_load checks the file (magic, version,
 * sizes, hash) and that its parameters equal the handle's bit for bit, then
 * copies theta to the device buffer and returns next_traj (synchronises).
 * A bad or mismatched file is QEDHMC_EINVAL with nothing written. */
qedhmc_status qedhmc_checkpoint_save(qedhmc_t h, const double *theta,
                                     uint64_t next_traj, const char *path);
qedhmc_status qedhmc_checkpoint_info(const char *path, qedhmc_params *params,
                                     uint64_t *next_traj);
qedhmc_status qedhmc_checkpoint_load(qedhmc_t h, const char *path,
                                     double *theta, uint64_t *next_traj);

/* ------------------------------------------------------------------------
 * Batched chains: many independent Markov chains, each on its own lattice
 * (sizes may differ), advanced together on one device.  Every chain runs
 * exactly the single-lattice trajectory of qedhmc_hmc_trajectory (same
 * heat bath streams from its own seed, same leapfrog, same Metropolis); the
 * chains' CG solves share each kernel launch (one launch performs one
 * iteration of every chain still running), with per-chain scalars,
 * reliable updates and stopping.  Methods, "HQMC algorithm"; the batching
 * itself is not in the paper.
 *
 * Layout: all chains' arrays are concatenated in chain order.  theta_all,
 * momenta and forces: double, chain c at offset theta_off[c] (2*Nt*L*L
 * doubles per chain); complex vectors: chain c at complex offset vec_off[c]
 * (Nt*L*L elements).  The offsets come from qedhmc_batch_layout.
 *
 * Limits: every lattice must fit one workgroup per time slice with at most
 * two 2x2 cells per thread (L <= 44; QEDHMC_EUNSUPPORTED otherwise).
 * Preconditioning is not offered on batches. */
typedef struct qedhmc_batch *qedhmc_batch_t;

/* Create n_chains handles from params[0..n_chains-1] (each validated as by
 * qedhmc_init_lattice) on one stream, and pick the tile shape of the batched
 * CG kernels by timing every candidate on these lattices.  Synchronises the
 * stream.  On failure nothing is left allocated and *out is NULL. */
qedhmc_status qedhmc_batch_create(const qedhmc_params *params,
                                  int32_t n_chains, void *stream,
                                  qedhmc_batch_t *out);
qedhmc_status qedhmc_batch_destroy(qedhmc_batch_t b);

/* Offsets into the concatenated arrays, host int64[n_chains + 1] each; the
 * last entry is the total length. */
qedhmc_status qedhmc_batch_layout(qedhmc_batch_t b, int64_t *theta_off,
                                  int64_t *vec_off);

/* The tile shape the autotuner chose for the CG recursion in precision
 * prec (cells per thread, threads per workgroup, LDS exchange buffers; a
 * workgroup runs threads / G consecutive time slices of one chain, G the
 * smallest power of two from 16 up with G x cells per thread at least the
 * slice's L^2 / 4 cells) and
 * the measured time per batched CG iteration of each of the four candidate
 * shapes in microseconds (host float[4]; 0 for a candidate that does not
 * fit). */
qedhmc_status qedhmc_batch_tile(qedhmc_batch_t b, qedhmc_precision prec,
                                int32_t *cells_per_thread, int32_t *threads,
                                int32_t *exchange_buffers, float *us_per_iter);

/* Solve M^dag M x_c = rhs_c for every chain c at once (as qedhmc_cg_solve
 * without preconditioner).  theta_all, rhs_all, x_all: device, concatenated;
 * iters, true_rel: host arrays of n_chains.  QEDHMC_ENOCONV when any chain
 * did not converge (every x still written). */
qedhmc_status qedhmc_batch_cg_solve(qedhmc_batch_t b, const double *theta_all,
                                    const double *rhs_all, double *x_all,
                                    double tol, int32_t maxit,
                                    qedhmc_precision prec, int32_t *iters,
                                    double *true_rel);

/* One trajectory of every chain (as qedhmc_hmc_trajectory with
 * QEDHMC_PC_NONE).  theta_all: device, concatenated, updated per chain on
 * acceptance; out: host array of n_chains results. */
qedhmc_status qedhmc_batch_trajectory(qedhmc_batch_t b, double *theta_all,
                                      uint64_t traj_index, int32_t n_steps,
                                      double traj_len, double tol,
                                      int32_t maxit, qedhmc_precision prec,
                                      qedhmc_traj_result *out);

/* ------------------------------------------------------------------------
 * Production loop (Methods, "HQMC algorithm": N_leapfrog = 3 leapfrog steps
 * per trajectory, the step size tuned to keep a moderate acceptance rate),
 * the gauge observables it logs (Supplemental Material SV), the flux
 * correlator (Results, Eq. (33)) and the autocorrelation of a logged series.
 * ------------------------------------------------------------------------ */

/* S_tau and S_plaq, the two terms of the handle's gauge action at theta:
 * S_tau = 1/(J dtau) sum (theta_{tau+1} - theta_tau)^2 (non-compact; the
 * compact action's 1 - cos of the difference), S_plaq = K dtau sum cos(curl
 * theta) over the plaquettes.  Host outputs; synchronises. */
qedhmc_status qedhmc_gauge_observables(qedhmc_t h, const double *theta,
                                       double *S_tau, double *S_plaq);

/* C_out[dtau] = 1/(L^2 Nt) sum_{tau, plaquettes} sin Phi(tau + dtau)
 * sin Phi(tau), dtau = 0 .. Nt - 1, tau periodic (Eq. (33) averaged over the
 * time origin); C_out: device double[Nt].  Enqueued, not synchronised. */
qedhmc_status qedhmc_flux_correlator(qedhmc_t h, const double *theta,
                                     double *C_out);

typedef struct {
    uint64_t first_traj;     /* trajectory index of the first trajectory     */
    int32_t n_therm, n_meas; /* thermalisation (dt adapted), then measured   */
    int32_t n_steps;         /* leapfrog steps per trajectory (3 in the paper) */
    int32_t maxit;           /* CG iteration budget per solve                */
    double dt0;              /* initial leapfrog step                        */
    double target_accept;    /* in (0, 1): acceptance the step is tuned to   */
    double gain;             /* >= 0: step-size adaptation gain              */
    double tol;              /* CG true relative residual                    */
    qedhmc_precision prec;
    qedhmc_precond pc;
} qedhmc_prod_params;

typedef struct {
    uint64_t traj;
    double dt;               /* leapfrog step of this trajectory             */
    double dH;
    double S_tau, S_plaq;    /* of the chain's configuration after the
                                Metropolis decision                          */
    int32_t accepted, cg_iters, status, reserved;
} qedhmc_prod_record;

/* n_therm + n_meas chained trajectories from theta_inout (updated in place).
 * Trajectory k has index first_traj + k and n_steps steps of dt.  During
 * thermalisation, after each trajectory, dt <- dt exp(gain (min(1, e^{-dH})
 * - target_accept)), the factor clipped to [1/2, 2]; dt is frozen for the
 * measured trajectories.  records: host array of n_therm + n_meas.
 * C_flux_mean (nullable): device double[Nt], the flux correlator averaged
 * over the measured configurations.  dt_final (nullable, host): the frozen
 * step.  Synchronises.  ENOCONV when some trajectory had an unconverged solve
 * (that trajectory was rejected; the loop went on). */
qedhmc_status qedhmc_production(qedhmc_t h, double *theta_inout,
                                const qedhmc_prod_params *params,
                                qedhmc_prod_record *records,
                                double *C_flux_mean, double *dt_final);

/* Host analysis of a series x[0..n): rho[k] = C(k)/C(0) for k = 0 .. kmax,
 * C(k) = 1/(n-k) sum_t (x_t - mean)(x_{t+k} - mean); tau_int = 1/2 +
 * sum_{k=1..W} rho[k] with the smallest window W >= 5 tau_int (Sokal);
 * tau_exp from the least-squares fit of log rho[k] = -k/tau_exp over the
 * k >= 1 before rho first drops below 0.1 (0 if none).  1 <= kmax < n.
 * No device work. */
qedhmc_status qedhmc_autocorrelation(const double *series, int32_t n,
                                     int32_t kmax, double *rho,
                                     double *tau_int, double *tau_exp);

/* ------------------------------------------------------------------------
 * Stochastic estimation of fermionic observables (Methods, "Stochastic
 * estimation of fermionic observables", Eq. (Cij_est) and the FFT
 * translational average after it; Supplemental Material SIV).
 *
 * G = M^{-1} is the Green's function of one gauge configuration.  With n_rv
 * probes xi_p (E[xi^* xi^T] = 1) and X_p = G xi_p, computed as
 * (M^dag M)^{-1} M^dag xi_p, the spin correlator of SIV,
 *   C_S(i, j) = Gbar(i, j) G(i, j),  Gbar(i, j) = delta_ij - G(j, i),
 * averaged over translations of the periodic space-time torus,
 *   C_S(Delta) = (1/N) sum_i C_S(i, i + Delta),
 * is estimated without bias as delta_{Delta,0} T1 - T2(Delta):
 *   T1 = (1/(n_rv N)) sum_p sum_i X_p,i conj(xi_p,i),
 *   T2 = average over ordered probe pairs p != q of (1/N) sum_i a_i b_{i+Delta},
 *        a = X_p conj(xi_q), b = X_q conj(xi_p),
 * each correlation evaluated by three-dimensional DFTs (N = L^2 Nt sites).
 * ------------------------------------------------------------------------ */
typedef struct qedhmc_se *qedhmc_se_t;

/* A context for n_rv probes on one lattice: a multi-RHS CG (n_rv right-hand
 * sides whose iterations share one gauge field) and the transform workspace.
 * 2 <= n_rv, n_rv L^2 Nt < 2^32, L <= 44 (EUNSUPPORTED beyond).  The probes'
 * Philox key is params->seed.  Work is enqueued on stream. */
qedhmc_status qedhmc_se_create(const qedhmc_params *params, int32_t n_rv,
                               void *stream, qedhmc_se_t *out);
qedhmc_status qedhmc_se_destroy(qedhmc_se_t se);

/* xi_all: device complex FP64 [n_rv][Nt][L][L], written with the probes of
 * measurement meas_index: Re, Im ~ N(0, 1/2), Philox purpose 4, counter
 * element p * N + n, index words meas_index. */
qedhmc_status qedhmc_se_probes(qedhmc_se_t se, uint64_t meas_index,
                               double *xi_all);

/* X_p = (M^dag M)^{-1} M^dag xi_p for every probe, at relative true residual
 * tol (FP64, or the mixed path with QEDHMC_FP32), at most maxit iterations
 * each.  xi_all, X_all: device complex FP64 [n_rv][Nt][L][L], not aliased;
 * theta as for qedhmc_apply_M.  iters, true_rel: host arrays of n_rv, written
 * per probe.  Synchronises.  ENOCONV if any probe missed tol (all outputs
 * still written). */
qedhmc_status qedhmc_se_solve(qedhmc_se_t se, const double *theta,
                              const double *xi_all, double *X_all, double tol,
                              int32_t maxit, qedhmc_precision prec,
                              int32_t *iters, double *true_rel);

/* C_out = the estimate of C_S(Delta) from xi_all and X_all (as written by
 * qedhmc_se_probes and qedhmc_se_solve, or any probes and X_p = G xi_p):
 * device complex FP64 [Nt][L][L] indexed by Delta = (dtau, dy, dx), all
 * arithmetic in FP64 in a fixed order.  Enqueued on the stream; does not
 * synchronise. */
qedhmc_status qedhmc_se_spin_correlator(qedhmc_se_t se, const double *xi_all,
                                        const double *X_all, double *C_out);

/* ------------------------------------------------------------------------
 * Learned preconditioner (not in the paper; its fixed preconditioner of
 * Methods, "CG method and preconditioner", is the fallback): a network
 * z = N(theta, r) of six 3x3x3 convolutions over the (tau, y, x) lattice,
 * channels 6 -> 32 -> 32 -> 32 -> 32 -> 32 -> 2, SiLU after every layer but
 * the last.  Input channels per site: cos, sin of theta on the +x and +y
 * bonds leaving it and Re, Im of r / s, s = |r| / sqrt(N); output
 * z = s (o_0 + i o_1).  Padding periodic in x, y and tau, except that the
 * first layer's residual channels change sign when they wrap in tau.
 *
 * Parameters (host float array of qedhmc_net_param_count() entries): per
 * layer in order, W[Cout][Cin][27] with tap k = 9 (dt + 1) + 3 (dy + 1) +
 * (dx + 1) reading the input at (tau + dt, y + dy, x + dx), then b[Cout].
 * A network is bound to one lattice handle (its stream and sizes); copy the
 * parameters to use them on another lattice. */
typedef struct qedhmc_net *qedhmc_net_t;

/* Arithmetic of the network: FP32 on the vector ALUs throughout, or BF16
 * MFMA products (BF16 weights and activations, FP32 accumulation) for the
 * four 32 -> 32 layers with the first and last layers in FP32.  Training
 * runs in FP32 (FP32 master weights and Adam moments). */
typedef enum { QEDHMC_NET_FP32 = 0, QEDHMC_NET_BF16 = 1 } qedhmc_net_arith;

int64_t qedhmc_net_param_count(void);
/* Allocate a network on lattice h with all parameters zero. */
qedhmc_status qedhmc_net_create(qedhmc_t h, qedhmc_net_t *out);
qedhmc_status qedhmc_net_destroy(qedhmc_net_t n);
/* Copy parameters in / out (host layout above; count must match). */
qedhmc_status qedhmc_net_set_params(qedhmc_net_t n, const float *host,
                                    int64_t count);
qedhmc_status qedhmc_net_get_params(qedhmc_net_t n, float *host,
                                    int64_t count);
/* Zero the Adam moments and step counter. */
qedhmc_status qedhmc_net_reset_optimizer(qedhmc_net_t n);

/* z = N(theta, r); r, z: device complex FP64 [Nt][L][L]. */
qedhmc_status qedhmc_net_apply(qedhmc_net_t n, const double *theta,
                               const double *r, double *z,
                               qedhmc_net_arith arith);

/* One training step on the triple (theta, r, e), e the solution of
 * M^dag M e = r: loss = |N(theta, r) - e|^2 / |e|^2 into *loss (host), the
 * gradient of the loss into grad_host (host float array in the parameter
 * layout, nullable; the gradient before the update), then one Adam step
 * (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr).  FP32 arithmetic
 * only (QEDHMC_EUNSUPPORTED otherwise). */
qedhmc_status qedhmc_net_train_step(qedhmc_net_t n, const double *theta,
                                    const double *r, const double *e,
                                    double lr, qedhmc_net_arith arith,
                                    double *loss, float *grad_host);

/* One training step in residual form on the pair (theta, r): loss =
 * |O z - r|^2 / |r|^2 with z = N(theta, r) and O = M^dag M (the FP64 fused
 * operator of the handle) -- the error z - e of the triple (theta, r, e),
 * O e = r, measured as |O (z - e)| / |O e|, which needs no e.  It weighs the
 * error along each eigenvector of O by the eigenvalue instead of letting the
 * lowest modes dominate.  Gradient (2 s O (O z - r) / |r|^2 at the outputs,
 * s the output scale) into grad_host (nullable), then one Adam step as
 * above.  r: device complex FP64 [Nt][L][L], e.g. a residual r_k of one of
 * the method's own solves.  FP32 arithmetic only. */
qedhmc_status qedhmc_net_train_step_residual(qedhmc_net_t n,
                                             const double *theta,
                                             const double *r, double lr,
                                             qedhmc_net_arith arith,
                                             double *loss,
                                             float *grad_host);

/* Flexible CG on M^dag M x = rhs preconditioned by the network (Notay's
 * flexible CG: alpha = <p, r> / <p, O p>, beta = -<O p, z'> / <p, O p>),
 * from x = 0, stopping on the FP64 true residual |rhs - O x| / |rhs| <= tol.
 * The residual judges the network: when |r| has not at least halved
 * over the last 10 iterations the solve continues with the fallback
 * preconditioner (QEDHMC_PC_PAPER or QEDHMC_PC_NONE) and *switched_at
 * (host, nullable) receives that iteration (-1 if the network kept it).
 * The paper's preconditioner as fallback runs its stencil passes in FP32
 * (flexible CG tolerates the inexact preconditioner).
 * All vectors FP64 complex on the device.  ENOCONV as for qedhmc_cg_solve. */
qedhmc_status qedhmc_fcg_solve(qedhmc_net_t n, const double *theta,
                               const double *rhs, double *x, double tol,
                               int32_t maxit, qedhmc_net_arith arith,
                               qedhmc_precond fallback, int32_t *iters,
                               double *true_rel_resid, int32_t *switched_at);

/* Bind network n (created on this handle) as the handle's learned
 * preconditioner: QEDHMC_PC_LEARNED in qedhmc_cg_solve and
 * qedhmc_hmc_trajectory then runs flexible CG with z = N(theta, r) in
 * arithmetic arith, judged by the residual as in qedhmc_fcg_solve, with
 * fallback QEDHMC_PC_PAPER or QEDHMC_PC_NONE.  n = NULL unbinds.  The handle
 * keeps a reference only: destroying the network unbinds it; the network
 * must not outlive the handle.  EINVAL when n belongs to another handle or an
 * enum is out of range.  (North-star extension; the paper's fixed
 * preconditioner of Methods, "CG method and preconditioner", is the
 * fallback.) */
qedhmc_status qedhmc_set_learned_precond(qedhmc_t h, qedhmc_net_t n,
                                         qedhmc_net_arith arith,
                                         qedhmc_precond fallback);

/* Kernel timing for measurement (not part of the method).  qedhmc_profile
 * with every > 0 times every every-th launch of the timed kernel classes
 * with the start and end events of the dispatch itself
 * (hipExtLaunchKernelGGL) and clears the accumulators; every = 0 turns it
 * off.  qedhmc_profile_read returns, for kernel class k (QEDHMC_K_*), the
 * number of timed launches and their summed duration in milliseconds, after
 * synchronising the stream. */
typedef enum {
    QEDHMC_K_MDAGM_FP32 = 0,   /* standalone fused M^dag M, complex FP32 */
    QEDHMC_K_MDAGM_FP64 = 1,   /* standalone fused M^dag M, complex FP64 */
    QEDHMC_K_FORCE = 2,        /* fermion force kernel (either precision) */
    QEDHMC_K_CG_FP32 = 3,      /* one fused CG iteration (M^dag M + updates), FP32 */
    QEDHMC_K_CG_FP64 = 4,      /* one fused CG iteration, FP64 */
    QEDHMC_K_PCG_MV_FP32 = 5,  /* M^dag M + inner products of a PCG iteration, FP32 */
    QEDHMC_K_PCG_MV_FP64 = 6,  /* the same, FP64 */
    QEDHMC_K_NET_MFMA = 7,     /* one 32 -> 32 network layer, BF16 MFMA */
    QEDHMC_K_NET_FP32 = 8,     /* one 32 -> 32 network layer, FP32 */
    QEDHMC_K_PC_SPEC_FP32 = 9, /* tau sum + inverse DFT of the spectral paper preconditioner, FP32 */
    QEDHMC_K_PC_SPEC_FP64 = 10,/* the same, FP64 */
    QEDHMC_K_COUNT = 11
} qedhmc_kernel_class;

qedhmc_status qedhmc_profile(qedhmc_t h, int32_t every);
qedhmc_status qedhmc_profile_read(qedhmc_t h, int32_t kernel_class,
                                  int64_t *count, double *total_ms);

#ifdef __cplusplus
}
#endif

#endif /* QEDHMC_H */
