/*
 * qed_oracle.c -- plain, slow, FP64 CPU oracle for the hybrid quantum Monte
 * Carlo (HQMC) hot path of lattice QED3: a U(1) gauge field theta on the
 * spatial bonds of an L x L x N_tau space-time lattice coupled to two
 * identical fermion flavours (one complex pseudofermion).
 *
 * TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
 * CPU-baseline leg call this file; the product library never does, and this
 * file shares no code, header or table with it.
 *
 * Everything is written from the paper's definitions (Methods: "Model and
 * partition function", "HQMC algorithm", "CG method and preconditioner",
 * "Matrix-free representation of M^dagger M v"; Supplemental Material SI),
 * one step at a time, with no blocking or fusion.  Where the paper is silent
 * or ambiguous, the reading taken is stated at the function.
 *
 * Conventions
 *   site         s = y*L + x                      (x, y in [0, L), periodic)
 *   space-time   n = tau*Vs + s                   (tau in [0, Nt); the paper
 *                                                  counts slices from 1)
 *   gauge field  theta[(d*Nt + tau)*Vs + s]       angle on the bond from s to
 *                                                  s + e_d (d=0: x, d=1: y)
 *   vectors      v[n], complex double
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* Lattice and couplings.  dtau: Trotter step; t: hopping amplitude;
 * J, K: couplings of the gauge action; noncompact: 0 for the compact
 * Lagrangian L_B^c, 1 for the non-compact L_B^nc of Results, Eq. (3). */
typedef struct {
    int32_t L, Nt;
    double dtau, t, J, K;
    int32_t noncompact;
} oracle_lat;

/* ------------------------------------------------------------------------ */
/* Bond families (Fig. 1 and Eq. 24): the spatial bonds split into four     */
/* families whose 2x2 hopping blocks commute within the family:             */
/*   f0: x-bonds leaving even x      f1: x-bonds leaving odd x              */
/*   f2: y-bonds leaving even y      f3: y-bonds leaving odd y              */
/* Entry = (i, j, bond index d*Vs + s), listed in increasing origin site s. */
/* Needs even L (odd L makes a family touch a site twice).                  */
/* ------------------------------------------------------------------------ */
void oracle_bond_tables(int32_t L, int32_t *tab /* [4][Vs/2][3] */)
{
    const int Vs = L * L, half = Vs / 2;
    int cnt[4] = {0, 0, 0, 0};
    for (int s = 0; s < Vs; s++) {
        const int x = s % L, y = s / L;
        /* bond along x from s */
        int f = (x % 2 == 0) ? 0 : 1;
        int32_t *e = tab + 3 * (f * half + cnt[f]++);
        e[0] = s;
        e[1] = y * L + (x + 1) % L;
        e[2] = 0 * Vs + s;
        /* bond along y from s */
        f = (y % 2 == 0) ? 2 : 3;
        e = tab + 3 * (f * half + cnt[f]++);
        e[0] = s;
        e[1] = ((y + 1) % L) * L + x;
        e[2] = 1 * Vs + s;
    }
}

/* exp(a * T_ij) on every bond of family f in slice tau, in place on the
 * slice vector v[Vs]: each bond block is cosh(a) 1 + sinh(a) T_ij with
 * T_ij = [[0, e^{i theta}], [e^{-i theta}, 0]] (Methods, block formula after
 * Eq. 24).  a = t * dtau / 2 for a half factor. */
static void apply_factor(const oracle_lat *p, const int32_t *tab, int f,
                         double a, const double *theta, int tau, cplx *v)
{
    const int Vs = p->L * p->L, half = Vs / 2;
    const double c = cosh(a), sh = sinh(a);
    for (int k = 0; k < half; k++) {
        const int32_t *e = tab + 3 * (f * half + k);
        const int i = e[0], j = e[1], b = e[2];
        const int d = b / Vs, s = b % Vs;
        const double th = theta[((size_t)d * p->Nt + tau) * Vs + s];
        const cplx h = sh * cexp(I * th);
        const cplx vi = v[i], vj = v[j];
        v[i] = c * vi + h * vj;
        v[j] = conj(h) * vi + c * vj;
    }
}

/* Symmetric checkerboard product for slice tau (Eq. 24):
 *   B_tau = E3(h) E2(h) E1(h) E0(2h) E1(h) E2(h) E3(h),  h = t dtau / 2,
 * with the paper's V1..V4 read as families f0..f3 and the two central
 * half factors of V1 merged into one full factor (exact, they commute).
 * The product is a palindrome, so the factors are applied to v in the
 * listed order. */
static void apply_B(const oracle_lat *p, const int32_t *tab,
                    const double *theta, int tau, cplx *v)
{
    const double h = 0.5 * p->t * p->dtau;
    static const int fam[7] = {3, 2, 1, 0, 1, 2, 3};
    for (int m = 0; m < 7; m++)
        apply_factor(p, tab, fam[m], fam[m] == 0 ? 2.0 * h : h, theta, tau, v);
}

static int32_t *make_tables(int L)
{
    int32_t *tab = malloc(sizeof(int32_t) * 3 * 2 * L * L);
    oracle_bond_tables(L, tab);
    return tab;
}

/* B_tau v for one slice (exported for dense checks). */
void oracle_apply_B(const oracle_lat *p, const double *theta, int32_t tau,
                    const cplx *in, cplx *out)
{
    int32_t *tab = make_tables(p->L);
    memcpy(out, in, sizeof(cplx) * p->L * p->L);
    apply_B(p, tab, theta, tau, out);
    free(tab);
}

/* One factor E_f(a) for one slice (exported for the force checks). */
void oracle_apply_factor(const oracle_lat *p, const double *theta, int32_t tau,
                         int32_t f, double a, cplx *v)
{
    int32_t *tab = make_tables(p->L);
    apply_factor(p, tab, f, a, theta, tau, v);
    free(tab);
}

/* Space-time matrix M (Eq. M_alpha), block bidiagonal with the
 * antiperiodic corner:
 *   (M v)_0   = v_0   + B_{Nt-1} v_{Nt-1}
 *   (M v)_tau = v_tau - B_{tau-1} v_{tau-1}          (tau >= 1)
 * and its adjoint (B_tau is Hermitian):
 *   (M^dag w)_tau    = w_tau - B_tau w_{tau+1}       (tau <= Nt-2)
 *   (M^dag w)_{Nt-1} = w_{Nt-1} + B_{Nt-1} w_0 */
static void apply_M_tab(const oracle_lat *p, const int32_t *tab,
                        const double *theta, const cplx *in, cplx *out,
                        int dagger)
{
    const int Vs = p->L * p->L, Nt = p->Nt;
    cplx *tmp = malloc(sizeof(cplx) * Vs);
    for (int tau = 0; tau < Nt; tau++) {
        int src, bslice;
        double sign;
        if (!dagger) {
            src = (tau + Nt - 1) % Nt;
            bslice = src;
            sign = (tau == 0) ? +1.0 : -1.0;
        } else {
            src = (tau + 1) % Nt;
            bslice = tau;
            sign = (tau == Nt - 1) ? +1.0 : -1.0;
        }
        memcpy(tmp, in + (size_t)src * Vs, sizeof(cplx) * Vs);
        apply_B(p, tab, theta, bslice, tmp);
        for (int s = 0; s < Vs; s++)
            out[(size_t)tau * Vs + s] = in[(size_t)tau * Vs + s] + sign * tmp[s];
    }
    free(tmp);
}

void oracle_apply_M(const oracle_lat *p, const double *theta, const cplx *in,
                    cplx *out, int32_t dagger)
{
    int32_t *tab = make_tables(p->L);
    apply_M_tab(p, tab, theta, in, out, dagger);
    free(tab);
}

/* O v = M^dag (M v), unfused (the definition; CG section). */
static void apply_MdagM_tab(const oracle_lat *p, const int32_t *tab,
                            const double *theta, const cplx *in, cplx *out,
                            cplx *scratch)
{
    apply_M_tab(p, tab, theta, in, scratch, 0);
    apply_M_tab(p, tab, theta, scratch, out, 1);
}

void oracle_apply_MdagM(const oracle_lat *p, const double *theta,
                        const cplx *in, cplx *out)
{
    const size_t N = (size_t)p->L * p->L * p->Nt;
    int32_t *tab = make_tables(p->L);
    cplx *scr = malloc(sizeof(cplx) * N);
    apply_MdagM_tab(p, tab, theta, in, out, scr);
    free(scr);
    free(tab);
}

static double dot_re(const cplx *a, const cplx *b, size_t n)
{
    double s = 0.0;
    for (size_t k = 0; k < n; k++) s += creal(conj(a[k]) * b[k]);
    return s;
}

/* Optional preconditioner z = P r supplied by the caller (NULL: none). */
typedef void (*oracle_precond_fn)(void *ctx, const cplx *r, cplx *z);

/* Preconditioned conjugate gradient on O X = rhs (Eq. pCG), started from
 * X_0 = 0.  Readings: d_0 = z_0 = P r_0 (standard PCG; the printed d_0 = r_0
 * is only right without a preconditioner); stop when the recursive residual
 * satisfies |r| <= tol |rhs|, then recompute r = rhs - O X and, if that true
 * residual is still above tol, continue from it with d = P r.  Returns 0 on
 * convergence, 1 when maxit iterations were spent. */
int32_t oracle_cg_solve_pc(const oracle_lat *p, const double *theta,
                           const cplx *rhs, cplx *X, double tol, int32_t maxit,
                           oracle_precond_fn pc, void *pc_ctx, int32_t *iters,
                           double *true_rel_resid)
{
    const size_t N = (size_t)p->L * p->L * p->Nt;
    int32_t *tab = make_tables(p->L);
    cplx *r = malloc(sizeof(cplx) * N), *z = malloc(sizeof(cplx) * N);
    cplx *d = malloc(sizeof(cplx) * N), *Od = malloc(sizeof(cplx) * N);
    cplx *scr = malloc(sizeof(cplx) * N);
    const double bnorm = sqrt(dot_re(rhs, rhs, N));
    int it = 0, status = 1;
    double rel = 0.0;

    for (size_t k = 0; k < N; k++) { X[k] = 0.0; r[k] = rhs[k]; }
    if (bnorm == 0.0) { status = 0; goto done; }
    for (;;) {
        /* (re)start from the current residual */
        if (pc) pc(pc_ctx, r, z); else memcpy(z, r, sizeof(cplx) * N);
        memcpy(d, z, sizeof(cplx) * N);
        double rz = dot_re(r, z, N);
        while (it < maxit && sqrt(dot_re(r, r, N)) > tol * bnorm) {
            apply_MdagM_tab(p, tab, theta, d, Od, scr);
            const double zeta = rz / dot_re(d, Od, N);
            for (size_t k = 0; k < N; k++) {
                X[k] += zeta * d[k];
                r[k] -= zeta * Od[k];
            }
            if (pc) pc(pc_ctx, r, z); else memcpy(z, r, sizeof(cplx) * N);
            const double rz_new = dot_re(r, z, N);
            const double rho = rz_new / rz;
            rz = rz_new;
            for (size_t k = 0; k < N; k++) d[k] = z[k] + rho * d[k];
            it++;
        }
        /* true residual */
        apply_MdagM_tab(p, tab, theta, X, Od, scr);
        for (size_t k = 0; k < N; k++) r[k] = rhs[k] - Od[k];
        rel = sqrt(dot_re(r, r, N)) / bnorm;
        if (rel <= tol) { status = 0; break; }
        if (it >= maxit) break;
    }
done:
    if (iters) *iters = it;
    if (true_rel_resid) *true_rel_resid = rel;
    free(r); free(z); free(d); free(Od); free(scr); free(tab);
    return status;
}

int32_t oracle_cg_solve(const oracle_lat *p, const double *theta,
                        const cplx *rhs, cplx *X, double tol, int32_t maxit,
                        int32_t *iters, double *true_rel_resid)
{
    return oracle_cg_solve_pc(p, theta, rhs, X, tol, maxit, NULL, NULL, iters,
                              true_rel_resid);
}

/* ------------------------------------------------------------------------ */
/* Fermion force (Supplemental Material SI, Eq. force&CG and fermion_force) */
/*   S_F = eta^dag (M^dag M)^{-1} eta,   X = (M^dag M)^{-1} eta,  Y = M X   */
/*   F_b = -dS_F/dtheta_b = 2 Re[ Y^dag (dM/dtheta_b) X ]                   */
/* Reading: the paper's first line calls +dS_F/dtheta the force while the   */
/* leapfrog uses F = -dH/dtheta; the sign here is the one Hamilton's        */
/* equations need.  theta_{b,tau} enters only B_tau, which sits in block    */
/* row tau+1 of M with the coefficient -1 (+1 for the wrapping block), so   */
/*   F_{b,tau} = 2 Re[ Yt_tau^dag (dB_tau/dtheta_b) X_tau ],                */
/*   Yt_tau = -Y_{tau+1} (tau < Nt-1),  Yt_{Nt-1} = +Y_0,                   */
/* and dB_tau/dtheta_b is the product rule over the seven factors of        */
/* Eq. 24 (SI): B = L_m E_m R_m  =>  2 Re[(L_m^dag Yt)^dag dE_m (R_m X)].   */
/* ------------------------------------------------------------------------ */
void oracle_fermion_force(const oracle_lat *p, const double *theta,
                          const cplx *X, double *F /* [2][Nt][Vs] */)
{
    const int L = p->L, Vs = L * L, Nt = p->Nt, half = Vs / 2;
    const size_t N = (size_t)Vs * Nt;
    const double h = 0.5 * p->t * p->dtau;
    static const int fam[7] = {3, 2, 1, 0, 1, 2, 3}; /* factor m, left to right */
    int32_t *tab = make_tables(L);
    cplx *Y = malloc(sizeof(cplx) * N);
    cplx *u = malloc(sizeof(cplx) * 8 * Vs); /* u[m] = R_m X_tau, m = 0..6 */
    cplx *w = malloc(sizeof(cplx) * 8 * Vs); /* w[m] = L_m^dag Yt_tau     */

    apply_M_tab(p, tab, theta, X, Y, 0);
    memset(F, 0, sizeof(double) * 2 * N);
    for (int tau = 0; tau < Nt; tau++) {
        /* R_6 = 1; R_{m-1} = E_m R_m */
        memcpy(u + 6 * Vs, X + (size_t)tau * Vs, sizeof(cplx) * Vs);
        for (int m = 6; m >= 1; m--) {
            memcpy(u + (m - 1) * Vs, u + m * Vs, sizeof(cplx) * Vs);
            apply_factor(p, tab, fam[m], fam[m] == 0 ? 2 * h : h, theta, tau,
                         u + (m - 1) * Vs);
        }
        /* L_0 = 1; L_{m+1}^dag = E_m L_m^dag (every factor is Hermitian) */
        const int tn = (tau + 1) % Nt;
        const double sgn = (tau == Nt - 1) ? +1.0 : -1.0;
        for (int s = 0; s < Vs; s++) w[s] = sgn * Y[(size_t)tn * Vs + s];
        for (int m = 0; m < 6; m++) {
            memcpy(w + (m + 1) * Vs, w + m * Vs, sizeof(cplx) * Vs);
            apply_factor(p, tab, fam[m], fam[m] == 0 ? 2 * h : h, theta, tau,
                         w + (m + 1) * Vs);
        }
        for (int m = 0; m < 7; m++) {
            const int f = fam[m];
            const double sh = sinh(f == 0 ? 2 * h : h);
            const cplx *um = u + m * Vs, *wm = w + m * Vs;
            for (int k = 0; k < half; k++) {
                const int32_t *e = tab + 3 * (f * half + k);
                const int i = e[0], j = e[1], b = e[2];
                const int d = b / Vs, s = b % Vs;
                const size_t idx = ((size_t)d * Nt + tau) * Vs + s;
                const double th = theta[idx];
                /* d/dtheta of the block [[c, sh e^{i th}], [sh e^{-i th}, c]] */
                const cplx dij = I * sh * cexp(I * th);
                const cplx dji = -I * sh * cexp(-I * th);
                const cplx val = conj(wm[i]) * dij * um[j] + conj(wm[j]) * dji * um[i];
                F[idx] += 2.0 * creal(val);
            }
        }
    }
    free(Y); free(u); free(w); free(tab);
}

/* ------------------------------------------------------------------------ */
/* Compact gauge action (Results, L_B^c) integrated over imaginary time:    */
/*   S_B = dtau sum_tau L_B^c                                               */
/*       = 1/(J dtau) sum_{d,tau,s} [1 - cos(theta_{d,tau+1,s}-theta_{d,tau,s})]
 *         + K dtau sum_{tau,s} cos Phi_{tau,s}                              */
/* with tau periodic and the plaquette flux (curl, counter-clockwise,       */
/* theta_ji = -theta_ij)                                                    */
/*   Phi_{tau,s} = th_x(s) + th_y(s+x) - th_x(s+y) - th_y(s).               */
/* ------------------------------------------------------------------------ */
static double plaq(const oracle_lat *p, const double *theta, int tau, int s)
{
    const int L = p->L, Vs = L * L, Nt = p->Nt;
    const int x = s % L, y = s / L;
    const int sx = y * L + (x + 1) % L, sy = ((y + 1) % L) * L + x;
    const double *tx = theta + (size_t)(0 * Nt + tau) * Vs;
    const double *ty = theta + (size_t)(1 * Nt + tau) * Vs;
    return tx[s] + ty[sx] - tx[sy] - ty[s];
}

double oracle_bosonic_action(const oracle_lat *p, const double *theta)
{
    const int L = p->L, Vs = L * L, Nt = p->Nt;
    double kin = 0.0, pot = 0.0;
    for (int d = 0; d < 2; d++)
        for (int tau = 0; tau < Nt; tau++)
            for (int s = 0; s < Vs; s++) {
                const double a = theta[((size_t)d * Nt + (tau + 1) % Nt) * Vs + s];
                const double b = theta[((size_t)d * Nt + tau) * Vs + s];
                /* compact: 1 - cos of the time difference (L_B^c);
                 * non-compact: its square, same prefactor (Eq. 3) */
                kin += p->noncompact ? (a - b) * (a - b) : 1.0 - cos(a - b);
            }
    for (int tau = 0; tau < Nt; tau++)
        for (int s = 0; s < Vs; s++) pot += cos(plaq(p, theta, tau, s));
    return kin / (p->J * p->dtau) + p->K * p->dtau * pot;
}

/* F_B = -dS_B/dtheta, accumulated term by term from the same sums. */
void oracle_bosonic_force(const oracle_lat *p, const double *theta, double *F)
{
    const int L = p->L, Vs = L * L, Nt = p->Nt;
    const size_t nb = (size_t)2 * Nt * Vs;
    memset(F, 0, sizeof(double) * nb);
    const double cj = 1.0 / (p->J * p->dtau);
    for (int d = 0; d < 2; d++)
        for (int tau = 0; tau < Nt; tau++)
            for (int s = 0; s < Vs; s++) {
                const size_t ia = ((size_t)d * Nt + (tau + 1) % Nt) * Vs + s;
                const size_t ib = ((size_t)d * Nt + tau) * Vs + s;
                /* term 1 - cos(a - b): d/da = sin(a-b), d/db = -sin(a-b);
                 * term (a - b)^2:      d/da = 2(a-b),   d/db = -2(a-b) */
                const double g = p->noncompact ? 2.0 * (theta[ia] - theta[ib]) : sin(theta[ia] - theta[ib]);
                F[ia] -= cj * g;
                F[ib] += cj * g;
            }
    for (int tau = 0; tau < Nt; tau++)
        for (int s = 0; s < Vs; s++) {
            const int x = s % L, y = s / L;
            const int sx = y * L + (x + 1) % L, sy = ((y + 1) % L) * L + x;
            /* K dtau cos(Phi): d/dPhi = -K dtau sin(Phi); force = +K dtau sin(Phi) dPhi/dtheta */
            const double g = p->K * p->dtau * sin(plaq(p, theta, tau, s));
            F[((size_t)0 * Nt + tau) * Vs + s] += g;
            F[((size_t)1 * Nt + tau) * Vs + sx] += g;
            F[((size_t)0 * Nt + tau) * Vs + sy] -= g;
            F[((size_t)1 * Nt + tau) * Vs + s] -= g;
        }
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,       */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of     */
/* two 32x32->64 multiplies with the Weyl key schedule.                     */
/* ------------------------------------------------------------------------ */
void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                          uint32_t out[4])
{
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; r++) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    }
    memcpy(out, c, sizeof(c));
}

/* Random-number streams of one trajectory.  Counter = (element, trajectory
 * low word, purpose, trajectory high word), key = (seed low, seed high).
 * Purposes: 1 momenta, 2 pseudofermion source R, 3 Metropolis uniform,
 * 4 probe vectors of the stochastic estimation (the "trajectory" words then
 * hold the measurement index). */
enum { PURPOSE_MOMENTUM = 1, PURPOSE_SOURCE = 2, PURPOSE_METROPOLIS = 3, PURPOSE_PROBE = 4 };

static void draw(uint64_t seed, uint64_t traj, uint32_t purpose, uint32_t elem,
                 uint32_t out[4])
{
    const uint32_t ctr[4] = {elem, (uint32_t)traj, purpose, (uint32_t)(traj >> 32)};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    oracle_philox4x32_10(ctr, key, out);
}

/* 53-bit uniform in [0, 1) from two 32-bit words. */
static double u53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

/* Box-Muller: two independent N(0,1) from one Philox block. */
static void gauss2(const uint32_t x[4], double *g1, double *g2)
{
    const double u1 = u53(x[0], x[1]), u2 = u53(x[2], x[3]);
    const double rad = sqrt(-2.0 * log(1.0 - u1));
    const double ang = 2.0 * M_PI * u2;
    *g1 = rad * cos(ang);
    *g2 = rad * sin(ang);
}

/* Heat bath of step (i): p ~ exp(-p^2), i.e. N(0, 1/2) per bond, and R with
 * density exp(-|R|^2), i.e. Re, Im ~ N(0, 1/2) per site.  Bond pair
 * (2k, 2k+1) and site k take block k of their purpose. */
void oracle_heatbath(const oracle_lat *p, uint64_t seed, uint64_t traj,
                     double *mom /* [2N] */, cplx *R /* [N] */)
{
    const size_t N = (size_t)p->L * p->L * p->Nt;
    const double r2 = 1.0 / sqrt(2.0);
    uint32_t x[4];
    double g1, g2;
    for (size_t k = 0; k < N; k++) {
        draw(seed, traj, PURPOSE_MOMENTUM, (uint32_t)k, x);
        gauss2(x, &g1, &g2);
        mom[2 * k] = r2 * g1;
        mom[2 * k + 1] = r2 * g2;
    }
    for (size_t k = 0; k < N; k++) {
        draw(seed, traj, PURPOSE_SOURCE, (uint32_t)k, x);
        gauss2(x, &g1, &g2);
        R[k] = r2 * g1 + I * (r2 * g2);
    }
}

/* Probe vectors of the stochastic estimation (Methods, "Stochastic
 * estimation of fermionic observables"): entries i.i.d. complex Gaussian with
 * E[xi_i^* xi_j] = delta_ij (Re, Im ~ N(0, 1/2)).  Probe k, site n takes the
 * block of element k * N + n (n_rv * N < 2^32). */
void oracle_probes(const oracle_lat *p, uint64_t seed, uint64_t meas, int32_t n_rv,
                   cplx *xi /* [n_rv][N] */)
{
    const size_t N = (size_t)p->L * p->L * p->Nt;
    const double r2 = 1.0 / sqrt(2.0);
    uint32_t x[4];
    double g1, g2;
    for (size_t e = 0; e < (size_t)n_rv * N; e++) {
        draw(seed, meas, PURPOSE_PROBE, (uint32_t)e, x);
        gauss2(x, &g1, &g2);
        xi[e] = r2 * g1 + I * (r2 * g2);
    }
}

double oracle_metropolis_uniform(uint64_t seed, uint64_t traj)
{
    uint32_t x[4];
    draw(seed, traj, PURPOSE_METROPOLIS, 0u, x);
    return u53(x[0], x[1]);
}

/* ------------------------------------------------------------------------ */
/* One HQMC trajectory, steps (i)-(iv) of the Methods with the leapfrog of   */
/* Eq. leapfrog and H of Eq. H_hmc:                                         */
/*   H = S_B(theta) + sum p^2 + eta^dag (M^dag M)^{-1} eta                  */
/* Every solve starts from X = 0 (keeps the MD reversible); the fermion     */
/* action at both ends is Re eta^dag X from the solve at that theta.        */
/* theta is overwritten by the proposal on acceptance and left as it was on */
/* rejection.  mom/R/eta_out may be NULL; when given they receive the drawn */
/* momenta (before MD), the source R and eta = M^dag R.                     */
/* ------------------------------------------------------------------------ */
typedef struct {
    double dH, H0, H1, SB0, SB1, SF0, SF1, K0, K1, u;
    int32_t accepted, n_solves, cg_iters_total, cg_iters_max, status;
    double max_true_resid;
} oracle_traj;

static void total_force(const oracle_lat *p, const double *theta,
                        const cplx *X, double *F, double *Fb, size_t nb)
{
    oracle_fermion_force(p, theta, X, F);
    oracle_bosonic_force(p, theta, Fb);
    for (size_t b = 0; b < nb; b++) F[b] += Fb[b];
}

static void solve_track(const oracle_lat *p, const double *theta, const cplx *eta,
                        cplx *X, double tol, int maxit, oracle_precond_fn pc,
                        void *pc_ctx, oracle_traj *res)
{
    int32_t it = 0;
    double rel = 0.0;
    const int32_t st = oracle_cg_solve_pc(p, theta, eta, X, tol, maxit, pc, pc_ctx, &it, &rel);
    res->n_solves++;
    res->cg_iters_total += it;
    if (it > res->cg_iters_max) res->cg_iters_max = it;
    if (rel > res->max_true_resid) res->max_true_resid = rel;
    if (st) res->status = st;
}

void oracle_hmc_trajectory_pc(const oracle_lat *p, double *theta, uint64_t seed,
                              uint64_t traj, int32_t n_steps, double traj_len,
                              double tol, int32_t maxit, oracle_precond_fn pc,
                              void *pc_ctx, oracle_traj *res, double *mom_out,
                              cplx *R_out, cplx *eta_out)
{
    const size_t N = (size_t)p->L * p->L * p->Nt, nb = 2 * N;
    const double dt = traj_len / n_steps;
    double *th0 = malloc(sizeof(double) * nb), *mom = malloc(sizeof(double) * nb);
    double *F = malloc(sizeof(double) * nb), *Fb = malloc(sizeof(double) * nb);
    cplx *R = malloc(sizeof(cplx) * N), *eta = malloc(sizeof(cplx) * N);
    cplx *X = malloc(sizeof(cplx) * N);
    memset(res, 0, sizeof(*res));
    memcpy(th0, theta, sizeof(double) * nb);

    /* (i) heat bath and eta = M^dag R */
    oracle_heatbath(p, seed, traj, mom, R);
    if (mom_out) memcpy(mom_out, mom, sizeof(double) * nb);
    if (R_out) memcpy(R_out, R, sizeof(cplx) * N);
    oracle_apply_M(p, theta, R, eta, 1);
    if (eta_out) memcpy(eta_out, eta, sizeof(cplx) * N);

    /* H at the start */
    solve_track(p, theta, eta, X, tol, maxit, pc, pc_ctx, res);
    res->SF0 = dot_re(eta, X, N);
    res->SB0 = oracle_bosonic_action(p, theta);
    res->K0 = 0.0;
    for (size_t b = 0; b < nb; b++) res->K0 += mom[b] * mom[b];
    res->H0 = res->SB0 + res->K0 + res->SF0;

    /* (ii) leapfrog, Eq. leapfrog: dtheta/dt = 2p, dp/dt = F */
    total_force(p, theta, X, F, Fb, nb);
    for (int n = 0; n < n_steps; n++) {
        for (size_t b = 0; b < nb; b++) mom[b] += 0.5 * dt * F[b];
        for (size_t b = 0; b < nb; b++) theta[b] += 2.0 * dt * mom[b];
        solve_track(p, theta, eta, X, tol, maxit, pc, pc_ctx, res);
        total_force(p, theta, X, F, Fb, nb);
        for (size_t b = 0; b < nb; b++) mom[b] += 0.5 * dt * F[b];
    }

    /* H at the end */
    res->SF1 = dot_re(eta, X, N);
    res->SB1 = oracle_bosonic_action(p, theta);
    res->K1 = 0.0;
    for (size_t b = 0; b < nb; b++) res->K1 += mom[b] * mom[b];
    res->H1 = res->SB1 + res->K1 + res->SF1;
    res->dH = res->H1 - res->H0;

    /* (iii) Metropolis: accept with probability min(1, exp(-dH)) */
    res->u = oracle_metropolis_uniform(seed, traj);
    res->accepted = (res->dH <= 0.0 || res->u < exp(-res->dH)) ? 1 : 0;
    if (!res->accepted) memcpy(theta, th0, sizeof(double) * nb);

    free(th0); free(mom); free(F); free(Fb); free(R); free(eta); free(X);
}

void oracle_hmc_trajectory(const oracle_lat *p, double *theta, uint64_t seed,
                           uint64_t traj, int32_t n_steps, double traj_len,
                           double tol, int32_t maxit, oracle_traj *res,
                           double *mom_out, cplx *R_out, cplx *eta_out)
{
    oracle_hmc_trajectory_pc(p, theta, seed, traj, n_steps, traj_len, tol, maxit,
                             NULL, NULL, res, mom_out, R_out, eta_out);
}

/* Leapfrog from given (theta, mom, eta) with dense-free CG solves; returns
 * H before and after without any Metropolis step (used by the dt^2 and
 * reversibility checks).  theta and mom are updated in place. */
void oracle_leapfrog(const oracle_lat *p, double *theta, double *mom,
                     const cplx *eta, int32_t n_steps, double traj_len,
                     double tol, int32_t maxit, double *H_before,
                     double *H_after)
{
    const size_t N = (size_t)p->L * p->L * p->Nt, nb = 2 * N;
    const double dt = traj_len / n_steps;
    double *F = malloc(sizeof(double) * nb), *Fb = malloc(sizeof(double) * nb);
    cplx *X = malloc(sizeof(cplx) * N);
    oracle_traj res;
    memset(&res, 0, sizeof(res));
    double K = 0.0;

    solve_track(p, theta, eta, X, tol, maxit, NULL, NULL, &res);
    for (size_t b = 0; b < nb; b++) K += mom[b] * mom[b];
    *H_before = oracle_bosonic_action(p, theta) + K + dot_re(eta, X, N);
    total_force(p, theta, X, F, Fb, nb);
    for (int n = 0; n < n_steps; n++) {
        for (size_t b = 0; b < nb; b++) mom[b] += 0.5 * dt * F[b];
        for (size_t b = 0; b < nb; b++) theta[b] += 2.0 * dt * mom[b];
        solve_track(p, theta, eta, X, tol, maxit, NULL, NULL, &res);
        total_force(p, theta, X, F, Fb, nb);
        for (size_t b = 0; b < nb; b++) mom[b] += 0.5 * dt * F[b];
    }
    K = 0.0;
    for (size_t b = 0; b < nb; b++) K += mom[b] * mom[b];
    *H_after = oracle_bosonic_action(p, theta) + K + dot_re(eta, X, N);
    free(F); free(Fb); free(X);
}
