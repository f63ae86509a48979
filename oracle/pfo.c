/*
 * pfo.c -- plain FP64 CPU reference solver ("the oracle").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the HIP library, and the HIP library never
 * calls it.
 *
 * What it computes: one time step of the ternary phase-field lattice
 * Boltzmann method of Ghorbanpour Arani et al. (arXiv 2207.09431), Sec. 2:
 *   - Cahn-Hilliard populations hbar^i (i = 1..n_h) with constant or
 *     variable mobility (Sec. 2.1, Eqs. (5)-(7); Sec. 2.2, Eqs. (18)-(21)),
 *   - pressure/momentum populations gbar (Sec. 2.2, Eqs. (12)-(16)),
 *   - moments (Eqs. (22)-(24)),
 *   - a per-cell relaxation time from the truncated power law whose strain
 *     rate comes from the non-equilibrium second moment of gbar, evaluated
 *     with the previous step's tau (Sec. 2.3, Eqs. (25)-(33)),
 *   - streaming, periodic in x, half-way bounce-back walls in y.
 * Everything is stored literally (gbar and every hbar population) and the
 * step runs as separate plain loops in the order of the method.  Built with
 * -O2 -ffp-contract=off and no fast-math.
 *
 * Readings where the paper is silent or garbled (the same list is kept with
 * the design notes):
 *   R1  pressure moment: p = sum gbar + (1/2) c_s^2 u.grad(rho)  (the factor
 *       1/2 is required for sum gbar_eq to equal sum gbar; Eq. (24) prints
 *       it without the 1/2).
 *   R2  g_eq = w p + rho c_s^2 (Gamma - w), from Eqs. (9) and (13).
 *   R3  rho = sum_k rho_k C_k with each C_k limited to [0, 1]: inside a
 *       curved interface the bulk C of the dispersed phase settles slightly
 *       above 1, and the unlimited sum turns negative at density ratio 1000.
 *   R4  mixture viscosity from the harmonic rule 1/nu = sum_k C_k / nu_k (each
 *       C_k limited to [0, 1]), clamped to [min nu_k, max nu_k].  The two-layer
 *       flow of Sec. 3.3 (Table 3) discriminates: across a diffuse interface
 *       of two layers in series the stress is continuous and the shear rates
 *       add, and the linear rule sum_k C_k nu_k misses the layered closed form
 *       by 2-8 times the printed errors.  Switch mix_linear=1 takes the
 *       linear rule.
 *   R5  the power law gives a kinematic viscosity nu_P = K gdot^(n-1).
 *   R6  strain rate D = -Pi/(2 (tau+1/2) rho c_s^4) with Pi the second moment
 *       of gbar - gbar_eq (Chapman-Enskog form for the transformed
 *       populations).  Switch strain_literal=1 multiplies Pi by
 *       2tau/(2tau+1) in addition (Eq. (29) fed into Eq. (25) literally).
 *   R7  tau in the strain rate is the cell's tau of the previous step; the
 *       initial tau is the one at zero shear.  tau_iterations = m > 0 adds m
 *       fixed-point passes of the implicit relation (Eq. (32)) from there.
 *   R8  truncation is a clamp of nu_P to [nu_min, nu_max]; gdot = 0 is taken
 *       explicitly (nu_max if n<1, nu_min if n>1).
 *   R9  stencils: isotropic central differences (CD) for every gradient and
 *       Laplacian, for mu, the moments and both equilibria; the explicit
 *       forcing terms of the collisions take every (e_a - u).grad phi of rho
 *       and C_k as a mixed directional derivative (MD), in the gbar forcing
 *       and for grad C_i in the hbar forcing alike.  With MD in the gbar
 *       forcing but CD in the hbar forcing the scheme diverges within 50 steps
 *       at density ratio 1000 even for a flat interface.  Switches:
 *       gforce_cd=1 (CD in the gbar forcing), hforce_mode=1 (CD in the hbar
 *       forcing), hforce_mode=2 (MD also for grad p and the force in the
 *       hbar forcing), force_potential=1 (force written -sum_k C_k grad mu_k).
 *   R11 sum_i mu_i grad C_i in the forcing runs over all three components.
 *   R12 the second half of the diffusion source (Eq. (18), terms at x+e) is
 *       added at the receiving node with time-t fields there; a population
 *       bounced at a wall is received by its own source node.
 *   R13 variable-mobility divergence uses the product form of Eq. (21),
 *       with the CD gradient of the field C_i - C_i^2 for grad C_i - grad C_i^2;
 *       inside the mobility C_i is limited to [0, 1] so that D_i >= 0.  Switch mobility_flux=1 uses the
 *       conservative link form sum_a w_a (M(x)+M(x+e_a)) (mu(x+e_a)-mu(x))/c_s^2.
 *   R14 wall ghosts for stencils mirror the first rows (zero normal
 *       derivative) for C, mu and p; x is periodic.
 *   R15 half-way bounce-back, walls at rest at y = -1/2 and y = ny - 1/2.
 *   R16 body force F_b = rho (fx, -g); fx = 0 reproduces Eq. (12).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "pfo.h"

/* Per-node loops are split over rows with OpenMP when the library is built
 * with it, for domains of 2048 nodes or more (smaller ones run on the calling
 * thread: starting a parallel region costs more than such a loop).  Each
 * node is computed by one thread with the same operations, so the results do
 * not depend on the thread count.  (Testing only: speed.)  OMP_FOR is used
 * only where the context `c` is in scope. */
#ifdef _OPENMP
#include <omp.h>
#define OMP_FOR _Pragma("omp parallel for schedule(static) if(c->n >= 2048)")
#else
#define OMP_FOR
#endif

void pfo_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int pfo_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* D2Q9 lattice, Sec. 2.2 Eqs. (10)-(11): alpha = 0 rest, 1-4 axes, 5-8 diagonals. */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double CS2 = 1.0 / 3.0;

struct pfo_ctx {
    pfo_params p;
    int nx, ny, n;           /* n = nx*ny */
    double *g;               /* [9][n] gbar */
    double *h;               /* [n_h][9][n] hbar */
    double *tau;             /* [n] tau of the previous step */
    /* work fields, recomputed every step */
    double *C;               /* [3][n] */
    double *rho;             /* [n] */
    double *gradC;           /* [3][2][n] */
    double *lapC;            /* [3][n] */
    double *gradM;           /* [3][2][n]  CD gradient of C_i - C_i^2 (C_i limited to [0,1]) */
    double *mu;              /* [3][n] */
    double *gradmu;          /* [3][2][n] */
    double *lapmu;           /* [3][n] */
    double *dif;             /* [2][n]  divergence of D_i grad mu_i */
    double *gradrho;         /* [2][n] */
    double *Fs;              /* [2][n]  sum mu grad C + F_b */
    double *u;               /* [2][n] */
    double *pr;              /* [n] pressure p */
    double *gradp;           /* [2][n] */
    double *tmp;             /* [n] */
    double *gpost;           /* [9][n] */
    double *hpost;           /* [n_h][9][n] */
    double *taunew;          /* [n] */
    double *gold;            /* [9][n] gbar before streaming (open x only) */
};

/* ---------------------------------------------------------------- indexing */
static inline int wrapx(int x, int nx) {
    while (x < 0) x += nx;
    while (x >= nx) x -= nx;
    return x;
}
/* mirror about the walls at y=-1/2 and y=ny-1/2 (R14) */
static inline int mirrory(int y, int ny) {
    while (y < 0 || y >= ny) {
        if (y < 0) y = -y - 1;
        if (y >= ny) y = 2 * ny - 1 - y;
    }
    return y;
}
/* x is periodic, or with open x (velocity inlet at x = 0, outflow at
 * x = nx-1) mirrored about x = -1/2 and x = nx - 1/2 like the walls */
static inline double at(const double *f, int x, int y, int nx, int ny, int ox) {
    return f[mirrory(y, ny) * nx + (ox ? mirrory(x, nx) : wrapx(x, nx))];
}
#define OX (c->p.open_x)

/* ------------------------------------------------------------- stencils (R9)
 * Isotropic central gradient: grad phi = sum_a w_a e_a [phi(x+e_a)-phi(x-e_a)] / (2 c_s^2).
 * Isotropic Laplacian:        lap phi  = sum_a w_a [phi(x+e_a) - 2 phi(x) + phi(x-e_a)] / c_s^2.
 * Mixed directional derivative along e_a (mean of the central and the
 * second-order biased forms):
 *   d_a phi = [-phi(x+2e) + 5 phi(x+e) - 3 phi(x) - phi(x-e)] / 4.
 * Mixed gradient: grad^MD phi = sum_a w_a e_a d_a phi / c_s^2.
 */
static void grad_cd_at(const double *f, int x, int y, int nx, int ny, int ox, double *gx, double *gy) {
    double sx = 0.0, sy = 0.0;
    for (int a = 1; a < 9; ++a) {
        double d = at(f, x + EX[a], y + EY[a], nx, ny, ox) - at(f, x - EX[a], y - EY[a], nx, ny, ox);
        sx += W[a] * EX[a] * d;
        sy += W[a] * EY[a] * d;
    }
    *gx = sx / (2.0 * CS2);
    *gy = sy / (2.0 * CS2);
}
static double lap_cd_at(const double *f, int x, int y, int nx, int ny, int ox) {
    double c = at(f, x, y, nx, ny, ox), s = 0.0;
    for (int a = 1; a < 9; ++a)
        s += W[a] * (at(f, x + EX[a], y + EY[a], nx, ny, ox) - 2.0 * c + at(f, x - EX[a], y - EY[a], nx, ny, ox));
    return s / CS2;
}
static double dir_md_at(const double *f, int x, int y, int a, int nx, int ny, int ox) {
    return (-at(f, x + 2 * EX[a], y + 2 * EY[a], nx, ny, ox) + 5.0 * at(f, x + EX[a], y + EY[a], nx, ny, ox)
            - 3.0 * at(f, x, y, nx, ny, ox) - at(f, x - EX[a], y - EY[a], nx, ny, ox)) / 4.0;
}
static double dir_cd_at(const double *f, int x, int y, int a, int nx, int ny, int ox) {
    return (at(f, x + EX[a], y + EY[a], nx, ny, ox) - at(f, x - EX[a], y - EY[a], nx, ny, ox)) / 2.0;
}
static void grad_md_at(const double *f, int x, int y, int nx, int ny, int ox, double *gx, double *gy) {
    double sx = 0.0, sy = 0.0;
    for (int a = 1; a < 9; ++a) {
        double d = dir_md_at(f, x, y, a, nx, ny, ox);
        sx += W[a] * EX[a] * d;
        sy += W[a] * EY[a] * d;
    }
    *gx = sx / CS2;
    *gy = sy / CS2;
}

/* -------------------------------------------------------- thermodynamics
 * Capillary coefficients Sigma_i = s_ij + s_ik - s_jk and 3/Sigma_T =
 * sum 1/Sigma_i (Sec. 2.1, below Eq. (2) and Eq. (7)).
 */
static void capillary(const pfo_params *p, double S[3], double *ST) {
    S[0] = p->sigma12 + p->sigma13 - p->sigma23;
    S[1] = p->sigma12 + p->sigma23 - p->sigma13;
    S[2] = p->sigma13 + p->sigma23 - p->sigma12;
    *ST = 3.0 / (1.0 / S[0] + 1.0 / S[1] + 1.0 / S[2]);
}

/* Bulk free energy E0 (Sec. 2.1, Eq. (3)). */
static double bulk_E0(const pfo_params *p, const double S[3], double c1, double c2, double c3) {
    return p->sigma12 * c1 * c1 * c2 * c2 + p->sigma13 * c1 * c1 * c3 * c3
         + p->sigma23 * c2 * c2 * c3 * c3
         + c1 * c2 * c3 * (S[0] * c1 + S[1] * c2 + S[2] * c3)
         + p->Lambda * c1 * c1 * c2 * c2 * c3 * c3;
}

/* Partial derivatives of E0 with C1, C2, C3 treated as independent. */
static void bulk_dE0(const pfo_params *p, const double S[3], double c1, double c2, double c3, double d[3]) {
    double sc = S[0] * c1 + S[1] * c2 + S[2] * c3;
    d[0] = 2.0 * p->sigma12 * c1 * c2 * c2 + 2.0 * p->sigma13 * c1 * c3 * c3
         + c2 * c3 * sc + c1 * c2 * c3 * S[0] + 2.0 * p->Lambda * c1 * c2 * c2 * c3 * c3;
    d[1] = 2.0 * p->sigma12 * c1 * c1 * c2 + 2.0 * p->sigma23 * c2 * c3 * c3
         + c1 * c3 * sc + c1 * c2 * c3 * S[1] + 2.0 * p->Lambda * c1 * c1 * c2 * c3 * c3;
    d[2] = 2.0 * p->sigma13 * c1 * c1 * c3 + 2.0 * p->sigma23 * c2 * c2 * c3
         + c1 * c2 * sc + c1 * c2 * c3 * S[2] + 2.0 * p->Lambda * c1 * c1 * c2 * c2 * c3;
}

/* Chemical potentials (Sec. 2.1, Eq. (5)):
 * mu_i = (4 Sigma_T / xi) sum_{j != i} (dE0/dC_i - dE0/dC_j) / Sigma_j - (3/4) xi Sigma_i lap C_i. */
static void chem_potential(const pfo_params *p, const double c[3], const double lap[3], double mu[3]) {
    double S[3], ST, d[3];
    capillary(p, S, &ST);
    bulk_dE0(p, S, c[0], c[1], c[2], d);
    for (int i = 0; i < 3; ++i) {
        double s = 0.0;
        for (int j = 0; j < 3; ++j)
            if (j != i) s += (d[i] - d[j]) / S[j];
        mu[i] = 4.0 * ST / p->xi * s - 0.75 * p->xi * S[i] * lap[i];
    }
}

/* A concentration limited to its physical range [0, 1] (R3, R13). */
static double clip01(double c) { return c < 0.0 ? 0.0 : (c > 1.0 ? 1.0 : c); }

/* Mixture density rho = sum_k rho_k C_k with each C_k limited to [0, 1] (R3). */
static double mixture_density(const pfo_params *p, double c1, double c2, double c3) {
    return p->rho[0] * clip01(c1) + p->rho[1] * clip01(c2) + p->rho[2] * clip01(c3);
}

/* Mobility D_i (Sec. 2.1, Eq. (6)) with C_i limited to [0, 1] (R13); D0 is
 * the auxiliary scale. */
static double mobility_shape(double ci) {
    double c = clip01(ci);
    return c * (1.0 - c);
}
static double mobility(const pfo_params *p, const double S[3], int i, double ci) {
    double m = p->D0 / S[i];
    return p->variable_mobility ? m * mobility_shape(ci) : m;
}

/* -------------------------------------------------------------- rheology
 * Truncated power law (Sec. 2.3, Eqs. (31), (33), reading R8), kinematic (R5). */
static double powerlaw_nu(const pfo_params *p, double gdot) {
    double nu;
    if (gdot <= 0.0) {
        if (p->n < 1.0) return p->nu_max;
        if (p->n > 1.0) return p->nu_min;
        nu = p->K;
    } else {
        nu = p->K * pow(gdot, p->n - 1.0);
    }
    if (nu < p->nu_min) nu = p->nu_min;
    if (nu > p->nu_max) nu = p->nu_max;
    return nu;
}

/* Mixture relaxation time tau = nu / c_s^2 (Sec. 2.2 below Eq. (14); R4). */
static double mixture_tau(const pfo_params *p, const double c[3], double gdot) {
    double nuk[3];
    for (int k = 0; k < 3; ++k) nuk[k] = (k == p->powerlaw_comp) ? powerlaw_nu(p, gdot) : p->nu[k];
    double nu;
    if (p->mix_linear) {
        nu = c[0] * nuk[0] + c[1] * nuk[1] + c[2] * nuk[2];
    } else {
        double q = 0.0;
        for (int k = 0; k < 3; ++k) q += clip01(c[k]) / nuk[k];
        nu = 1.0 / q;   /* q > 0: the limited C_k sum to at least 1/3 */
    }
    double lo = nuk[0], hi = nuk[0];
    for (int k = 1; k < 3; ++k) { if (nuk[k] < lo) lo = nuk[k]; if (nuk[k] > hi) hi = nuk[k]; }
    if (nu < lo) nu = lo;
    if (nu > hi) nu = hi;
    return nu / CS2;
}

/* Shear rate from the non-equilibrium second moment (Sec. 2.3, Eqs. (25)-(29), R6):
 * D = -Pi / (2 (tau+1/2) rho c_s^4), gdot = sqrt(2 D:D). */
static double shear_rate(const pfo_params *p, const double Pi[3] /* xx, yy, xy */, double tau, double rho) {
    double f = -1.0 / (2.0 * (tau + 0.5) * rho * CS2 * CS2);
    if (p->strain_literal) f *= 2.0 * tau / (2.0 * tau + 1.0);
    double dxx = f * Pi[0], dyy = f * Pi[1], dxy = f * Pi[2];
    return sqrt(2.0 * (dxx * dxx + dyy * dyy + 2.0 * dxy * dxy));
}

/* Gamma_a(u) = f_eq / rho (Sec. 2.2, Eq. (9)). */
static double Gamma(int a, double ux, double uy) {
    double eu = EX[a] * ux + EY[a] * uy;
    return W[a] * (1.0 + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - (ux * ux + uy * uy) / (2.0 * CS2));
}

/* ------------------------------------------------------------ allocation */
static void *zalloc(size_t n) { void *q = calloc(n ? n : 1, sizeof(double)); return q; }

int pfo_create(const pfo_params *prm, pfo_ctx **out) {
    if (!prm || !out) return -1;
    if (prm->nx < 5 || prm->ny < 5 || (prm->n_h != 1 && prm->n_h != 2)) return -1;
    if (prm->open_x != 0 && prm->open_x != 1) return -1;
    for (int k = 0; k < 3; ++k) if (!(prm->rho[k] > 0.0)) return -1;
    pfo_ctx *c = (pfo_ctx *)calloc(1, sizeof(pfo_ctx));
    if (!c) return -3;
    c->p = *prm;
    c->nx = prm->nx; c->ny = prm->ny; c->n = prm->nx * prm->ny;
    size_t n = (size_t)c->n, nh = (size_t)prm->n_h;
    c->g = zalloc(9 * n); c->h = zalloc(nh * 9 * n); c->tau = zalloc(n);
    c->C = zalloc(3 * n); c->rho = zalloc(n); c->gradC = zalloc(6 * n); c->lapC = zalloc(3 * n);
    c->gradM = zalloc(6 * n); c->mu = zalloc(3 * n); c->gradmu = zalloc(6 * n); c->lapmu = zalloc(3 * n);
    c->dif = zalloc(2 * n); c->gradrho = zalloc(2 * n); c->Fs = zalloc(2 * n); c->u = zalloc(2 * n);
    c->pr = zalloc(n); c->gradp = zalloc(2 * n); c->tmp = zalloc(n);
    c->gpost = zalloc(9 * n); c->hpost = zalloc(nh * 9 * n); c->taunew = zalloc(n);
    c->gold = prm->open_x ? zalloc(9 * n) : NULL;
    if (!c->g || !c->h || !c->tau || !c->C || !c->rho || !c->gradC || !c->lapC || !c->gradM || !c->mu ||
        !c->gradmu || !c->lapmu || !c->dif || !c->gradrho || !c->Fs || !c->u || !c->pr || !c->gradp ||
        !c->tmp || !c->gpost || !c->hpost || !c->taunew || (prm->open_x && !c->gold)) {
        pfo_destroy(c);
        return -3;
    }
    *out = c;
    return 0;
}

void pfo_destroy(pfo_ctx *c) {
    if (!c) return;
    free(c->g); free(c->h); free(c->tau); free(c->C); free(c->rho); free(c->gradC); free(c->lapC);
    free(c->gradM); free(c->mu); free(c->gradmu); free(c->lapmu); free(c->dif); free(c->gradrho);
    free(c->Fs); free(c->u); free(c->pr); free(c->gradp); free(c->tmp); free(c->gpost); free(c->hpost);
    free(c->taunew); free(c->gold);
    free(c);
}

/* ------------------------------------------------- per-step field stages */

/* Stage 1: phase moments C_i = sum_a hbar^i_a (Eq. (22)), C_3 = 1 - C_1 - C_2
 * (Eq. (1)), C_2 = 0 when only one phase field is carried, rho (R3). */
static void stage_phase(pfo_ctx *c) {
    int n = c->n, nh = c->p.n_h;
    OMP_FOR
    for (int q = 0; q < n; ++q) {
        double ci[2] = {0.0, 0.0};
        for (int i = 0; i < nh; ++i) {
            double s = 0.0;
            for (int a = 0; a < 9; ++a) s += c->h[((size_t)i * 9 + a) * n + q];
            ci[i] = s;
        }
        c->C[0 * n + q] = ci[0];
        c->C[1 * n + q] = ci[1];
        c->C[2 * n + q] = 1.0 - ci[0] - ci[1];
        c->rho[q] = mixture_density(&c->p, ci[0], ci[1], c->C[2 * n + q]);
    }
}

/* Stage 2: CD stencils of C_i, of C_i - C_i^2 and of rho; Stage 3: mu_i. */
static void stage_chem(pfo_ctx *c) {
    int nx = c->nx, ny = c->ny, n = c->n;
    for (int k = 0; k < 3; ++k) {
        const double *f = c->C + (size_t)k * n;
        OMP_FOR
        for (int q = 0; q < n; ++q) c->tmp[q] = mobility_shape(f[q]);
        OMP_FOR
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int q = y * nx + x;
                grad_cd_at(f, x, y, nx, ny, OX, &c->gradC[(2 * k) * n + q], &c->gradC[(2 * k + 1) * n + q]);
                c->lapC[k * n + q] = lap_cd_at(f, x, y, nx, ny, OX);
                grad_cd_at(c->tmp, x, y, nx, ny, OX, &c->gradM[(2 * k) * n + q], &c->gradM[(2 * k + 1) * n + q]);
            }
    }
    OMP_FOR
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int q = y * nx + x;
            grad_cd_at(c->rho, x, y, nx, ny, OX, &c->gradrho[q], &c->gradrho[n + q]);
            double ck[3] = {c->C[q], c->C[n + q], c->C[2 * n + q]};
            double lk[3] = {c->lapC[q], c->lapC[n + q], c->lapC[2 * n + q]};
            double m[3];
            chem_potential(&c->p, ck, lk, m);
            for (int k = 0; k < 3; ++k) c->mu[k * n + q] = m[k];
        }
}

/* Stage 4-5: CD stencils of mu_i (ghost mu mirrors the wall rows, R14) and the
 * diffusion source Dif_i = div(D_i grad mu_i) (Eq. (21), R13). */
static void stage_diffusion(pfo_ctx *c) {
    int nx = c->nx, ny = c->ny, n = c->n;
    double S[3], ST;
    capillary(&c->p, S, &ST);
    for (int k = 0; k < 3; ++k) {
        const double *f = c->mu + (size_t)k * n;
        OMP_FOR
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int q = y * nx + x;
                grad_cd_at(f, x, y, nx, ny, OX, &c->gradmu[(2 * k) * n + q], &c->gradmu[(2 * k + 1) * n + q]);
                c->lapmu[k * n + q] = lap_cd_at(f, x, y, nx, ny, OX);
            }
    }
    for (int i = 0; i < c->p.n_h; ++i) {
        const double *ci = c->C + (size_t)i * n, *mi = c->mu + (size_t)i * n;
        OMP_FOR
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int q = y * nx + x;
                double v;
                if (c->p.mobility_flux) {
                    /* conservative link form of div(M grad mu) */
                    double s = 0.0, m0 = mobility(&c->p, S, i, ci[q]);
                    for (int a = 1; a < 9; ++a) {
                        double m1 = mobility(&c->p, S, i, at(ci, x + EX[a], y + EY[a], nx, ny, OX));
                        s += W[a] * (m0 + m1) * (at(mi, x + EX[a], y + EY[a], nx, ny, OX) - mi[q]);
                    }
                    v = s / CS2;
                } else {
                    v = mobility(&c->p, S, i, ci[q]) * c->lapmu[i * n + q];
                    if (c->p.variable_mobility) {
                        double ax = c->gradM[(2 * i) * n + q];
                        double ay = c->gradM[(2 * i + 1) * n + q];
                        v += c->p.D0 / S[i] * (ax * c->gradmu[(2 * i) * n + q] + ay * c->gradmu[(2 * i + 1) * n + q]);
                    }
                }
                c->dif[i * n + q] = v;
            }
    }
}

/* Surface-tension force sum_k mu_k grad C_k (Eq. (12)); with force_potential
 * the equivalent potential form -sum_k C_k grad mu_k. */
static void surface_force(const pfo_ctx *c, int q, double *fx, double *fy) {
    int n = c->n;
    double sx = 0.0, sy = 0.0;
    for (int k = 0; k < 3; ++k) {
        if (c->p.force_potential) {
            sx -= c->C[k * n + q] * c->gradmu[(2 * k) * n + q];
            sy -= c->C[k * n + q] * c->gradmu[(2 * k + 1) * n + q];
        } else {
            sx += c->mu[k * n + q] * c->gradC[(2 * k) * n + q];
            sy += c->mu[k * n + q] * c->gradC[(2 * k + 1) * n + q];
        }
    }
    *fx = sx;
    *fy = sy;
}

/* Stage 6: force, velocity and pressure moments (Eqs. (12), (23), (24), R1),
 * then the CD gradient of p (ghost p mirrors the wall rows). */
static void stage_hydro(pfo_ctx *c) {
    int nx = c->nx, ny = c->ny, n = c->n;
    OMP_FOR
    for (int q = 0; q < n; ++q) {
        double fx, fy;
        surface_force(c, q, &fx, &fy);
        fx += c->rho[q] * c->p.fx;
        fy -= c->rho[q] * c->p.g;
        c->Fs[q] = fx;
        c->Fs[n + q] = fy;
        double s = 0.0, jx = 0.0, jy = 0.0;
        for (int a = 0; a < 9; ++a) {
            double ga = c->g[(size_t)a * n + q];
            s += ga;
            jx += EX[a] * ga;
            jy += EY[a] * ga;
        }
        double ux = (jx / CS2 + 0.5 * fx) / c->rho[q];
        double uy = (jy / CS2 + 0.5 * fy) / c->rho[q];
        c->u[q] = ux;
        c->u[n + q] = uy;
        c->pr[q] = s + 0.5 * CS2 * (ux * c->gradrho[q] + uy * c->gradrho[n + q]);
    }
    OMP_FOR
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int q = y * nx + x;
            grad_cd_at(c->pr, x, y, nx, ny, OX, &c->gradp[q], &c->gradp[n + q]);
        }
}

/* Equilibria at node q for direction a (Eqs. (13), (16), (20), R2). */
typedef struct {
    double ux, uy, rho, p, grx, gry, Fx, Fy;
} node_macro;

static double gbar_eq(const node_macro *m, int a) {
    double G = Gamma(a, m->ux, m->uy);
    double geq = W[a] * m->p + m->rho * CS2 * (G - W[a]);
    double ex = EX[a] - m->ux, ey = EY[a] - m->uy;
    double fcd = CS2 * (ex * m->grx + ey * m->gry) * (G - W[a]) + (ex * m->Fx + ey * m->Fy) * G;
    return geq - 0.5 * fcd;
}

/* Stage 7-11 at every node: rheology and collisions. */
static void stage_collide(pfo_ctx *c) {
    int nx = c->nx, ny = c->ny, n = c->n, nh = c->p.n_h;
    const pfo_params *P = &c->p;
    OMP_FOR
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int q = y * nx + x;
            node_macro m = {c->u[q], c->u[n + q], c->rho[q], c->pr[q], c->gradrho[q], c->gradrho[n + q],
                            c->Fs[q], c->Fs[n + q]};
            double geq[9], G[9];
            for (int a = 0; a < 9; ++a) { geq[a] = gbar_eq(&m, a); G[a] = Gamma(a, m.ux, m.uy); }

            /* rheology: second moment of gbar - gbar_eq, previous tau (R6-R8) */
            double Pi[3] = {0.0, 0.0, 0.0};
            for (int a = 0; a < 9; ++a) {
                double ne = c->g[(size_t)a * n + q] - geq[a];
                Pi[0] += ne * EX[a] * EX[a];
                Pi[1] += ne * EY[a] * EY[a];
                Pi[2] += ne * EX[a] * EY[a];
            }
            double gdot = shear_rate(P, Pi, c->tau[q], m.rho);
            double ck[3] = {c->C[q], c->C[n + q], c->C[2 * n + q]};
            double tau = mixture_tau(P, ck, gdot);
            /* optional fixed-point passes of the implicit relation tau =
             * tau(gdot(tau)) of Eq. (32), from the previous step's tau */
            for (int it = 0; it < P->tau_iterations; ++it) tau = mixture_tau(P, ck, shear_rate(P, Pi, tau, m.rho));
            c->taunew[q] = tau;

            /* directional derivatives along every e_a and the matching gradients
             * of rho and C_k: mixed differences by default, central ones with
             * gforce_cd (R9) */
            double drho[9], dC[9][3], gmdx, gmdy, gcx[3], gcy[3];
            if (P->gforce_cd) {
                gmdx = m.grx; gmdy = m.gry;
                for (int k = 0; k < 3; ++k) { gcx[k] = c->gradC[(2 * k) * n + q]; gcy[k] = c->gradC[(2 * k + 1) * n + q]; }
                for (int a = 0; a < 9; ++a) {
                    drho[a] = EX[a] * gmdx + EY[a] * gmdy;
                    for (int k = 0; k < 3; ++k) dC[a][k] = EX[a] * gcx[k] + EY[a] * gcy[k];
                }
            } else {
                grad_md_at(c->rho, x, y, nx, ny, OX, &gmdx, &gmdy);
                for (int k = 0; k < 3; ++k) grad_md_at(c->C + (size_t)k * n, x, y, nx, ny, OX, &gcx[k], &gcy[k]);
                for (int a = 0; a < 9; ++a) {
                    drho[a] = dir_md_at(c->rho, x, y, a, nx, ny, OX);
                    for (int k = 0; k < 3; ++k) dC[a][k] = dir_md_at(c->C + (size_t)k * n, x, y, a, nx, ny, OX);
                }
            }

            /* gbar collision with the explicit forcing (Eq. (14)):
             * F_a = c_s^2 [(e-u).grad rho] (Gamma_a - w_a) + [(e-u).(sum mu grad C + F_b)] Gamma_a */
            double mu[3] = {c->mu[q], c->mu[n + q], c->mu[2 * n + q]};
            double fbx = m.rho * P->fx, fby = -m.rho * P->g;
            double omega = 1.0 / (tau + 0.5);
            double Fdir[9];   /* (e_a - u).(sum mu grad C + F_b) with directional derivatives */
            for (int a = 0; a < 9; ++a) {
                double t1 = CS2 * (drho[a] - (m.ux * gmdx + m.uy * gmdy)) * (G[a] - W[a]);
                double t2 = 0.0;
                if (P->force_potential) {
                    for (int k = 0; k < 3; ++k) {
                        double dm, gmx, gmy;
                        if (P->gforce_cd) {
                            gmx = c->gradmu[(2 * k) * n + q]; gmy = c->gradmu[(2 * k + 1) * n + q];
                            dm = EX[a] * gmx + EY[a] * gmy;
                        } else {
                            dm = dir_md_at(c->mu + (size_t)k * n, x, y, a, nx, ny, OX);
                            grad_md_at(c->mu + (size_t)k * n, x, y, nx, ny, OX, &gmx, &gmy);
                        }
                        t2 -= ck[k] * (dm - (m.ux * gmx + m.uy * gmy));
                    }
                } else {
                    for (int k = 0; k < 3; ++k) t2 += mu[k] * (dC[a][k] - (m.ux * gcx[k] + m.uy * gcy[k]));
                }
                t2 += (EX[a] - m.ux) * fbx + (EY[a] - m.uy) * fby;
                Fdir[a] = t2;
                double F = t1 + t2 * G[a];
                double ga = c->g[(size_t)a * n + q];
                c->gpost[(size_t)a * n + q] = ga - omega * (ga - geq[a]) + F;
            }

            /* hbar collision (Eqs. (18)-(20)) with the source-side half of the
             * diffusion term.  Forcing (e-u).X_i Gamma_a with
             * X_i = grad C_i - C_i/(rho c_s^2) (grad p - sum mu grad C - F_b);
             * the equilibrium uses central differences, the explicit forcing
             * takes (e-u).grad C_i as a mixed directional derivative like the
             * gbar forcing (hforce_mode 0, R9), central differences throughout
             * (hforce_mode 1), or mixed derivatives for grad p and the force
             * too (hforce_mode 2). */
            double omh = 1.0 / (P->tau_h + 0.5);
            double bx = c->gradp[q] - m.Fx, by = c->gradp[n + q] - m.Fy; /* grad p - sum mu grad C - F_b */
            double dp[9], gpx = 0.0, gpy = 0.0;
            if (P->hforce_mode == 2) {
                grad_md_at(c->pr, x, y, nx, ny, OX, &gpx, &gpy);
                for (int a = 0; a < 9; ++a) dp[a] = dir_md_at(c->pr, x, y, a, nx, ny, OX);
            }
            for (int i = 0; i < nh; ++i) {
                double cc = ck[i];
                double Xx = c->gradC[(2 * i) * n + q] - cc / (m.rho * CS2) * bx;
                double Xy = c->gradC[(2 * i + 1) * n + q] - cc / (m.rho * CS2) * by;
                double difi = c->dif[i * n + q];
                for (int a = 0; a < 9; ++a) {
                    double ex = EX[a] - m.ux, ey = EY[a] - m.uy;
                    double fX;    /* (e_a - u).X_i */
                    if (P->hforce_mode == 1) {
                        fX = ex * Xx + ey * Xy;
                    } else if (P->hforce_mode == 2) {
                        fX = (dC[a][i] - (m.ux * gcx[i] + m.uy * gcy[i]))
                           - cc / (m.rho * CS2) * ((dp[a] - (m.ux * gpx + m.uy * gpy)) - Fdir[a]);
                    } else {
                        fX = (dC[a][i] - (m.ux * gcx[i] + m.uy * gcy[i])) - cc / (m.rho * CS2) * (ex * bx + ey * by);
                    }
                    double heq = cc * G[a] - 0.5 * (ex * Xx + ey * Xy) * G[a];
                    double ha = c->h[((size_t)i * 9 + a) * n + q];
                    c->hpost[((size_t)i * 9 + a) * n + q] = ha - omh * (ha - heq) + fX * G[a] + 0.5 * difi * G[a];
                }
            }
        }
}

/* Streamed value of population a at node (x, y) in the interior rule:
 * periodic (or, with open x, any source inside the domain), half-way
 * bounce-back when the source lies beyond a wall (R15). */
static double streamed_g(const pfo_ctx *c, int a, int x, int y) {
    int sy = y - EY[a], sx = x - EX[a], n = c->n;
    if (sy < 0 || sy >= c->ny) return c->gpost[(size_t)OPP[a] * n + y * c->nx + x];
    return c->gpost[(size_t)a * n + sy * c->nx + wrapx(sx, c->nx)];
}
static double streamed_h(const pfo_ctx *c, int i, int a, int x, int y) {
    int sy = y - EY[a], sx = x - EX[a], n = c->n;
    if (sy < 0 || sy >= c->ny) return c->hpost[((size_t)i * 9 + OPP[a]) * n + y * c->nx + x];
    return c->hpost[((size_t)i * 9 + a) * n + sy * c->nx + wrapx(sx, c->nx)];
}

/* Open x (Sec. 3.2: velocity inlet on the left, convective outflow on the
 * right; the paper cites these conditions without printing them, so they
 * are derived here for the transformed populations).  A population whose
 * source lies beyond a wall is bounced back first (R15); the others whose
 * source lies beyond x = 0 or x = nx-1 are set here.
 *   Inlet (x = 0; pure component 3 flows in with u = (u_in, 0)): every
 *   unknown a (e_ax = +1) takes gbar_a = gbar_abar + gbar_eq,a - gbar_eq,abar,
 *   the odd part of the equilibrium at u_in (the node's density,
 *   grad rho = 0, the body force as the only force).  That makes
 *   sum_a e_ax gbar_a = c_s^2 (rho u_in - F_x / 2), so the next velocity
 *   moment returns u_in; with both diagonals unknown, the pair 5 / 8 shares
 *   a correction that sets sum_a e_ay gbar_a = -c_s^2 F_y / 2 as well (the
 *   Zou-He non-equilibrium bounce-back); at a corner, where one diagonal
 *   comes from the wall, the other diagonal and the axis population take
 *   the corrections that meet both components.  The unknown hbar_a are 0 plus the receiving node's diffusion
 *   half (no component 1 or 2 enters).
 *   Outflow (x = nx-1): the unknown a (e_ax = -1) follow the convective
 *   condition d/dt + U d/dx = 0, discretised as
 *   gbar_a(t+1) = [gbar_a(t) + U gbar_a(x-1, t+1)] / (1 + U), U the node's
 *   u_x at time t (not below 0), with their pressure part w_a p replaced:
 *   w_a [p_e - (p(x, t) + U p(x-1, t)) / (1 + U)] is added, p_e = 2 p(x-1, t)
 *   - p(x-2, t) the linear extrapolation of the pressure.  (Applied to the
 *   whole population, the convective condition also transports the pressure,
 *   dp/dt = -U dp/dx, which in a developed channel flow with its constant
 *   pressure drop makes the pressure, and the mass held by the weakly
 *   compressible lattice, grow without bound while less leaves than enters.)
 *   hbar_a copies its neighbour's new value (zero normal gradient). */
static void open_x_columns(pfo_ctx *c) {
    int nx = c->nx, ny = c->ny, n = c->n, nh = c->p.n_h;
    const pfo_params *P = &c->p;
    for (int y = 0; y < ny; ++y) {
        /* inlet */
        int q = y * nx;
        double rho = c->rho[q];
        node_macro m = {P->u_in, 0.0, rho, 0.0, 0.0, 0.0, rho * P->fx, -rho * P->g};
        double g[9];
        int unknown[9] = {0};
        for (int a = 0; a < 9; ++a) {
            int sy = y - EY[a];
            g[a] = c->g[(size_t)a * n + q];      /* already streamed (interior rule) */
            if (EX[a] == 1 && sy >= 0 && sy < ny) unknown[a] = 1;
        }
        for (int a = 0; a < 9; ++a)
            if (unknown[a]) g[a] = g[OPP[a]] + gbar_eq(&m, a) - gbar_eq(&m, OPP[a]);
        double jx = (rho * P->u_in - 0.5 * m.Fx) * CS2, jy = (0.0 - 0.5 * m.Fy) * CS2;
        double rx = jx, ry = jy;
        for (int a = 0; a < 9; ++a) { rx -= EX[a] * g[a]; ry -= EY[a] * g[a]; }
        if (unknown[5] && unknown[8]) {
            /* the pair shares the y correction (x unchanged); rx is 0 up to rounding */
            g[5] += 0.5 * ry;
            g[8] -= 0.5 * ry;
            g[1] += rx;
        } else {
            /* a corner: one diagonal comes from the wall, the other (d) and the
             * axis population meet both components */
            int d = unknown[5] ? 5 : 8;
            g[d] += EY[d] * ry;
            g[1] += rx - EY[d] * ry;
        }
        for (int a = 0; a < 9; ++a) c->g[(size_t)a * n + q] = g[a];
        for (int i = 0; i < nh; ++i)
            for (int a = 0; a < 9; ++a)
                if (unknown[a])
                    c->h[((size_t)i * 9 + a) * n + q] = 0.5 * c->dif[i * n + q] * Gamma(a, c->u[q], c->u[n + q]);
        /* outflow */
        q = y * nx + nx - 1;
        int qn = q - 1;
        double U = c->u[q] > 0.0 ? c->u[q] : 0.0;
        double pt = 2.0 * c->pr[qn] - c->pr[qn - 1];   /* linear extrapolation of p at time t */
        for (int a = 0; a < 9; ++a) {
            int sy = y - EY[a];
            if (EX[a] != -1 || sy < 0 || sy >= ny) continue;
            double gnext = streamed_g(c, a, nx - 2, y);
            c->g[(size_t)a * n + q] = (c->gold[(size_t)a * n + q] + U * gnext) / (1.0 + U)
                                      + W[a] * (pt - (c->pr[q] + U * c->pr[qn]) / (1.0 + U));
            for (int i = 0; i < nh; ++i)
                c->h[((size_t)i * 9 + a) * n + q] = streamed_h(c, i, a, nx - 2, y)
                    + 0.5 * c->dif[i * n + qn] * Gamma(a, c->u[qn], c->u[n + qn]);
        }
    }
}

/* Stage 12-13: streaming (periodic x, half-way bounce-back in y, R15) and the
 * receiving-node half of the diffusion term (R12); with open x the boundary
 * columns are completed by open_x_columns. */
static void stage_stream(pfo_ctx *c) {
    int nx = c->nx, ny = c->ny, n = c->n, nh = c->p.n_h;
    if (OX) memcpy(c->gold, c->g, sizeof(double) * 9 * (size_t)n);
    OMP_FOR
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int q = y * nx + x;
            double ux = c->u[q], uy = c->u[n + q];
            for (int a = 0; a < 9; ++a) {
                c->g[(size_t)a * n + q] = streamed_g(c, a, x, y);
                double G = Gamma(a, ux, uy);
                for (int i = 0; i < nh; ++i)
                    c->h[((size_t)i * 9 + a) * n + q] = streamed_h(c, i, a, x, y) + 0.5 * c->dif[i * n + q] * G;
            }
            c->tau[q] = c->taunew[q];
        }
    if (OX) open_x_columns(c);
}

static void macro_from_state(pfo_ctx *c) {
    stage_phase(c);
    stage_chem(c);
    stage_diffusion(c);
    stage_hydro(c);
}

int pfo_step(pfo_ctx *c, int64_t nsteps) {
    if (!c || nsteps < 0) return -1;
    for (int64_t s = 0; s < nsteps; ++s) {
        macro_from_state(c);
        stage_collide(c);
        stage_stream(c);
    }
    return 0;
}

/* Initial state from C, u, p (u, p may be NULL for zero): populations at
 * their equilibria, tau at zero shear (R7). */
int pfo_init_fields(pfo_ctx *c, const double *C, const double *u, const double *p) {
    if (!c || !C) return -1;
    int nx = c->nx, ny = c->ny, n = c->n, nh = c->p.n_h;
    for (int q = 0; q < n; ++q) {
        double ci[2] = {C[q], nh == 2 ? C[n + q] : 0.0};
        if (!isfinite(ci[0]) || !isfinite(ci[1])) return -4;
        c->C[q] = ci[0];
        c->C[n + q] = ci[1];
        c->C[2 * n + q] = 1.0 - ci[0] - ci[1];
        c->rho[q] = mixture_density(&c->p, ci[0], ci[1], c->C[2 * n + q]);
        c->u[q] = u ? u[q] : 0.0;
        c->u[n + q] = u ? u[n + q] : 0.0;
        c->pr[q] = p ? p[q] : 0.0;
    }
    stage_chem(c);
    stage_diffusion(c);
    /* force; the gbar populations do not exist yet */
    for (int q = 0; q < n; ++q) {
        double fx, fy;
        surface_force(c, q, &fx, &fy);
        c->Fs[q] = fx + c->rho[q] * c->p.fx;
        c->Fs[n + q] = fy - c->rho[q] * c->p.g;
    }
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int q = y * nx + x;
            grad_cd_at(c->pr, x, y, nx, ny, OX, &c->gradp[q], &c->gradp[n + q]);
        }
    for (int q = 0; q < n; ++q) {
        node_macro m = {c->u[q], c->u[n + q], c->rho[q], c->pr[q], c->gradrho[q], c->gradrho[n + q],
                        c->Fs[q], c->Fs[n + q]};
        for (int a = 0; a < 9; ++a) c->g[(size_t)a * n + q] = gbar_eq(&m, a);
        double bx = c->gradp[q] - m.Fx, by = c->gradp[n + q] - m.Fy;
        for (int i = 0; i < nh; ++i) {
            double cc = c->C[i * n + q];
            double Xx = c->gradC[(2 * i) * n + q] - cc / (m.rho * CS2) * bx;
            double Xy = c->gradC[(2 * i + 1) * n + q] - cc / (m.rho * CS2) * by;
            for (int a = 0; a < 9; ++a) {
                double G = Gamma(a, m.ux, m.uy);
                c->h[((size_t)i * 9 + a) * n + q] = cc * G - 0.5 * ((EX[a] - m.ux) * Xx + (EY[a] - m.uy) * Xy) * G;
            }
        }
        double ck[3] = {c->C[q], c->C[n + q], c->C[2 * n + q]};
        c->tau[q] = mixture_tau(&c->p, ck, 0.0);
    }
    return 0;
}

/* Macroscopic fields of the current state (stages 1-6). Any output may be NULL. */
int pfo_macroscopic(pfo_ctx *c, double *rho, double *u, double *p, double *phi) {
    if (!c) return -1;
    macro_from_state(c);
    int n = c->n;
    if (rho) memcpy(rho, c->rho, sizeof(double) * n);
    if (u) memcpy(u, c->u, sizeof(double) * 2 * n);
    if (p) memcpy(p, c->pr, sizeof(double) * n);
    if (phi) memcpy(phi, c->C, sizeof(double) * (size_t)c->p.n_h * n);
    return 0;
}

/* Every derived field of the current state, for unit tests of single stages.
 * out must hold PFO_NFIELDS planes of nx*ny doubles, in the order listed in
 * pfo.h. */
int pfo_fields(pfo_ctx *c, double *out) {
    if (!c || !out) return -1;
    macro_from_state(c);
    size_t n = (size_t)c->n;
    double *o = out;
    memcpy(o, c->C, 3 * n * sizeof(double)); o += 3 * n;
    memcpy(o, c->rho, n * sizeof(double)); o += n;
    memcpy(o, c->gradC, 6 * n * sizeof(double)); o += 6 * n;
    memcpy(o, c->lapC, 3 * n * sizeof(double)); o += 3 * n;
    memcpy(o, c->mu, 3 * n * sizeof(double)); o += 3 * n;
    memcpy(o, c->gradmu, 6 * n * sizeof(double)); o += 6 * n;
    memcpy(o, c->lapmu, 3 * n * sizeof(double)); o += 3 * n;
    memcpy(o, c->dif, 2 * n * sizeof(double)); o += 2 * n;
    memcpy(o, c->Fs, 2 * n * sizeof(double)); o += 2 * n;
    memcpy(o, c->u, 2 * n * sizeof(double)); o += 2 * n;
    memcpy(o, c->pr, n * sizeof(double)); o += n;
    memcpy(o, c->gradp, 2 * n * sizeof(double)); o += 2 * n;
    memcpy(o, c->gradrho, 2 * n * sizeof(double)); o += 2 * n;
    return 0;
}

/* Mass, mass of cells with C>0.5, centroid and mean velocity of component comp
 * (Sec. 3.1 for the thresholded mass; Sec. 4.2, Eqs. (43)-(44)).  The
 * centroid is the plain C-weighted mean of the node coordinates: a bubble
 * that straddles the periodic seam in x reports a mean between its two
 * halves.  Returns -1 for component 1 (C_2) when only one phase field is
 * carried, -4 when the component's mass is zero or a sum is not finite. */
int pfo_bubble_centroid_velocity(pfo_ctx *c, int comp, double out[6]) {
    if (!c || !out || comp < 0 || comp > 2) return -1;
    if (comp == 1 && c->p.n_h == 1) return -1;
    macro_from_state(c);
    int nx = c->nx, ny = c->ny, n = c->n;
    double m = 0.0, mh = 0.0, sx = 0.0, sy = 0.0, su = 0.0, sv = 0.0;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int q = y * nx + x;
            double cg = c->C[comp * n + q];
            m += cg;
            if (cg > 0.5) mh += cg;
            sx += cg * x;
            sy += cg * y;
            su += cg * c->u[q];
            sv += cg * c->u[n + q];
        }
    if (!(m != 0.0) || !isfinite(m) || !isfinite(mh) || !isfinite(sx) || !isfinite(sy) || !isfinite(su) ||
        !isfinite(sv))
        return -4;
    out[0] = m; out[1] = mh;
    out[2] = sx / m; out[3] = sy / m; out[4] = su / m; out[5] = sv / m;
    return 0;
}

size_t pfo_state_doubles(const pfo_ctx *c) {
    return c ? (size_t)c->n * (9 + 9 * (size_t)c->p.n_h + 1) : 0;
}

/* State = gbar[9][n], hbar[n_h][9][n], tau[n]. */
int pfo_get_state(const pfo_ctx *c, double *dst) {
    if (!c || !dst) return -1;
    size_t n = (size_t)c->n, nh = (size_t)c->p.n_h;
    memcpy(dst, c->g, 9 * n * sizeof(double));
    memcpy(dst + 9 * n, c->h, nh * 9 * n * sizeof(double));
    memcpy(dst + 9 * n + nh * 9 * n, c->tau, n * sizeof(double));
    return 0;
}

int pfo_set_state(pfo_ctx *c, const double *src) {
    if (!c || !src) return -1;
    size_t n = (size_t)c->n, nh = (size_t)c->p.n_h;
    memcpy(c->g, src, 9 * n * sizeof(double));
    memcpy(c->h, src + 9 * n, nh * 9 * n * sizeof(double));
    memcpy(c->tau, src + 9 * n + nh * 9 * n, n * sizeof(double));
    return 0;
}

/* Test hooks: lattice tables, single stencils on a caller field, E0 and mu. */
void pfo_lattice(int *ex, int *ey, double *w, int *opp) {
    for (int a = 0; a < 9; ++a) { ex[a] = EX[a]; ey[a] = EY[a]; w[a] = W[a]; opp[a] = OPP[a]; }
}

int pfo_stencil(const double *f, int nx, int ny, int kind, int a, double *out) {
    if (!f || !out || nx < 1 || ny < 1) return -1;
    int n = nx * ny;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int q = y * nx + x;
            switch (kind) {
                case 0: grad_cd_at(f, x, y, nx, ny, 0, &out[q], &out[n + q]); break;
                case 1: out[q] = lap_cd_at(f, x, y, nx, ny, 0); break;
                case 2: out[q] = dir_md_at(f, x, y, a, nx, ny, 0); break;
                case 3: grad_md_at(f, x, y, nx, ny, 0, &out[q], &out[n + q]); break;
                case 4: out[q] = dir_cd_at(f, x, y, a, nx, ny, 0); break;
                default: return -1;
            }
        }
    return 0;
}

double pfo_bulk_energy(const pfo_params *p, double c1, double c2, double c3) {
    double S[3], ST;
    capillary(p, S, &ST);
    return bulk_E0(p, S, c1, c2, c3);
}

void pfo_chem_potential(const pfo_params *p, const double c[3], const double lap[3], double mu[3]) {
    chem_potential(p, c, lap, mu);
}

double pfo_mixture_tau(const pfo_params *p, const double c[3], double gdot) {
    return mixture_tau(p, c, gdot);
}
