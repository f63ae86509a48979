/*
 * pfo.h -- FP64 reference solver for the phase-field power-law lattice
 * Boltzmann step of arXiv 2207.09431, Sec. 2.  TEST INFRASTRUCTURE ONLY:
 * loaded by the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark; never by the HIP library.
 *
 * All arrays are host float64, row-major (ny, nx), x fastest.  Functions
 * return 0 on success, -1 for an invalid argument, -3 when out of memory,
 * -4 for a non-finite input.
 */
#ifndef PFO_H
#define PFO_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nx, ny;            /* lattice; x periodic, walls below y=0 and above y=ny-1 */
    int32_t n_h;               /* phase fields carried: 1 (C2 = 0) or 2 */
    double rho[3];             /* component densities */
    double nu[3];              /* Newtonian kinematic viscosities */
    int32_t powerlaw_comp;     /* component following the power law, or -1 */
    double K, n, nu_min, nu_max;
    double sigma12, sigma13, sigma23, Lambda;
    double xi, D0;
    int32_t variable_mobility;
    double tau_h;
    double g;                  /* F_b = rho (fx, -g) */
    double fx;
    int32_t strain_literal;    /* reading switches, 0 = default reading */
    int32_t mobility_flux;
    int32_t hforce_mode;
    int32_t gforce_cd;
    int32_t force_potential;
    int32_t mix_linear;
    int32_t tau_iterations;    /* 0: previous-step tau (R7); m: m fixed-point passes */
    int32_t open_x;            /* 0: x periodic; 1: velocity inlet at x = 0, convective outflow at x = nx-1 */
    double u_in;               /* inlet velocity along x (open_x = 1) */
} pfo_params;

typedef struct pfo_ctx pfo_ctx;

/* Planes written by pfo_fields, each nx*ny doubles:
 * C[3], rho, gradC[3][2], lapC[3], mu[3], gradmu[3][2], lapmu[3], dif[2],
 * Fs[2], u[2], p, gradp[2], gradrho[2]. */
#define PFO_NFIELDS 36

int pfo_create(const pfo_params *p, pfo_ctx **out);
void pfo_destroy(pfo_ctx *c);
int pfo_init_fields(pfo_ctx *c, const double *C, const double *u, const double *p);
int pfo_step(pfo_ctx *c, int64_t nsteps);
int pfo_macroscopic(pfo_ctx *c, double *rho, double *u, double *p, double *phi);
int pfo_fields(pfo_ctx *c, double *out);
/* -1: bad comp (1 with n_h = 1); -4: zero mass or a non-finite sum */
int pfo_bubble_centroid_velocity(pfo_ctx *c, int comp, double out[6]);
size_t pfo_state_doubles(const pfo_ctx *c);
int pfo_get_state(const pfo_ctx *c, double *dst);
int pfo_set_state(pfo_ctx *c, const double *src);

void pfo_lattice(int *ex, int *ey, double *w, int *opp);
int pfo_stencil(const double *f, int nx, int ny, int kind, int a, double *out);
double pfo_bulk_energy(const pfo_params *p, double c1, double c2, double c3);
void pfo_chem_potential(const pfo_params *p, const double c[3], const double lap[3], double mu[3]);
double pfo_mixture_tau(const pfo_params *p, const double c[3], double gdot);

/* Threads of the per-node loops (OpenMP build); results do not depend on it. */
void pfo_set_threads(int n);
int pfo_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
