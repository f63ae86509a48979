/*
 * pflbm.h -- C ABI of the MI355X (gfx950) phase-field power-law lattice
 * Boltzmann step.
 *
 * Method (Ghorbanpour Arani et al., arXiv 2207.09431, Sec. 2): D2Q9
 * pressure/momentum populations gbar (Sec. 2.2, Eqs. (12)-(16), (23)-(24))
 * coupled to Cahn-Hilliard populations hbar^i (Eqs. (17)-(22)) of the ternary
 * free energy (Sec. 2.1, Eqs. (1)-(7)), with a per-cell relaxation time from a
 * truncated power-law viscosity whose shear rate comes from the
 * non-equilibrium second moment of gbar with the previous step's tau
 * (Sec. 2.3, Eqs. (25)-(33)).  x is periodic; the rows y = 0 and y = ny-1 are
 * next to half-way bounce-back walls at rest.
 *
 * Conventions
 *  - Every call returns a pflbm_status; no C++ exception crosses the ABI.
 *  - Device memory is owned by the caller.  The library keeps the state in
 *    the caller's workspace (pflbm_workspace_bytes) and allocates no device
 *    memory; the workspace must stay valid until pflbm_destroy.  The library
 *    owns only the host-side context.
 *  - Work is enqueued on the HIP stream given to pflbm_create (NULL = the
 *    null stream).  Calls are asynchronous unless stated otherwise.
 *  - Host arrays are float64, row-major (ny, nx) with x fastest, and are
 *    copied during the call.  Device outputs are float32, row-major (ny, nx).
 *  - One context may be used by one host thread at a time.
 */
#ifndef PFLBM_H
#define PFLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PFLBM_OK = 0,
    PFLBM_ERR_INVALID_ARG = -1,   /* a parameter or argument is out of range */
    PFLBM_ERR_WORKSPACE = -2,     /* workspace NULL, too small or misaligned */
    PFLBM_ERR_DEVICE = -3,        /* a HIP call failed */
    PFLBM_ERR_NONFINITE = -4,     /* non-finite input, or the state became non-finite */
    PFLBM_ERR_STATE = -5,         /* call out of order (e.g. step before init_fields) */
    PFLBM_ERR_UNSUPPORTED = -6    /* valid request the library does not provide */
} pflbm_status;

typedef struct pflbm_ctx pflbm_ctx;

/*
 * Physical and numerical parameters of one domain (one "case").
 * Components: C1 and C2 are carried by hbar^1, hbar^2; C3 = 1 - C1 - C2
 * (Sec. 2.1, Eq. (1)).  With n_h = 1 only C1 is carried and C2 = 0.
 */
typedef struct {
    int32_t nx, ny;            /* lattice size, both >= 5 */
    int32_t n_h;               /* 1 or 2 phase fields carried */
    double rho[3];             /* component densities, > 0 */
    double nu[3];              /* Newtonian kinematic viscosities nu_k = c_s^2 tau_k, > 0 */
    int32_t powerlaw_comp;     /* component whose viscosity is the power law (0..2), or -1 */
    double K, n;               /* power law nu_P = K gdot^(n-1) (Sec. 2.3, Eq. (31)); finite, > 0
                                  when powerlaw_comp >= 0 */
    double nu_min, nu_max;     /* truncation of nu_P (Eq. (33)); 0 < nu_min <= nu_max */
    double sigma12, sigma13, sigma23; /* pairwise surface tensions (Sec. 2.1) */
    double Lambda;             /* six-fold term of the bulk free energy (Eq. (3)) */
    double xi;                 /* interface thickness (Eq. (2)), finite, > 0 */
    double D0;                 /* mobility scale (Eq. (6)); xi/300 in the paper; finite, >= 0 */
    int32_t variable_mobility; /* 0: D_i = D0/Sigma_i, 1: D_i = D0/Sigma_i C_i (1-C_i) (Eq. (6)) */
    double tau_h;              /* relaxation time of hbar (0.5 in the paper); finite, > 0 */
    double g;                  /* gravity: F_b = rho (fx, -g) (Eq. (12)) */
    double fx;                 /* horizontal body acceleration (0 in the paper's bubble runs) */
    int32_t storage;           /* 0: gbar deviations in float32; 1: float16 pair moments (see below) */
    int32_t store_h;           /* 0: keep only C_i when tau_h = 0.5 (exact), 1: store hbar */
    int32_t tau_iterations;    /* 0: tau from the shear rate taken with the previous step's tau
                                  (the paper's explicit update, Sec. 2.3); m in 1..8: m fixed-point
                                  passes tau <- tau(gdot(tau)) of the implicit relation Eq. (32),
                                  started from the previous step's tau */
    int32_t hforce_cd;         /* stencil of (e_a - u).grad C_i in the hbar forcing (Eq. (18)):
                                  0 mixed directional differences (default), 1 central differences.
                                  The paper names both kinds (Sec. 2.2, after Eq. (21)) without
                                  assigning them to terms.  With variable mobility (Eq. (6)) use 1:
                                  in a phase where D_i vanishes the mixed form amplifies oblique
                                  modes (up to 1.148 per step), the central form does not */
    int32_t open_x;            /* 0: x periodic.  1: velocity inlet at x = 0 and convective outflow at
                                  x = nx-1 (Sec. 3.2; compact state forms only, store_h = 0).  The
                                  inlet brings pure component 3 in with u = (u_in, 0): the unknown
                                  gbar take the odd part of the equilibrium at u_in plus the
                                  corrections that make both velocity moments exact, the unknown
                                  hbar carry no component 1 or 2.  The outflow applies
                                  d/dt + U d/dx = 0 (U the node's u_x, not below 0) to the unknown
                                  gbar with their pressure part replaced by the linear
                                  extrapolation of p, and copies the neighbour's hbar.  Stencil
                                  ghosts beyond the ends mirror the end columns */
    double u_in;               /* inlet velocity (open_x = 1) */
    int32_t mobility_flux;     /* form of the diffusion source div(D_i grad mu_i) (Sec. 2.2, Eq. (21)):
                                  0 the product form D_i lap mu_i + grad D_i . grad mu_i, 1 the
                                  conservative link form sum_a w_a (D_i(x) + D_i(x+e_a))
                                  (mu_i(x+e_a) - mu_i(x)) / c_s^2, whose links cancel in pairs so
                                  that the component totals keep no source of the method's own (with
                                  variable mobility the product form does not, Eq. (6)); identical
                                  to the product form in the continuum */
} pflbm_params;

/*
 * State forms.  gbar is kept as its level s = sum_a gbar_a (float64, stored
 * against the liquid's hydrostatic profile rho_3 g (y_c - y), y_c the
 * mid-height) and the deviations from the rest-state weights
 * d_a = gbar_a - w_a s, a = 1..8 (d_0 follows from sum_a d_a = 0); C_i is
 * kept in float64 and tau in float32.
 *  - storage = 0: d_a in float32 (104 B moved per lattice update, two-phase).
 *  - storage = 1: the momentum j = sum_a e_a d_a in float32 and the six pair
 *    moments (d1+d3, d2+d4, d5+d7, d6+d8, d5-d7, d6-d8) * 2^14 rounded to
 *    float16 (nearest even): 80 B per update; the arithmetic stays float32.
 *    Float16 rounding then reaches only moments that the collision relaxes.
 *    Requires store_h = 0.
 *  - store_h = 0 (requires tau_h = 0.5): hbar relaxes at rate 1, so the
 *    post-collision hbar depends only on time-t fields and keeping C_i alone
 *    is exact.  store_h = 1 keeps hbar as 9 n_h float32 planes of the
 *    deviations hbar_a - w_a C_i (C_i itself stays float64), for any tau_h.
 */

/*
 * Workspace bytes for the given cases (device memory, 256-byte aligned base).
 * Returns 0 when the parameters are invalid.
 */
size_t pflbm_workspace_bytes(const pflbm_params* cases, int32_t ncases);

/*
 * Creates a context for `ncases` domains (ncases = 1 is the plain path; more
 * cases are advanced together by every launch).  All cases must share n_h,
 * storage and store_h.  `d_workspace` is caller-owned device memory of at
 * least pflbm_workspace_bytes(cases, ncases) bytes; `hip_stream` is a
 * hipStream_t or NULL.  Errors: INVALID_ARG for out-of-range parameters
 * (nx or ny < 5, n_h not 1 or 2, rho_k <= 0, nu_k <= 0, nu_min <= 0 or
 * nu_min > nu_max, K <= 0 with a power-law component, xi <= 0, D0 < 0,
 * tau_h <= 0, a Sigma_i <= 0, store_h = 0 with tau_h != 0.5, storage not
 * 0 or 1, tau_iterations outside 0..8, hforce_cd, open_x or mobility_flux not 0 or 1, a
 * non-finite u_in with open_x, nx rounded up to 64 times ny at or above 2^29
 * nodes);
 * UNSUPPORTED for storage = 1 with store_h = 1, or open_x with store_h = 1; WORKSPACE when the
 * workspace is NULL, small or misaligned; DEVICE when a HIP call fails.
 */
int32_t pflbm_create(const pflbm_params* cases, int32_t ncases, void* d_workspace, size_t bytes,
                     void* hip_stream, pflbm_ctx** out);

/*
 * Initial state of one case from host fields (Sec. 4.2: quiescent start,
 * tanh interface of Eq. (42) supplied by the caller): C holds n_h planes,
 * u two planes (u_x then u_y) or NULL for zero, p one plane or NULL for zero,
 * each plane nx * ny doubles (the ABI reads exactly that many; the caller
 * guarantees the sizes).  Populations start at their equilibria
 * (Eqs. (16), (20)) and tau at its zero-shear value; the case's non-finite
 * flag is cleared.  Synchronises.  Errors: NONFINITE for a non-finite input.
 */
int32_t pflbm_init_fields(pflbm_ctx* ctx, int32_t case_id, const double* C, const double* u,
                          const double* p);

/*
 * Advances every case by nsteps time steps (collision, streaming,
 * bounce-back, Eqs. (14), (18)); asynchronous.  Errors: STATE before every
 * case has been initialised.
 */
int32_t pflbm_step(pflbm_ctx* ctx, int64_t nsteps);

/*
 * Macroscopic fields of one case (Eqs. (22)-(24)) into caller device
 * buffers, each row-major (ny, nx) float32: rho (1 plane), u (2 planes:
 * u_x, u_y), p (1 plane), phi (n_h planes: C_1..C_n_h).  Any pointer may be
 * NULL to skip that output.  Asynchronous.
 */
int32_t pflbm_macroscopic(pflbm_ctx* ctx, int32_t case_id, float* d_rho, float* d_u, float* d_p,
                          float* d_phi);

/*
 * Bubble diagnostics of component `comp` (0..2) of one case, summed in
 * float64 on the device (Sec. 3.1 thresholded mass; Sec. 4.2,
 * Eqs. (43)-(44)): out = { sum C, sum of C over cells with C > 0.5,
 * centroid x, centroid y, mean u_x, mean u_y } with weights C (unclipped;
 * component 2 is C_3 = 1 - C_1 - C_2).  The centroid is the plain C-weighted
 * mean of the node coordinates (x in [0, nx), y in [0, ny)): a bubble that
 * straddles the periodic seam in x reports a mean between its two halves.
 * Synchronises the stream.  Errors: INVALID_ARG for comp = 1 when n_h = 1
 * (C_2 is not carried); NONFINITE when the case's state or a summed quantity
 * is not finite (the case's sticky flag, below), or when the component's
 * mass is zero (no centroid).
 */
int32_t pflbm_bubble_centroid_velocity(pflbm_ctx* ctx, int32_t case_id, int32_t comp, double out[6]);

/*
 * The same diagnostics for callers that cannot allocate device memory or
 * touch their own workspace's scratch region at this point (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation).
 * Identical arguments, results (bitwise: the same kernels in the same order)
 * and errors as pflbm_bubble_centroid_velocity; the reduction's partial sums
 * and results are kept in a static device array of the library
 * (1024 x 6 + 8 doubles = 49,216 bytes per GPU, held until the process
 * ends) instead of the workspace.  Calls no allocating routine.  Every call
 * on one GPU shares that array: calls that overlap on one GPU (different
 * streams or host threads) race and must be serialised by the caller; each
 * call overwrites every slot it reads, so no clearing is needed between
 * calls.  Errors additionally: WORKSPACE if a reduction would need more than
 * the array's 1024 partial rows (the reduction caps its grid there, so no
 * domain size does).  Synchronises the stream.
 */
int32_t pflbm_bubble_centroid_velocity_noalloc(pflbm_ctx* ctx, int32_t case_id, int32_t comp, double out[6]);

/*
 * Divergence detection (sticky NONFINITE).  Every case carries a device flag
 * that the once-per-call kernels (pflbm_macroscopic,
 * pflbm_bubble_centroid_velocity, pflbm_export_populations and the scan
 * below) set when they meet a non-finite value in the state or in the fields
 * derived from it.  A synchronising call that finds a case's flag set makes
 * it sticky on the host: from then on pflbm_bubble_centroid_velocity of that
 * case, pflbm_check_state and pflbm_autotune return NONFINITE, until
 * pflbm_init_fields (that case) or pflbm_set_state (every case) clears it.
 * pflbm_step stays asynchronous and does not test the flag (cases of a batch
 * are independent: the others can still be advanced).
 *
 * pflbm_check_state scans the complete state of every case (one read of
 * it), synchronises, and returns NONFINITE if any case is flagged, OK
 * otherwise; STATE before every case has been initialised.
 * pflbm_case_nonfinite returns 1 if case_id is flagged on the host (as of
 * the last synchronising call), 0 if not, INVALID_ARG for a bad case_id;
 * it does not touch the device.
 */
int32_t pflbm_check_state(pflbm_ctx* ctx);
int32_t pflbm_case_nonfinite(const pflbm_ctx* ctx, int32_t case_id);

/*
 * Checkpoint: copies the complete state of every case (device to device)
 * into/out of a caller buffer of pflbm_state_bytes bytes.  Asynchronous.
 * pflbm_set_state clears every case's non-finite flag (the restored state
 * is scanned again by the next diagnostic call).
 */
size_t pflbm_state_bytes(const pflbm_ctx* ctx);
int32_t pflbm_get_state(pflbm_ctx* ctx, void* d_dst, size_t bytes);
int32_t pflbm_set_state(pflbm_ctx* ctx, const void* d_src, size_t bytes);

/*
 * Raw population planes of one case for inspection, as float32 (ny, nx)
 * planes copied into a caller device buffer: 9 planes of gbar_a
 * (a = 0..8, D2Q9 order of Eq. (11)), then n_h planes of C_i, then tau.
 * Asynchronous.
 */
int32_t pflbm_export_populations(pflbm_ctx* ctx, int32_t case_id, float* d_out);

/*
 * Kernel variants (tile shapes) of the step.  pflbm_set_variant selects the
 * variant used by pflbm_step; -1 restores the default.  pflbm_variant_name
 * returns NULL for an unknown index.
 */
int32_t pflbm_num_variants(const pflbm_ctx* ctx);
const char* pflbm_variant_name(const pflbm_ctx* ctx, int32_t index);
int32_t pflbm_set_variant(pflbm_ctx* ctx, int32_t index);

/*
 * Times every variant on the current state for `steps` launches each, in
 * two passes over the variants (each variant's faster pass counts), and
 * selects the fastest for pflbm_step.  The state is left unchanged (each
 * timed launch recomputes the same step into the spare buffer).  `best`
 * receives the chosen index; `ms_per_variant` (NULL or pflbm_num_variants
 * floats) receives the mean milliseconds per step of that pass, -1 for a
 * variant that does not apply.  Synchronises the stream.  Errors: STATE before init_fields;
 * NONFINITE (after tuning) when a case is flagged non-finite; DEVICE when a
 * launch or event fails, after which the variant in use before the call is
 * selected again.
 */
int32_t pflbm_autotune(pflbm_ctx* ctx, int32_t steps, int32_t* best, float* ms_per_variant);

/*
 * Launch mode of pflbm_step: 0 launches every step separately; an even
 * steps_per_graph > 0 captures that many steps once into a hipGraph and
 * replays it (whole graphs first, single launches for the remainder).  The
 * graph is rebuilt when the variant changes.  Results are identical to plain
 * launches.
 */
int32_t pflbm_set_graph(pflbm_ctx* ctx, int32_t steps_per_graph);

/* Stream of the step kernel (hipStream_t as void*), for timing with events. */
void* pflbm_stream(const pflbm_ctx* ctx);

/* Algorithmic bytes moved per lattice update by the step kernel. */
double pflbm_bytes_per_update(const pflbm_ctx* ctx);

/*
 * Destroys any captured hipGraph, waits for the context's stream and frees
 * the host-side context (the caller's workspace is left alone).  Errors:
 * INVALID_ARG for NULL; DEVICE when the final synchronisation fails (the
 * context is freed either way).
 */
int32_t pflbm_destroy(pflbm_ctx* ctx);

/* Static text for a pflbm_status value ("unknown status" otherwise). */
const char* pflbm_status_string(int32_t status);

#ifdef __cplusplus
}
#endif
#endif /* PFLBM_H */
