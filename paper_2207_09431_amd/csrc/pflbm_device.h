// pflbm_device.h -- device-side building blocks of the gfx950 step kernels.
//
// Lattice, per-case parameter block, thermodynamics (Sec. 2.1), equilibria
// and forcing (Sec. 2.2) and the truncated power law (Sec. 2.3) of
// arXiv 2207.09431, in float32.  Private to the HIP library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pflbm {

// D2Q9 in the order of Sec. 2.2, Eq. (11): 0 rest, 1-4 axes, 5-8 diagonals.
// The float32 weights are 4/9 and 1/9 rounded to nearest and 1/36 one unit
// in the last place below its nearest value (0x3CE38E38 instead of
// 0x3CE38E39), so that they sum to exactly 1: with the nearest values the
// sum is 1 + 7.45e-9, and every source term whose weighted sum is meant to
// return its own value (sum_a Gamma_a H = H) gains 7.45e-9 H per node and
// step, a systematic drift of the component mass.
struct Lat {
    static constexpr int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static constexpr int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    static constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    static constexpr float w[9] = {4.0f / 9.0f, 1.0f / 9.0f, 1.0f / 9.0f, 1.0f / 9.0f, 1.0f / 9.0f,
                                   0x1.c71c7p-6f, 0x1.c71c7p-6f, 0x1.c71c7p-6f, 0x1.c71c7p-6f};
};
constexpr float kCs2 = 1.0f / 3.0f;

// Per-case block in device memory.  State planes are row-major (ny, pitch);
// `plane` is the element stride between planes.  The gbar state is kept as
// s = sum_a gbar_a in plane 0 (less the reference p_ref below) and the
// deviations d_a = gbar_a - w_a s
// (a = 1..8) in planes 1..8 (float32; the float16 form is described below);
// d_0 = -sum_{a>0} d_a.  The phase
// fields C_i are accumulated in float64 planes: their per-step change is far
// below the float32 spacing near C = 1, and rounding it into a float32 state
// drifts the component mass.
struct CaseDev {
    int nx, ny, pitch, n_h;
    long long plane;
    double* P[2];       // s - p_ref (float64), one plane each (ping-pong)
    float* S[2];        // d_a in plane a-1 (a = 1..8), or j_x, j_y in planes 0, 1 of the float16 form
    double* C[2];       // n_h planes each (float64)
    float* T[2];        // tau of the previous step
    float* H[2];        // stored-hbar form: q_a = hbar_a - w_a C_i, 9*n_h planes each, else null
    // float16 storage form: S holds s, j_x, j_y (float32) and Q the six pair
    // moments of the deviations (float16, scaled by qscale); null otherwise
    _Float16* Q[2];
    float qscale, qinv;
    float rho[3], nu[3], inu[3];   // inu = 1 / nu
    float inuF[3], nuloF, nuhiF;  // inu with 0 for the power-law component; min, max of the other nu
    int plc;            // power-law component or -1
    int vm;             // variable mobility
    int tau_iters;      // fixed-point passes of the implicit tau (0: previous step's tau)
    int hcd;            // central differences for grad C_i in the hbar forcing
    int openx;          // velocity inlet at x = 0 and outflow at x = nx-1 (else x periodic)
    float u_in;         // inlet velocity
    int mflux;          // conservative link form of the diffusion source
    float K, nexp, numin, numax;
    float sig12, sig13, sig23, lam;
    float Sig[3];
    float xi;
    float mob[2];       // D0 / Sigma_i for the carried components
    float omh;          // 1 / (tau_h + 1/2)
    float g, fx;
    // float64 coefficients of the bulk chemical potential; dA_j = 4 Sigma_T / (xi Sigma_j)
    double dsig12, dsig13, dsig23, dlam, dSig[3], dA[3];
    double drho[3];     // component densities in float64
    // The state keeps s' = s - p_ref(y) with p_ref(y) = pref_g (pref_yc - y),
    // the hydrostatic pressure of the liquid (pref_g = rho_3 g, pref_yc the
    // mid-height): in a tall domain under gravity s reaches rho g H / 2, and
    // float32 spacing at that size is comparable to the gas momentum at
    // density ratio 1000.  The reference is exact bookkeeping: every use adds
    // it back or takes its exact differences.
    float pref_g, pref_yc;
    // set to 1 by any once-per-call kernel that meets a non-finite value in
    // this case's state or in the fields derived from it; cleared by the host
    // (init_fields, set_state)
    unsigned int* flag;
};

__device__ __forceinline__ float pref(const CaseDev& cd, int y) { return cd.pref_g * (cd.pref_yc - (float)y); }
__device__ __forceinline__ double pref_d(const CaseDev& cd, int y) {
    return (double)cd.pref_g * ((double)cd.pref_yc - (double)y);
}

struct TileDev {
    int case_id, x0, y0, pad;
};

__device__ __forceinline__ float clip01(float c) { return fminf(fmaxf(c, 0.0f), 1.0f); }

__device__ __forceinline__ int wrap_x(int x, int nx) {
    // x lies within a few tile widths of [0, nx): no integer division
    while (x < 0) x += nx;
    while (x >= nx) x -= nx;
    return x;
}
// Branch-free wrap for tile regions: exact for x in [-nx, 2 nx); larger x
// (halo nodes of a ragged last tile more than nx beyond the edge, whose
// values never reach an output) are clamped to a valid column.
__device__ __forceinline__ int wrap_x_tile(int x, int nx) {
    x = x < 0 ? x + nx : (x >= nx ? x - nx : x);
    return x < nx ? x : nx - 1;
}
// Mirror about the walls at y = -1/2 and y = ny - 1/2 (zero normal
// derivative of the stencil fields); rows farther than ny away are clamped.
__device__ __forceinline__ int mirror_y(int y, int ny) {
    if (y < 0) y = -y - 1;
    if (y >= ny) y = 2 * ny - 1 - y;
    return y < 0 ? 0 : (y >= ny ? ny - 1 : y);
}

// Float16 storage form.  s stays float64 (plane P) and the momentum
// j = sum_a e_a d_a float32 (it is
// conserved by the collision, so rounding it would persist, and at density
// ratio 1000 it is a small difference of the deviations); the rest of the
// deviations is kept as six pair moments in float16,
//   m = (d1+d3, d2+d4, d5+d7, d6+d8, d5-d7, d6-d8),
// whose rounding only reaches non-conserved moments, which the collision
// relaxes.  Scale 2^14: |m| up to 4 stays finite, values down to 4e-9 stay
// normal, and the scaling is exact.
constexpr float kQScale = 16384.0f;
constexpr int kQPlanes = 6;    // float16 planes
constexpr int kSPlanes16 = 2;  // float32 planes: j_x, j_y

__device__ __forceinline__ void pack_devs(const float d[9], float& jx, float& jy, float m[6]) {
    const float x5 = d[5] - d[7], x6 = d[6] - d[8];
    jx = (d[1] - d[3]) + (x5 - x6);
    jy = (d[2] - d[4]) + (x5 + x6);
    m[0] = d[1] + d[3];
    m[1] = d[2] + d[4];
    m[2] = d[5] + d[7];
    m[3] = d[6] + d[8];
    m[4] = x5;
    m[5] = x6;
}
__device__ __forceinline__ void unpack_devs(float jx, float jy, const float m[6], float d[9]) {
    const float x1 = jx - (m[4] - m[5]), y1 = jy - (m[4] + m[5]);
    d[1] = 0.5f * (m[0] + x1);
    d[3] = 0.5f * (m[0] - x1);
    d[2] = 0.5f * (m[1] + y1);
    d[4] = 0.5f * (m[1] - y1);
    d[5] = 0.5f * (m[2] + m[4]);
    d[7] = 0.5f * (m[2] - m[4]);
    d[6] = 0.5f * (m[3] + m[5]);
    d[8] = 0.5f * (m[3] - m[5]);
}

// Deviations d_1..d_8 of buffer `par` at element offset `off`, in either
// storage form (used by the once-per-call kernels).
__device__ __forceinline__ void load_devs(const CaseDev& cd, int par, long long off, float d[9]) {
    if (cd.Q[par]) {
        float m[6];
        for (int k = 0; k < kQPlanes; ++k) m[k] = (float)cd.Q[par][k * cd.plane + off] * cd.qinv;
        unpack_devs(cd.S[par][off], cd.S[par][cd.plane + off], m, d);
    } else {
        for (int a = 1; a < 9; ++a) d[a] = cd.S[par][(a - 1) * cd.plane + off];
    }
}
__device__ __forceinline__ void store_devs(const CaseDev& cd, int par, long long off, const float d[9]) {
    if (cd.Q[par]) {
        float jx, jy, m[6];
        pack_devs(d, jx, jy, m);
        cd.S[par][off] = jx;
        cd.S[par][cd.plane + off] = jy;
        for (int k = 0; k < kQPlanes; ++k) cd.Q[par][k * cd.plane + off] = (_Float16)(m[k] * cd.qscale);
    } else {
        for (int a = 1; a < 9; ++a) cd.S[par][(a - 1) * cd.plane + off] = d[a];
    }
}

// Mixture density with concentrations limited to [0, 1], formed in float64
// from the float64 phase fields: inside a bubble C_1 = 1 - O(1e-5), and
// 1 - C_1 in float32 would carry a relative error of O(1e-3) into a liquid
// term that is a few percent of the gas density.
__device__ __forceinline__ float mix_rho(const CaseDev& cd, double c1, double c2) {
    const double a = fmin(fmax(c1, 0.0), 1.0), b = fmin(fmax(c2, 0.0), 1.0);
    const double c = fmin(fmax(1.0 - c1 - c2, 0.0), 1.0);
    return (float)(cd.drho[0] * a + cd.drho[1] * b + cd.drho[2] * c);
}

// Isotropic central stencils from the nine values of a D2Q9 neighbourhood in
// lattice order (f[0] the node, f[a] at x + e_a):
//   grad f = sum_a w_a e_a [f(x+e_a) - f(x-e_a)] / (2 c_s^2),
//   lap f  = sum_a w_a [f(x+e_a) - 2 f(x) + f(x-e_a)] / c_s^2,
// each direction pair contributing once with twice its weight.  The step
// kernel evaluates the same expressions on its LDS tiles, so that the fields
// exported or reduced once per call round exactly as the step's own.
__device__ __forceinline__ void cd_grad9(const float f[9], float& gx, float& gy) {
    const float d1 = f[1] - f[3], d2 = f[2] - f[4], d5 = f[5] - f[7], d6 = f[6] - f[8];
    gx = (1.0f / 3.0f) * d1 + (1.0f / 12.0f) * (d5 - d6);
    gy = (1.0f / 3.0f) * d2 + (1.0f / 12.0f) * (d5 + d6);
}
// The Laplacian of the float64 phase field, rounded once.
__device__ __forceinline__ float cd_lap9_d(const double f[9]) {
    const double c = f[0];
    const double s1 = (f[1] - c) + (f[3] - c), s2 = (f[2] - c) + (f[4] - c);
    const double s5 = (f[5] - c) + (f[7] - c), s6 = (f[6] - c) + (f[8] - c);
    return (float)((2.0 / 3.0) * (s1 + s2) + (1.0 / 6.0) * (s5 + s6));
}

// Hardware reciprocal (1 ulp), instead of the correctly rounded division
// sequence: float32 rounding of this size is far below the method's needs.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Global-memory views of the state planes: the pointers come out of the case
// block, so without the address-space cast the compiler falls back to flat
// loads and stores.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}

// Global access at a uniform base plus a 32-bit byte offset: the compiler
// then uses the SGPR-base form of the global load/store, so one 32-bit offset
// per node serves every plane (no 64-bit address arithmetic per access).
// Every plane of a case is below 4 GiB (checked when the context is created).
template <class T>
__device__ __forceinline__ T gld(const T* base, uint32_t boff) {
    typedef const __attribute__((address_space(1))) char* gcp;
    typedef const __attribute__((address_space(1))) T* gtp;
    return *(gtp)((gcp)base + boff);
}
template <class T>
__device__ __forceinline__ void gst(T* base, uint32_t boff, T v) {
    typedef __attribute__((address_space(1))) char* gcp;
    typedef __attribute__((address_space(1))) T* gtp;
    *(gtp)((gcp)base + boff) = v;
}

// Chemical potentials of the ternary free energy (Sec. 2.1, Eqs. (3), (5)):
// mu_i = sum_{j != i} (dE0/dC_i - dE0/dC_j) a_j - (3/4) xi Sigma_i lap C_i
// with a_j = 4 Sigma_T / (xi Sigma_j).  The bulk part is evaluated in float64
// from the float64 concentrations: near equilibrium mu is a small difference
// of the bulk and gradient parts, and its float32 error reaches the gas
// velocity amplified by the density ratio.  With one phase field (C_2 = 0)
// only mu_1 and mu_3 enter the step; the terms that vanish with C_2 are left
// out, which changes no rounding.
template <int NH>
__device__ __forceinline__ void chem_potential(const CaseDev& cd, double c1, double c2, float l1, float l2,
                                               float mu[3]) {
    const double c3 = 1.0 - c1 - c2;
    const float b = 0.75f * cd.xi;
    if (NH == 1) {
        const double d0 = 2.0 * cd.dsig13 * c1 * c3 * c3;
        const double d1 = c1 * c3 * (cd.dSig[0] * c1 + cd.dSig[2] * c3);
        const double d2 = 2.0 * cd.dsig13 * c1 * c1 * c3;
        mu[0] = (float)((d0 - d1) * cd.dA[1] + (d0 - d2) * cd.dA[2]) - b * cd.Sig[0] * l1;
        mu[1] = 0.0f;
        mu[2] = (float)((d2 - d0) * cd.dA[0] + (d2 - d1) * cd.dA[1]) + b * cd.Sig[2] * l1;
    } else {
        const double S0 = cd.dSig[0], S1 = cd.dSig[1], S2 = cd.dSig[2];
        const double sc = S0 * c1 + S1 * c2 + S2 * c3;
        const double c123 = c1 * c2 * c3;
        const double d0 = 2.0 * cd.dsig12 * c1 * c2 * c2 + 2.0 * cd.dsig13 * c1 * c3 * c3 + c2 * c3 * sc + c123 * S0
                        + 2.0 * cd.dlam * c1 * c2 * c2 * c3 * c3;
        const double d1 = 2.0 * cd.dsig12 * c1 * c1 * c2 + 2.0 * cd.dsig23 * c2 * c3 * c3 + c1 * c3 * sc + c123 * S1
                        + 2.0 * cd.dlam * c1 * c1 * c2 * c3 * c3;
        const double d2 = 2.0 * cd.dsig13 * c1 * c1 * c3 + 2.0 * cd.dsig23 * c2 * c2 * c3 + c1 * c2 * sc + c123 * S2
                        + 2.0 * cd.dlam * c1 * c1 * c2 * c2 * c3;
        mu[0] = (float)((d0 - d1) * cd.dA[1] + (d0 - d2) * cd.dA[2]) - b * cd.Sig[0] * l1;
        mu[1] = (float)((d1 - d0) * cd.dA[0] + (d1 - d2) * cd.dA[2]) - b * cd.Sig[1] * l2;
        mu[2] = (float)((d2 - d0) * cd.dA[0] + (d2 - d1) * cd.dA[1]) + b * cd.Sig[2] * (l1 + l2);
    }
}

// Truncated power law, kinematic (Sec. 2.3, Eqs. (31), (33)).
__device__ __forceinline__ float powerlaw_nu(const CaseDev& cd, float gdot) {
    float nu;
    if (gdot <= 0.0f) {
        if (cd.nexp < 1.0f) return cd.numax;
        if (cd.nexp > 1.0f) return cd.numin;
        nu = cd.K;
    } else {
        // hardware log2/exp2: gdot > 0 here, and for a denormal gdot (< 1e-38)
        // the clamp below decides the result anyway
        nu = cd.K * __builtin_amdgcn_exp2f((cd.nexp - 1.0f) * __builtin_amdgcn_logf(gdot));
    }
    return fminf(fmaxf(nu, cd.numin), cd.numax);
}

// Mixture tau = nu / c_s^2 with the harmonic rule 1/nu = sum_k C_k / nu_k
// (each C_k limited to [0, 1]) clamped to [min nu_k, max nu_k]: two layers in
// series share the stress and add their shear rates, which the layered flow
// of Sec. 3.3 (Table 3) reproduces.
__device__ __forceinline__ float mixture_tau(const CaseDev& cd, float c1, float c2, float c3, float gdot) {
    // the components of fixed viscosity (their inverse weights precomputed,
    // the power-law component's set to 0), then the power-law component
    float q = fmaf(clip01(c1), cd.inuF[0], fmaf(clip01(c2), cd.inuF[1], clip01(c3) * cd.inuF[2]));
    float lo = cd.nuloF, hi = cd.nuhiF;
    if (cd.plc >= 0) {
        const float np = powerlaw_nu(cd, gdot);
        const float cp = cd.plc == 0 ? c1 : (cd.plc == 1 ? c2 : c3);
        q = fmaf(clip01(cp), rcp(np), q);
        lo = fminf(lo, np);
        hi = fmaxf(hi, np);
    }
    const float nu = fminf(fmaxf(rcp(q), lo), hi);   // q > 0: the limited C_k sum to at least 1/3
    return 3.0f * nu;
}

}  // namespace pflbm
