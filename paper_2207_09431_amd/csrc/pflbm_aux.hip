// pflbm_aux.hip -- initial state, macroscopic export and float64 reductions.
//
// These kernels run once per call (not per time step); one thread handles one
// node and reads its stencil neighbours straight from global memory.
#include "pflbm_internal.h"

namespace pflbm {

namespace {

constexpr int kBlock = 256;

// C_1, C_2 of node (x, y) (mirror/wrap applied by the caller)
__device__ __forceinline__ void load_c(const CaseDev& cd, const double* C, int x, int y, double& c1, double& c2) {
    const long long off = (long long)y * cd.pitch + x;
    c1 = C[off];
    c2 = cd.n_h == 2 ? C[cd.plane + off] : 0.0;
}

struct NodeStencil {
    float c[2], gcx[2], gcy[2], lc[2];
    float rho, grx, gry;
    float mu[3];
};

// Central-difference stencils of C_i and rho and the chemical potentials at
// an in-domain node, from a C field given by `get(x, y, c1, c2)`, in the
// arithmetic of the step kernel's phase B: grad C_i from the float32-rounded
// C_i, lap C_i from the float64 field (rounded once), rho from the float64
// C_i, grad rho from the float32 rho of the neighbours.
template <class Get>
__device__ __forceinline__ NodeStencil stencil_at(const CaseDev& cd, int x, int y, Get get) {
    NodeStencil n;
    double q1[9], q2[9];
    float f1[9], f2[9], r[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const int xa = x + Lat::ex[a];
        get(cd.openx ? mirror_y(xa, cd.nx) : wrap_x(xa, cd.nx), mirror_y(y + Lat::ey[a], cd.ny), q1[a], q2[a]);
        f1[a] = (float)q1[a];
        f2[a] = (float)q2[a];
        r[a] = mix_rho(cd, q1[a], q2[a]);
    }
    n.c[0] = f1[0];
    n.c[1] = f2[0];
    n.rho = r[0];
    cd_grad9(f1, n.gcx[0], n.gcy[0]);
    n.lc[0] = cd_lap9_d(q1);
    if (cd.n_h == 2) {
        cd_grad9(f2, n.gcx[1], n.gcy[1]);
        n.lc[1] = cd_lap9_d(q2);
    } else {
        n.gcx[1] = n.gcy[1] = n.lc[1] = 0.0f;
    }
    cd_grad9(r, n.grx, n.gry);
    if (cd.n_h == 1) chem_potential<1>(cd, q1[0], q2[0], n.lc[0], n.lc[1], n.mu);
    else chem_potential<2>(cd, q1[0], q2[0], n.lc[0], n.lc[1], n.mu);
    return n;
}

// sum_k mu_k grad C_k + F_b with grad C_3 = -grad C_1 - grad C_2, in the
// step kernel's order of operations.
__device__ __forceinline__ void node_force(const CaseDev& cd, const NodeStencil& n, float& fx, float& fy) {
    fx = (n.mu[0] - n.mu[2]) * n.gcx[0] + n.rho * cd.fx;
    fy = (n.mu[0] - n.mu[2]) * n.gcy[0] - n.rho * cd.g;
    if (cd.n_h == 2) {
        fx += (n.mu[1] - n.mu[2]) * n.gcx[1];
        fy += (n.mu[1] - n.mu[2]) * n.gcy[1];
    }
}

// rho, u, p of an in-domain node from the current state (Eqs. (23), (24)),
// rounded as in the step kernel.
__device__ __forceinline__ void node_macro(const CaseDev& cd, int par, int x, int y, NodeStencil& n, float& ux,
                                           float& uy, float& p) {
    const double* C = cd.C[par];
    n = stencil_at(cd, x, y, [&](int xx, int yy, double& a, double& b) { load_c(cd, C, xx, yy, a, b); });
    const long long off = (long long)y * cd.pitch + x;
    float d[9];
    load_devs(cd, par, off, d);
    const double s = cd.P[par][off];
    const float jx = d[1] - d[3] + d[5] - d[6] - d[7] + d[8];
    const float jy = d[2] - d[4] + d[5] + d[6] - d[7] - d[8];
    float fx, fy;
    node_force(cd, n, fx, fy);
    const float rr = rcp(n.rho);
    ux = (3.0f * jx + 0.5f * fx) * rr;
    uy = (3.0f * jy + 0.5f * fy) * rr;
    // the step keeps p - p_ref; the reference is added back in float64
    const float pr = (float)s + 0.5f * kCs2 * (ux * n.grx + uy * n.gry);
    p = (float)((double)pr + pref_d(cd, y));
}

// Marks the case's non-finite flag: a plain per-lane global store of 1 by
// every lane that found a non-finite value (all write the same word).
__device__ __forceinline__ void mark_nonfinite(const CaseDev& cd, bool bad) {
    if (bad) *cd.flag = 1u;
}

__global__ __launch_bounds__(kBlock) void init_kernel(const CaseDev* __restrict__ cdp, int par,
                                                      const double* __restrict__ Cin, const double* __restrict__ uin,
                                                      const double* __restrict__ pin) {
    const CaseDev& cd = *cdp;
    const int nx = cd.nx, ny = cd.ny;
    const long long q = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (q >= (long long)nx * ny) return;
    const int y = (int)(q / nx), x = (int)(q - (long long)y * nx);
    const long long n = (long long)nx * ny;
    auto getc = [&](int xx, int yy, double& a, double& b) {
        const long long k = (long long)yy * nx + xx;
        a = Cin[k];
        b = cd.n_h == 2 ? Cin[n + k] : 0.0;
    };
    const NodeStencil st = stencil_at(cd, x, y, getc);
    const float ux = uin ? (float)uin[q] : 0.0f, uy = uin ? (float)uin[n + q] : 0.0f;
    const double p = pin ? pin[q] : 0.0;
    float gpx = 0.f, gpy = 0.f;
    if (pin) {
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            const int xp = x + Lat::ex[a], xm = x - Lat::ex[a];
            const double pp = pin[(long long)mirror_y(y + Lat::ey[a], ny) * nx + (cd.openx ? mirror_y(xp, nx) : wrap_x(xp, nx))];
            const double pm = pin[(long long)mirror_y(y - Lat::ey[a], ny) * nx + (cd.openx ? mirror_y(xm, nx) : wrap_x(xm, nx))];
            const float dp = (float)(pp - pm);
            gpx += Lat::w[a] * Lat::ex[a] * dp;
            gpy += Lat::w[a] * Lat::ey[a] * dp;
        }
        gpx *= 1.5f;
        gpy *= 1.5f;
    }
    const float rho = st.rho;
    float Fx, Fy;
    node_force(cd, st, Fx, Fy);
    const float uu = ux * ux + uy * uy, ugr = ux * st.grx + uy * st.gry, uF = ux * Fx + uy * Fy;
    const float ps = 0.5f * kCs2 * ugr;                      // p - sum gbar_eq
    const float rc2 = rho * kCs2;
    const long long off = (long long)y * cd.pitch + x;
    cd.P[par][off] = p - (double)ps - pref_d(cd, y);
    float A[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const float eu = Lat::ex[a] * ux + Lat::ey[a] * uy;
        A[a] = 3.0f * eu + 4.5f * eu * eu - 1.5f * uu;
    }
    float dq[9];
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        const float wa = Lat::w[a];
        const float egr = Lat::ex[a] * st.grx + Lat::ey[a] * st.gry - ugr;
        const float eF = Lat::ex[a] * Fx + Lat::ey[a] * Fy - uF;
        dq[a] = wa * ps + rc2 * wa * A[a] - 0.5f * (kCs2 * egr * wa * A[a] + eF * wa * (1.0f + A[a]));
    }
    store_devs(cd, par, off, dq);
    double* C = cd.C[par];
    for (int i = 0; i < cd.n_h; ++i) C[i * cd.plane + off] = Cin[(long long)i * n + q];
    if (cd.H[par]) {
        const float bx = gpx - Fx, by = gpy - Fy;
        for (int i = 0; i < cd.n_h; ++i) {
            const float kk = st.c[i] / rc2;
            const float Xx = st.gcx[i] - kk * bx, Xy = st.gcy[i] - kk * by;
            const float uX = ux * Xx + uy * Xy;
#pragma unroll
            for (int a = 0; a < 9; ++a) {
                const float G = Lat::w[a] * (1.0f + A[a]);
                const float eX = Lat::ex[a] * Xx + Lat::ey[a] * Xy - uX;
                // stored as the deviation q_a = hbar_a - w_a C of the equilibrium
                cd.H[par][(long long)(i * 9 + a) * cd.plane + off] = st.c[i] * Lat::w[a] * A[a] - 0.5f * eX * G;
            }
        }
    }
    cd.T[par][off] = mixture_tau(cd, st.c[0], st.c[1], 1.0f - st.c[0] - st.c[1], 0.0f);
}

__global__ __launch_bounds__(kBlock) void macro_kernel(const CaseDev* __restrict__ cdp, int par, float* rho,
                                                       float* u, float* p, float* phi) {
    const CaseDev& cd = *cdp;
    const int nx = cd.nx, ny = cd.ny;
    const long long q = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (q >= (long long)nx * ny) return;
    const int y = (int)(q / nx), x = (int)(q - (long long)y * nx);
    const long long n = (long long)nx * ny;
    NodeStencil st;
    float ux, uy, pp;
    node_macro(cd, par, x, y, st, ux, uy, pp);
    mark_nonfinite(cd, !(isfinite(ux) && isfinite(uy) && isfinite(pp) && isfinite(st.c[0]) && isfinite(st.c[1])));
    if (rho) rho[q] = st.rho;
    if (u) { u[q] = ux; u[n + q] = uy; }
    if (p) p[q] = pp;
    if (phi)
        for (int i = 0; i < cd.n_h; ++i) phi[i * n + q] = st.c[i];
}

__global__ __launch_bounds__(kBlock) void export_kernel(const CaseDev* __restrict__ cdp, int par, float* out) {
    const CaseDev& cd = *cdp;
    const int nx = cd.nx, ny = cd.ny;
    const long long q = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (q >= (long long)nx * ny) return;
    const int y = (int)(q / nx), x = (int)(q - (long long)y * nx);
    const long long n = (long long)nx * ny, off = (long long)y * cd.pitch + x;
    const float s = (float)(cd.P[par][off] + pref_d(cd, y));
    float d0 = 0.f, dd[9];
    load_devs(cd, par, off, dd);
    for (int a = 1; a < 9; ++a) {
        const float da = dd[a];
        d0 -= da;
        out[a * n + q] = Lat::w[a] * s + da;
    }
    out[q] = Lat::w[0] * s + d0;
    bool ok = isfinite(s) && isfinite(d0);
    for (int i = 0; i < cd.n_h; ++i) {
        const double c = cd.C[par][i * cd.plane + off];
        ok = ok && isfinite(c);
        out[(9 + i) * n + q] = (float)c;
    }
    const float tau = cd.T[par][off];
    out[(9 + cd.n_h) * n + q] = tau;
    mark_nonfinite(cd, !(ok && isfinite(tau)));
}

// Scans the state of one case (level, deviations or pair moments, C_i, tau,
// stored hbar) for non-finite values and marks the case's flag.
__global__ __launch_bounds__(kBlock) void check_kernel(const CaseDev* __restrict__ cdp, int par) {
    const CaseDev& cd = *cdp;
    const int nx = cd.nx, ny = cd.ny;
    const long long q = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (q >= (long long)nx * ny) return;
    const int y = (int)(q / nx), x = (int)(q - (long long)y * nx);
    const long long off = (long long)y * cd.pitch + x;
    bool ok = isfinite(cd.P[par][off]) && isfinite(cd.T[par][off]);
    if (cd.Q[par]) {
        ok = ok && isfinite(cd.S[par][off]) && isfinite(cd.S[par][cd.plane + off]);
        for (int k = 0; k < kQPlanes; ++k) ok = ok && isfinite((float)cd.Q[par][k * cd.plane + off]);
    } else {
        for (int a = 0; a < 8; ++a) ok = ok && isfinite(cd.S[par][a * cd.plane + off]);
    }
    for (int i = 0; i < cd.n_h; ++i) ok = ok && isfinite(cd.C[par][i * cd.plane + off]);
    if (cd.H[par])
        for (int k = 0; k < 9 * cd.n_h; ++k) ok = ok && isfinite(cd.H[par][k * cd.plane + off]);
    mark_nonfinite(cd, !ok);
}

// Clears n flags (a fill kernel rather than a memset node, so that the call
// may sit inside a captured graph).
__global__ void clear_flags_kernel(unsigned int* __restrict__ flags, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flags[i] = 0u;
}

// Neumaier-compensated float64 accumulation.
struct Acc {
    double s, c;
    __device__ void add(double v) {
        const double t = s + v;
        c += fabs(s) >= fabs(v) ? (s - t) + v : (v - t) + s;
        s = t;
    }
    __device__ double value() const { return s + c; }
};

__global__ __launch_bounds__(kBlock) void reduce_kernel(const CaseDev* __restrict__ cdp, int par, int comp,
                                                        double* __restrict__ partials) {
    const CaseDev& cd = *cdp;
    const int nx = cd.nx, ny = cd.ny;
    const long long n = (long long)nx * ny;
    Acc acc[6] = {};
    for (long long q = (long long)blockIdx.x * kBlock + threadIdx.x; q < n; q += (long long)gridDim.x * kBlock) {
        const int y = (int)(q / nx), x = (int)(q - (long long)y * nx);
        NodeStencil st;
        float ux, uy, pp;
        node_macro(cd, par, x, y, st, ux, uy, pp);
        // the phase fields in float64, straight from the state (unclipped)
        const long long off = (long long)y * cd.pitch + x;
        const double c1 = cd.C[par][off], c2 = cd.n_h == 2 ? cd.C[par][cd.plane + off] : 0.0;
        const double cg = comp == 0 ? c1 : (comp == 1 ? c2 : 1.0 - c1 - c2);
        mark_nonfinite(cd, !(isfinite(ux) && isfinite(uy) && isfinite(pp) && isfinite(c1) && isfinite(c2)));
        acc[0].add(cg);
        if (cg > 0.5) acc[1].add(cg);
        acc[2].add(cg * x);
        acc[3].add(cg * y);
        acc[4].add(cg * ux);
        acc[5].add(cg * uy);
    }
    // wavefront reduction: a butterfly over the 64 lanes (lane 0's sum, the
    // one kept, is formed in the same order on every run), then one value per
    // wave through LDS, added in wave order
    constexpr int kWaves = kBlock / 64;
    __shared__ double sh[6][kWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        double v = acc[k].value();
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
        if (lane == 0) sh[k][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        double v = 0.0;
        for (int w = 0; w < kWaves; ++w) v += sh[threadIdx.x][w];
        partials[blockIdx.x * 6 + threadIdx.x] = v;
    }
}

__global__ void reduce_final_kernel(const double* __restrict__ partials, int nblocks, double* __restrict__ out) {
    const int k = threadIdx.x;
    if (k >= 6) return;
    Acc a = {};
    for (int b = 0; b < nblocks; ++b) a.add(partials[b * 6 + k]);
    out[k] = a.value();
}

unsigned grid_for(const CaseDev& cd) {
    const long long n = (long long)cd.nx * cd.ny;
    return (unsigned)((n + kBlock - 1) / kBlock);
}

}  // namespace

hipError_t launch_init(const CaseDev* cd_dev, const CaseDev& cd, int par, const double* C, const double* u,
                       const double* p, hipStream_t stream) {
    hipLaunchKernelGGL(init_kernel, dim3(grid_for(cd)), dim3(kBlock), 0, stream, cd_dev, par, C, u, p);
    return hipGetLastError();
}

hipError_t launch_macro(const CaseDev* cd_dev, const CaseDev& cd, int par, float* rho, float* u, float* p,
                        float* phi, hipStream_t stream) {
    hipLaunchKernelGGL(macro_kernel, dim3(grid_for(cd)), dim3(kBlock), 0, stream, cd_dev, par, rho, u, p, phi);
    return hipGetLastError();
}

hipError_t launch_export(const CaseDev* cd_dev, const CaseDev& cd, int par, float* out, hipStream_t stream) {
    hipLaunchKernelGGL(export_kernel, dim3(grid_for(cd)), dim3(kBlock), 0, stream, cd_dev, par, out);
    return hipGetLastError();
}

hipError_t launch_check(const CaseDev* cd_dev, const CaseDev& cd, int par, hipStream_t stream) {
    hipLaunchKernelGGL(check_kernel, dim3(grid_for(cd)), dim3(kBlock), 0, stream, cd_dev, par);
    return hipGetLastError();
}

hipError_t launch_clear_flags(unsigned int* flags, int n, hipStream_t stream) {
    hipLaunchKernelGGL(clear_flags_kernel, dim3((n + 63) / 64), dim3(64), 0, stream, flags, n);
    return hipGetLastError();
}

int reduce_blocks(const CaseDev& cd) {
    const long long n = (long long)cd.nx * cd.ny;
    long long b = (n + kBlock - 1) / kBlock;
    return (int)(b < 1024 ? b : 1024);
}

hipError_t launch_reduce(const CaseDev* cd_dev, const CaseDev& cd, int par, int comp, double* partials,
                         double* result, hipStream_t stream) {
    const int nb = reduce_blocks(cd);
    hipLaunchKernelGGL(reduce_kernel, dim3(nb), dim3(kBlock), 0, stream, cd_dev, par, comp, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(64), 0, stream, partials, nb, result);
    return hipGetLastError();
}

}  // namespace pflbm
