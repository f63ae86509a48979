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
// an in-domain node, from a C field given by `get(x, y, c1, c2)`.
template <class Get>
__device__ __forceinline__ NodeStencil stencil_at(const CaseDev& cd, int x, int y, Get get) {
    NodeStencil n;
    double d1, d2;
    get(x, y, d1, d2);
    const float c1 = (float)d1, c2 = (float)d2;
    n.c[0] = c1;
    n.c[1] = c2;
    n.rho = mix_rho(cd, d1, d2);
    float sx[2] = {0.f, 0.f}, sy[2] = {0.f, 0.f}, sl[2] = {0.f, 0.f}, rx = 0.f, ry = 0.f;
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        double q1, q2, r1, r2;
        get(wrap_x(x + Lat::ex[a], cd.nx), mirror_y(y + Lat::ey[a], cd.ny), q1, q2);
        get(wrap_x(x - Lat::ex[a], cd.nx), mirror_y(y - Lat::ey[a], cd.ny), r1, r2);
        const float p1 = (float)q1, p2 = (float)q2, m1 = (float)r1, m2 = (float)r2;
        const float w = Lat::w[a];
        sx[0] += w * Lat::ex[a] * (p1 - m1);
        sy[0] += w * Lat::ey[a] * (p1 - m1);
        sl[0] += w * ((p1 - c1) + (m1 - c1));
        sx[1] += w * Lat::ex[a] * (p2 - m2);
        sy[1] += w * Lat::ey[a] * (p2 - m2);
        sl[1] += w * ((p2 - c2) + (m2 - c2));
        const float dr = mix_rho(cd, q1, q2) - mix_rho(cd, r1, r2);
        rx += w * Lat::ex[a] * dr;
        ry += w * Lat::ey[a] * dr;
    }
    for (int i = 0; i < 2; ++i) {
        n.gcx[i] = 1.5f * sx[i];
        n.gcy[i] = 1.5f * sy[i];
        n.lc[i] = 3.0f * sl[i];
    }
    n.grx = 1.5f * rx;
    n.gry = 1.5f * ry;
    if (cd.n_h == 1) chem_potential<1>(cd, d1, d2, n.lc[0], n.lc[1], n.mu);
    else chem_potential<2>(cd, d1, d2, n.lc[0], n.lc[1], n.mu);
    return n;
}

// rho, u, p of an in-domain node from the current state (Eqs. (23), (24)).
__device__ __forceinline__ void node_macro(const CaseDev& cd, int par, int x, int y, NodeStencil& n, float& ux,
                                           float& uy, float& p) {
    const double* C = cd.C[par];
    n = stencil_at(cd, x, y, [&](int xx, int yy, double& a, double& b) { load_c(cd, C, xx, yy, a, b); });
    const long long off = (long long)y * cd.pitch + x;
    float d[9];
    load_devs(cd, par, off, d);
    const float s = (float)(cd.P[par][off] + pref_d(cd, y));
    const float jx = d[1] - d[3] + d[5] - d[6] - d[7] + d[8];
    const float jy = d[2] - d[4] + d[5] + d[6] - d[7] - d[8];
    const float mu13 = n.mu[0] - n.mu[2], mu23 = n.mu[1] - n.mu[2];
    const float fx = mu13 * n.gcx[0] + mu23 * n.gcx[1] + n.rho * cd.fx;
    const float fy = mu13 * n.gcy[0] + mu23 * n.gcy[1] - n.rho * cd.g;
    ux = (3.0f * jx + 0.5f * fx) / n.rho;
    uy = (3.0f * jy + 0.5f * fy) / n.rho;
    p = s + 0.5f * kCs2 * (ux * n.grx + uy * n.gry);
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
            const double pp = pin[(long long)mirror_y(y + Lat::ey[a], ny) * nx + wrap_x(x + Lat::ex[a], nx)];
            const double pm = pin[(long long)mirror_y(y - Lat::ey[a], ny) * nx + wrap_x(x - Lat::ex[a], nx)];
            const float dp = (float)(pp - pm);
            gpx += Lat::w[a] * Lat::ex[a] * dp;
            gpy += Lat::w[a] * Lat::ey[a] * dp;
        }
        gpx *= 1.5f;
        gpy *= 1.5f;
    }
    const float rho = st.rho;
    const float mu13 = st.mu[0] - st.mu[2], mu23 = st.mu[1] - st.mu[2];
    const float Fx = mu13 * st.gcx[0] + mu23 * st.gcx[1] + rho * cd.fx;
    const float Fy = mu13 * st.gcy[0] + mu23 * st.gcy[1] - rho * cd.g;
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
    for (int i = 0; i < cd.n_h; ++i) out[(9 + i) * n + q] = (float)cd.C[par][i * cd.plane + off];
    out[(9 + cd.n_h) * n + q] = cd.T[par][off];
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
        acc[0].add(cg);
        if (cg > 0.5) acc[1].add(cg);
        acc[2].add(cg * x);
        acc[3].add(cg * y);
        acc[4].add(cg * ux);
        acc[5].add(cg * uy);
    }
    __shared__ double sh[6][kBlock];
    for (int k = 0; k < 6; ++k) sh[k][threadIdx.x] = acc[k].value();
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 6; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 6; ++k) partials[blockIdx.x * 6 + k] = sh[k][0];
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
