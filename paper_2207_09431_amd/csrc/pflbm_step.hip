// pflbm_step.hip -- fused collide-stream step kernel for gfx950.
//
// One work-group advances a TX x TY tile of output nodes by one time step of
// the method of arXiv 2207.09431, Sec. 2 (pull streaming).  The tile stages
// its neighbourhood through LDS in four phases:
//   A  C_i and rho on the tile plus a 3-node halo (periodic x, mirrored rows
//      beyond the walls);
//   B  on the 2-node halo: central-difference stencils of C_i and rho, the
//      chemical potentials (Eq. (5)), the velocity and pressure moments
//      (Eqs. (23), (24) with the 1/2 factor on u.grad rho) from the gbar state;
//   C  on the 1-node halo: grad p, grad mu, lap mu, the diffusion source of
//      Eq. (21) (product form, or in the extended instances optionally the
//      conservative link form), mixed directional derivatives of rho and
//      C_i, the shear rate from the non-equilibrium second moment with the
//      previous tau
//      (Eqs. (25)-(29)), the truncated power-law viscosity (Eqs. (31), (33))
//      mixed harmonically across the interface into tau (optionally with
//      fixed-point passes of Eq. (32)) and the post-collision populations of
//      gbar (Eq. (14)) and hbar (Eq. (18));
//   D  on the tile: gather the post-collision populations (half-way
//      bounce-back at the walls), add the receiving-node half of the
//      diffusion term and write the new state.
// gbar is carried as its level s = sum gbar (float64, against the liquid's
// hydrostatic profile) plus float32 deviations d_a = gbar_a - w_a s, so that
// the momentum moment is formed from small numbers (at density ratio 1000
// the gas momentum is orders of magnitude below the level).  All global loads
// of a tile are issued in phase A; phase C reads its node's state from LDS,
// where phase B parks it.
#include <type_traits>

#include "pflbm_internal.h"

namespace pflbm {

// Isotropic central stencils over the four lattice direction pairs on an LDS
// array with row pitch W: grad f = sum_a w_a e_a [f(x+e_a) - f(x-e_a)] / (2 c_s^2)
// and lap f = sum_a w_a [f(x+e_a) - 2 f(x) + f(x-e_a)] / c_s^2, each pair
// (a, opposite of a) contributing once with twice its weight.
template <int W>
__device__ __forceinline__ void cd_grad(const float* f, int i, float& gx, float& gy) {
    const float d1 = f[i + 1] - f[i - 1], d2 = f[i + W] - f[i - W];
    const float d5 = f[i + W + 1] - f[i - W - 1], d6 = f[i + W - 1] - f[i - W + 1];
    gx = (1.0f / 3.0f) * d1 + (1.0f / 12.0f) * (d5 - d6);
    gy = (1.0f / 3.0f) * d2 + (1.0f / 12.0f) * (d5 + d6);
}
// The Laplacian of the float64 phase field, rounded once: it sets the
// gradient part of mu, which inside a bubble (C = 1 - O(1e-5)) is as small as
// the bulk part, and the float32 copy's spacing there would be a 1 % error.
template <int W>
__device__ __forceinline__ float cd_lap_d(const double* f, int i) {
    const double c = f[i];
    const double s1 = (f[i + 1] - c) + (f[i - 1] - c), s2 = (f[i + W] - c) + (f[i - W] - c);
    const double s5 = (f[i + W + 1] - c) + (f[i - W - 1] - c), s6 = (f[i + W - 1] - c) + (f[i - W + 1] - c);
    return (float)((2.0 / 3.0) * (s1 + s2) + (1.0 / 6.0) * (s5 + s6));
}
template <int W>
__device__ __forceinline__ float cd_lap(const float* f, int i) {
    const float c = f[i];
    const float s1 = (f[i + 1] - c) + (f[i - 1] - c), s2 = (f[i + W] - c) + (f[i - W] - c);
    const float s5 = (f[i + W + 1] - c) + (f[i - W - 1] - c), s6 = (f[i + W - 1] - c) + (f[i - W + 1] - c);
    return (2.0f / 3.0f) * (s1 + s2) + (1.0f / 6.0f) * (s5 + s6);
}
// e_a . v for a compile-time lattice vector (no multiplications by 0 or 1).
__device__ __forceinline__ float edot(int ex, int ey, float vx, float vy) {
    if (ex == 0 && ey == 0) return 0.0f;
    if (ex == 0) return ey > 0 ? vy : -vy;
    if (ey == 0) return ex > 0 ? vx : -vx;
    const float t = ex > 0 ? vx : -vx;
    return ey > 0 ? t + vy : t - vy;
}
// The mixed directional derivatives of md_all (below) from the float64
// phase field: near C = 1 the float32 copy is
// spaced 6e-8, which the 5/4-weighted stencil turns into derivative noise of
// that size, a random walk of the component mass and a velocity error at the
// bubble rims; the stencil is therefore taken in float64 and rounded once.
// Returns four times the derivatives (q_a = 4 d_a f, exact scaling) so that
// each takes three float64 operations; the callers fold the 1/4 into their
// coefficients, and the gradient is the true one.
template <int W>
__device__ __forceinline__ void md_all_d4(const double* f, int i, float q[9], float& gx, float& gy) {
    q[0] = 0.0f;
    const double m3 = -3.0 * f[i];
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        const int o = Lat::ey[a] * W + Lat::ex[a];
        q[a] = (float)((fma(5.0, f[i + o], -f[i + 2 * o]) - f[i - o]) + m3);
    }
    const float p5 = q[5] - q[7], p6 = q[6] - q[8];
    gx = (1.0f / 12.0f) * (q[1] - q[3]) + (1.0f / 48.0f) * (p5 - p6);
    gy = (1.0f / 12.0f) * (q[2] - q[4]) + (1.0f / 48.0f) * (p5 + p6);
}

// Mixed directional derivatives along e_1..e_8 (mean of the central and the
// second-order biased differences) and the mixed gradient
// grad^MD f = sum_a w_a e_a d_a f / c_s^2 built from them.
template <int W>
__device__ __forceinline__ void md_all(const float* f, int i, float d[9], float& gx, float& gy) {
    d[0] = 0.0f;
    const float fc = -0.75f * f[i];
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        const int o = Lat::ey[a] * W + Lat::ex[a];
        // [-f(x+2e) + 5 f(x+e) - 3 f(x) - f(x-e)] / 4
        d[a] = fmaf(0.25f, fmaf(5.0f, f[i + o], -f[i + 2 * o]) - f[i - o], fc);
    }
    const float p5 = d[5] - d[7], p6 = d[6] - d[8];
    gx = (1.0f / 3.0f) * (d[1] - d[3]) + (1.0f / 12.0f) * (p5 - p6);
    gy = (1.0f / 3.0f) * (d[2] - d[4]) + (1.0f / 12.0f) * (p5 + p6);
}

// Thread-to-node order on a region of width TX + 2h: the TX middle columns
// first, a row of TX nodes per TX threads, so that (for TX = 32) every
// half-wave (32 lanes) reads 32 consecutive LDS words of one row and the
// stencil reads of the other regions (row pitches TX + 2..6) meet no bank
// conflict; the 2h edge columns of every row follow.  Returns the
// region-linear index.
template <int TX, int H>
__device__ __forceinline__ int region_node(int n, int rows, int& rx, int& ry) {
    constexpr int W = TX + 2 * H;
    const int main = rows * TX;
    if (n < main) {
        ry = n / TX;
        rx = n - ry * TX + H;
    } else {
        const int e = n - main;
        ry = e / (2 * H);
        const int c = e - ry * (2 * H);
        rx = c < H ? c : TX + c;
    }
    return ry * W + rx;
}

template <int TX, int TY, int NH, bool SH, bool F16, int NT, bool EXT>
__global__ __launch_bounds__(NT) void step_kernel(const CaseDev* __restrict__ cases,
                                                  const TileDev* __restrict__ tiles, int ntiles, int par) {
    constexpr int W3 = TX + 6, H3 = TY + 6, N3 = W3 * H3;
    constexpr int W2 = TX + 4, H2 = TY + 4, N2 = W2 * H2;
    constexpr int W1 = TX + 2, H1 = TY + 2, N1 = W1 * H1;
    constexpr int NMU = NH + 1;      // mu_1 (, mu_2), mu_3

    __shared__ float sC[NH][N3];
    __shared__ double sCd[NH][N3];   // the float64 phase field on R3
    __shared__ float sR[N3];
    __shared__ float sMu[NMU][N2];
    __shared__ float sUx[N2], sUy[N2], sP[N2];
    __shared__ float sD[9][N1];      // post-collision deviations d*_a
    __shared__ double sS[N1];        // s - p_ref at the source (float64)
    // post-collision hbar: without the (1-omega_h) hbar part when hbar is
    // stored, else as its deviation from w_a C at the source
    __shared__ float sH[NH][9][N1];
    __shared__ float sDif[NH][N1];

    // XCD-aware order: consecutive tiles land on the same XCD (work-groups are
    // dealt to the 8 XCDs round-robin).
    int t;
    {
        const int i = blockIdx.x, k = i & 7, j = i >> 3, q = ntiles >> 3, r = ntiles & 7;
        t = k * q + (k < r ? k : r) + j;
    }
    const TileDev tile = tiles[t];
    const CaseDev& cd = cases[tile.case_id];
    const int nx = cd.nx, ny = cd.ny, pitch = cd.pitch;
    const long long plane = cd.plane;
    const int x0 = tile.x0, y0 = tile.y0;
    const double* Pin = cd.P[par];
    const float* Sin = cd.S[par];
    const double* Cin = cd.C[par];
    const float* Tin = cd.T[par];
    double* Pout = cd.P[par ^ 1];
    float* Sout = cd.S[par ^ 1];
    double* Cout = cd.C[par ^ 1];
    float* Tout = cd.T[par ^ 1];
    const float* Hin = cd.H[par];
    float* Hout = cd.H[par ^ 1];
    const _Float16* Qin = cd.Q[par];
    _Float16* Qout = cd.Q[par ^ 1];
    const float qinv = cd.qinv, qscale = cd.qscale;
    const int tid = threadIdx.x;
    // open x (velocity inlet at x = 0, outflow at x = nx-1; extended
    // instances): stencil ghosts mirror in x like the walls' rows, and the
    // boundary columns are completed in phase D
    const bool openx = EXT && cd.openx != 0;
    // tiles whose regions reach beyond an open end (uniform per work-group)
    const bool xedge = openx && (x0 < 3 || x0 + TX + 3 > nx);

    // ---------------- phase A: C_i and rho on R3
    // All global loads of phases A and B are issued here, phase A's first, so
    // that the latency of the gbar loads (consumed in phase B) overlaps
    // phase A.  Thread tid owns the R3 nodes idx = tid + k NT (linear order)
    // and the R2 nodes numbered tid + k NT in the row order of region_node,
    // the order in which phase B consumes them.  The loads are unconditional (surplus threads and rows beyond the walls
    // read a valid node and discard it) so that no branch forces an early wait.
    constexpr int KA = (N3 + NT - 1) / NT, KB = (N2 + NT - 1) / NT;
    constexpr int ND = F16 ? 2 + kQPlanes : 8;
    double ca[KA][NH];
    double ps[KB];
    float pd[KB][ND], pt[KB];
    // Element offset of region node (rx, ry) of the region with halo h: tiles
    // whose regions stay clear of the walls and of the periodic seam take the
    // plain offset, the others wrap x and mirror y.
    auto loads = [&](auto plain_tag) {
        constexpr bool PLAIN = decltype(plain_tag)::value;
        auto node = [&](int rx, int ry, int h) -> uint32_t {
            if (PLAIN) return (uint32_t)((y0 - h + ry) * pitch + (x0 - h + rx));
            const int xr = x0 - h + rx;
            return (uint32_t)(mirror_y(y0 - h + ry, ny) * pitch + (openx ? mirror_y(xr, nx) : wrap_x_tile(xr, nx)));
        };
#pragma unroll
        for (int k = 0; k < KA; ++k) {
            const int idx = min(tid + k * NT, N3 - 1);
            const int ry = idx / W3, rx = idx - ry * W3;
            const uint32_t eo = node(rx, ry, 3);
#pragma unroll
            for (int i = 0; i < NH; ++i) ca[k][i] = gld(Cin + i * plane, eo * 8u);
        }
        // gbar state of the R2 nodes: s, the momentum and (used for the R1
        // nodes) the rest of the deviations and tau
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            int rx, ry;
            region_node<TX, 2>(min(tid + k * NT, N2 - 1), H2, rx, ry);
            const uint32_t eo = node(rx, ry, 2);
            ps[k] = gld(Pin, eo * 8u);
            if (F16) {
                pd[k][0] = gld(Sin, eo * 4u);
                pd[k][1] = gld(Sin + plane, eo * 4u);
#pragma unroll
                for (int q = 0; q < kQPlanes; ++q) pd[k][2 + q] = (float)gld(Qin + q * plane, eo * 2u);
            } else {
#pragma unroll
                for (int a = 1; a < 9; ++a) pd[k][a - 1] = gld(Sin + (a - 1) * plane, eo * 4u);
            }
            pt[k] = gld(Tin, eo * 4u);
        }
    };
    if (x0 >= 3 && x0 + TX + 3 <= nx && y0 >= 3 && y0 + TY + 3 <= ny) loads(std::true_type{});
    else loads(std::false_type{});
    // surplus threads (idx >= N3) repeat node N3 - 1: same address, same value
#pragma unroll
    for (int k = 0; k < KA; ++k) {
        const int idx = min(tid + k * NT, N3 - 1);
        const double d1 = ca[k][0];
        const double d2 = NH == 2 ? ca[k][NH - 1] : 0.0;
        sC[0][idx] = (float)d1;
        sCd[0][idx] = d1;
        if (NH == 2) { sC[NH - 1][idx] = (float)d2; sCd[NH - 1][idx] = d2; }
        sR[idx] = mix_rho(cd, d1, d2);
    }
    __syncthreads();

    // ---------------- phase B: mu, u, p on R2; the gbar state and tau of the
    // R1 nodes are parked in sD, sS and sDif, which phase C reads and then
    // overwrites node by node
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        if (tid + k * NT >= N2) continue;
        int rx, ry;
        const int idx = region_node<TX, 2>(tid + k * NT, H2, rx, ry);
        const int i3 = (ry + 1) * W3 + rx + 1;
        const int gyr = y0 - 2 + ry;
        float gcx[2] = {0.f, 0.f}, gcy[2] = {0.f, 0.f}, lc[2] = {0.f, 0.f};
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            cd_grad<W3>(sC[i], i3, gcx[i], gcy[i]);
            lc[i] = cd_lap_d<W3>(sCd[i], i3);
        }
        float mu[3];
        chem_potential<NH>(cd, sCd[0][i3], NH == 2 ? sCd[NH - 1][i3] : 0.0, lc[0], lc[1], mu);
        sMu[0][idx] = mu[0];
        if (NH == 2) sMu[1][idx] = mu[1];
        sMu[NH][idx] = mu[2];
        if (gyr >= 0 && gyr < ny) {
            const double s = ps[k];
            float jx, jy;
            float d[9];
            if (F16) {
                jx = pd[k][0];
                jy = pd[k][1];
            } else {
#pragma unroll
                for (int a = 1; a < 9; ++a) d[a] = pd[k][a - 1];
                jx = d[1] - d[3] + d[5] - d[6] - d[7] + d[8];
                jy = d[2] - d[4] + d[5] + d[6] - d[7] - d[8];
            }
            const bool in_r1 = rx >= 1 && rx <= W2 - 2 && ry >= 1 && ry <= H2 - 2;
            const int i1 = (ry - 1) * W1 + rx - 1;
            if (in_r1) {
                if (F16) {
                    float m[kQPlanes];
#pragma unroll
                    for (int q = 0; q < kQPlanes; ++q) m[q] = pd[k][2 + q] * qinv;
                    unpack_devs(jx, jy, m, d);
                }
#pragma unroll
                for (int a = 1; a < 9; ++a) sD[a][i1] = d[a];
                sS[i1] = s;
                sDif[0][i1] = pt[k];
            }
            float grx, gry;
            cd_grad<W3>(sR, i3, grx, gry);
            const float rho = sR[i3];
            // sum_k mu_k grad C_k with grad C_3 = -grad C_1 - grad C_2
            float fx = (mu[0] - mu[2]) * gcx[0] + rho * cd.fx;
            float fy = (mu[0] - mu[2]) * gcy[0] - rho * cd.g;
            if (NH == 2) {
                fx += (mu[1] - mu[2]) * gcx[1];
                fy += (mu[1] - mu[2]) * gcy[1];
            }
            const float rr = rcp(rho);
            const float ux = (3.0f * jx + 0.5f * fx) * rr;
            const float uy = (3.0f * jy + 0.5f * fy) * rr;
            sUx[idx] = ux;
            sUy[idx] = uy;
            if (in_r1) {
                // grad C_i, grad rho and the force of the R1 nodes, parked in
                // the hbar planes (written only later, by phase C)
                sH[0][0][i1] = gcx[0];
                sH[0][1][i1] = gcy[0];
                sH[0][2][i1] = grx;
                sH[0][3][i1] = gry;
                sH[0][4][i1] = fx;
                sH[0][5][i1] = fy;
                if (NH == 2) {
                    sH[0][6][i1] = gcx[1];
                    sH[0][7][i1] = gcy[1];
                }
            }
            sP[idx] = (float)s + 0.5f * kCs2 * (ux * grx + uy * gry);
        }
    }
    __syncthreads();
    // with open x the two ghost columns beyond each end mirror the end
    // columns for grad p (same row: no reference difference)
    if (openx && (x0 < 2 || x0 + TX + 2 > nx)) {
        for (int idx = tid; idx < N2; idx += NT) {
            const int ry = idx / W2, rx = idx - ry * W2;
            const int gxr = x0 - 2 + rx, gyr = y0 - 2 + ry;
            if ((gxr < 0 || (gxr >= nx && gxr < nx + 2)) && gyr >= 0 && gyr < ny)
                sP[idx] = sP[ry * W2 + (mirror_y(gxr, nx) - (x0 - 2))];
        }
        __syncthreads();
    }
    // the two ghost rows beyond each wall mirror the wall rows for grad p
    // (rows farther out are never read); only tiles next to a wall have them
    if (y0 < 2 || y0 + TY + 2 > ny) {
        for (int idx = tid; idx < N2; idx += NT) {
            const int ry = idx / W2, rx = idx - ry * W2;
            const int gyr = y0 - 2 + ry;
            if ((gyr < 0 && gyr >= -2) || (gyr >= ny && gyr < ny + 2)) {
                // p mirrors; sP holds p - p_ref, so the reference's difference is added
                const int ym = mirror_y(gyr, ny);
                sP[idx] = sP[(ym - (y0 - 2)) * W2 + rx] + cd.pref_g * (float)(gyr - ym);
            }
        }
        __syncthreads();
    }

    // ---------------- phase C: collisions on R1
    for (int n = tid; n < N1; n += NT) {
        int rx, ry;
        const int idx = region_node<TX, 1>(n, H1, rx, ry);
        const int gyr = y0 - 1 + ry;
        if (gyr < 0 || gyr >= ny) continue;   // nodes beyond the walls are never sources
        // nor, with open x, nodes beyond the ends (their populations are replaced)
        if (xedge) {
            if (x0 - 1 + rx < 0 || x0 - 1 + rx >= nx) continue;
        }
        const int i2 = (ry + 1) * W2 + rx + 1;
        const int i3 = (ry + 2) * W3 + rx + 2;

        float d[9];
#pragma unroll
        for (int a = 1; a < 9; ++a) d[a] = sD[a][idx];
        d[0] = -(d[1] + d[2] + d[3] + d[4] + d[5] + d[6] + d[7] + d[8]);
        const float tprev = sDif[0][idx];

        // central gradients of C_i and rho and the force (parked by phase B),
        // moments and potentials of the node
        float c[2] = {0.f, 0.f}, gcx[2] = {0.f, 0.f}, gcy[2] = {0.f, 0.f};
#pragma unroll
        for (int i = 0; i < NH; ++i) c[i] = sC[i][i3];
        gcx[0] = sH[0][0][idx];
        gcy[0] = sH[0][1][idx];
        if (NH == 2) {
            gcx[1] = sH[0][6][idx];
            gcy[1] = sH[0][7][idx];
        }
        const float grx = sH[0][2][idx], gry = sH[0][3][idx];
        const float Fx = sH[0][4][idx], Fy = sH[0][5][idx];
        const float c3 = 1.0f - c[0] - c[1];
        const float rho = sR[i3];
        float gpx, gpy;
        cd_grad<W2>(sP, i2, gpx, gpy);
        gpy -= cd.pref_g;   // sP holds p - p_ref, and grad p_ref = (0, -rho_3 g) exactly
        const float mu1 = sMu[0][i2], mu3 = sMu[NH][i2];
        const float mu2 = NH == 2 ? sMu[1][i2] : 0.0f;
        const float ux = sUx[i2], uy = sUy[i2];

        // diffusion source Dif_i = div(D_i grad mu_i) in the product form of Eq. (21)
        float dif[2] = {0.f, 0.f};
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            float mx, my;
            cd_grad<W2>(sMu[i], i2, mx, my);
            const float lapmu = cd_lap<W2>(sMu[i], i2);
            if (EXT && cd.mflux) {
                // conservative link form (extended instances):
                //   sum_a w_a (D(x) + D(x+e_a)) (mu(x+e_a) - mu(x)) / c_s^2,
                // D = mob C (1 - C) with C limited to [0, 1], or mob when constant
                auto shape = [&](int j) {
                    if (!cd.vm) return 1.0f;
                    const float q = clip01(sC[i][j]);
                    return q - q * q;
                };
                const float m0 = shape(i3), u0 = sMu[i][i2];
                float acc = 0.0f;
#pragma unroll
                for (int a = 1; a < 9; ++a) {
                    const int o2 = Lat::ey[a] * W2 + Lat::ex[a], o3 = Lat::ey[a] * W3 + Lat::ex[a];
                    acc = fmaf(Lat::w[a] * (m0 + shape(i3 + o3)), sMu[i][i2 + o2] - u0, acc);
                }
                dif[i] = cd.mob[i] * (3.0f * acc);
            } else if (cd.vm) {
                // grad of C_i - C_i^2 with C_i limited to [0, 1]
                auto sf = [&](int j) { const float q = clip01(sC[i][j]); return q - q * q; };
                const float e1 = sf(i3 + 1) - sf(i3 - 1), e2 = sf(i3 + W3) - sf(i3 - W3);
                const float e5 = sf(i3 + W3 + 1) - sf(i3 - W3 - 1), e6 = sf(i3 + W3 - 1) - sf(i3 - W3 + 1);
                const float sgx = (1.0f / 3.0f) * e1 + (1.0f / 12.0f) * (e5 - e6);
                const float sgy = (1.0f / 3.0f) * e2 + (1.0f / 12.0f) * (e5 + e6);
                const float cl = clip01(c[i]);
                dif[i] = cd.mob[i] * (cl * (1.0f - cl) * lapmu + (sgx * mx + sgy * my));
            } else {
                dif[i] = cd.mob[i] * lapmu;
            }
        }

        // mixed directional derivatives along every e_a (radius 2) and their gradients
        float drho[9], dc[2][9], mrx, mry, mcx[2] = {0.f, 0.f}, mcy[2] = {0.f, 0.f};
        md_all<W3>(sR, i3, drho, mrx, mry);
#pragma unroll
        for (int i = 0; i < NH; ++i) md_all_d4<W3>(sCd[i], i3, dc[i], mcx[i], mcy[i]);   // dc = 4 d_a C_i
        if (NH == 1) {
#pragma unroll
            for (int a = 0; a < 9; ++a) dc[1][a] = 0.0f;
        } else {
            // two phase fields: each d_a C_i waits in that component's own hbar
            // planes at this node (free once the parked values were read) and is
            // read back where it is used, so that the collision does not hold
            // both sets of nine in registers
#pragma unroll
            for (int i = 0; i < NH; ++i)
#pragma unroll
                for (int a = 1; a < 9; ++a) sH[i][a][idx] = dc[i][a];
        }

        // force, equilibrium and the non-equilibrium part.  With
        // A_a = Gamma_a / w_a - 1 (so w_a A_a = Gamma_a - w_a) the deviation
        // equilibrium  w_a ps + w_a A_a (rho c_s^2 - c_s^2 (e_a-u).grad rho / 2)
        //              - (e_a-u).F Gamma_a / 2
        // is w_a (E_a + A_a R_a) with E_a = ps - (e_a-u).F / 2 and
        // R_a = rho c_s^2 - (e_a-u).(c_s^2 grad rho + F) / 2, both affine in e_a.
        const float mu13 = mu1 - mu3, mu23 = mu2 - mu3;
        const float fbx = rho * cd.fx, fby = -rho * cd.g;
        const float uu = ux * ux + uy * uy;
        const float ugr = ux * grx + uy * gry;
        const float uF = ux * Fx + uy * Fy;
        const float ps = 0.5f * kCs2 * ugr;          // p - s
        const float hFx = 0.5f * Fx, hFy = 0.5f * Fy;
        const float Vx = fmaf(0.5f * kCs2, grx, hFx), Vy = fmaf(0.5f * kCs2, gry, hFy);
        const float E0 = fmaf(0.5f, uF, ps);
        const float R0 = fmaf(rho, kCs2, E0);        // rho c_s^2 + c_s^2 u.grad rho / 2 + u.F / 2
        const float uu15 = -1.5f * uu;
        float A[9], ne[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const int ex = Lat::ex[a], ey = Lat::ey[a];
            const float eu = edot(ex, ey, ux, uy);
            A[a] = fmaf(eu, fmaf(4.5f, eu, 3.0f), uu15);
            const float R = R0 - edot(ex, ey, Vx, Vy);
            const float E = E0 - edot(ex, ey, hFx, hFy);
            ne[a] = fmaf(-Lat::w[a], fmaf(A[a], R, E), d[a]);
        }
        // The zeroth and first moments of the non-equilibrium part vanish
        // exactly (u and p are the moments of this gbar); the float32 rounding
        // left in them, m0 and m, is projected out, ne_a -> ne_a - w_a (m0 +
        // 3 e_a.m), so that the collision conserves the pressure and momentum
        // moments to the rounding of small numbers instead of leaking a
        // systematic residue every step.  The projection lowers Pi_xx and
        // Pi_yy by c_s^2 m0 and is applied inside the collision below.
        const float m0 = ((ne[0] + ne[1]) + (ne[2] + ne[3])) + ((ne[4] + ne[5]) + (ne[6] + ne[7])) + ne[8];
        const float mx = (ne[1] - ne[3]) + ((ne[5] - ne[7]) + (ne[8] - ne[6]));
        const float my = (ne[2] - ne[4]) + ((ne[5] - ne[7]) + (ne[6] - ne[8]));
        const float pdiag = ne[5] + ne[6] + ne[7] + ne[8];
        const float pxx = fmaf(-kCs2, m0, ne[1] + ne[3] + pdiag), pyy = fmaf(-kCs2, m0, ne[2] + ne[4] + pdiag);
        const float pxy = ne[5] - ne[6] + ne[7] - ne[8];
        // shear rate: D = -Pi / (2 (tau_prev + 1/2) rho c_s^4), gdot = sqrt(2 D:D)
        const float fs = 4.5f * rcp((tprev + 0.5f) * rho);
        // hardware square root (1 ulp): the rate enters only the power law
        const float pin = __builtin_amdgcn_sqrtf(2.0f * (pxx * pxx + pyy * pyy + 2.0f * pxy * pxy));
        float tau = mixture_tau(cd, c[0], c[1], c3, fs * pin);
        // optional fixed-point passes of the implicit relation tau = tau(gdot(tau))
        // (Sec. 2.3, Eq. (32)), started from the previous step's tau; only in
        // the extended instances, so that the default path has no loop here
        if (EXT)
            for (int it = 0; it < cd.tau_iters; ++it)
                tau = mixture_tau(cd, c[0], c[1], c3, 4.5f * rcp((tau + 0.5f) * rho) * pin);
        const float om = rcp(tau + 0.5f);

        // gbar collision with the mixed-difference forcing:
        //   d*_a = d_a - om (ne_a - w_a (m0 + 3 e_a.m)) + c_s^2 (d_a rho - u.grad^MD rho) w_a A_a
        //          + [sum_k mu_k (d_a C_k - u.grad^MD C_k) + (e_a-u).F_b] w_a (1 + A_a)
        //        = d_a - om ne_a + w_a [Z_a + t_a + A_a (K_a + t_a)]
        const float umr = ux * mrx + uy * mry;
        const float um1 = ux * mcx[0] + uy * mcy[0], um2 = ux * mcx[1] + uy * mcy[1];
        float T0 = -(ux * fbx + uy * fby) - mu13 * um1;
        if (NH == 2) T0 -= mu23 * um2;
        const float Z0 = om * m0, Zx = 3.0f * om * mx, Zy = 3.0f * om * my;
        const float cum = -kCs2 * umr;
        const float mu13q = 0.25f * mu13, mu23q = 0.25f * mu23;   // dc holds 4 d_a C
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const int ex = Lat::ex[a], ey = Lat::ey[a];
            const float K = fmaf(kCs2, drho[a], cum);
            const float dc0 = NH == 2 ? (a == 0 ? 0.0f : sH[0][a][idx]) : dc[0][a];
            float t = fmaf(mu13q, dc0, T0 + edot(ex, ey, fbx, fby));
            if (NH == 2) t = fmaf(mu23q, a == 0 ? 0.0f : sH[1][a][idx], t);
            const float br = fmaf(A[a], K + t, (Z0 + edot(ex, ey, Zx, Zy)) + t);
            sD[a][idx] = fmaf(Lat::w[a], br, fmaf(-om, ne[a], d[a]));
        }

        // hbar collision: equilibrium with central differences, forcing with the
        // mixed derivative of C_i and central grad p, source half of Dif.
        //   X = grad C_i - (C_i / (rho c_s^2)) (grad p - F),
        //   forcing (d_a C_i - u.grad^MD C_i) - (C_i/(rho c_s^2)) (e_a-u).(grad p - F)
        const float bx = gpx - Fx, by = gpy - Fy;
        const float ub = ux * bx + uy * by;
        const float r3 = 3.0f * rcp(rho);
        // The forcing's (e_a-u).grad C_i takes the mixed directional
        // derivatives (the default) or, with hforce_cd (extended instances),
        // central differences: then e_a.grad C_i joins the terms affine in
        // e_a.  One copy of the block per choice, selected by a uniform branch.
        auto hbar_block = [&](auto cd_tag) {
            constexpr bool HCD = decltype(cd_tag)::value;
#pragma unroll
            for (int i = 0; i < NH; ++i) {
                const float kk = c[i] * r3;                // C_i / (rho c_s^2)
                const float Xx = gcx[i] - kk * bx, Xy = gcy[i] - kk * by;
                const float uX = ux * Xx + uy * Xy;
                const float umc = HCD ? ux * gcx[i] + uy * gcy[i] : ((i == 0) ? um1 : um2);
                const float fgx = HCD ? gcx[i] : 0.0f, fgy = HCD ? gcy[i] : 0.0f;
                if (SH) {
                    // stored hbar_a = w_a C + q_a: hbar*_a = w_a C + (1 - omega_h) q_a + Q_a with
                    //   Q_a = omega_h w_a A_a C + Gamma_a [-omega_h (e_a-u).X / 2 + forcing + Dif / 2]
                    //       = w_a [H_a + A_a (omega_h C + H_a)];  Q_a is parked, the q_a term is
                    // added by the receiver, and w_a C streams in float64 there
                    const float oh = cd.omh;
                    const float H0 = fmaf(0.5f * oh, uX, fmaf(kk, ub, 0.5f * dif[i])) - umc;
                    const float Hx = fmaf(0.5f * oh, Xx, kk * bx) - fgx, Hy = fmaf(0.5f * oh, Xy, kk * by) - fgy;
                    const float oc = oh * c[i];
#pragma unroll
                    for (int a = 0; a < 9; ++a) {
                        const float dca = NH == 2 ? (a == 0 ? 0.0f : sH[i][a][idx]) : dc[i][a];
                        const float H = (HCD ? H0 : fmaf(0.25f, dca, H0)) - edot(Lat::ex[a], Lat::ey[a], Hx, Hy);
                        sH[i][a][idx] = Lat::w[a] * fmaf(A[a], oc + H, H);
                    }
                } else {
                    // omega_h = 1: hbar* - w_a C = w_a A_a C + Gamma_a H_a
                    //   = w_a [H_a + A_a (C + H_a)],  H_a = -(e_a-u).X / 2 + forcing + Dif / 2
                    // (the weight is applied here: applied by the receiver instead, inside
                    // its sum, it triples the component mass drift, measured)
                    const float H0 = fmaf(0.5f, uX, fmaf(kk, ub, 0.5f * dif[i])) - umc;
                    const float Hx = fmaf(0.5f, Xx, kk * bx) - fgx, Hy = fmaf(0.5f, Xy, kk * by) - fgy;
#pragma unroll
                    for (int a = 0; a < 9; ++a) {
                        const float dca = NH == 2 ? (a == 0 ? 0.0f : sH[i][a][idx]) : dc[i][a];
                        const float H = (HCD ? H0 : fmaf(0.25f, dca, H0)) - edot(Lat::ex[a], Lat::ey[a], Hx, Hy);
                        sH[i][a][idx] = Lat::w[a] * fmaf(A[a], c[i] + H, H);
                    }
                }
                sDif[i][idx] = dif[i];
            }
        };
        if (EXT && cd.hcd) hbar_block(std::true_type{});
        else hbar_block(std::false_type{});
        // tau is written for the tile's own nodes
        const int ox = rx - 1, oy = ry - 1;
        if (ox >= 0 && ox < TX && oy >= 0 && oy < TY && x0 + ox < nx)
            gst(Tout, (uint32_t)(gyr * pitch + x0 + ox) * 4u, tau);
    }
    __syncthreads();

    // ---------------- phase D: gather, bounce-back, destination term, write.
    // Only tiles holding row 0 or row ny-1 have bounced populations; the
    // others take the gather offsets as compile-time constants.
    auto phase_d = [&](auto wall_tag) {
        constexpr bool WALL = decltype(wall_tag)::value;
        for (int idx = tid; idx < TX * TY; idx += NT) {
            const int oy = idx / TX, ox = idx - oy * TX;
            const int gx = x0 + ox, gyr = y0 + oy;
            if (gx >= nx || gyr >= ny) continue;
            const int i1 = (oy + 1) * W1 + ox + 1;
            const int i2 = (oy + 2) * W2 + ox + 2;
            const uint32_t eo = (uint32_t)(gyr * pitch + gx);
            float dv[9];
            int src[9], dir[9];
            bool bb[9];
#pragma unroll
            for (int a = 0; a < 9; ++a) {
                const int sy = gyr - Lat::ey[a];
                bb[a] = WALL && (sy < 0 || sy >= ny);
                src[a] = bb[a] ? i1 : i1 - Lat::ey[a] * W1 - Lat::ex[a];
                dir[a] = bb[a] ? Lat::opp[a] : a;
            }
            // s(y) = sum_a w_a s(z_a) + sum_a d*_a(z_a), formed around the node's
            // own s.  The stored s' = s - p_ref: a source one row below carries
            // p_ref(z) - p_ref(y) = rho_3 g e_y exactly (zero for a bounced one)
            const double sy0 = sS[i1];
            const double pg = cd.pref_g;
            // level differences to the sources, exact in float64 and then small
            // enough for float32: ds_a = s(z_a) - s(y) (with the reference's)
            float ds[9], ssum = 0.f, dsum = 0.f;
#pragma unroll
            for (int a = 0; a < 9; ++a) {
                double sv = sS[src[a]] - sy0;
                if (!bb[a] && Lat::ey[a] != 0) sv += Lat::ey[a] > 0 ? pg : -pg;
                ds[a] = (float)sv;
                dv[a] = sD[dir[a]][src[a]];
                if constexpr (!WALL) {
                    // interior tiles: the sums in the same pass (same order of additions)
                    if (a > 0) ssum += Lat::w[a] * ds[a];
                    dsum += dv[a];
                }
            }
            // region index of the output node on R3
            const int j3 = (oy + 3) * W3 + ox + 3;
            // open ends: populations whose source lies beyond x = 0 or nx-1
            // (and not beyond a wall) are set by the inlet or outflow condition
            const bool inlet = WALL && openx && gx == 0, outlet = WALL && openx && gx == nx - 1;
            bool unk[9];
#pragma unroll
            for (int a = 0; a < 9; ++a) unk[a] = (inlet && Lat::ex[a] == 1 && !bb[a]) || (outlet && Lat::ex[a] == -1 && !bb[a]);
            if (inlet) {
                // velocity inlet, pure component 3 entering with u = (u_in, 0):
                // gbar_a = gbar_abar + (gbar_eq,a - gbar_eq,abar) at u_in (grad rho = 0,
                // the body force as the force), then corrections that make both
                // velocity moments exact
                const float rho = sR[j3], Fx = rho * cd.fx, Fy = -rho * cd.g, ui = cd.u_in;
                float mx = 0.f, my = 0.f;
#pragma unroll
                for (int a = 0; a < 9; ++a) {
                    if (unk[a]) {
                        const int b = Lat::opp[a];
                        const float eu = Lat::ex[a] * ui, eF = edot(Lat::ex[a], Lat::ey[a], Fx, Fy);
                        const float odd = 2.0f * rho * eu - eF * (1.0f + 4.5f * eu * eu - 1.5f * ui * ui) + 3.0f * (ui * Fx) * eu;
                        ds[a] = ds[b];
                        dv[a] = dv[b] + Lat::w[a] * odd;
                    }
                }
#pragma unroll
                for (int a = 1; a < 9; ++a) {
                    const float v = fmaf(Lat::w[a], ds[a], dv[a]);
                    mx += Lat::ex[a] * v;
                    my += Lat::ey[a] * v;
                }
                const float rx_ = kCs2 * (rho * ui - 0.5f * Fx) - mx, ry_ = kCs2 * (-0.5f * Fy) - my;
                if (unk[5] && unk[8]) {
                    dv[5] += 0.5f * ry_;
                    dv[8] -= 0.5f * ry_;
                    dv[1] += rx_;
                } else {
                    const int d = unk[5] ? 5 : 8;
                    dv[d] += Lat::ey[d] * ry_;
                    dv[1] += rx_ - Lat::ey[d] * ry_;
                }
            } else if (outlet) {
                // convective outflow on the unknown populations, their pressure
                // part replaced by the linear extrapolation of p:
                // gbar_a = [gbar_a(t) + U gbar_a(x-1, t+1)] / (1 + U)
                //          + w_a [p_e - (p(x, t) + U p(x-1, t)) / (1 + U)]
                const float U = fmaxf(sUx[i2], 0.0f), iu = 1.0f / (1.0f + U);
                float dold[9];
                if (F16) {
                    float m[kQPlanes];
#pragma unroll
                    for (int q = 0; q < kQPlanes; ++q) m[q] = (float)gld(Qin + q * plane, eo * 2u) * qinv;
                    unpack_devs(gld(Sin, eo * 4u), gld(Sin + plane, eo * 4u), m, dold);
                } else {
#pragma unroll
                    for (int a = 1; a < 9; ++a) dold[a] = gld(Sin + (a - 1) * plane, eo * 4u);
                }
                const float pcorr = (2.0f * sP[i2 - 1] - sP[i2 - 2]) - (sP[i2] + U * sP[i2 - 1]) * iu;
#pragma unroll
                for (int a = 1; a < 9; ++a) {
                    if (unk[a]) {
                        // the neighbour x-1 receives population a from (x, y - e_ay)
                        const int s2 = i1 - Lat::ey[a] * W1;
                        double sv = sS[s2] - sy0;
                        if (Lat::ey[a] != 0) sv += Lat::ey[a] > 0 ? pg : -pg;
                        const float ds2 = (float)sv;
                        const float g2 = fmaf(Lat::w[a], ds2, sD[a][s2]);
                        ds[a] = 0.0f;
                        dv[a] = fmaf(Lat::w[a], pcorr, (dold[a] + U * g2) * iu);
                    }
                }
            }
            if constexpr (WALL) {
#pragma unroll
                for (int a = 0; a < 9; ++a) {
                    if (a > 0 && !bb[a]) ssum += Lat::w[a] * ds[a];
                    dsum += dv[a];
                }
            }
            const float dnew = ssum + dsum;               // s(t+1) - s(y)
            gst(Pout, eo * 8u, sy0 + (double)dnew);
            // d_a(y) = w_a (s(z_a) - s(t+1)) + d*_a(z_a)
            float da[9];
#pragma unroll
            for (int a = 1; a < 9; ++a) da[a] = Lat::w[a] * (ds[a] - dnew) + dv[a];
            if (F16) {
                float jx, jy, m[kQPlanes];
                pack_devs(da, jx, jy, m);
                gst(Sout, eo * 4u, jx);
                gst(Sout + plane, eo * 4u, jy);
#pragma unroll
                for (int k = 0; k < kQPlanes; ++k)
                    gst(Qout + k * plane, eo * 2u, (_Float16)(m[k] * qscale));   // nearest even
            } else {
#pragma unroll
                for (int a = 1; a < 9; ++a) gst(Sout + (a - 1) * plane, eo * 4u, da[a]);
            }

#pragma unroll
            for (int i = 0; i < NH; ++i) {
                const float hd = 0.5f * sDif[i][i1];
                if (!SH && (inlet || outlet)) {
                    // open ends: an entering population carries no component 1 or
                    // 2 (only the receiving node's diffusion half, which the hd
                    // below adds); a leaving one copies its neighbour x-1's new
                    // value (zero normal gradient)
                    const double cy = sCd[i][j3];
                    const float ux = sUx[i2], uy = sUy[i2], uu = ux * ux + uy * uy;
                    const float nxu = sUx[i2 - 1], nyu = sUy[i2 - 1], nuu = nxu * nxu + nyu * nyu;
                    const float nhd = 0.5f * sDif[i][i1 - 1];
                    double dsum = 0.0;
                    float qsum = 0.f;
#pragma unroll
                    for (int a = 0; a < 9; ++a) {
                        if (unk[a] && inlet) {
                            dsum -= (double)Lat::w[a] * cy;
                        } else if (unk[a]) {
                            const float eu = Lat::ex[a] * ux + Lat::ey[a] * uy, neu = Lat::ex[a] * nxu + Lat::ey[a] * nyu;
                            const float G = Lat::w[a] * (1.0f + 3.0f * eu + 4.5f * eu * eu - 1.5f * uu);
                            const float nG = Lat::w[a] * (1.0f + 3.0f * neu + 4.5f * neu * neu - 1.5f * nuu);
                            dsum += (double)Lat::w[a] * (sCd[i][j3 - Lat::ey[a] * W3] - cy);
                            qsum += sH[i][a][i1 - Lat::ey[a] * W1] + (nhd * nG - hd * G);
                        } else {
                            qsum += sH[i][dir[a]][src[a]];
                            if (a > 0 && !bb[a])
                                dsum += (double)Lat::w[a] * (sCd[i][j3 - Lat::ey[a] * W3 - Lat::ex[a]] - cy);
                        }
                    }
                    gst(Cout + i * plane, eo * 8u, cy + (dsum + (double)(qsum + hd)));
                } else if (SH) {
                    // hbar_a(y) = w_a C(z_a) + (1 - omega_h) q_b(z_a) + Q_b(z_a) + Dif(y)/2 Gamma_a(y);
                    // C(t+1) = sum_a hbar_a(y) accumulated in float64 around C(y), and the
                    // new deviations q_a = hbar_a - w_a C(t+1)
                    const float ux = sUx[i2], uy = sUy[i2], uu = ux * ux + uy * uy;
                    const double cy = sCd[i][j3];
                    float hv[9];
                    double dz[9], csum = 0.0;
#pragma unroll
                    for (int a = 0; a < 9; ++a) {
                        const float eu = Lat::ex[a] * ux + Lat::ey[a] * uy;
                        const float G = Lat::w[a] * (1.0f + 3.0f * eu + 4.5f * eu * eu - 1.5f * uu);
                        const int sxg = wrap_x(gx - (bb[a] ? 0 : Lat::ex[a]), nx);
                        const int syg = bb[a] ? gyr : gyr - Lat::ey[a];
                        const uint32_t so = (uint32_t)(syg * pitch + sxg);
                        hv[a] = sH[i][dir[a]][src[a]] + (1.0f - cd.omh) * gld(Hin + (i * 9 + dir[a]) * plane, so * 4u) +
                                hd * G;
                        dz[a] = bb[a] ? 0.0 : sCd[i][j3 - Lat::ey[a] * W3 - Lat::ex[a]] - cy;
                        csum += (double)Lat::w[a] * dz[a] + (double)hv[a];
                    }
                    gst(Cout + i * plane, eo * 8u, cy + csum);
#pragma unroll
                    for (int a = 0; a < 9; ++a)
                        gst(Hout + (i * 9 + a) * plane, eo * 4u, (float)((double)Lat::w[a] * (dz[a] - csum) + (double)hv[a]));
                } else {
                    // C(t+1) = C(y) + sum_a [w_a (C(z_a) - C(y)) + (hbar*_b(z_a) - w_b C(z_a))]
                    //          + Dif(y)/2 sum_a Gamma_a(y)      (sum_a Gamma_a = 1 exactly for D2Q9)
                    const double cy = sCd[i][j3];
                    double dsum = 0.0;
                    float qsum = 0.f;
#pragma unroll
                    for (int a = 0; a < 9; ++a) {
                        qsum += sH[i][dir[a]][src[a]];
                        if (a > 0 && !bb[a])
                            dsum += (double)Lat::w[a] * (sCd[i][j3 - Lat::ey[a] * W3 - Lat::ex[a]] - cy);
                    }
                    gst(Cout + i * plane, eo * 8u, cy + (dsum + (double)(qsum + hd)));
                }
            }
        }
    };
    if (y0 == 0 || y0 + TY >= ny || (openx && (x0 == 0 || x0 + TX >= nx))) phase_d(std::true_type{});
    else phase_d(std::false_type{});
}

// Step variants selectable at run time: tile shape x phase-field count x
// state form (compact float32, stored hbar float32, compact float16; each
// plain and extended).  The extended instances add the fixed-point passes of
// the implicit tau, central differences in the hbar forcing, open x ends and
// the link form of the diffusion source;
// the plain ones carry none of that code (each costs ~1 % even unexecuted,
// measured).  A tile
// shape whose LDS footprint exceeds the 160 KiB of a gfx950 CU for two phase
// fields is offered for one phase field only.
using StepFn = void (*)(const CaseDev*, const TileDev*, int, int);
struct StepVariant {
    int tx, ty, nt;
    StepFn k[2][kStepForms];   // [n_h - 1][form]
};

#define PFLBM_K(TX, TY, NH, SH, F16, NT, I) step_kernel<TX, TY, NH, SH, F16, NT, I>
#define PFLBM_FORMS(TX, TY, NH, NT)                                                                  \
    {PFLBM_K(TX, TY, NH, false, false, NT, false), PFLBM_K(TX, TY, NH, true, false, NT, false),      \
     PFLBM_K(TX, TY, NH, false, true, NT, false), PFLBM_K(TX, TY, NH, false, false, NT, true),        \
     PFLBM_K(TX, TY, NH, true, false, NT, true), PFLBM_K(TX, TY, NH, false, true, NT, true)}
#define PFLBM_V2(TX, TY, NT) {TX, TY, NT, {PFLBM_FORMS(TX, TY, 1, NT), PFLBM_FORMS(TX, TY, 2, NT)}}
#define PFLBM_V1(TX, TY, NT) {TX, TY, NT, {PFLBM_FORMS(TX, TY, 1, NT), {}}}

static const StepVariant kVariants[] = {
    PFLBM_V2(32, 16, 512),
    PFLBM_V2(32, 16, 256),
    PFLBM_V2(32, 8, 256),
    // one pass per phase but the first for a 32 x 8 tile: with two phase
    // fields (67 KB of LDS, two work-groups per CU) the fastest on large domains
    PFLBM_V2(32, 8, 512),
    PFLBM_V2(64, 8, 512),
    PFLBM_V1(64, 16, 512),
    PFLBM_V1(64, 16, 1024),
    // small tiles for small domains: more work-groups where 32 x 16 tiles
    // leave most compute units idle (a 64 x 128 domain is 16 such tiles,
    // 128 tiles of 8 x 8); with 256 threads every phase of an 8 x 8 tile,
    // and all but the first of a 16 x 8 tile, takes one pass, which
    // shortens the step of a lone tile
    PFLBM_V2(16, 8, 128),
    PFLBM_V2(16, 16, 256),
    PFLBM_V2(8, 8, 128),
    PFLBM_V2(8, 8, 256),
    PFLBM_V2(16, 8, 256),
};

int step_variant_count() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }

bool step_variant_shape(int v, int nh, int* tx, int* ty, int* nt) {
    if (v < 0 || v >= step_variant_count() || (nh != 1 && nh != 2)) return false;
    const StepVariant& sv = kVariants[v];
    if (sv.k[nh - 1][0] == nullptr) return false;
    *tx = sv.tx;
    *ty = sv.ty;
    *nt = sv.nt;
    return true;
}

hipError_t launch_step(int v, int nh, int form, const CaseDev* cases, const TileDev* tiles, int ntiles, int par,
                       hipStream_t stream) {
    if (v < 0 || v >= step_variant_count() || (nh != 1 && nh != 2) || form < 0 || form >= kStepForms ||
        ntiles <= 0)
        return hipErrorInvalidValue;
    const StepFn k = kVariants[v].k[nh - 1][form];
    if (!k) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k, dim3(ntiles), dim3(kVariants[v].nt), 0, stream, cases, tiles, ntiles, par);
    return hipGetLastError();
}

}  // namespace pflbm
