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
//      Eq. (21), mixed directional derivatives of rho and C_i, the shear rate
//      from the non-equilibrium second moment with the previous tau
//      (Eqs. (25)-(29)), the truncated power-law tau (Eqs. (31)-(33)) and the
//      post-collision populations of gbar (Eq. (14)) and hbar (Eq. (18));
//   D  on the tile: gather the post-collision populations (half-way
//      bounce-back at the walls), add the receiving-node half of the
//      diffusion term and write the new state.
// gbar is carried as s = sum gbar plus deviations d_a = gbar_a - w_a s so that
// the momentum moment is formed from small numbers (float32 at density
// ratio 1000).
#include "pflbm_internal.h"

namespace pflbm {

template <int TX, int TY, int NH, bool SH, int NT>
__global__ __launch_bounds__(NT) void step_kernel(const CaseDev* __restrict__ cases,
                                                  const TileDev* __restrict__ tiles, int ntiles, int par) {
    constexpr int W3 = TX + 6, H3 = TY + 6, N3 = W3 * H3;
    constexpr int W2 = TX + 4, H2 = TY + 4, N2 = W2 * H2;
    constexpr int W1 = TX + 2, H1 = TY + 2, N1 = W1 * H1;
    constexpr int NMU = 3;

    __shared__ float sC[NH][N3];
    __shared__ double sCd[NH][N3];   // the float64 phase field on R3
    __shared__ float sR[N3];
    __shared__ float sMu[NMU][N2];
    __shared__ float sUx[N2], sUy[N2], sP[N2];
    __shared__ float sD[9][N1];      // post-collision deviations d*_a
    __shared__ float sS[N1];         // s = sum gbar at the source
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
    const auto Sin = gmem<const float>(cd.S[par]);
    const auto Cin = gmem<const double>(cd.C[par]);
    const auto Tin = gmem<const float>(cd.T[par]);
    const auto Sout = gmem<float>(cd.S[par ^ 1]);
    const auto Cout = gmem<double>(cd.C[par ^ 1]);
    const auto Tout = gmem<float>(cd.T[par ^ 1]);
    const auto Hin = gmem<const float>(cd.H[par]);
    const auto Hout = gmem<float>(cd.H[par ^ 1]);
    const int tid = threadIdx.x;

    // ---------------- phase A: C_i and rho on R3
    for (int idx = tid; idx < N3; idx += NT) {
        const int ry = idx / W3, rx = idx - ry * W3;
        const int gx = wrap_x(x0 - 3 + rx, nx), gy = mirror_y(y0 - 3 + ry, ny);
        const long long off = (long long)gy * pitch + gx;
        const double d1 = Cin[off];
        const double d2 = NH == 2 ? Cin[plane + off] : 0.0;
        const float c1 = (float)d1, c2 = (float)d2;
        sC[0][idx] = c1;
        sCd[0][idx] = d1;
        if (NH == 2) { sC[NH - 1][idx] = c2; sCd[NH - 1][idx] = d2; }
        sR[idx] = mix_rho(cd, c1, c2);
    }
    __syncthreads();

    // ---------------- phase B: mu, u, p on R2
    for (int idx = tid; idx < N2; idx += NT) {
        const int ry = idx / W2, rx = idx - ry * W2;
        const int i3 = (ry + 1) * W3 + rx + 1;
        const int gyr = y0 - 2 + ry;
        float c[2], gcx[2], gcy[2], lc[2];
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            float sx = 0.f, sy = 0.f, sl = 0.f;
            const float cc = sC[i][i3];
#pragma unroll
            for (int a = 1; a < 9; ++a) {
                const float fp = sC[i][i3 + Lat::ey[a] * W3 + Lat::ex[a]];
                const float fm = sC[i][i3 - Lat::ey[a] * W3 - Lat::ex[a]];
                sx += Lat::w[a] * Lat::ex[a] * (fp - fm);
                sy += Lat::w[a] * Lat::ey[a] * (fp - fm);
                sl += Lat::w[a] * ((fp - cc) + (fm - cc));
            }
            c[i] = cc;
            gcx[i] = 1.5f * sx;
            gcy[i] = 1.5f * sy;
            lc[i] = 3.0f * sl;
        }
        if (NH == 1) { c[1] = 0.f; gcx[1] = 0.f; gcy[1] = 0.f; lc[1] = 0.f; }
        float mu[3];
        chem_potential<NH>(cd, sCd[0][i3], NH == 2 ? sCd[NH - 1][i3] : 0.0, lc[0], lc[1], mu);
#pragma unroll
        for (int k = 0; k < 3; ++k) sMu[k][idx] = mu[k];
        if (gyr >= 0 && gyr < ny) {
            const int gx = wrap_x(x0 - 2 + rx, nx);
            const long long off = (long long)gyr * pitch + gx;
            float d[9];
#pragma unroll
            for (int a = 1; a < 9; ++a) d[a] = Sin[a * plane + off];
            const float s = Sin[off];
            const float jx = d[1] - d[3] + d[5] - d[6] - d[7] + d[8];
            const float jy = d[2] - d[4] + d[5] + d[6] - d[7] - d[8];
            float grx = 0.f, gry = 0.f;
#pragma unroll
            for (int a = 1; a < 9; ++a) {
                const float df = sR[i3 + Lat::ey[a] * W3 + Lat::ex[a]] - sR[i3 - Lat::ey[a] * W3 - Lat::ex[a]];
                grx += Lat::w[a] * Lat::ex[a] * df;
                gry += Lat::w[a] * Lat::ey[a] * df;
            }
            grx *= 1.5f;
            gry *= 1.5f;
            const float rho = sR[i3];
            // sum_k mu_k grad C_k with grad C_3 = -grad C_1 - grad C_2
            const float fx = (mu[0] - mu[2]) * gcx[0] + (mu[1] - mu[2]) * gcx[1] + rho * cd.fx;
            const float fy = (mu[0] - mu[2]) * gcy[0] + (mu[1] - mu[2]) * gcy[1] - rho * cd.g;
            const float rr = rcp(rho);
            const float ux = (3.0f * jx + 0.5f * fx) * rr;
            const float uy = (3.0f * jy + 0.5f * fy) * rr;
            sUx[idx] = ux;
            sUy[idx] = uy;
            sP[idx] = s + 0.5f * kCs2 * (ux * grx + uy * gry);
        }
    }
    __syncthreads();
    // the two ghost rows beyond each wall mirror the wall rows for grad p
    // (rows farther out are never read)
    for (int idx = tid; idx < N2; idx += NT) {
        const int ry = idx / W2, rx = idx - ry * W2;
        const int gyr = y0 - 2 + ry;
        if ((gyr < 0 && gyr >= -2) || (gyr >= ny && gyr < ny + 2)) {
            const int rm = mirror_y(gyr, ny) - (y0 - 2);
            sP[idx] = sP[rm * W2 + rx];
        }
    }
    __syncthreads();

    // ---------------- phase C: collisions on R1
    for (int idx = tid; idx < N1; idx += NT) {
        const int ry = idx / W1, rx = idx - ry * W1;
        const int gyr = y0 - 1 + ry;
        if (gyr < 0 || gyr >= ny) continue;   // nodes beyond the walls are never sources
        const int i2 = (ry + 1) * W2 + rx + 1;
        const int i3 = (ry + 2) * W3 + rx + 2;
        const int gx = wrap_x(x0 - 1 + rx, nx);
        const long long off = (long long)gyr * pitch + gx;

        float d[9];
#pragma unroll
        for (int a = 1; a < 9; ++a) d[a] = Sin[a * plane + off];
        const float s = Sin[off];
        d[0] = -(d[1] + d[2] + d[3] + d[4] + d[5] + d[6] + d[7] + d[8]);
        const float tprev = Tin[off];

        float c[2], gcx[2], gcy[2];
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            float sx = 0.f, sy = 0.f;
#pragma unroll
            for (int a = 1; a < 9; ++a) {
                const float df = sC[i][i3 + Lat::ey[a] * W3 + Lat::ex[a]] - sC[i][i3 - Lat::ey[a] * W3 - Lat::ex[a]];
                sx += Lat::w[a] * Lat::ex[a] * df;
                sy += Lat::w[a] * Lat::ey[a] * df;
            }
            c[i] = sC[i][i3];
            gcx[i] = 1.5f * sx;
            gcy[i] = 1.5f * sy;
        }
        if (NH == 1) { c[1] = 0.f; gcx[1] = 0.f; gcy[1] = 0.f; }
        const float c3 = 1.0f - c[0] - c[1];
        const float rho = sR[i3];
        float grx = 0.f, gry = 0.f;
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            const float df = sR[i3 + Lat::ey[a] * W3 + Lat::ex[a]] - sR[i3 - Lat::ey[a] * W3 - Lat::ex[a]];
            grx += Lat::w[a] * Lat::ex[a] * df;
            gry += Lat::w[a] * Lat::ey[a] * df;
        }
        grx *= 1.5f;
        gry *= 1.5f;

        float mu[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) mu[k] = sMu[k][i2];
        const float ux = sUx[i2], uy = sUy[i2], p = sP[i2];
        float gpx = 0.f, gpy = 0.f;
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            const float df = sP[i2 + Lat::ey[a] * W2 + Lat::ex[a]] - sP[i2 - Lat::ey[a] * W2 - Lat::ex[a]];
            gpx += Lat::w[a] * Lat::ex[a] * df;
            gpy += Lat::w[a] * Lat::ey[a] * df;
        }
        gpx *= 1.5f;
        gpy *= 1.5f;

        // diffusion source Dif_i = div(D_i grad mu_i) in the product form of Eq. (21)
        float dif[2];
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            float mx = 0.f, my = 0.f, ml = 0.f, sx = 0.f, sy = 0.f;
            const float mc = sMu[i][i2];
#pragma unroll
            for (int a = 1; a < 9; ++a) {
                const float fp = sMu[i][i2 + Lat::ey[a] * W2 + Lat::ex[a]];
                const float fm = sMu[i][i2 - Lat::ey[a] * W2 - Lat::ex[a]];
                mx += Lat::w[a] * Lat::ex[a] * (fp - fm);
                my += Lat::w[a] * Lat::ey[a] * (fp - fm);
                ml += Lat::w[a] * ((fp - mc) + (fm - mc));
            }
            const float lapmu = 3.0f * ml;
            if (cd.vm) {
#pragma unroll
                for (int a = 1; a < 9; ++a) {
                    const float cp = clip01(sC[i][i3 + Lat::ey[a] * W3 + Lat::ex[a]]);
                    const float cm = clip01(sC[i][i3 - Lat::ey[a] * W3 - Lat::ex[a]]);
                    const float df = (cp - cp * cp) - (cm - cm * cm);
                    sx += Lat::w[a] * Lat::ex[a] * df;
                    sy += Lat::w[a] * Lat::ey[a] * df;
                }
                const float cl = clip01(c[i]);
                dif[i] = cd.mob[i] * (cl * (1.0f - cl) * lapmu + 2.25f * (sx * mx + sy * my));
            } else {
                dif[i] = cd.mob[i] * lapmu;
            }
        }

        // mixed directional derivatives along every e_a (radius 2)
        float drho[9], dc[2][9];
        drho[0] = 0.f;
        dc[0][0] = 0.f;
        dc[1][0] = 0.f;
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            const int o1 = Lat::ey[a] * W3 + Lat::ex[a];
            drho[a] = 0.25f * (-sR[i3 + 2 * o1] + 5.0f * sR[i3 + o1] - 3.0f * sR[i3] - sR[i3 - o1]);
#pragma unroll
            for (int i = 0; i < NH; ++i)
                dc[i][a] = 0.25f * (-sC[i][i3 + 2 * o1] + 5.0f * sC[i][i3 + o1] - 3.0f * sC[i][i3] - sC[i][i3 - o1]);
            if (NH == 1) dc[1][a] = 0.f;
        }
        float mrx = 0.f, mry = 0.f, m1x = 0.f, m1y = 0.f, m2x = 0.f, m2y = 0.f;
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            mrx += Lat::w[a] * Lat::ex[a] * drho[a];
            mry += Lat::w[a] * Lat::ey[a] * drho[a];
            m1x += Lat::w[a] * Lat::ex[a] * dc[0][a];
            m1y += Lat::w[a] * Lat::ey[a] * dc[0][a];
            m2x += Lat::w[a] * Lat::ex[a] * dc[1][a];
            m2y += Lat::w[a] * Lat::ey[a] * dc[1][a];
        }
        mrx *= 3.0f; mry *= 3.0f; m1x *= 3.0f; m1y *= 3.0f; m2x *= 3.0f; m2y *= 3.0f;

        // force, equilibria (deviation form) and the non-equilibrium second moment
        const float mu13 = mu[0] - mu[2], mu23 = mu[1] - mu[2];
        const float fbx = rho * cd.fx, fby = -rho * cd.g;
        const float Fx = mu13 * gcx[0] + mu23 * gcx[1] + fbx;
        const float Fy = mu13 * gcy[0] + mu23 * gcy[1] + fby;
        const float uu = ux * ux + uy * uy;
        const float ugr = ux * grx + uy * gry;
        const float uF = ux * Fx + uy * Fy;
        const float ps = 0.5f * kCs2 * ugr;          // p - s
        const float rc2 = rho * kCs2;
        float A[9], deq[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const float eu = Lat::ex[a] * ux + Lat::ey[a] * uy;
            A[a] = 3.0f * eu + 4.5f * eu * eu - 1.5f * uu;     // Gamma_a / w_a - 1
            const float egr = Lat::ex[a] * grx + Lat::ey[a] * gry - ugr;
            const float eF = Lat::ex[a] * Fx + Lat::ey[a] * Fy - uF;
            const float wa = Lat::w[a];
            deq[a] = wa * ps + rc2 * wa * A[a] - 0.5f * (kCs2 * egr * wa * A[a] + eF * wa * (1.0f + A[a]));
        }
        float pxx = 0.f, pyy = 0.f, pxy = 0.f;
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            const float ne = d[a] - deq[a];
            pxx += Lat::ex[a] * Lat::ex[a] * ne;
            pyy += Lat::ey[a] * Lat::ey[a] * ne;
            pxy += Lat::ex[a] * Lat::ey[a] * ne;
        }
        // shear rate: D = -Pi / (2 (tau_prev + 1/2) rho c_s^4), gdot = sqrt(2 D:D)
        const float fs = 4.5f * rcp((tprev + 0.5f) * rho);
        const float gdot = fs * sqrtf(2.0f * (pxx * pxx + pyy * pyy + 2.0f * pxy * pxy));
        const float tau = mixture_tau(cd, c[0], c[1], c3, gdot);
        const float om = rcp(tau + 0.5f);

        // gbar collision with the mixed-difference forcing
        const float umr = ux * mrx + uy * mry;
        const float um1 = ux * m1x + uy * m1y, um2 = ux * m2x + uy * m2y;
        const float ufb = ux * fbx + uy * fby;
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const float wa = Lat::w[a];
            const float t1 = kCs2 * (drho[a] - umr) * wa * A[a];
            const float t2 = mu13 * (dc[0][a] - um1) + mu23 * (dc[1][a] - um2)
                           + (Lat::ex[a] * fbx + Lat::ey[a] * fby - ufb);
            const float Fa = t1 + t2 * wa * (1.0f + A[a]);
            sD[a][idx] = d[a] - om * (d[a] - deq[a]) + Fa;
        }
        sS[idx] = s;

        // hbar collision: equilibrium with central differences, forcing with the
        // mixed derivative of C_i and central grad p, source half of Dif
        const float bx = gpx - Fx, by = gpy - Fy;
        const float ub = ux * bx + uy * by;
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            const float kk = c[i] * 3.0f * rcp(rho);
            const float Xx = gcx[i] - kk * bx, Xy = gcy[i] - kk * by;
            const float uX = ux * Xx + uy * Xy;
            const float umc = (i == 0) ? um1 : um2;
#pragma unroll
            for (int a = 0; a < 9; ++a) {
                const float G = Lat::w[a] * (1.0f + A[a]);
                const float eX = Lat::ex[a] * Xx + Lat::ey[a] * Xy - uX;
                const float fX = (dc[i][a] - umc) - kk * (Lat::ex[a] * bx + Lat::ey[a] * by - ub);
                if (SH) {
                    const float heq = c[i] * G - 0.5f * eX * G;
                    sH[i][a][idx] = cd.omh * heq + fX * G + 0.5f * dif[i] * G;
                } else {
                    // omega_h = 1: hbar* - w_a C = w_a A_a C + (-(e-u).X/2 + (e-u).X^MD + Dif/2) Gamma_a
                    sH[i][a][idx] = Lat::w[a] * A[a] * c[i] + (-0.5f * eX + fX + 0.5f * dif[i]) * G;
                }
            }
            sDif[i][idx] = dif[i];
        }
        (void)p;
        // tau is written for the tile's own nodes
        const int ox = rx - 1, oy = ry - 1;
        if (ox >= 0 && ox < TX && oy >= 0 && oy < TY && x0 + ox < nx) Tout[off] = tau;
    }
    __syncthreads();

    // ---------------- phase D: gather, bounce-back, destination term, write
    for (int idx = tid; idx < TX * TY; idx += NT) {
        const int oy = idx / TX, ox = idx - oy * TX;
        const int gx = x0 + ox, gyr = y0 + oy;
        if (gx >= nx || gyr >= ny) continue;
        const int i1 = (oy + 1) * W1 + ox + 1;
        const int i2 = (oy + 2) * W2 + ox + 2;
        const long long off = (long long)gyr * pitch + gx;
        const float ux = sUx[i2], uy = sUy[i2], uu = ux * ux + uy * uy;
        float sv[9], dv[9];
        int src[9], dir[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const int sy = gyr - Lat::ey[a];
            if (sy < 0 || sy >= ny) { src[a] = i1; dir[a] = Lat::opp[a]; }
            else { src[a] = i1 - Lat::ey[a] * W1 - Lat::ex[a]; dir[a] = a; }
        }
        float snew = 0.f, dsum = 0.f;
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            sv[a] = sS[src[a]];
            dv[a] = sD[dir[a]][src[a]];
            snew += Lat::w[a] * sv[a];
            dsum += dv[a];
        }
        snew += dsum;
        Sout[off] = snew;
#pragma unroll
        for (int a = 1; a < 9; ++a) Sout[a * plane + off] = Lat::w[a] * (sv[a] - snew) + dv[a];

        // region index of the output node and of each source on R3 (for C)
        const int j3 = (oy + 3) * W3 + ox + 3;
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            const float hd = 0.5f * sDif[i][i1];
            if (SH) {
                float csum = 0.f;
#pragma unroll
                for (int a = 0; a < 9; ++a) {
                    const float eu = Lat::ex[a] * ux + Lat::ey[a] * uy;
                    const float G = Lat::w[a] * (1.0f + 3.0f * eu + 4.5f * eu * eu - 1.5f * uu);
                    float hv = sH[i][dir[a]][src[a]] + hd * G;
                    const int sxg = wrap_x(gx - (dir[a] == a ? Lat::ex[a] : 0), nx);
                    const int syg = dir[a] == a ? gyr - Lat::ey[a] : gyr;
                    const long long so = (long long)syg * pitch + sxg;
                    hv += (1.0f - cd.omh) * Hin[(long long)(i * 9 + dir[a]) * plane + so];
                    Hout[(long long)(i * 9 + a) * plane + off] = hv;
                    csum += hv;
                }
                Cout[(long long)i * plane + off] = (double)csum;
            } else {
                // C(t+1) = C(y) + sum_a [w_a (C(z_a) - C(y)) + (hbar*_b(z_a) - w_b C(z_a))] + Dif(y)/2 sum_a Gamma_a(y)
                const double cy = sCd[i][j3];
                double dsum = 0.0;
                float qsum = 0.f, gsum = 0.f;
#pragma unroll
                for (int a = 0; a < 9; ++a) {
                    const float eu = Lat::ex[a] * ux + Lat::ey[a] * uy;
                    gsum += Lat::w[a] * (1.0f + 3.0f * eu + 4.5f * eu * eu - 1.5f * uu);
                    qsum += sH[i][dir[a]][src[a]];
                    if (dir[a] == a) dsum += (double)Lat::w[a] * (sCd[i][j3 - Lat::ey[a] * W3 - Lat::ex[a]] - cy);
                }
                Cout[(long long)i * plane + off] = cy + (dsum + (double)(qsum + hd * gsum));
            }
        }
    }
}

// Step variants selectable at run time: tile shape x phase-field count x
// hbar storage.  A tile shape whose LDS footprint exceeds the 160 KiB of a
// gfx950 CU for two phase fields is offered for one phase field only.
struct StepVariant {
    int tx, ty, nt;
    void (*k1[2])(const CaseDev*, const TileDev*, int, int);   // n_h = 1: compact, stored hbar
    void (*k2[2])(const CaseDev*, const TileDev*, int, int);   // n_h = 2
};

#define PFLBM_K(TX, TY, NH, SH, NT) step_kernel<TX, TY, NH, SH, NT>
#define PFLBM_V2(TX, TY, NT)                                                                        \
    {TX, TY, NT, {PFLBM_K(TX, TY, 1, false, NT), PFLBM_K(TX, TY, 1, true, NT)},                      \
     {PFLBM_K(TX, TY, 2, false, NT), PFLBM_K(TX, TY, 2, true, NT)}}
#define PFLBM_V1(TX, TY, NT)                                                                        \
    {TX, TY, NT, {PFLBM_K(TX, TY, 1, false, NT), PFLBM_K(TX, TY, 1, true, NT)}, {nullptr, nullptr}}

static const StepVariant kVariants[] = {
    PFLBM_V2(32, 16, 512),
    PFLBM_V2(32, 16, 256),
    PFLBM_V2(32, 8, 256),
    PFLBM_V2(64, 8, 512),
    PFLBM_V1(64, 16, 512),
    PFLBM_V1(64, 16, 1024),
};

int step_variant_count() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }

bool step_variant_shape(int v, int nh, int* tx, int* ty, int* nt) {
    if (v < 0 || v >= step_variant_count() || (nh != 1 && nh != 2)) return false;
    const StepVariant& sv = kVariants[v];
    if ((nh == 1 ? sv.k1[0] : sv.k2[0]) == nullptr) return false;
    *tx = sv.tx;
    *ty = sv.ty;
    *nt = sv.nt;
    return true;
}

hipError_t launch_step(int v, int nh, bool sh, const CaseDev* cases, const TileDev* tiles, int ntiles, int par,
                       hipStream_t stream) {
    if (v < 0 || v >= step_variant_count() || (nh != 1 && nh != 2) || ntiles <= 0) return hipErrorInvalidValue;
    const StepVariant& sv = kVariants[v];
    auto k = (nh == 1 ? sv.k1 : sv.k2)[sh ? 1 : 0];
    if (!k) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k, dim3(ntiles), dim3(sv.nt), 0, stream, cases, tiles, ntiles, par);
    return hipGetLastError();
}

}  // namespace pflbm
