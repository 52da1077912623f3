// Pointwise first-order GHG right-hand side (App. A.1 eqs. gdot, Phidot,
// Pidot with gamma_0 = gamma_2 = 1, gamma_1 = -1), fused with the Cartesian
// chain rule (Sec. 2.2), the freezing-incoming boundary operator on the outer
// sphere (App. A.3) and the RK4 stage combination (Sec. 2.5).
//
// One thread per grid point.  The right-hand side is linear in the
// derivatives, so it is evaluated in two phases: first every term built from
// the undifferentiated variables (3+1 split, inverse metrics, Christoffel
// symbols, quadratic terms, constraint damping, gauge terms), then the
// derivative terms, streamed variable by variable so that only the 50 (58)
// accumulators stay live.
#include "internal.h"

namespace sg {

namespace {

__device__ __forceinline__ int pr(int a, int b) {
    // symmetric pair index, order tt tx ty tz xx xy xz yy yz zz
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    return lo == 0 ? hi : (lo == 1 ? 3 + hi : (lo == 2 ? 5 + hi : 9));
}

template <int NV>
__global__ __launch_bounds__(256) void k_rhs(KShell s, const double* __restrict__ u,
                                             const double* __restrict__ du, int cart,
                                             double* __restrict__ out, const double* __restrict__ ubase,
                                             double* __restrict__ acc, double dt, int stage) {
    const long long np = s.npts;
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int k = (int)(p % s.n_r);
    const int i = (int)((p / s.n_r) % s.n_th);
    const int j = (int)(p / ((long long)s.n_r * s.n_th));

    // ---- variables ---------------------------------------------------------
    double g[4][4], P[4][4], F[3][4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = a; b < 4; ++b) {
            const int q = pr(a, b);
            g[a][b] = g[b][a] = u[q * np + p];
            P[a][b] = P[b][a] = u[(10 + q) * np + p];
#pragma unroll
            for (int x = 0; x < 3; ++x) F[x][a][b] = F[x][b][a] = u[(20 + 10 * x + q) * np + p];
        }

    // ---- 3+1 split (eqs. normal, abgfromgab) -------------------------------
    const double gxx = g[1][1], gxy = g[1][2], gxz = g[1][3], gyy = g[2][2], gyz = g[2][3], gzz = g[3][3];
    const double cxx = gyy * gzz - gyz * gyz, cxy = gxz * gyz - gxy * gzz, cxz = gxy * gyz - gxz * gyy;
    const double cyy = gxx * gzz - gxz * gxz, cyz = gxy * gxz - gxx * gyz, czz = gxx * gyy - gxy * gxy;
    const double idet = 1.0 / (gxx * cxx + gxy * cxy + gxz * cxz);
    double gi[3][3] = {{cxx * idet, cxy * idet, cxz * idet},
                       {cxy * idet, cyy * idet, cyz * idet},
                       {cxz * idet, cyz * idet, czz * idet}};
    double bl[3] = {g[0][1], g[0][2], g[0][3]};
    double bu[3];
#pragma unroll
    for (int x = 0; x < 3; ++x) bu[x] = gi[x][0] * bl[0] + gi[x][1] * bl[1] + gi[x][2] * bl[2];
    const double al = sqrt(bu[0] * bl[0] + bu[1] * bl[1] + bu[2] * bl[2] - g[0][0]);
    const double ial = 1.0 / al, ial2 = ial * ial;
    double gI[4][4];
    gI[0][0] = -ial2;
#pragma unroll
    for (int x = 0; x < 3; ++x) {
        gI[0][x + 1] = gI[x + 1][0] = bu[x] * ial2;
#pragma unroll
        for (int y = 0; y < 3; ++y) gI[x + 1][y + 1] = gi[x][y] - bu[x] * bu[y] * ial2;
    }
    const double nu[4] = {ial, -bu[0] * ial, -bu[1] * ial, -bu[2] * ial};
    const double nl0 = -al;   // n_a = (-alpha, 0, 0, 0)

    // ---- Christoffel symbols (eq. Gamma), d_t g from eq. gdot ---------------
    double Dg[4][4][4];   // Dg[c][a][b] = d_c g_ab
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            Dg[0][a][b] = -al * P[a][b] + bu[0] * F[0][a][b] + bu[1] * F[1][a][b] + bu[2] * F[2][a][b];
#pragma unroll
            for (int x = 0; x < 3; ++x) Dg[x + 1][a][b] = F[x][a][b];
        }
    double Gm[4][4][4];   // Gm[c][a][b] = Gamma_cab
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) Gm[c][a][b] = 0.5 * (Dg[a][b][c] + Dg[b][a][c] - Dg[c][a][b]);
    double Gc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        double t = 0.0;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) t += gI[a][b] * Gm[c][a][b];
        Gc[c] = t;
    }

    // ---- gauge source H_a and d_a H_b ---------------------------------------
    const long long blk = (long long)NV * np;
    double Hl[4], dH[4][4];
    if (NV == 58) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            Hl[b] = u[(50 + b) * np + p];
            dH[0][b] = u[(54 + b) * np + p];   // d_t H_b = Q_b
        }
    } else {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            Hl[b] = s.H[b * np + p];
            dH[0][b] = 0.0;                     // static gauge (eq. gauge)
        }
    }
    {
        const double r = s.rk[k], st = s.sth[i], ct = s.cth[i], sp = s.sph[j], cp = s.cph[j];
        const double ir = 1.0 / r, irs = 1.0 / (r * st);
        const double J[3][3] = {{st * cp, ct * cp * ir, -sp * irs}, {st * sp, ct * sp * ir, cp * irs}, {ct, -st * ir, 0.0}};
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            if (NV == 58) {
                const long long q = (long long)(50 + b) * np + p;
                const double d0 = du[q], d1 = du[blk + q], d2 = du[2 * blk + q];
                if (cart) {
                    dH[1][b] = d0; dH[2][b] = d1; dH[3][b] = d2;
                } else {
#pragma unroll
                    for (int x = 0; x < 3; ++x) dH[x + 1][b] = J[x][0] * d0 + J[x][1] * d1 + J[x][2] * d2;
                }
            } else {
#pragma unroll
                for (int x = 0; x < 3; ++x) dH[x + 1][b] = s.dH[(x * 4 + b) * np + p];
            }
        }
    }
    double Hu[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) Hu[c] = gI[c][0] * Hl[0] + gI[c][1] * Hl[1] + gI[c][2] * Hl[2] + gI[c][3] * Hl[3];
    double C[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) C[c] = Hl[c] + Gc[c];
    const double nC = nu[0] * C[0] + nu[1] * C[1] + nu[2] * C[2] + nu[3] * C[3];

    // ---- undifferentiated terms of eq. Pidot --------------------------------
    double rP[10], rF[3][10], rg[10];
    {
        // Z[x][c][b] = g^cd Phi_xbd,  W[c][b] = g^cd Pi_db
        double Z[3][4][4], Wp[4][4];
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                Wp[c][b] = gI[c][0] * P[0][b] + gI[c][1] * P[1][b] + gI[c][2] * P[2][b] + gI[c][3] * P[3][b];
#pragma unroll
                for (int x = 0; x < 3; ++x)
                    Z[x][c][b] = gI[c][0] * F[x][b][0] + gI[c][1] * F[x][b][1] + gI[c][2] * F[x][b][2] + gI[c][3] * F[x][b][3];
            }
        // Fu[y][a][c] = gamma^xy Phi_xac  (raised derivative index)
        double Fu[3][4][4];
#pragma unroll
        for (int y = 0; y < 3; ++y)
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c) Fu[y][a][c] = gi[y][0] * F[0][a][c] + gi[y][1] * F[1][a][c] + gi[y][2] * F[2][a][c];
        // Gu[b][c][e] = g^cd g^ef Gamma_bdf
        double Gh[4][4][4];
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int f = 0; f < 4; ++f)
                    Gh[b][c][f] = gI[c][0] * Gm[b][0][f] + gI[c][1] * Gm[b][1][f] + gI[c][2] * Gm[b][2][f] + gI[c][3] * Gm[b][3][f];
        // v^y = n^c Pi_cx gamma^xy
        double vP[3];
#pragma unroll
        for (int x = 0; x < 3; ++x) vP[x] = nu[0] * P[0][x + 1] + nu[1] * P[1][x + 1] + nu[2] * P[2][x + 1] + nu[3] * P[3][x + 1];
        double vu[3];
#pragma unroll
        for (int y = 0; y < 3; ++y) vu[y] = gi[y][0] * vP[0] + gi[y][1] * vP[1] + gi[y][2] * vP[2];
        double nnP = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int d = 0; d < 4; ++d) nnP += nu[c] * nu[d] * P[c][d];

#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = a; b < 4; ++b) {
                const int q = pr(a, b);
                double quad = 0.0;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
#pragma unroll
                    for (int y = 0; y < 3; ++y) quad += Fu[y][a][c] * Z[y][c][b];
                    quad -= P[a][c] * Wp[c][b];
                    double gg = 0.0;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        double ge = 0.0;
#pragma unroll
                        for (int f = 0; f < 4; ++f) ge += Gh[b][c][f] * gI[f][e];
                        gg += Gm[a][c][e] * ge;
                    }
                    quad -= gg;
                }
                double nabH = 0.5 * (dH[a][b] + dH[b][a]);
#pragma unroll
                for (int c = 0; c < 4; ++c) nabH -= Hu[c] * Gm[c][a][b];
                double bF = bu[0] * F[0][a][b] + bu[1] * F[1][a][b] + bu[2] * F[2][a][b];
                double damp = -g[a][b] * nC;
                if (b == 0) damp += C[a] * nl0;
                if (a == 0) damp += C[b] * nl0;
                rP[q] = 2.0 * al * quad - 2.0 * al * nabH - 0.5 * al * nnP * P[a][b]
                        - al * (vu[0] * F[0][a][b] + vu[1] * F[1][a][b] + vu[2] * F[2][a][b])
                        + al * damp + bF;
                rg[q] = -al * P[a][b] + bF;
            }
    }

    // ---- undifferentiated terms of eq. Phidot --------------------------------
    {
        // w[x][y] = n^c Phi_x(y)c,  wu[x][z] = w[x][y] gamma^yz
        double nnF[3], wu[3][3];
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            double t = 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int d = 0; d < 4; ++d) t += nu[c] * nu[d] * F[x][c][d];
            nnF[x] = t;
            double w[3];
#pragma unroll
            for (int y = 0; y < 3; ++y)
                w[y] = nu[0] * F[x][y + 1][0] + nu[1] * F[x][y + 1][1] + nu[2] * F[x][y + 1][2] + nu[3] * F[x][y + 1][3];
#pragma unroll
            for (int z = 0; z < 3; ++z) wu[x][z] = w[0] * gi[0][z] + w[1] * gi[1][z] + w[2] * gi[2][z];
        }
#pragma unroll
        for (int x = 0; x < 3; ++x)
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = a; b < 4; ++b) {
                    const int q = pr(a, b);
                    rF[x][q] = 0.5 * al * nnF[x] * P[a][b]
                               + al * (wu[x][0] * F[0][a][b] + wu[x][1] * F[1][a][b] + wu[x][2] * F[2][a][b])
                               - al * F[x][a][b];
                }
    }

    // ---- derivative terms, streamed ------------------------------------------
    {
        const double r = s.rk[k], st = s.sth[i], ct = s.cth[i], sp = s.sph[j], cp = s.cph[j];
        const double ir = 1.0 / r, irs = 1.0 / (r * st);
        const double J[3][3] = {{st * cp, ct * cp * ir, -sp * irs}, {st * sp, ct * sp * ir, cp * irs}, {ct, -st * ir, 0.0}};
        auto cartd = [&](int mu, double d[3]) {
            const long long q = (long long)mu * np + p;
            const double d0 = du[q], d1 = du[blk + q], d2 = du[2 * blk + q];
            if (cart) {
                d[0] = d0; d[1] = d1; d[2] = d2;
            } else {
#pragma unroll
                for (int x = 0; x < 3; ++x) d[x] = J[x][0] * d0 + J[x][1] * d1 + J[x][2] * d2;
            }
        };
#pragma unroll
        for (int q = 0; q < 10; ++q) {
            double d[3];
            cartd(q, d);                                   // d_x g_q
            rP[q] -= bu[0] * d[0] + bu[1] * d[1] + bu[2] * d[2];
#pragma unroll
            for (int x = 0; x < 3; ++x) rF[x][q] += al * d[x];
            cartd(10 + q, d);                              // d_x Pi_q
            rP[q] += bu[0] * d[0] + bu[1] * d[1] + bu[2] * d[2];
#pragma unroll
            for (int x = 0; x < 3; ++x) rF[x][q] -= al * d[x];
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                cartd(20 + 10 * x + q, d);                 // d_y Phi_xq
                rF[x][q] += bu[0] * d[0] + bu[1] * d[1] + bu[2] * d[2];
                rP[q] -= al * (gi[x][0] * d[0] + gi[x][1] * d[1] + gi[x][2] * d[2]);
            }
        }
    }

    // ---- outer boundary: freeze incoming characteristic fields (App. A.3) ----
    if (k == s.n_r - 1) {
        const double xh[3] = {s.sth[i] * s.cph[j], s.sth[i] * s.sph[j], s.cth[i]};
        double su_[3];
#pragma unroll
        for (int x = 0; x < 3; ++x) su_[x] = gi[x][0] * xh[0] + gi[x][1] * xh[1] + gi[x][2] * xh[2];
        const double inorm = 1.0 / sqrt(su_[0] * xh[0] + su_[1] * xh[1] + su_[2] * xh[2]);
        double sl[3], su[3];
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            sl[x] = xh[x] * inorm;
            su[x] = su_[x] * inorm;
        }
#pragma unroll
        for (int q = 0; q < 10; ++q) {
            const double sF = su[0] * rF[0][q] + su[1] * rF[1][q] + su[2] * rF[2][q];
            const double w = 0.5 * (-rg[q] + rP[q] + sF);
            rP[q] = 0.5 * (rg[q] + rP[q] + sF);
#pragma unroll
            for (int x = 0; x < 3; ++x) rF[x][q] = sl[x] * w;
        }
    }

    // ---- output / RK4 stage combination (Sec. 2.5) ---------------------------
    auto emit = [&](int mu, double kv) {
        const long long q = (long long)mu * np + p;
        if (stage == 0) {
            out[q] = kv;
        } else if (stage == 1) {          // k1 at u: acc = u + dt/6 k1, us = u + dt/2 k1
            const double u0 = u[q];
            acc[q] = u0 + dt * (1.0 / 6.0) * kv;
            out[q] = u0 + 0.5 * dt * kv;
        } else if (stage == 2) {          // k2 at us: acc += dt/3 k2, us = u + dt/2 k2
            acc[q] += dt * (1.0 / 3.0) * kv;
            out[q] = ubase[q] + 0.5 * dt * kv;
        } else if (stage == 3) {          // k3: acc += dt/3 k3, us = u + dt k3
            acc[q] += dt * (1.0 / 3.0) * kv;
            out[q] = ubase[q] + dt * kv;
        } else {                          // k4: u = acc + dt/6 k4
            out[q] = acc[q] + dt * (1.0 / 6.0) * kv;
        }
    };
#pragma unroll
    for (int q = 0; q < 10; ++q) emit(q, rg[q]);
#pragma unroll
    for (int q = 0; q < 10; ++q) emit(10 + q, rP[q]);
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int q = 0; q < 10; ++q) emit(20 + 10 * x + q, rF[x][q]);
    if (NV == 58) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            emit(50 + b, dH[0][b]);   // d_t H_b = Q_b
            emit(54 + b, 0.0);        // d_t Q_b = 0
        }
    }
}

// Initial data of App. A.3 from the metric and its Cartesian derivatives
// dg[x][q] (x < 3, q < 10): Phi_xq = d_x g_q, Pi_q = beta^x Phi_xq / alpha
// (d_t g = 0), H_a = -Gamma_a.
__global__ __launch_bounds__(256) void k_initial(KShell s, const double* __restrict__ g10,
                                                 const double* __restrict__ dg, double* __restrict__ u,
                                                 double* __restrict__ H) {
    const long long np = s.npts;
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    double g[4][4], F[3][4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = a; b < 4; ++b) {
            const int q = pr(a, b);
            g[a][b] = g[b][a] = g10[q * np + p];
#pragma unroll
            for (int x = 0; x < 3; ++x) F[x][a][b] = F[x][b][a] = dg[(x * 10 + q) * np + p];
        }
    const double gxx = g[1][1], gxy = g[1][2], gxz = g[1][3], gyy = g[2][2], gyz = g[2][3], gzz = g[3][3];
    const double cxx = gyy * gzz - gyz * gyz, cxy = gxz * gyz - gxy * gzz, cxz = gxy * gyz - gxz * gyy;
    const double cyy = gxx * gzz - gxz * gxz, cyz = gxy * gxz - gxx * gyz, czz = gxx * gyy - gxy * gxy;
    const double idet = 1.0 / (gxx * cxx + gxy * cxy + gxz * cxz);
    const double gi[3][3] = {{cxx * idet, cxy * idet, cxz * idet}, {cxy * idet, cyy * idet, cyz * idet}, {cxz * idet, cyz * idet, czz * idet}};
    const double bl[3] = {g[0][1], g[0][2], g[0][3]};
    double bu[3];
    for (int x = 0; x < 3; ++x) bu[x] = gi[x][0] * bl[0] + gi[x][1] * bl[1] + gi[x][2] * bl[2];
    const double al = sqrt(bu[0] * bl[0] + bu[1] * bl[1] + bu[2] * bl[2] - g[0][0]);
    const double ial2 = 1.0 / (al * al);
    double gI[4][4];
    gI[0][0] = -ial2;
    for (int x = 0; x < 3; ++x) {
        gI[0][x + 1] = gI[x + 1][0] = bu[x] * ial2;
        for (int y = 0; y < 3; ++y) gI[x + 1][y + 1] = gi[x][y] - bu[x] * bu[y] * ial2;
    }
    double P[4][4];
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) P[a][b] = (bu[0] * F[0][a][b] + bu[1] * F[1][a][b] + bu[2] * F[2][a][b]) / al;
    // d_t g = 0: Dg[0] = 0, Dg[x+1] = F[x]
    for (int c = 0; c < 4; ++c) {
        double t = 0.0;
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                const double dab_c = (a == 0 ? 0.0 : F[a - 1][b][c]);
                const double dba_c = (b == 0 ? 0.0 : F[b - 1][a][c]);
                const double dc_ab = (c == 0 ? 0.0 : F[c - 1][a][b]);
                t += gI[a][b] * 0.5 * (dab_c + dba_c - dc_ab);
            }
        if (H) H[c * np + p] = -t;
        if (s.n_v == 58) u[(50 + c) * np + p] -= t;
    }
    for (int a = 0; a < 4; ++a)
        for (int b = a; b < 4; ++b) {
            const int q = pr(a, b);
            u[q * np + p] = g[a][b];
            u[(10 + q) * np + p] = P[a][b];
            for (int x = 0; x < 3; ++x) u[(20 + 10 * x + q) * np + p] = F[x][a][b];
        }
}

__global__ __launch_bounds__(256) void k_finite(const double* __restrict__ u, size_t n, int* flag) {
    int bad = 0;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        bad |= !isfinite(u[e]);
    if (bad) atomicOr(flag, 1);
}

}  // namespace

hipError_t launch_rhs(const KShell& s, const double* u, const double* du, bool cart, double* out,
                      const double* ubase, double* acc, double dt, int stage, hipStream_t st) {
    const unsigned blocks = (unsigned)((s.npts + 255) / 256);
    if (s.n_v == 58)
        hipLaunchKernelGGL(k_rhs<58>, dim3(blocks), dim3(256), 0, st, s, u, du, cart ? 1 : 0, out, ubase, acc, dt, stage);
    else
        hipLaunchKernelGGL(k_rhs<50>, dim3(blocks), dim3(256), 0, st, s, u, du, cart ? 1 : 0, out, ubase, acc, dt, stage);
    return hipGetLastError();
}

hipError_t launch_initial(const KShell& s, const double* g10, const double* dg, double* u, double* H,
                          hipStream_t st) {
    const unsigned blocks = (unsigned)((s.npts + 255) / 256);
    hipLaunchKernelGGL(k_initial, dim3(blocks), dim3(256), 0, st, s, g10, dg, u, H);
    return hipGetLastError();
}

hipError_t launch_finite_check(const double* u, size_t n, int* flag, hipStream_t st) {
    hipLaunchKernelGGL(k_finite, dim3(1024), dim3(256), 0, st, u, n, flag);
    return hipGetLastError();
}

}  // namespace sg
