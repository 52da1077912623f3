// Pointwise first-order GHG right-hand side (App. A.1 eqs. gdot, Phidot,
// Pidot with gamma_0 = gamma_2 = 1, gamma_1 = -1), fused with the Cartesian
// chain rule (Sec. 2.2), the freezing-incoming boundary operator on the outer
// sphere (App. A.3) and the RK4 stage combination (Sec. 2.5).
//
// The derivative terms and the boundary operator couple only the fields of
// one symmetric index pair ab (g_ab, Pi_ab, Phi_xab); the quadratic terms of
// eq. Pidot for a pair need only rows a and b.  The work of a grid point is
// therefore split by pair across the waves of a workgroup (see k_rhs).
#include "internal.h"
#include "constraints.h"

namespace sg {

namespace {

__host__ __device__ constexpr int pr(int a, int b) {
    // symmetric pair index, order tt tx ty tz xx xy xz yy yz zz
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    return lo == 0 ? hi : (lo == 1 ? 3 + hi : (lo == 2 ? 5 + hi : 9));
}

// Symmetric pair q = (a, b), a <= b, in storage order.
__host__ __device__ constexpr int pair_a(int q) { return q < 4 ? 0 : (q < 7 ? 1 : (q < 9 ? 2 : 3)); }
__host__ __device__ constexpr int pair_b(int q) { return q < 4 ? q : (q < 7 ? q - 3 : (q < 9 ? q - 5 : 3)); }
static_assert(pair_a(5) == 1 && pair_b(5) == 2 && pair_a(8) == 2 && pair_b(8) == 3, "pair order");

template <int Q>
struct PairC {
    static constexpr int value = Q;
};

constexpr int kPts = 64;      // grid points per workgroup
constexpr int kWaves = 4;     // waves per workgroup

// Workgroup = 64 consecutive grid points (one per lane) x 4 waves; at 256
// VGPRs and 56 KB of LDS two workgroups share a CU.  The points' variables
// are staged in LDS ([item][lane], conflict-free); every wave recomputes the
// 3+1 quantities in registers, a few per-point vectors shared by all pairs
// are formed once into LDS, and then wave w evaluates everything that belongs
// to its symmetric pairs ab (three pairs for waves 0 and 1, two for 2 and 3,
// all sharing one index): the sources and derivative terms of d_t g_ab,
// d_t Pi_ab and d_t Phi_xab, the boundary operator (which couples only fields
// of one pair) and the RK4 stage update.
template <int NV, typename TD>
__global__ __launch_bounds__(kWaves * 64, 2) void k_rhs(KShell s, const double* __restrict__ u,
                                             const double* __restrict__ du, const TD* __restrict__ dang, int cart,
                                             double* __restrict__ out, const double* __restrict__ ubase,
                                             double* __restrict__ acc, double dt, int stage, long long blk) {
    // blockIdx.y: shell of a run of identical shells stored one after the
    // other; blk: stride between the derivative blocks (d_r, d_theta, d_phi).
    {
        const long long so = (long long)blockIdx.y * NV * s.npts;
        u += so;
        du += so;
        dang += so;
        out += so;
        if (ubase) ubase += so;
        if (acc) acc += so;
        s.H += (long long)blockIdx.y * 4 * s.npts;
        s.dH += (long long)blockIdx.y * 12 * s.npts;
    }
    __shared__ double su[NV][kPts];          // state of the 64 points
    __shared__ double sH[4][kPts];           // H_a
    __shared__ double sdH[4][4][kPts];       // d_a H_b (a = t from the state or 0)
    __shared__ double sdtg[10][kPts];        // d_t g_ab, eq. gdot
    __shared__ double sC[4][kPts];           // C_a = H_a + Gamma_a
    __shared__ double sHu[4][kPts];          // H^a = g^ab H_b
    __shared__ double sv[7][kPts];           // n.n.Pi, (n^c Pi_cx gamma^xy)_y, n.n.Phi_x
    __shared__ double swu[3][3][kPts];       // n^c Phi_x(y)c gamma^yz

    const long long np = s.npts;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const long long p0 = (long long)blockIdx.x * kPts;
    const long long p = p0 + lane;
    const bool ok = p < np;
    // Every global load below uses pc, a point inside the shell for every
    // lane (lanes past the end read the last point and store nothing), so
    // that the loads of a phase sit in one basic block with no per-lane
    // branch and are all in flight before the first wait: the kernel is
    // bound by how many memory latencies a wave waits out one after another.
    const long long pc = ok ? p : np - 1;

    // ---- per-thread geometry (every thread's point is its lane: the staging
    // loops below step by a multiple of 64) ------------------------------------
    const int k = ok ? (int)(p % s.n_r) : 0;
    const int i = ok ? (int)((p / s.n_r) % s.n_th) : 0;
    const int j = ok ? (int)(p / ((long long)s.n_r * s.n_th)) : 0;
    const double st = s.sth[i], ct = s.cth[i], sp = s.sph[j], cp = s.cph[j];

    // ---- stage the variables; points past the end get Minkowski data --------
    {
        constexpr int kT = (NV + kWaves - 1) / kWaves;
        double v[kT];
#pragma unroll
        for (int t = 0; t < kT; ++t) v[t] = u[(long long)min(w + t * kWaves, NV - 1) * np + pc];
#pragma unroll
        for (int t = 0; t < kT; ++t) {
            const int f = w + t * kWaves;
            if (f < NV) su[f][lane] = ok ? v[t] : ((f == 0) ? -1.0 : ((f == 4 || f == 7 || f == 9) ? 1.0 : 0.0));
        }
    }
    if (NV == 50) {
        // rows f = w + 4 t of the [16][64] block H_a (f < 4), d_x H_b (f >= 4)
        double v[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int f = w + 4 * t;
            v[t] = (f < 4) ? s.H[(long long)f * np + pc] : s.dH[(long long)(f - 4) * np + pc];
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int f = w + 4 * t;
            const double h = ok ? v[t] : 0.0;
            if (f < 4) {
                sH[f][lane] = h;
                sdH[0][f][lane] = 0.0;                            // static gauge, eq. gauge
            } else {
                const int x = (f - 4) >> 2, b = (f - 4) & 3;      // Cartesian d_x H_b
                sdH[x + 1][b][lane] = h;
            }
        }
    }
    __syncthreads();

    // ---- 3+1 split (eqs. normal, abgfromgab) ----------------------------------
    auto G = [&](int a, int b) -> double { return su[pr(a, b)][lane]; };
    auto PI = [&](int a, int b) -> double { return su[10 + pr(a, b)][lane]; };
    auto PH = [&](int x, int a, int b) -> double { return su[20 + 10 * x + pr(a, b)][lane]; };
    const double gxx = G(1, 1), gxy = G(1, 2), gxz = G(1, 3), gyy = G(2, 2), gyz = G(2, 3), gzz = G(3, 3);
    const double cxx = gyy * gzz - gyz * gyz, cxy = gxz * gyz - gxy * gzz, cxz = gxy * gyz - gxz * gyy;
    const double cyy = gxx * gzz - gxz * gxz, cyz = gxy * gxz - gxx * gyz, czz = gxx * gyy - gxy * gxy;
    const double idet = 1.0 / (gxx * cxx + gxy * cxy + gxz * cxz);
    const double gi[3][3] = {{cxx * idet, cxy * idet, cxz * idet},
                             {cxy * idet, cyy * idet, cyz * idet},
                             {cxz * idet, cyz * idet, czz * idet}};
    const double bl[3] = {G(0, 1), G(0, 2), G(0, 3)};
    double bu[3];
#pragma unroll
    for (int x = 0; x < 3; ++x) bu[x] = gi[x][0] * bl[0] + gi[x][1] * bl[1] + gi[x][2] * bl[2];
    const double al = sqrt(bu[0] * bl[0] + bu[1] * bl[1] + bu[2] * bl[2] - G(0, 0));
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
    // Derivatives of u_mu at this thread's point: load3 issues the three
    // loads (no wait), tocart forms the Cartesian d_x u_mu, x = 0..2, by the
    // chain rule of Sec. 2.2 (eq. dvdx) with the analytic Jacobian
    // d(r, theta, phi)/d(x, y, z)
    auto load3 = [&](int mu, double d[3]) {
        const long long q = (long long)mu * np + pc;
        d[0] = du[q];
        d[1] = (double)dang[q];
        d[2] = (double)dang[blk + q];
    };
    const double ir = 1.0 / s.rk[k], irs = ir / st;
    auto tocart = [&](double d[3]) {
        if (!cart) {
            const double d0 = d[0], d1 = d[1], d2 = d[2];
            d[0] = st * cp * d0 + ct * cp * ir * d1 - sp * irs * d2;
            d[1] = st * sp * d0 + ct * sp * ir * d1 + cp * irs * d2;
            d[2] = ct * d0 - st * ir * d1;
        }
    };

    // ---- shared per-point quantities, phase 1 --------------------------------
    if (w == 0) {
#pragma unroll
        for (int q = 0; q < 10; ++q) {
            const int a = pair_a(q), b = pair_b(q);
            sdtg[q][lane] = -al * PI(a, b) + bu[0] * PH(0, a, b) + bu[1] * PH(1, a, b) + bu[2] * PH(2, a, b);
        }
    } else if (w == 1) {
        if (NV == 58) {
            double d[4][3];
#pragma unroll
            for (int b = 0; b < 4; ++b) load3(50 + b, d[b]);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                sH[b][lane] = su[50 + b][lane];
                sdH[0][b][lane] = su[54 + b][lane];              // d_t H_b = Q_b
                tocart(d[b]);
#pragma unroll
                for (int x = 0; x < 3; ++x) sdH[x + 1][b][lane] = d[b][x];
            }
        }
    } else if (w == 2) {
        double nnP = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int d = 0; d < 4; ++d) nnP += nu[c] * nu[d] * PI(c, d);
        sv[0][lane] = nnP;
        double vP[3];
#pragma unroll
        for (int x = 0; x < 3; ++x)
            vP[x] = nu[0] * PI(0, x + 1) + nu[1] * PI(1, x + 1) + nu[2] * PI(2, x + 1) + nu[3] * PI(3, x + 1);
#pragma unroll
        for (int y = 0; y < 3; ++y) sv[1 + y][lane] = gi[y][0] * vP[0] + gi[y][1] * vP[1] + gi[y][2] * vP[2];
    } else if (w == 3) {
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            double t = 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int d = 0; d < 4; ++d) t += nu[c] * nu[d] * PH(x, c, d);
            sv[4 + x][lane] = t;
            double wv[3];
#pragma unroll
            for (int y = 0; y < 3; ++y)
                wv[y] = nu[0] * PH(x, y + 1, 0) + nu[1] * PH(x, y + 1, 1) + nu[2] * PH(x, y + 1, 2) + nu[3] * PH(x, y + 1, 3);
#pragma unroll
            for (int z = 0; z < 3; ++z) swu[x][z][lane] = wv[0] * gi[0][z] + wv[1] * gi[1][z] + wv[2] * gi[2][z];
        }
    }
    __syncthreads();

    // d_c g_ab (c = t from eq. gdot, c = x: Phi) and Gamma_cab (eq. Gamma)
    auto Dg = [&](int c, int a, int b) -> double { return c == 0 ? sdtg[pr(a, b)][lane] : PH(c - 1, a, b); };
    auto Gam = [&](int c, int a, int b) -> double { return 0.5 * (Dg(a, b, c) + Dg(b, a, c) - Dg(c, a, b)); };

    // ---- shared per-point quantities, phase 2 --------------------------------
    if (w == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double t = 0.0;
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) t += gI[a][b] * Gam(c, a, b);
            sC[c][lane] = sH[c][lane] + t;   // C_c = H_c + Gamma_c
        }
    } else if (w == 1) {
#pragma unroll
        for (int c = 0; c < 4; ++c)
            sHu[c][lane] = gI[c][0] * sH[0][lane] + gI[c][1] * sH[1][lane] + gI[c][2] * sH[2][lane] + gI[c][3] * sH[3][lane];
    }
    __syncthreads();
    const double nC = nu[0] * sC[0][lane] + nu[1] * sC[1][lane] + nu[2] * sC[2][lane] + nu[3] * sC[3][lane];

    // derivative loads of pair q (g_ab, Pi_ab, Phi_xab; no wait)
    auto load_pair = [&](int q, double (&d)[5][3]) {
        load3(q, d[0]);
        load3(10 + q, d[1]);
#pragma unroll
        for (int y = 0; y < 3; ++y) load3(20 + 10 * y + q, d[2 + y]);
    };
    // sources, derivative terms, boundary operator and stage update of pair
    // (a, b), given its quadratic bracket and its loaded derivatives d; the
    // derivative loads of the wave's next pair (NC >= 0) are issued into dn
    // together with this pair's stage-update reads, so their latency overlaps
    // this pair's stores
    auto pair_tail = [&](auto AC, auto BC, double quad, double (&d)[5][3], auto NC, double (&dn)[5][3]) {
        constexpr int a = decltype(AC)::value < decltype(BC)::value ? decltype(AC)::value : decltype(BC)::value;
        constexpr int b = decltype(AC)::value < decltype(BC)::value ? decltype(BC)::value : decltype(AC)::value;
        constexpr int q = pr(a, b);
        double(&dg)[3] = d[0];
        double(&dP)[3] = d[1];
        double dF[3][3];
#pragma unroll
        for (int y = 0; y < 3; ++y)
#pragma unroll
            for (int x = 0; x < 3; ++x) dF[y][x] = d[2 + y][x];
        tocart(dg);
        tocart(dP);
#pragma unroll
        for (int y = 0; y < 3; ++y) tocart(dF[y]);
        double nabH = 0.5 * (sdH[a][b][lane] + sdH[b][a][lane]);
#pragma unroll
        for (int c = 0; c < 4; ++c) nabH -= sHu[c][lane] * Gam(c, a, b);
        const double Pab = PI(a, b);
        const double Fab[3] = {PH(0, a, b), PH(1, a, b), PH(2, a, b)};
        const double bF = bu[0] * Fab[0] + bu[1] * Fab[1] + bu[2] * Fab[2];
        double damp = -G(a, b) * nC;
        if (b == 0) damp += sC[a][lane] * nl0;
        if (a == 0) damp += sC[b][lane] * nl0;
        // eq. Pidot
        double rP = 2.0 * al * quad - 2.0 * al * nabH - 0.5 * al * sv[0][lane] * Pab
                    - al * (sv[1][lane] * Fab[0] + sv[2][lane] * Fab[1] + sv[3][lane] * Fab[2]) + al * damp + bF;
        rP += -(bu[0] * dg[0] + bu[1] * dg[1] + bu[2] * dg[2]) + (bu[0] * dP[0] + bu[1] * dP[1] + bu[2] * dP[2]);
#pragma unroll
        for (int x = 0; x < 3; ++x) rP -= al * (gi[x][0] * dF[x][0] + gi[x][1] * dF[x][1] + gi[x][2] * dF[x][2]);
        // eq. Phidot
        double rF[3];
#pragma unroll
        for (int x = 0; x < 3; ++x)
            rF[x] = 0.5 * al * sv[4 + x][lane] * Pab
                    + al * (swu[x][0][lane] * Fab[0] + swu[x][1][lane] * Fab[1] + swu[x][2][lane] * Fab[2]) - al * Fab[x]
                    + al * dg[x] - al * dP[x] + bu[0] * dF[x][0] + bu[1] * dF[x][1] + bu[2] * dF[x][2];
        // eq. gdot
        double rg = -al * Pab + bF;
        // outer boundary: freeze incoming characteristic fields (App. A.3); an
        // interface sphere of nested shells is coupled by k_patch instead
        if (k == s.n_r - 1 && !s.kraw_out) {
            const double xh[3] = {st * cp, st * sp, ct};
            double su_[3];
#pragma unroll
            for (int x = 0; x < 3; ++x) su_[x] = gi[x][0] * xh[0] + gi[x][1] * xh[1] + gi[x][2] * xh[2];
            const double inorm = 1.0 / sqrt(su_[0] * xh[0] + su_[1] * xh[1] + su_[2] * xh[2]);
            const double sF = (su_[0] * rF[0] + su_[1] * rF[1] + su_[2] * rF[2]) * inorm;
            const double wv = 0.5 * (-rg + rP + sF);
            rP = 0.5 * (rg + rP + sF);
#pragma unroll
            for (int x = 0; x < 3; ++x) rF[x] = xh[x] * inorm * wv;
        }
        double av[5], bv[5];
        if (stage >= 2) {
#pragma unroll
            for (int m = 0; m < 5; ++m) av[m] = acc[(long long)(q + 10 * m) * np + pc];
        }
        if (stage == 2 || stage == 3) {
#pragma unroll
            for (int m = 0; m < 5; ++m) bv[m] = ubase[(long long)(q + 10 * m) * np + pc];
        }
        if constexpr (decltype(NC)::value >= 0) load_pair(decltype(NC)::value, dn);
        if (ok) {
            const long long nang = np / s.n_r, ang = p / s.n_r;   // angular point of this lane
            double* kraw = (k == s.n_r - 1) ? s.kraw_out : (k == 0 ? s.kraw_in : nullptr);
            auto emit = [&](int m, double kv) {
                const int mu = q + 10 * m;
                const long long o = (long long)mu * np + p;
                if (kraw) kraw[mu * nang + ang] = kv;
                if (stage == 0) {
                    out[o] = kv;
                } else if (stage == 1) {        // k1 at u: acc = u + dt/6 k1, us = u + dt/2 k1
                    const double u0 = su[mu][lane];
                    acc[o] = u0 + dt * (1.0 / 6.0) * kv;
                    out[o] = u0 + 0.5 * dt * kv;
                } else if (stage == 2) {        // k2 at us: acc += dt/3 k2, us = u + dt/2 k2
                    acc[o] = av[m] + dt * (1.0 / 3.0) * kv;
                    out[o] = bv[m] + 0.5 * dt * kv;
                } else if (stage == 3) {        // k3: acc += dt/3 k3, us = u + dt k3
                    acc[o] = av[m] + dt * (1.0 / 3.0) * kv;
                    out[o] = bv[m] + dt * kv;
                } else {                        // k4: u = acc + dt/6 k4
                    out[o] = av[m] + dt * (1.0 / 6.0) * kv;
                }
            };
            emit(0, rg);
            emit(1, rP);
#pragma unroll
            for (int x = 0; x < 3; ++x) emit(2 + x, rF[x]);
            if constexpr (NV == 58 && q == 6) {   // d_t H_c = Q_c, d_t Q_c = 0
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const long long o = (long long)(50 + c) * np + p;
                    const double kv = c < 4 ? sdH[0][c][lane] : 0.0;
                    if (kraw) kraw[(50 + c) * nang + ang] = kv;
                    const double u0 = su[50 + c][lane];
                    if (stage == 0) {
                        out[o] = kv;
                    } else if (stage == 1) {
                        acc[o] = u0 + dt * (1.0 / 6.0) * kv;
                        out[o] = u0 + 0.5 * dt * kv;
                    } else if (stage == 2) {
                        acc[o] += dt * (1.0 / 3.0) * kv;
                        out[o] = ubase[o] + 0.5 * dt * kv;
                    } else if (stage == 3) {
                        acc[o] += dt * (1.0 / 3.0) * kv;
                        out[o] = ubase[o] + dt * kv;
                    } else {
                        out[o] = acc[o] + dt * (1.0 / 6.0) * kv;
                    }
                }
            }
        }
    };
    // ---- the wave's two symmetric pairs (a1, b) and (a2, b) share the index b,
    // so the b-dependent contractions of the quadratic term are formed once;
    // all indices are compile-time constants in each instance of the body, so
    // every LDS offset and every branch on the indices folds away -------------
    auto wave_pairs = [&](auto BC, auto A1C, auto A2C, auto A3C) {
        constexpr int b = decltype(BC)::value, a1 = decltype(A1C)::value, a2 = decltype(A2C)::value;
        constexpr int a3 = decltype(A3C)::value < 0 ? a2 : decltype(A3C)::value;   // < 0: no third pair
        constexpr bool three = decltype(A3C)::value >= 0;
        // quadratic bracket of eq. Pidot for (a, b),
        //   g^cd (gamma^ij Phi_iac Phi_jbd - Pi_ac Pi_bd) - g^cd g^ef Gamma_ace Gamma_bdf
        //   = Phi_xac Z_xc - Pi_ac V_c - Gamma_ace Y^ce,
        // with Z_xc = g^cd gamma^xy Phi_ybd, V_c = g^cd Pi_bd and
        // Y = G Gamma_b G (Gamma_b the 4x4 matrix Gamma_bdf), all of row b.
        // Contractions streamed so that few values are live at a time (the
        // register budget decides how many workgroups share a CU): Phi part
        // per spatial x, Pi part per c, Gamma part per column e of G Gamma_b.
        constexpr int q1 = pr(a1, b), q2 = pr(a2, b), q3 = three ? pr(a3, b) : -1;
        double dA[5][3], dB[5][3];
        load_pair(q1, dA);
        __builtin_amdgcn_sched_barrier(0);
        double quad1 = 0.0, quad2 = 0.0, quad3 = 0.0;
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            double pbx[4];   // gamma^xy Phi_ybd
#pragma unroll
            for (int d = 0; d < 4; ++d) pbx[d] = gi[x][0] * PH(0, b, d) + gi[x][1] * PH(1, b, d) + gi[x][2] * PH(2, b, d);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double z = gI[c][0] * pbx[0] + gI[c][1] * pbx[1] + gI[c][2] * pbx[2] + gI[c][3] * pbx[3];
                quad1 += PH(x, a1, c) * z;
                quad2 += PH(x, a2, c) * z;
                if (three) quad3 += PH(x, a3, c) * z;
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double v = gI[c][0] * PI(b, 0) + gI[c][1] * PI(b, 1) + gI[c][2] * PI(b, 2) + gI[c][3] * PI(b, 3);
            quad1 -= PI(a1, c) * v;
            quad2 -= PI(a2, c) * v;
            if (three) quad3 -= PI(a3, c) * v;
        }
        {
            double gb[4][4];   // Gamma_bdf (symmetric in d, f)
#pragma unroll
            for (int d = 0; d < 4; ++d)
#pragma unroll
                for (int f = d; f < 4; ++f) gb[d][f] = gb[f][d] = Gam(b, d, f);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                double t[4];   // Gamma_bdf g^fe
#pragma unroll
                for (int d = 0; d < 4; ++d)
                    t[d] = gb[d][0] * gI[0][e] + gb[d][1] * gI[1][e] + gb[d][2] * gI[2][e] + gb[d][3] * gI[3][e];
#pragma unroll
                for (int c = 0; c <= e; ++c) {   // Y^ce = g^cd t_d, symmetric: off-diagonal twice
                    const double y = (c == e ? 1.0 : 2.0) *
                                     (gI[c][0] * t[0] + gI[c][1] * t[1] + gI[c][2] * t[2] + gI[c][3] * t[3]);
                    quad1 -= Gam(a1, c, e) * y;
                    quad2 -= Gam(a2, c, e) * y;
                    if (three) quad3 -= Gam(a3, c, e) * y;
                }
                }
        }
        // the barriers keep each pair's loads where they are placed
        // (register pressure)
        __builtin_amdgcn_sched_barrier(0);
        pair_tail(A1C, BC, quad1, dA, PairC<q2>{}, dB);
        __builtin_amdgcn_sched_barrier(0);
        pair_tail(A2C, BC, quad2, dB, PairC<q3>{}, dA);
        if constexpr (three) {
            __builtin_amdgcn_sched_barrier(0);
            pair_tail(PairC<a3>{}, BC, quad3, dA, PairC<-1>{}, dB);
        }
    };
    using None = PairC<-1>;
    switch (w) {   // pairs tt tx ty | xx xy xz | yy yz | zz tz
        case 0: wave_pairs(PairC<0>{}, PairC<0>{}, PairC<1>{}, PairC<2>{}); break;
        case 1: wave_pairs(PairC<1>{}, PairC<1>{}, PairC<2>{}, PairC<3>{}); break;
        case 2: wave_pairs(PairC<2>{}, PairC<2>{}, PairC<3>{}, None{}); break;
        default: wave_pairs(PairC<3>{}, PairC<3>{}, PairC<0>{}, None{}); break;
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

// Constraint fields of App. A.1 at every point of a shell, reduced per
// workgroup: C_a = H_a + Gamma_a and C_iab = d_i g_ab - Phi_iab with d_i g_ab
// the Cartesian spectral derivative dg[i * dblk + pair * npts + point] (dblk:
// stride between the x, y, z blocks).  part[blk][4] = (max |C_a|, sum C_a^2,
// max |C_iab|, sum C_iab^2) over the workgroup's points.
__global__ __launch_bounds__(256) void k_constraints(KShell s, const double* __restrict__ u,
                                                     const double* __restrict__ dg, long long dblk,
                                                     double* __restrict__ part) {
    __shared__ double red[4][256];
    const long long np = s.npts;
    const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
    double mxa = 0.0, ssa = 0.0, mxi = 0.0, ssi = 0.0;
    if (p < np) {
        gauge_constraint(s, u, p, mxa, ssa);
#pragma unroll
        for (int x = 0; x < 3; ++x)
#pragma unroll
            for (int q = 0; q < 10; ++q) {
                const double ci = dg[x * dblk + q * np + p] - u[(20 + 10 * x + q) * np + p];
                mxi = fmax(mxi, fabs(ci));
                ssi += ci * ci;
            }
    }
    reduce4(red, mxa, ssa, mxi, ssi);
    if (threadIdx.x < 4) part[(long long)blockIdx.x * 4 + threadIdx.x] = red[threadIdx.x][0];
}

// norms[0..3] = (max |C_a|, rms C_a, max |C_iab|, rms C_iab) from n_part
// workgroup partials; rms over 4 (resp. 30) components x npts points.
__global__ __launch_bounds__(256) void k_constraint_norms(const double* __restrict__ part, int n_part,
                                                          long long npts, double* __restrict__ norms) {
    __shared__ double red[4][256];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < n_part; b += 256) {
        v[0] = fmax(v[0], part[b * 4]);
        v[1] += part[b * 4 + 1];
        v[2] = fmax(v[2], part[b * 4 + 2]);
        v[3] += part[b * 4 + 3];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + h]);
            red[1][threadIdx.x] += red[1][threadIdx.x + h];
            red[2][threadIdx.x] = fmax(red[2][threadIdx.x], red[2][threadIdx.x + h]);
            red[3][threadIdx.x] += red[3][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        norms[0] = red[0][0];
        norms[1] = sqrt(red[1][0] / (4.0 * (double)npts));
        norms[2] = red[2][0];
        norms[3] = sqrt(red[3][0] / (30.0 * (double)npts));
    }
}

// Interface of nested shells a (inside) and b (outside) sharing a sphere
// (the outlook of Sec. 1 and Sec. 5; the interface condition is this
// library's reading): both copies of the sphere get one right-hand side.  For
// every symmetric pair the raw right-hand sides are taken apart into the
// characteristic fields of App. A.2 (eq. characteristics) with s_i the unit
// normal from a into b: u^0 = g (speed 0), u^1+- = -g + Pi +- s^k Phi_k
// (speeds +-alpha - b), u^2_i = P^k_i Phi_k (speed -b), b = s_k beta^k; each
// is taken from the side it travels from (speed > 0: a, < 0: b, 0: the mean)
// and transformed back:
//   d g = u^0,  d Pi = u^0 + (u^1+ + u^1-)/2,  d Phi_i = s_i (u^1+ - u^1-)/2 + u^2_i.
// The gauge fields of the 58-field form (no spatial derivatives) take the
// mean.  The copies' stage outputs were formed from the raw right-hand
// sides; they are corrected here by the stage coefficients times the
// difference (stage 0: the output is the right-hand side).
// Thread (angular point, pair q): blockIdx.y = q for the ten symmetric pairs,
// q = 10 for the gauge fields of the 58-field form; every load of a thread is
// issued before the first use (a patch launch is a few dozen workgroups, so
// the time is the threads' chains of memory latencies).
__global__ __launch_bounds__(256) void k_patch(KShell sa, KShell sb, const double* __restrict__ ua,
                                               const double* __restrict__ ka, const double* __restrict__ kb,
                                               double* __restrict__ out_a, double* __restrict__ acc_a,
                                               double* __restrict__ out_b, double* __restrict__ acc_b, double dt,
                                               int stage) {
    const long long nang = (long long)sa.n_th * sa.n_ph;
    const long long ang = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int q = blockIdx.y;
    if (ang >= nang) return;
    const long long pa = (long long)(sa.n_r - 1) + sa.n_r * ang, pb = (long long)sb.n_r * ang;
    const long long npa = sa.npts, npb = sb.npts;
    double co = 1.0, cacc = 0.0;   // stage coefficients of out and acc (RK4, Sec. 2.5)
    if (stage == 1) { co = 0.5 * dt; cacc = dt / 6.0; }
    else if (stage == 2) { co = 0.5 * dt; cacc = dt / 3.0; }
    else if (stage == 3) { co = dt; cacc = dt / 3.0; }
    else if (stage == 4) { co = dt / 6.0; }
    // the thread's fields, their two raw right-hand sides and stage values
    constexpr int kF = 8;
    int mu[kF];
    int nf;
    if (q < 10) {
        nf = 5;
        mu[0] = q;
        mu[1] = 10 + q;
        mu[2] = 20 + q;
        mu[3] = 30 + q;
        mu[4] = 40 + q;
    } else {
        nf = sa.n_v - 50;
#pragma unroll
        for (int t = 0; t < kF; ++t) mu[t] = 50 + t;
    }
    double k_a[kF], k_b[kF], oa_[kF], ob_[kF], aa_[kF], ab_[kF];
#pragma unroll
    for (int t = 0; t < kF; ++t) {
        if (t < nf) {
            k_a[t] = ka[mu[t] * nang + ang];
            k_b[t] = kb[mu[t] * nang + ang];
            if (stage != 0) {
                oa_[t] = out_a[mu[t] * npa + pa];
                ob_[t] = out_b[mu[t] * npb + pb];
            }
            if (cacc != 0.0) {
                aa_[t] = acc_a[mu[t] * npa + pa];
                ab_[t] = acc_b[mu[t] * npb + pb];
            }
        }
    }
    double kp[kF];
    if (q < 10) {
        // 3+1 quantities of the state at the sphere (the copies are equal)
        const int i = (int)(ang % sa.n_th), j = (int)(ang / sa.n_th);
        double g[10];
#pragma unroll
        for (int c = 0; c < 10; ++c) g[c] = ua[c * npa + pa];
        const double gxx = g[4], gxy = g[5], gxz = g[6], gyy = g[7], gyz = g[8], gzz = g[9];
        const double cxx = gyy * gzz - gyz * gyz, cxy = gxz * gyz - gxy * gzz, cxz = gxy * gyz - gxz * gyy;
        const double cyy = gxx * gzz - gxz * gxz, cyz = gxy * gxz - gxx * gyz, czz = gxx * gyy - gxy * gxy;
        const double idet = 1.0 / (gxx * cxx + gxy * cxy + gxz * cxz);
        const double gi[3][3] = {{cxx * idet, cxy * idet, cxz * idet},
                                 {cxy * idet, cyy * idet, cyz * idet},
                                 {cxz * idet, cyz * idet, czz * idet}};
        const double bl[3] = {g[1], g[2], g[3]};
        double bu[3];
#pragma unroll
        for (int x = 0; x < 3; ++x) bu[x] = gi[x][0] * bl[0] + gi[x][1] * bl[1] + gi[x][2] * bl[2];
        const double al = sqrt(bu[0] * bl[0] + bu[1] * bl[1] + bu[2] * bl[2] - g[0]);
        const double st = sa.sth[i], ct = sa.cth[i], sp = sa.sph[j], cp = sa.cph[j];
        const double xh[3] = {st * cp, st * sp, ct};
        double su_[3];
#pragma unroll
        for (int x = 0; x < 3; ++x) su_[x] = gi[x][0] * xh[0] + gi[x][1] * xh[1] + gi[x][2] * xh[2];
        const double inorm = 1.0 / sqrt(su_[0] * xh[0] + su_[1] * xh[1] + su_[2] * xh[2]);
        double sl[3], sup[3];
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            sl[x] = xh[x] * inorm;
            sup[x] = su_[x] * inorm;
        }
        const double b = sl[0] * bu[0] + sl[1] * bu[1] + sl[2] * bu[2];
        // 0: from a, 1: from b, 0.5: mean (speed 0)
        auto pick = [](double v) { return v > 0.0 ? 0.0 : (v < 0.0 ? 1.0 : 0.5); };
        const double wp = pick(al - b), wm = pick(-al - b), wt = pick(-b);
        double c2[2][6];   // u^0, u^1+, u^1-, u^2_x, u^2_y, u^2_z of each side
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const double* kk = side ? k_b : k_a;
            const double dg = kk[0], dP = kk[1];
            const double dF[3] = {kk[2], kk[3], kk[4]};
            const double sF = sup[0] * dF[0] + sup[1] * dF[1] + sup[2] * dF[2];
            c2[side][0] = dg;
            c2[side][1] = -dg + dP + sF;
            c2[side][2] = -dg + dP - sF;
#pragma unroll
            for (int x = 0; x < 3; ++x) c2[side][3 + x] = dF[x] - sl[x] * sF;
        }
        const double u0 = 0.5 * (c2[0][0] + c2[1][0]);
        const double up = (1.0 - wp) * c2[0][1] + wp * c2[1][1];
        const double um = (1.0 - wm) * c2[0][2] + wm * c2[1][2];
        kp[0] = u0;
        kp[1] = u0 + 0.5 * (up + um);
#pragma unroll
        for (int x = 0; x < 3; ++x) kp[2 + x] = sl[x] * 0.5 * (up - um) + (1.0 - wt) * c2[0][3 + x] + wt * c2[1][3 + x];
    } else {
#pragma unroll
        for (int t = 0; t < kF; ++t) kp[t] = 0.5 * (k_a[t] + k_b[t]);
    }
#pragma unroll
    for (int t = 0; t < kF; ++t) {
        if (t >= nf) continue;
        const long long oa = mu[t] * npa + pa, ob = mu[t] * npb + pb;
        if (stage == 0) {
            out_a[oa] = kp[t];
            out_b[ob] = kp[t];
            continue;
        }
        const double da = kp[t] - k_a[t], db = kp[t] - k_b[t];
        out_a[oa] = oa_[t] + co * da;
        out_b[ob] = ob_[t] + co * db;
        if (cacc != 0.0) {
            acc_a[oa] = aa_[t] + cacc * da;
            acc_b[ob] = ab_[t] + cacc * db;
        }
    }
}

__global__ __launch_bounds__(256) void k_finite(const double* __restrict__ u, size_t n, int* flag) {
    int bad = 0;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        bad |= !isfinite(u[e]);
    if (bad) atomicOr(flag, 1);
}

}  // namespace

hipError_t launch_rhs(const KShell& s, int count, const double* u, const double* du, bool cart, double* out,
                      const double* ubase, double* acc, double dt, int stage, hipStream_t st) {
    const dim3 grid((unsigned)((s.npts + kPts - 1) / kPts), (unsigned)count);
    const long long blk = (long long)count * s.n_v * s.npts;
    const double* dang = du + blk;
    if (s.n_v == 58)
        hipLaunchKernelGGL((k_rhs<58, double>), grid, dim3(kWaves * 64), 0, st, s, u, du, dang, cart ? 1 : 0,
                           out, ubase, acc, dt, stage, blk);
    else
        hipLaunchKernelGGL((k_rhs<50, double>), grid, dim3(kWaves * 64), 0, st, s, u, du, dang, cart ? 1 : 0,
                           out, ubase, acc, dt, stage, blk);
    return hipGetLastError();
}

hipError_t launch_rhs_mixed(const KShell& s, int count, const double* u, const double* dr, const float* dang,
                            double* out, const double* ubase, double* acc, double dt, int stage, hipStream_t st) {
    const dim3 grid((unsigned)((s.npts + kPts - 1) / kPts), (unsigned)count);
    const long long blk = (long long)count * s.n_v * s.npts;
    if (s.n_v == 58)
        hipLaunchKernelGGL((k_rhs<58, float>), grid, dim3(kWaves * 64), 0, st, s, u, dr, dang, 0, out, ubase,
                           acc, dt, stage, blk);
    else
        hipLaunchKernelGGL((k_rhs<50, float>), grid, dim3(kWaves * 64), 0, st, s, u, dr, dang, 0, out, ubase,
                           acc, dt, stage, blk);
    return hipGetLastError();
}

hipError_t launch_initial(const KShell& s, const double* g10, const double* dg, double* u, double* H,
                          hipStream_t st) {
    const unsigned blocks = (unsigned)((s.npts + 255) / 256);
    hipLaunchKernelGGL(k_initial, dim3(blocks), dim3(256), 0, st, s, g10, dg, u, H);
    return hipGetLastError();
}

hipError_t launch_constraints(const KShell& s, const double* u, const double* dg, long long dblk, double* part,
                              double* norms, hipStream_t st) {
    const unsigned blocks = (unsigned)((s.npts + 255) / 256);
    hipLaunchKernelGGL(k_constraints, dim3(blocks), dim3(256), 0, st, s, u, dg, dblk, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_constraint_norms(s, part, norms, st);
}

hipError_t launch_constraint_norms(const KShell& s, const double* part, double* norms, hipStream_t st) {
    const unsigned blocks = (unsigned)((s.npts + 255) / 256);
    hipLaunchKernelGGL(k_constraint_norms, dim3(1), dim3(256), 0, st, part, (int)blocks, (long long)s.npts, norms);
    return hipGetLastError();
}

hipError_t launch_patch(const KShell& a, const KShell& b, const double* ua, const double* ka, const double* kb,
                        double* out_a, double* acc_a, double* out_b, double* acc_b, double dt, int stage,
                        hipStream_t st) {
    const long long nang = (long long)a.n_th * a.n_ph;
    if (a.n_v != 50 && a.n_v != 58) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_patch, dim3((unsigned)((nang + 255) / 256), a.n_v == 58 ? 11u : 10u), dim3(256), 0, st, a, b,
                       ua, ka, kb, out_a, acc_a, out_b, acc_b, dt, stage);
    return hipGetLastError();
}

hipError_t launch_finite_check(const double* u, size_t n, int* flag, hipStream_t st) {
    hipLaunchKernelGGL(k_finite, dim3(1024), dim3(256), 0, st, u, n, flag);
    return hipGetLastError();
}

}  // namespace sg
