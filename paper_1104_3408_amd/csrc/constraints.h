// Device helpers of the constraint monitor (App. A.1), shared by the
// constraint kernels of the library.
#pragma once

#include "internal.h"

namespace sg {

namespace {

// symmetric pair index, order tt tx ty tz xx xy xz yy yz zz
__host__ __device__ constexpr int cpair(int a, int b) {
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    return lo == 0 ? hi : (lo == 1 ? 3 + hi : (lo == 2 ? 5 + hi : 9));
}

// Gauge constraint of App. A.1 at point p: C_a = H_a + Gamma_a with
// Gamma_a = g^bc Gamma_abc and d_t g from eq. gdot; adds max |C_a| and
// sum C_a^2 over a = t x y z into mx, ss.
__device__ __forceinline__ void gauge_constraint(const KShell& s, const double* __restrict__ u, long long p,
                                                 double& mx, double& ss) {
    const long long np = s.npts;
    double g[4][4], Pi[4][4], F[3][4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = a; b < 4; ++b) {
            const int q = cpair(a, b);
            g[a][b] = g[b][a] = u[q * np + p];
            Pi[a][b] = Pi[b][a] = u[(10 + q) * np + p];
#pragma unroll
            for (int x = 0; x < 3; ++x) F[x][a][b] = F[x][b][a] = u[(20 + 10 * x + q) * np + p];
        }
    const double gxx = g[1][1], gxy = g[1][2], gxz = g[1][3], gyy = g[2][2], gyz = g[2][3], gzz = g[3][3];
    const double cxx = gyy * gzz - gyz * gyz, cxy = gxz * gyz - gxy * gzz, cxz = gxy * gyz - gxz * gyy;
    const double cyy = gxx * gzz - gxz * gxz, cyz = gxy * gxz - gxx * gyz, czz = gxx * gyy - gxy * gxy;
    const double idet = 1.0 / (gxx * cxx + gxy * cxy + gxz * cxz);
    const double gi[3][3] = {{cxx * idet, cxy * idet, cxz * idet},
                             {cxy * idet, cyy * idet, cyz * idet},
                             {cxz * idet, cyz * idet, czz * idet}};
    double bu[3];
#pragma unroll
    for (int x = 0; x < 3; ++x) bu[x] = gi[x][0] * g[0][1] + gi[x][1] * g[0][2] + gi[x][2] * g[0][3];
    const double al = sqrt(bu[0] * g[0][1] + bu[1] * g[0][2] + bu[2] * g[0][3] - g[0][0]);
    const double ial2 = 1.0 / (al * al);
    double gI[4][4];
    gI[0][0] = -ial2;
#pragma unroll
    for (int x = 0; x < 3; ++x) {
        gI[0][x + 1] = gI[x + 1][0] = bu[x] * ial2;
#pragma unroll
        for (int y = 0; y < 3; ++y) gI[x + 1][y + 1] = gi[x][y] - bu[x] * bu[y] * ial2;
    }
    double D[4][4][4];   // D[c][a][b] = d_c g_ab
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            D[0][a][b] = -al * Pi[a][b] + bu[0] * F[0][a][b] + bu[1] * F[1][a][b] + bu[2] * F[2][a][b];
#pragma unroll
            for (int x = 0; x < 3; ++x) D[x + 1][a][b] = F[x][a][b];
        }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        double t = 0.0;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) t += gI[a][b] * 0.5 * (D[a][b][c] + D[b][a][c] - D[c][a][b]);
        const double h = s.n_v == 58 ? u[(50 + c) * np + p] : s.H[c * np + p];
        const double ca = h + t;
        mx = fmax(mx, fabs(ca));
        ss += ca * ca;
    }
}

// Block reduction of four partials (max, sum, max, sum) over 256 threads;
// the result is left in red[k][0].
__device__ __forceinline__ void reduce4(double (*red)[256], double mxa, double ssa, double mxi, double ssi) {
    red[0][threadIdx.x] = mxa;
    red[1][threadIdx.x] = ssa;
    red[2][threadIdx.x] = mxi;
    red[3][threadIdx.x] = ssi;
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
}

}  // namespace

}  // namespace sg
