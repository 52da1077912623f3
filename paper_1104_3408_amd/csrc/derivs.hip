// Spectral derivative kernels on the field-major layout
// u[mu][j = phi][i = theta][k = r] (r fastest), Sec. 2.4.
//
// The paper applies D_1 by one GEMM on the reshaped array and D_2, D_3 by
// transpose -> GEMM -> transpose (eqs. D1, D2, D3).  Here every direction is a
// strided contraction staged through LDS, with no transposes:
//   d_r      contiguous radial lines, D_r (Chebyshev, eq. CDhat) in LDS;
//   d_theta  one workgroup per meridian circle (phi_j, phi_j + pi): both
//            half-planes in LDS, folded N_theta x 2 N_theta matrix of the
//            double cover (Sec. 2.1);
//   d_phi    one workgroup per (variable, 64 contiguous (theta, r) columns),
//            the N_phi rows of those columns in LDS.
// The same phi-axis kernel also applies the Fourier analysis and synthesis
// matrices of the filter (Sec. 3.1).
#include "internal.h"

namespace sg {

namespace {

constexpr int kLines = 8;      // radial lines per workgroup in d_r (N_r <= 80: <= 56 KB LDS)

__global__ __launch_bounds__(256) void k_dr(const double* __restrict__ in, double* __restrict__ out,
                                            const double* __restrict__ D, int n_r, long long n_lines) {
    extern __shared__ double sm[];
    double* sD = sm;
    double* sU = sm + n_r * n_r;
    const long long line0 = (long long)blockIdx.x * kLines;
    const int nl = (int)min((long long)kLines, n_lines - line0);
    for (int e = threadIdx.x; e < n_r * n_r; e += blockDim.x) sD[e] = D[e];
    const double* src = in + line0 * n_r;
    const int ne = nl * n_r;
    for (int e = threadIdx.x; e < ne; e += blockDim.x) sU[e] = src[e];
    __syncthreads();
    double* dst = out + line0 * n_r;
    for (int e = threadIdx.x; e < ne; e += blockDim.x) {
        const int l = e / n_r, k = e - l * n_r;
        const double* row = sD + k * n_r;
        const double* v = sU + l * n_r;
        double acc = 0.0;
        for (int kk = 0; kk < n_r; ++kk) acc = fma(row[kk], v[kk], acc);
        dst[e] = acc;
    }
}

// grid: (N_phi/2, n_fields, ceil(N_r/32)).  Output for phi_j and phi_j + pi,
// radial indices k0 .. k0+31 of the two half-planes staged in LDS.
constexpr int kKChunk = 32;
__global__ __launch_bounds__(256) void k_dtheta(const double* __restrict__ in, double* __restrict__ out,
                                                const double* __restrict__ H, int n_r, int n_th, int n_ph) {
    extern __shared__ double sm[];
    const int jp = blockIdx.x, mu = blockIdx.y;
    const int k0 = blockIdx.z * kKChunk;
    const int nk = min(kKChunk, n_r - k0);
    const int jq = jp + n_ph / 2;
    const long long plane = (long long)n_th * n_r;
    const long long fbase = (long long)mu * n_ph * plane;
    const int tile = n_th * kKChunk;
    double* sA = sm;
    double* sB = sm + tile;
    const double* a = in + fbase + jp * plane + k0;
    const double* b = in + fbase + jq * plane + k0;
    for (int e = threadIdx.x; e < tile; e += blockDim.x) {
        const int i = e / kKChunk, k = e - i * kKChunk;
        const bool ok = k < nk;
        sA[e] = ok ? a[(long long)i * n_r + k] : 0.0;
        sB[e] = ok ? b[(long long)i * n_r + k] : 0.0;
    }
    __syncthreads();
    const int n2 = 2 * n_th;
    double* oa = out + fbase + jp * plane + k0;
    double* ob = out + fbase + jq * plane + k0;
    for (int e = threadIdx.x; e < tile; e += blockDim.x) {
        const int i = e / kKChunk, k = e - i * kKChunk;
        if (k >= nk) continue;
        const double* h = H + (long long)i * n2;
        double accA = 0.0, accB = 0.0;
        for (int ip = 0; ip < n_th; ++ip) {
            const double h1 = h[ip], h2 = h[n_th + ip];
            const double va = sA[ip * kKChunk + k], vb = sB[ip * kKChunk + k];
            accA = fma(h1, va, fma(h2, vb, accA));
            accB = fma(h1, vb, fma(h2, va, accB));
        }
        oa[(long long)i * n_r + k] = accA;
        ob[(long long)i * n_r + k] = accB;
    }
}

// out[f][q][c] = sum_r W[q][r] in[f][r][c],  c < ncol, r < n_in, q < n_out.
// grid: (ceil(ncol/COLS), n_fields), 256 threads; the 256/COLS thread groups
// take q = w, w + 256/COLS, ... so W is read group-uniformly.
template <int COLS>
__global__ __launch_bounds__(256) void k_axis_phi(const double* __restrict__ in, double* __restrict__ out,
                                                  const double* __restrict__ W, int n_in, int n_out,
                                                  long long ncol) {
    extern __shared__ double sm[];
    const long long c0 = (long long)blockIdx.x * COLS;
    const int nc = (int)min((long long)COLS, ncol - c0);
    const int f = blockIdx.y;
    const double* src = in + (long long)f * n_in * ncol + c0;
    for (int e = threadIdx.x; e < n_in * COLS; e += blockDim.x) {
        const int r = e / COLS, c = e - r * COLS;
        sm[e] = (c < nc) ? src[(long long)r * ncol + c] : 0.0;
    }
    __syncthreads();
    constexpr int NG = 256 / COLS;
    const int c = threadIdx.x % COLS;
    const int w = threadIdx.x / COLS;
    double* dst = out + (long long)f * n_out * ncol + c0;
    for (int q = w; q < n_out; q += NG) {
        const double* wr = W + (long long)q * n_in;
        double acc = 0.0;
        for (int r = 0; r < n_in; ++r) acc = fma(wr[r], sm[r * COLS + c], acc);
        if (c < nc) dst[(long long)q * ncol + c] = acc;
    }
}

// (d_r, d_theta, d_phi) -> (d_x, d_y, d_z) in place, chain rule of Sec. 2.2
// eq. dvdx with the analytic Jacobian d(r, theta, phi)/d(x, y, z).
__global__ __launch_bounds__(256) void k_chain(KShell s, double* __restrict__ du, int n_fields) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= s.npts) return;
    const int k = (int)(p % s.n_r);
    const int i = (int)((p / s.n_r) % s.n_th);
    const int j = (int)(p / ((long long)s.n_r * s.n_th));
    const double r = s.rk[k], st = s.sth[i], ct = s.cth[i], sp = s.sph[j], cp = s.cph[j];
    const double ir = 1.0 / r, irs = 1.0 / (r * st);
    const double J[3][3] = {{st * cp, ct * cp * ir, -sp * irs}, {st * sp, ct * sp * ir, cp * irs}, {ct, -st * ir, 0.0}};
    const long long blk = (long long)n_fields * s.npts;
    for (int mu = 0; mu < n_fields; ++mu) {
        const long long q = (long long)mu * s.npts + p;
        const double a = du[q], b = du[blk + q], c = du[2 * blk + q];
        du[q] = J[0][0] * a + J[0][1] * b + J[0][2] * c;
        du[blk + q] = J[1][0] * a + J[1][1] * b + J[1][2] * c;
        du[2 * blk + q] = J[2][0] * a + J[2][1] * b;
    }
}

}  // namespace

hipError_t launch_dr(const KShell& s, const double* in, double* out, int n_fields, hipStream_t st) {
    const long long n_lines = (long long)n_fields * s.npts / s.n_r;
    const unsigned blocks = (unsigned)((n_lines + kLines - 1) / kLines);
    const size_t shm = sizeof(double) * (size_t(s.n_r) * s.n_r + size_t(kLines) * s.n_r);
    hipLaunchKernelGGL(k_dr, dim3(blocks), dim3(256), shm, st, in, out, s.Dr, s.n_r, n_lines);
    return hipGetLastError();
}

hipError_t launch_dtheta(const KShell& s, const double* in, double* out, int n_fields, hipStream_t st) {
    const size_t shm = sizeof(double) * 2 * size_t(s.n_th) * kKChunk;
    const unsigned kz = (unsigned)((s.n_r + kKChunk - 1) / kKChunk);
    hipLaunchKernelGGL(k_dtheta, dim3(s.n_ph / 2, n_fields, kz), dim3(256), shm, st, in, out, s.Hth, s.n_r,
                       s.n_th, s.n_ph);
    return hipGetLastError();
}

hipError_t launch_axis_phi(const double* in, double* out, const double* W, int n_in, int n_out,
                           long long ncol, int n_fields, hipStream_t st) {
    if (n_in <= 128) {
        const unsigned bx = (unsigned)((ncol + 63) / 64);
        hipLaunchKernelGGL(k_axis_phi<64>, dim3(bx, n_fields), dim3(256), sizeof(double) * size_t(n_in) * 64, st,
                           in, out, W, n_in, n_out, ncol);
    } else {
        const unsigned bx = (unsigned)((ncol + 31) / 32);
        hipLaunchKernelGGL(k_axis_phi<32>, dim3(bx, n_fields), dim3(256), sizeof(double) * size_t(n_in) * 32, st,
                           in, out, W, n_in, n_out, ncol);
    }
    return hipGetLastError();
}

hipError_t launch_chain(const KShell& s, double* du, int n_fields, hipStream_t st) {
    const unsigned blocks = (unsigned)((s.npts + 255) / 256);
    hipLaunchKernelGGL(k_chain, dim3(blocks), dim3(256), 0, st, s, du, n_fields);
    return hipGetLastError();
}

}  // namespace sg
