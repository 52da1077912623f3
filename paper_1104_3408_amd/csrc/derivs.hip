// Spectral derivative kernels on the field-major layout
// u[mu][j = phi][i = theta][k = r] (r fastest), Sec. 2.4.
//
// The paper applies D_1 by one GEMM on the reshaped array and D_2, D_3 by
// transpose -> GEMM -> transpose (eqs. D1, D2, D3).  Here every direction is a
// contraction over one axis with no transposes: a workgroup stages 64
// "columns" in LDS, one column per lane, and each wave produces a
// wave-uniform set of output rows.  The operator entries are therefore
// wave-uniform and come through the scalar cache into SGPRs: every FP64 FMA
// takes one SGPR and one VGPR operand, and each LDS value feeds all the
// wave's output rows.  (On gfx950 FP64 MFMA and FP64 vector FMA have the same
// peak, so the FP64 path uses this vector form; it handles any N without
// padding the data.)
//
// Operators are stored wave-blocked and zero-padded by the host:
// Wb[w][c][r] = W[w * R + r][c] (0 past the last row), so the R weights one
// wave needs for input c are contiguous and the inner loops carry no bounds
// checks.  A workgroup has nw = 8, 12 or 16 waves (blocked_shape picks nw and
// R from a target number of rows per wave): more waves per staged tile
// shorten each wave's load and FMA chains, which bound these kernels when a
// shell gives only a few workgroups per CU (measured against 4 waves with up
// to 20 rows each: d_phi 2.02 -> 1.44 ms on 8 shells of 65x64x128).  Each
// thread issues all of its tile loads (fully unrolled, in-bounds addresses,
// unused slots predicated off) before its first LDS store, so a wave waits
// out one memory latency per tile rather than one per loaded row.
//
//   d_r      columns = radial lines (contiguous), tile transposed in LDS;
//   d_theta  columns = (variable, phi_j with j < N_phi/2, r_k); the two
//            half-planes phi_j and phi_j + pi form one meridian circle of the
//            double cover (Sec. 2.1).  With S = f(phi_j) + f(phi_j + pi) and
//            A = f(phi_j) - f(phi_j + pi) the folded matrix [H_L | H_R] gives
//            d f(phi_j) = ((H_L + H_R) S + (H_L - H_R) A)/2 and
//            d f(phi_j + pi) = ((H_L + H_R) S - (H_L - H_R) A)/2, half the
//            work of applying the N_theta x 2 N_theta matrix to both planes;
//   phi axis columns = (variable, theta_i, r_k), rows = phi_j.  Used for
//            d_phi (with the column mean over phi removed first: the Fourier
//            rows annihilate constants, and near the poles this keeps the
//            rounding error of d_phi proportional to sin(theta), so the
//            1/(r sin theta) of the chain rule does not amplify it) and for
//            the Fourier analysis/synthesis matrices of the filter (Sec. 3.1).
#include <algorithm>

#include "internal.h"
#include "tile_dr.h"

namespace sg {

namespace {

template <int R>
__global__ __launch_bounds__(1024) void k_dr(const double* __restrict__ in, double* __restrict__ out,
                                            const double* __restrict__ Db, int n_r, long long n_lines) {
    extern __shared__ double sm[];
    dr_tile<R>(blockIdx.x, in, out, Db, n_r, n_lines, sm);
}

// d_theta on meridian pairs.  Column c = (f * half + jp) * n_r + k; 64
// columns per workgroup, wave w computes theta rows i = w R + r.  The mean
// of each meridian circle is removed first (the rows of the Fourier matrix
// sum to zero), in FP64 before any rounding to T: S_i - (sum_i S_i)/N_theta.
constexpr int kThMaxPerThread = 64 / kMinWaves;   // N_theta <= 64 rows over at least kMinWaves waves

template <int R, typename T, typename O>
__device__ __forceinline__ void dtheta_tile(long long tile, const double* __restrict__ in, O* __restrict__ out,
                                            const T* __restrict__ Hsb, int n_r, int n_th,
                                            int n_ph, long long n_cols, double* __restrict__ smd) {
    // smd: S [n_th][64], A [n_th][64] in T, then partial sums [nw][64] in FP64
    T* sm = reinterpret_cast<T*>(smd);
    T* sS = sm;
    T* sA = sm + n_th * 64;
    double* spart = reinterpret_cast<double*>(sm + 2 * n_th * 64);
    const int half = n_ph / 2;
    const long long plane = (long long)n_th * n_r;
    const long long c0 = tile * 64;
    // this thread's column; it loads rows ip = w, w + nw, ...
    const int lane = threadIdx.x & 63;
    const int w = wave_id();
    const int nw = blockDim.x >> 6;
    const long long c = c0 + lane;
    const bool cok = c < n_cols;
    long long f = 0;
    int jp = 0, k = 0;
    if (cok) {
        const long long fj = c / n_r;
        k = (int)(c - fj * n_r);
        f = fj / half;
        jp = (int)(fj - f * half);
    }
    const double* base = in + f * n_ph * plane + (long long)jp * plane + k;   // f = jp = k = 0 past the end
    // S and A of this thread's rows, then the circle mean of S from the
    // waves' partial sums; the tile holds S - mean (rounded once to T) and A
    double sv[kThMaxPerThread], av[kThMaxPerThread];
#pragma unroll
    for (int t = 0; t < kThMaxPerThread; ++t) {
        const int ip = w + nw * t;
        double a = 0.0, b = 0.0;
        if (ip < n_th) {
            a = base[(long long)ip * n_r];
            b = base[half * plane + (long long)ip * n_r];
        }
        sv[t] = a;
        av[t] = b;
    }
    double part = 0.0;
#pragma unroll
    for (int t = 0; t < kThMaxPerThread; ++t) {
        const double a = cok ? sv[t] : 0.0, b = cok ? av[t] : 0.0;
        sv[t] = a + b;
        av[t] = a - b;
        part += sv[t];
    }
    spart[w * 64 + lane] = part;
    __syncthreads();
    double mc = 0.0;
    for (int v = 0; v < nw; ++v) mc += spart[v * 64 + lane];
    mc /= n_th;
#pragma unroll
    for (int t = 0; t < kThMaxPerThread; ++t) {
        const int ip = w + nw * t;
        if (ip < n_th) {
            sS[ip * 64 + lane] = (T)(sv[t] - mc);
            sA[ip * 64 + lane] = (T)av[t];
        }
    }
    __syncthreads();
    // equator pairs (i, N_theta - 1 - i) -> (x + x', x - x') in place, for S and A
    const int hh = (n_th + 1) / 2;   // rows i < hh; the middle row of an odd N_theta stays
    for (int ip = w; ip < n_th / 2; ip += nw) {
        const int im = n_th - 1 - ip;
        const T s0 = sS[ip * 64 + lane], s1 = sS[im * 64 + lane];
        const T a0 = sA[ip * 64 + lane], a1 = sA[im * 64 + lane];
        sS[ip * 64 + lane] = s0 + s1;
        sS[im * 64 + lane] = s0 - s1;
        sA[ip * 64 + lane] = a0 + a1;
        sA[im * 64 + lane] = a0 - a1;
    }
    __syncthreads();
    // Hs and Ha are both anti-persymmetric (M[N-1-i][N-1-i'] = -M[i][i']: the
    // double-cover circle is symmetric about the equator and the derivative is
    // odd under the reflection), so with x+ = x_i' + x_{N-1-i'}, x- = x_i' - x_{N-1-i'}
    // (i' < N/2; the middle row of an odd N enters x+ alone),
    //   (M x)_i = Q x+ + P x-,  (M x)_{N-1-i} = P x- - Q x+,  i < N/2,
    // Q_ii' = (M_ii' + M_i,N-1-i') / 2, P_ii' = (M_ii' - M_i,N-1-i') / 2: half the
    // products of M.  Operator blocked as [w][i'][Qs (R), Ps (R), Qa (R), Pa (R)].
    const T* Ww = Hsb + (long long)w * hh * 4 * R;
    T qs[R], ps[R], qa[R], pa[R];
#pragma unroll
    for (int r = 0; r < R; ++r) qs[r] = ps[r] = qa[r] = pa[r] = (T)0;
    #pragma unroll 2
    for (int ip = 0; ip < hh; ++ip) {
        const int im = n_th - 1 - ip;   // = ip for the middle row (its P weights are 0)
        const T sp = sS[ip * 64 + lane], sm_ = sS[im * 64 + lane];
        const T ap = sA[ip * 64 + lane], am = sA[im * 64 + lane];
        const T* wr = Ww + ip * 4 * R;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            qs[r] = fma(wr[r], sp, qs[r]);
            ps[r] = fma(wr[R + r], sm_, ps[r]);
            qa[r] = fma(wr[2 * R + r], ap, qa[r]);
            pa[r] = fma(wr[3 * R + r], am, pa[r]);
        }
    }
    if (cok) {
        O* o = out + f * n_ph * plane + jp * plane + k;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = w * R + r;
            if (i < hh) {
                const T hs = qs[r] + ps[r], ha = qa[r] + pa[r];
                o[(long long)i * n_r] = (O)((T)0.5 * (hs + ha));
                o[half * plane + (long long)i * n_r] = (O)((T)0.5 * (hs - ha));
                const int im = n_th - 1 - i;
                if (im != i) {
                    const T hs2 = ps[r] - qs[r], ha2 = pa[r] - qa[r];
                    o[(long long)im * n_r] = (O)((T)0.5 * (hs2 + ha2));
                    o[half * plane + (long long)im * n_r] = (O)((T)0.5 * (hs2 - ha2));
                }
            }
        }
    }
}

// d_theta in FP64 on whole meridian plane pairs: workgroup `tile` = (f,
// j), j < N_phi / 2, stages the planes phi_j and phi_j + pi of field f
// (N_theta N_r contiguous values each, so every load and store covers whole
// cache lines; the column tile above cuts the radial runs of N_r values at
// arbitrary points) and forms d_theta of both planes for all N_r columns,
// lane = k.  Arithmetic as dtheta_tile: S - mean and A, the equator pairs,
// the operator of the equator-parity form.  LDS: 2 N_theta N_r doubles.
template <int R>
__device__ __forceinline__ void dtheta_plane_tile(long long tile, const double* __restrict__ in,
                                                  double* __restrict__ out, const double* __restrict__ Hsb,
                                                  int n_r, int n_th, int n_ph, double* __restrict__ sm) {
    const int half = n_ph / 2;
    const long long plane = (long long)n_th * n_r;
    const long long f = tile / half;
    const int jp = (int)(tile - f * half);
    const double* src0 = in + (f * n_ph + jp) * plane;
    const double* src1 = src0 + half * plane;
    const int np_ = n_th * n_r;
    const int nt = blockDim.x;
    const int tid = threadIdx.x;
    constexpr int U = 4;   // loads in flight per plane and thread
    for (int base = 0; base < np_; base += U * nt) {
        double a[U], b[U];
#pragma unroll
        for (int t = 0; t < U; ++t) {
            const int e = base + tid + t * nt;
            const int ec = e < np_ ? e : np_ - 1;   // in-bounds address for every thread
            a[t] = src0[ec];
            b[t] = src1[ec];
        }
#pragma unroll
        for (int t = 0; t < U; ++t) {
            const int e = base + tid + t * nt;
            if (e < np_) {
                sm[e] = a[t];
                sm[np_ + e] = b[t];
            }
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int w = wave_id();
    const int nw = nt >> 6;
    double* sS = sm;          // rows i, column k at i n_r + k: S - mean, then equator pairs
    double* sA = sm + np_;    // A, then equator pairs
    double* spart = sm + 2 * np_;   // [nw][n_r] partial sums of S
    // S = P0 + P1 and A = P0 - P1 in place; partial sums of S per column
    for (int k0 = 0; k0 < n_r; k0 += 64) {
        const int k = k0 + lane;
        double part = 0.0;
        if (k < n_r)
            for (int i = w; i < n_th; i += nw) {
                const double p0 = sS[i * n_r + k], p1 = sA[i * n_r + k];
                sS[i * n_r + k] = p0 + p1;
                sA[i * n_r + k] = p0 - p1;
                part += p0 + p1;
            }
        if (k < n_r) spart[w * n_r + k] = part;
    }
    __syncthreads();
    for (int k0 = 0; k0 < n_r; k0 += 64) {
        const int k = k0 + lane;
        if (k >= n_r) continue;
        double mc = 0.0;
        for (int v = 0; v < nw; ++v) mc += spart[v * n_r + k];
        mc /= n_th;
        for (int i = w; i < n_th / 2; i += nw) {   // S - mean, then the equator pairs of S and A
            const int im = n_th - 1 - i;
            const double s0 = sS[i * n_r + k] - mc, s1 = sS[im * n_r + k] - mc;
            const double a0 = sA[i * n_r + k], a1 = sA[im * n_r + k];
            sS[i * n_r + k] = s0 + s1;
            sS[im * n_r + k] = s0 - s1;
            sA[i * n_r + k] = a0 + a1;
            sA[im * n_r + k] = a0 - a1;
        }
        if ((n_th & 1) && w == (n_th / 2) % nw) sS[(n_th / 2) * n_r + k] -= mc;   // middle row of an odd N_theta
    }
    __syncthreads();
    const int hh = (n_th + 1) / 2;
    const double* Ww = Hsb + (long long)w * hh * 4 * R;
    double* o0 = out + (f * n_ph + jp) * plane;
    double* o1 = o0 + half * plane;
    for (int k0 = 0; k0 < n_r; k0 += 64) {
        const int k = k0 + lane;
        const int kc = k < n_r ? k : n_r - 1;
        double qs[R], ps[R], qa[R], pa[R];
#pragma unroll
        for (int r = 0; r < R; ++r) qs[r] = ps[r] = qa[r] = pa[r] = 0.0;
        #pragma unroll 2
        for (int ip = 0; ip < hh; ++ip) {
            const int im = n_th - 1 - ip;
            const double sp = sS[ip * n_r + kc], smm = sS[im * n_r + kc];
            const double ap = sA[ip * n_r + kc], am = sA[im * n_r + kc];
            const double* wr = Ww + ip * 4 * R;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                qs[r] = fma(wr[r], sp, qs[r]);
                ps[r] = fma(wr[R + r], smm, ps[r]);
                qa[r] = fma(wr[2 * R + r], ap, qa[r]);
                pa[r] = fma(wr[3 * R + r], am, pa[r]);
            }
        }
        if (k >= n_r) continue;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = w * R + r;
            if (i < hh) {
                const double hs = qs[r] + ps[r], ha = qa[r] + pa[r];
                o0[i * n_r + k] = 0.5 * (hs + ha);
                o1[i * n_r + k] = 0.5 * (hs - ha);
                const int im = n_th - 1 - i;
                if (im != i) {
                    const double hs2 = ps[r] - qs[r], ha2 = pa[r] - qa[r];
                    o0[im * n_r + k] = 0.5 * (hs2 + ha2);
                    o1[im * n_r + k] = 0.5 * (hs2 - ha2);
                }
            }
        }
    }
}

template <int R>
__global__ __launch_bounds__(1024) void k_dtheta_plane(const double* __restrict__ in, double* __restrict__ out,
                                                      const double* __restrict__ Hsb, int n_r, int n_th, int n_ph) {
    extern __shared__ double smd[];
    dtheta_plane_tile<R>(blockIdx.x, in, out, Hsb, n_r, n_th, n_ph, smd);
}

template <int R, typename T, typename O>
__global__ __launch_bounds__(1024) void k_dtheta(const double* __restrict__ in, O* __restrict__ out,
                                                const T* __restrict__ Hsb,
                                                int n_r, int n_th, int n_ph, long long n_cols) {
    extern __shared__ double smd[];
    dtheta_tile<R, T, O>(xcd_block(blockIdx.x, gridDim.x), in, out, Hsb, n_r, n_th, n_ph, n_cols, smd);
}

// out[f][q][c] = sum_r W[q][r] (in[f][r][c] - m_c),  m_c = mean of column c
// over r if center, else 0.  grid: (ceil(ncol/64), n_fields); wave w of nw
// computes rows q = w R + r.  Thread (w, c) loads rows r = w, w + nw, ... of
// column c once; the column mean is formed in FP64 from the waves' partial
// sums.  FP64 tiles keep the raw values and subtract
// the mean per lane; FP32 tiles store (value - mean) rounded once, so the
// rounding is relative to the deviation from the mean.
constexpr int kAxisMaxIn = 128;

template <int R, typename I, typename T, typename O, bool CIRC>
__device__ __forceinline__ void axis_tile(long long tile, int f, const I* __restrict__ in, O* __restrict__ out,
                                          const T* __restrict__ Wb, int n_in, int n_out, long long ncol, int center,
                                          double* __restrict__ smd) {
    // smd: tile [n_in][64] in T, then partial sums [nw][64] in FP64
    T* sm = reinterpret_cast<T*>(smd);
    double* spart = reinterpret_cast<double*>(sm + n_in * 64);
    const long long c0 = tile * 64;
    const int nc = (int)min((long long)64, ncol - c0);
    const I* src = in + (long long)f * n_in * ncol + c0;
    const int lane = threadIdx.x & 63;
    const int w = wave_id();
    const int nw = blockDim.x >> 6;
    const bool colok = lane < nc;
    // this thread's rows, then (center) the column mean from the waves'
    // partial sums; the tile holds value - mean, rounded once to T
    const int lc = colok ? lane : 0;   // an in-bounds column for every lane
    double v[kAxisMaxIn / kMinWaves];
#pragma unroll
    for (int t = 0; t < kAxisMaxIn / kMinWaves; ++t) {
        const int r = w + nw * t;
        v[t] = (r < n_in) ? (double)src[(long long)r * ncol + lc] : 0.0;
    }
    double mc = 0.0;
    if (center) {
        double part = 0.0;
#pragma unroll
        for (int t = 0; t < kAxisMaxIn / kMinWaves; ++t) part += v[t];
        spart[w * 64 + lane] = part;
        __syncthreads();
        for (int q = 0; q < nw; ++q) mc += spart[q * 64 + lane];
        mc /= n_in;
    }
#pragma unroll
    for (int t = 0; t < kAxisMaxIn / kMinWaves; ++t) {
        const int r = w + nw * t;
        if (r < n_in) sm[r * 64 + lane] = (T)(v[t] - mc);
    }
    __syncthreads();
    O* dst = out + (long long)f * n_out * ncol + c0;
    // operator rows are wave-uniform: scalar loads (an LDS copy with
    // broadcast reads measured 1.9x slower at N_phi = 64).  Blocked copy: the
    // rows of this wave for input ri at Ww + ri R; circulant: the sliding
    // window dv[n_in + q0 - ri ...] of a vector that stays in the scalar cache
    const T* Ww = CIRC ? Wb + n_in + w * R : Wb + (long long)w * n_in * R;
    T acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = (T)0;
    #pragma unroll 4   // operator loads run ahead of the FMAs (measured against 1, 2, default)
    for (int ri = 0; ri < n_in; ++ri) {
        const T v = sm[ri * 64 + lane];
        const T* wr = CIRC ? Ww - ri : Ww + ri * R;
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = fma(wr[r], v, acc[r]);
    }
    if (colok) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int q = w * R + r;
            if (q < n_out) dst[(long long)q * ncol + lane] = (O)acc[r];
        }
    }
}

template <int R, typename I, typename T, typename O, bool CIRC>
__global__ __launch_bounds__(1024) void k_axis(const I* __restrict__ in, O* __restrict__ out,
                                               const T* __restrict__ Wb, int n_in, int n_out, long long ncol,
                                               int center) {
    extern __shared__ double smd[];
    axis_tile<R, I, T, O, CIRC>(blockIdx.x, blockIdx.y, in, out, Wb, n_in, n_out, ncol, center, smd);
}

// d_phi in FP64 on the matrix cores (v_mfma_f64_16x16x4f64), for N_phi a
// multiple of 16: a dense N_phi x N_phi contraction of 2 N_phi flops per
// field-point, which at N_phi >= 96 keeps the vector units busier than the
// memory system.  Workgroup = 64 (theta, r) columns of one field (blockIdx.x
// column tile, blockIdx.y field) staged in LDS after the FP64 circle-mean
// removal of axis_tile; wave w forms output rows 16 w .. 16 w + 15 for the
// four 16-column blocks, accumulating over the inputs four at a time.
// Operand layout of the instruction (checked on the device with a one-wave
// probe): lane l feeds A[l % 16][l / 16] and B[l / 16][l % 16] and holds
// D[4 v + l / 16][l % 16] in item v of its result.  A[i][k] = D_phi[16 w + i][k0
// + k] = dv[N + 16 w + i - k0 - k] from the doubled circulant column dv,
// staged in LDS beside the tile (2 N values).
constexpr int kMfmaCols = 64;

__global__ __launch_bounds__(512) void k_dphi_mfma(const double* __restrict__ in, double* __restrict__ out,
                                                   const double* __restrict__ dv, int n, long long ncol) {
    extern __shared__ double smd[];
    double* sm = smd;                        // [n][64]: value - column mean
    const int lane = threadIdx.x & 63;
    const int w = wave_id();
    const int nw = blockDim.x >> 6;          // = n / 16
    double* spart = smd + n * kMfmaCols;     // [nw][64]: partial sums
    double* sdv = spart + nw * kMfmaCols;    // [2n]: the doubled circulant column
    for (int t = threadIdx.x; t < 2 * n; t += blockDim.x) sdv[t] = dv[t];
    const long long c0 = (long long)blockIdx.x * kMfmaCols;
    const int nc = (int)min((long long)kMfmaCols, ncol - c0);
    const long long f = blockIdx.y;
    const double* src = in + f * n * ncol + c0;
    const int lc = lane < nc ? lane : 0;   // an in-bounds column for every lane
    constexpr int kPer = 16;               // rows per thread: n / nw
    double v[kPer];
#pragma unroll
    for (int t = 0; t < kPer; ++t) v[t] = src[(long long)(w + nw * t) * ncol + lc];
    double part = 0.0;
#pragma unroll
    for (int t = 0; t < kPer; ++t) part += v[t];
    spart[w * kMfmaCols + lane] = part;
    __syncthreads();
    double mc = 0.0;
    for (int q = 0; q < nw; ++q) mc += spart[q * kMfmaCols + lane];
    mc /= n;
#pragma unroll
    for (int t = 0; t < kPer; ++t) sm[(w + nw * t) * kMfmaCols + lane] = v[t] - mc;
    __syncthreads();
    typedef double v4d __attribute__((ext_vector_type(4)));
    v4d acc[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[cb] = v4d{0.0, 0.0, 0.0, 0.0};
    const int li = lane & 15, lk = lane >> 4;
    const double* arow = sdv + n + 16 * w + li - lk;   // A[li][lk] at step k0: arow[-k0]
    #pragma unroll 4
    for (int k0 = 0; k0 < n; k0 += 4) {
        const double a = arow[-k0];
        const double* brow = sm + (k0 + lk) * kMfmaCols + li;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, brow[16 * cb], acc[cb], 0, 0, 0);
    }
    double* dst = out + f * n * ncol + c0;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        const int col = 16 * cb + li;
        if (col < nc) {
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) dst[(long long)(16 * w + 4 * vv + lk) * ncol + col] = acc[cb][vv];
        }
    }
}

// Contractions along phi in the parity form (MODE: kParAna, kParSyn,
// kParDphi).  About phi = 0 cos is even and sin odd, and the Fourier
// derivative matrix FD[q][c] = v[(q - c) mod N] has v odd, so with
// e_j = f_j + f_{N-j}, o_j = f_j - f_{N-j} (0 < j < N/2; e_0 = f_0,
// e_{N/2} = f_{N/2}):
//   analysis (Sec. 3.1 eq. Fanalysis): a_m = sum_{0 <= j <= N/2} C[m][j] e_j,
//     b_m = sum_{0 < j < N/2} S[m][j] o_j;
//   synthesis (eq. Fsynthesis): f_j = A_j + B_j, f_{N-j} = A_j - B_j with
//     A_j = sum_m C[j][m] a_m, B_j = sum_{m >= 1} S[j][m] b_m, 0 <= j <= N/2;
//   d_phi (Sec. 2.3, eq. D3; the circle mean removed first, the rows of FD
//     annihilate constants): y_q = A_q + B_q, y_{N-q} = B_q - A_q with
//     A_q = sum_{0 <= j <= N/2} C[q][j] e_j, B_q = sum_{0 < j < N/2} S[q][j] o_j,
//     C[q][j] = (v[q - j] + v[q + j]) / 2 (v[q], v[q - N/2] at j = 0, N/2),
//     S[q][j] = (v[q - j] - v[q + j]) / 2:
// half the products of the full matrices (and half the operator, which the
// waves read through the scalar cache).  Spectral rows are q = 0 (a_0),
// 2m - 1 (a_m), 2m (b_m).  Wave w forms the row pair (a_m, b_m), (A_j, B_j)
// resp. (A_q, B_q) for m, j resp. q = w R + r; the operator is wave-blocked
// as Wb[w][input][C (R values), S (R values)], zero past the last row and
// where S vanishes.  The analysis and d_phi rewrite the staged rows j, N - j
// into e_j, o_j in place.
constexpr int kParAna = 0, kParSyn = 1, kParDphi = 2;

template <int R, typename I, typename T, typename O, int MODE>
__device__ __forceinline__ void axis_par_tile(long long tile, int f, const I* __restrict__ in, O* __restrict__ out,
                                              const T* __restrict__ Wb, int n_ph, int m_keep, long long ncol,
                                              double* __restrict__ smd) {
    constexpr bool SYN = MODE == kParSyn;
    const int nw = blockDim.x >> 6;
    T* sm = reinterpret_cast<T*>(smd);   // [n_in][64], then (d_phi) partial sums [nw][64] in FP64
    double* spart = reinterpret_cast<double*>(sm + n_ph * 64);
    const int half = n_ph / 2;
    const int n_in = SYN ? 2 * m_keep + 1 : n_ph;
    const int n_out = MODE == kParAna ? 2 * m_keep + 1 : n_ph;
    const long long c0 = tile * 64;
    const int nc = (int)min((long long)64, ncol - c0);
    const I* src = in + (long long)f * n_in * ncol + c0;
    const int lane = threadIdx.x & 63;
    const int w = wave_id();
    const int lc = lane < nc ? lane : 0;   // an in-bounds column for every lane
    double v[kAxisMaxIn / kMinWaves];
#pragma unroll
    for (int t = 0; t < kAxisMaxIn / kMinWaves; ++t) {
        const int r = w + nw * t;
        v[t] = (r < n_in) ? (double)src[(long long)r * ncol + lc] : 0.0;
    }
    double mc = 0.0;
    if (MODE == kParDphi) {   // column mean over phi, in FP64 from the waves' partial sums
        double part = 0.0;
#pragma unroll
        for (int t = 0; t < kAxisMaxIn / kMinWaves; ++t) part += v[t];
        spart[w * 64 + lane] = part;
        __syncthreads();
        for (int q = 0; q < nw; ++q) mc += spart[q * 64 + lane];
        mc /= n_in;
    }
#pragma unroll
    for (int t = 0; t < kAxisMaxIn / kMinWaves; ++t) {
        const int r = w + nw * t;
        if (r < n_in) sm[r * 64 + lane] = (T)(v[t] - mc);
    }
    __syncthreads();
    if (!SYN) {
        for (int j = 1 + w; j < half; j += nw) {
            const T a = sm[j * 64 + lane], b = sm[(n_ph - j) * 64 + lane];
            sm[j * 64 + lane] = a + b;
            sm[(n_ph - j) * 64 + lane] = a - b;
        }
        __syncthreads();
    }
    const int n_loop = SYN ? m_keep + 1 : half + 1;
    const T* Ww = Wb + (long long)w * n_loop * 2 * R;
    T ac[R], as[R];
#pragma unroll
    for (int r = 0; r < R; ++r) ac[r] = as[r] = (T)0;
    #pragma unroll 4
    for (int jj = 0; jj < n_loop; ++jj) {
        // analysis, d_phi: e_jj and o_jj (rows jj, N - jj; jj = 0, N/2 carry no
        // S); synthesis: a_jj and b_jj (rows 2 jj - 1, 2 jj; a_0 at row 0, no b_0)
        const int rx = SYN ? (jj == 0 ? 0 : 2 * jj - 1) : jj;
        const int ry = SYN ? 2 * jj : ((jj == 0 || jj == half) ? jj : n_ph - jj);
        const T x = sm[rx * 64 + lane], y = sm[ry * 64 + lane];
        const T* wr = Ww + jj * 2 * R;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            ac[r] = fma(wr[r], x, ac[r]);
            as[r] = fma(wr[R + r], y, as[r]);
        }
    }
    if (lane >= nc) return;
    O* dst = out + (long long)f * n_out * ncol + c0 + lane;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int q = w * R + r;
        if (MODE == kParAna) {
            if (q <= m_keep) {
                dst[(long long)(q == 0 ? 0 : 2 * q - 1) * ncol] = (O)ac[r];
                if (q > 0) dst[(long long)(2 * q) * ncol] = (O)as[r];
            }
        } else if (q <= half) {
            const T sgn = MODE == kParSyn ? (T)1 : (T)-1;   // f_{N-j} = A - B, y_{N-q} = B - A
            dst[(long long)q * ncol] = (O)(ac[r] + as[r]);
            if (q > 0 && q < half) dst[(long long)(n_ph - q) * ncol] = (O)(sgn * (ac[r] - as[r]));
        }
    }
}

template <int R, typename I, typename T, typename O, int MODE>
__global__ __launch_bounds__(1024) void k_axis_par(const I* __restrict__ in, O* __restrict__ out,
                                                   const T* __restrict__ Wb, int n_ph, int m_keep, long long ncol) {
    extern __shared__ double smd[];
    axis_par_tile<R, I, T, O, MODE>(blockIdx.x, blockIdx.y, in, out, Wb, n_ph, m_keep, ncol, smd);
}

// The three coordinate derivatives of one run of shells in one launch:
// b_dr d_r tiles, b_th d_theta tiles and bx_ph column tiles per field of
// d_phi, interleaved over the grid so that the three kinds run side by side.
// Every workgroup has the same number of waves (the host uses this only when
// the three blocked shapes agree on it).  One launch instead of three on
// forked streams removes the cross-queue waits of the fork and join (about
// 20 us per stage at 33x32x64); measured step 0.474 -> 0.464 ms there.
// Giving each kind of tile its own XCDs (blockIdx mod 8) measured slower.
// (The array pointers are separate __restrict__ kernel arguments, not struct
// members: only then may the compiler read the operators through the scalar
// cache; from a struct they became vector loads and the launch ran 2x slower.)
struct D3Dims {
    long long n_lines, n_cols_th, ncol_ph;
    unsigned b_dr, b_th, bx_ph;
    int nf;
    int R_dr, R_th, R_ph, ph_par, th_plane;
    int n_r, n_th, n_ph;
};

// rows per wave the one-launch form is instantiated for: d_r and the parity
// d_phi up to 9, the circulant d_phi up to 12, the theta tile (four
// accumulator sets per row) up to 4; the workgroup's registers are the
// largest case's, so the cases stop at what the tile shapes in use need
constexpr int kFusedMaxR = 9, kFusedMaxRth = 4, kFusedMaxRcirc = 12;

template <typename T, typename O>
__global__ __launch_bounds__(1024) void k_derivs3(const double* __restrict__ in, double* __restrict__ out_r,
                                                 O* __restrict__ out_th, O* __restrict__ out_ph,
                                                 const double* __restrict__ Drb, const T* __restrict__ Hsb,
                                                 const T* __restrict__ Wph, D3Dims a) {
    extern __shared__ double smd[];
    // the three kinds of tiles interleaved evenly over the grid (Bresenham):
    // block b is the D(b)-th d_r tile if D(b + 1) > D(b), D(b) = floor(b b_dr / B);
    // otherwise the same rule splits the rest between d_theta and d_phi
    const unsigned long long B = (unsigned long long)a.b_dr + a.b_th + (unsigned long long)a.bx_ph * a.nf;
    const unsigned long long bb = blockIdx.x;   // (the XCD renumbering of k_dtheta measured slower here)
    const unsigned long long d0 = bb * a.b_dr / B, d1 = (bb + 1) * a.b_dr / B;
    const unsigned long long o = bb - d0, n_o = B - a.b_dr;   // index among the other tiles
    const unsigned long long t0 = n_o ? o * a.b_th / n_o : 0, t1 = n_o ? (o + 1) * a.b_th / n_o : 0;
    const bool is_dr = d1 > d0, is_th = !is_dr && t1 > t0;
    const unsigned long long t_dr = d0, t_th = t0, t_ph = o - t0;
    if (is_dr) {
        switch (a.R_dr) {
#define X(R) case R: dr_tile<R>(t_dr, in, out_r, Drb, a.n_r, a.n_lines, smd); break;
            X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9)
#undef X
        }
        return;
    }
    if (is_th) {
        if constexpr (sizeof(T) == sizeof(double)) {
            if (a.th_plane) {
                switch (a.R_th) {
#define X(R) case R: dtheta_plane_tile<R>(t_th, in, out_th, Hsb, a.n_r, a.n_th, a.n_ph, smd); break;
                    X(1) X(2) X(3) X(4)
#undef X
                }
                return;
            }
        }
        switch (a.R_th) {
#define X(R) case R: dtheta_tile<R, T, O>(t_th, in, out_th, Hsb, a.n_r, a.n_th, a.n_ph, a.n_cols_th, smd); break;
            X(1) X(2) X(3) X(4)
#undef X
        }
        return;
    }
    const long long bx = (long long)(t_ph % a.bx_ph);
    const int f = (int)(t_ph / a.bx_ph);
    if (a.ph_par) {
        switch (a.R_ph) {
#define X(R) case R: axis_par_tile<R, double, T, O, kParDphi>(bx, f, in, out_ph, Wph, a.n_ph, 0, a.ncol_ph, smd); break;
            X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9)
#undef X
        }
        return;
    }
    switch (a.R_ph) {
#define X(R) case R: axis_tile<R, double, T, O, true>(bx, f, in, out_ph, Wph, a.n_ph, a.n_ph, a.ncol_ph, 1, smd); break;
        X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12)
#undef X
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

std::vector<double> block_operator(const std::vector<double>& W, int n_out, int n_in, int R, int passes) {
    std::vector<double> Wb(size_t(passes) * 4 * n_in * R, 0.0);
    for (int p = 0; p < passes; ++p)
        for (int w = 0; w < 4; ++w)
            for (int c = 0; c < n_in; ++c)
                for (int r = 0; r < R; ++r) {
                    const int q = (p * 4 + w) * R + r;
                    if (q < n_out) Wb[((size_t(p) * 4 + w) * n_in + c) * R + r] = W[size_t(q) * n_in + c];
                }
    return Wb;
}

int blocked_shape(int n_out, int target, int& R, int& passes) {
    int nw = (n_out + target - 1) / target;
    nw = (nw + 3) / 4 * 4;
    if (nw < kMinWaves) nw = kMinWaves;
    if (nw > kMaxWaves) nw = kMaxWaves;
    R = (n_out + nw - 1) / nw;
    passes = nw / 4;
    return R <= kMaxRows ? 0 : -1;
}

#define SG_R_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) \
    X(17) X(18) X(19) X(20)

hipError_t launch_dr(const KShell& s, const double* in, double* out, int n_fields, hipStream_t st) {
    const long long n_lines = (long long)n_fields * s.npts / s.n_r;
    const unsigned blocks = (unsigned)((n_lines + 63) / 64);
    const size_t shm = sizeof(double) * size_t(s.n_r) * kDrStride;
    const unsigned nt = 64u * s.Dr_nw;
    switch (s.Dr_R) {
#define X(R) case R: hipLaunchKernelGGL(k_dr<R>, dim3(blocks), dim3(nt), shm, st, in, out, s.Drb, s.n_r, n_lines); break;
        SG_R_CASES(X)
#undef X
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, typename O>
static hipError_t dtheta_t(const KShell& s, const double* in, O* out, const T* Hsb, int n_fields,
                           hipStream_t st) {
    if constexpr (sizeof(T) == sizeof(double)) {
        if (s.th_plane) {   // whole meridian plane pairs per workgroup
            const unsigned blocks = (unsigned)((long long)n_fields * (s.n_ph / 2));
            const size_t shm = sizeof(double) * (2 * size_t(s.n_th) * s.n_r + size_t(s.Hth_nw) * s.n_r);
            switch (s.Hth_R) {
#define X(R) case R: hipLaunchKernelGGL((k_dtheta_plane<R>), dim3(blocks), dim3(64u * s.Hth_nw), shm, st, in, out, Hsb, s.n_r, s.n_th, s.n_ph); break;
                X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8)
#undef X
                default: return hipErrorInvalidValue;
            }
            return hipGetLastError();
        }
    }
    const long long n_cols = (long long)n_fields * (s.n_ph / 2) * s.n_r;
    const unsigned blocks = (unsigned)((n_cols + 63) / 64);
    if (s.n_th > s.Hth_nw * kThMaxPerThread) return hipErrorInvalidValue;
    const size_t shm = sizeof(T) * 2 * size_t(s.n_th) * 64 + size_t(s.Hth_nw) * 64 * sizeof(double);
    const unsigned nt = 64u * s.Hth_nw;
    switch (s.Hth_R) {
#define X(R) case R: hipLaunchKernelGGL((k_dtheta<R, T, O>), dim3(blocks), dim3(nt), shm, st, in, out, Hsb, s.n_r, s.n_th, s.n_ph, n_cols); break;
        SG_R_CASES(X)
#undef X
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dtheta(const KShell& s, const double* in, double* out, int n_fields, hipStream_t st) {
    return dtheta_t<double, double>(s, in, out, s.Hsb, n_fields, st);
}

hipError_t launch_dtheta_f32(const KShell& s, const double* in, float* out, int n_fields, hipStream_t st) {
    return dtheta_t<float, float>(s, in, out, s.Hsb_f, n_fields, st);
}

template <typename I, typename T, typename O>
static hipError_t axis_t(const AxisOp& op, const T* Wb, const I* in, O* out, long long ncol, int n_fields,
                         int center, hipStream_t st) {
    if (op.n_in > kAxisMaxIn || 4 * op.passes < kMinWaves) return hipErrorInvalidValue;
    const unsigned bx = (unsigned)((ncol + 63) / 64);
    const unsigned nt = 256u * op.passes;
    if (op.par) {   // parity form: phi analysis (par 1), synthesis (par 2), d_phi (par 3)
        const int n_ph = op.par == 2 ? op.n_out : op.n_in;
        const size_t shm = sizeof(T) * size_t(n_ph) * 64 + size_t(4 * op.passes) * 64 * sizeof(double);
        switch (op.R) {
#define X(R)                                                                                                   \
    case R:                                                                                                    \
        if (op.par == 1)                                                                                       \
            hipLaunchKernelGGL((k_axis_par<R, I, T, O, kParAna>), dim3(bx, n_fields), dim3(nt), shm, st, in,   \
                               out, Wb, n_ph, op.m_keep, ncol);                                                \
        else if (op.par == 2)                                                                                  \
            hipLaunchKernelGGL((k_axis_par<R, I, T, O, kParSyn>), dim3(bx, n_fields), dim3(nt), shm, st, in,   \
                               out, Wb, n_ph, op.m_keep, ncol);                                                \
        else                                                                                                   \
            hipLaunchKernelGGL((k_axis_par<R, I, T, O, kParDphi>), dim3(bx, n_fields), dim3(nt), shm, st, in,  \
                               out, Wb, n_ph, op.m_keep, ncol);                                                \
        break;
            SG_R_CASES(X)
#undef X
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if constexpr (sizeof(I) == sizeof(double) && sizeof(T) == sizeof(double) && sizeof(O) == sizeof(double)) {
        if (op.mfma && op.circ && center) {   // FP64 d_phi on the matrix cores
            const int n = op.n_in;
            if (n % 16 || n / 16 > 8 || n / 16 < 1) return hipErrorInvalidValue;
            const size_t shm_m = sizeof(double) * (size_t(n) * kMfmaCols + size_t(n / 16) * kMfmaCols + 2 * size_t(n));
            hipLaunchKernelGGL(k_dphi_mfma, dim3((unsigned)((ncol + kMfmaCols - 1) / kMfmaCols), (unsigned)n_fields),
                               dim3(64 * (n / 16)), shm_m, st, in, out, Wb, n, ncol);
            return hipGetLastError();
        }
    }
    const size_t shm = sizeof(T) * size_t(op.n_in) * 64 + size_t(4 * op.passes) * 64 * sizeof(double);
    switch (op.R) {
#define X(R)                                                                                                   \
    case R:                                                                                                    \
        if (op.circ)                                                                                           \
            hipLaunchKernelGGL((k_axis<R, I, T, O, true>), dim3(bx, n_fields), dim3(nt), shm, st, in, out, Wb, \
                               op.n_in, op.n_out, ncol, center);                                               \
        else                                                                                                   \
            hipLaunchKernelGGL((k_axis<R, I, T, O, false>), dim3(bx, n_fields), dim3(nt), shm, st, in, out,    \
                               Wb, op.n_in, op.n_out, ncol, center);                                           \
        break;
        SG_R_CASES(X)
#undef X
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_axis(const AxisOp& op, const double* in, double* out, long long ncol, int n_fields, int center,
                       hipStream_t st) {
    return axis_t<double, double, double>(op, op.Wb, in, out, ncol, n_fields, center, st);
}

hipError_t launch_axis_f32(const AxisOp& op, const double* in, float* out, long long ncol, int n_fields, int center,
                           hipStream_t st) {
    return axis_t<double, float, float>(op, op.Wb_f, in, out, ncol, n_fields, center, st);
}

hipError_t launch_axis_ff(const AxisOp& op, const float* in, float* out, long long ncol, int n_fields,
                          hipStream_t st) {
    return axis_t<float, float, float>(op, op.Wb_f, in, out, ncol, n_fields, 0, st);
}

template <typename T, typename O>
static hipError_t derivs3_t(const KShell& s, const AxisOp& dph, const T* Wph, const T* Hsb,
                            const double* in, double* out_r, O* out_th, O* out_ph, int n_fields, hipStream_t st) {
    const int nw = s.Dr_nw;
    if (s.Hth_nw != nw || 4 * dph.passes != nw || (dph.par != 3 && !dph.circ) || dph.mfma || dph.n_in != s.n_ph ||
        s.Dr_R > kFusedMaxR || s.Hth_R > kFusedMaxRth || dph.R > (dph.circ ? kFusedMaxRcirc : kFusedMaxR))
        return hipErrorNotSupported;   // shapes disagree: the caller launches the three kernels
    if (s.n_th > nw * kThMaxPerThread || dph.n_in > kAxisMaxIn) return hipErrorInvalidValue;
    D3Dims a;
    a.n_lines = (long long)n_fields * s.npts / s.n_r;
    a.n_cols_th = (long long)n_fields * (s.n_ph / 2) * s.n_r;
    a.ncol_ph = (long long)s.n_th * s.n_r;
    a.b_dr = (unsigned)((a.n_lines + 63) / 64);
    a.th_plane = sizeof(T) == sizeof(double) && s.th_plane;
    a.b_th = a.th_plane ? (unsigned)(n_fields * (s.n_ph / 2)) : (unsigned)((a.n_cols_th + 63) / 64);
    a.bx_ph = (unsigned)((a.ncol_ph + 63) / 64);
    a.nf = n_fields;
    a.R_dr = s.Dr_R;
    a.R_th = s.Hth_R;
    a.R_ph = dph.R;
    a.ph_par = dph.par == 3;
    a.n_r = s.n_r;
    a.n_th = s.n_th;
    a.n_ph = s.n_ph;
    const size_t part = size_t(nw) * 64 * sizeof(double);
    size_t shm = sizeof(double) * size_t(s.n_r) * kDrStride;
    shm = std::max(shm, a.th_plane ? sizeof(double) * (2 * size_t(s.n_th) * s.n_r + size_t(nw) * s.n_r)
                                   : sizeof(T) * 2 * size_t(s.n_th) * 64 + part);
    shm = std::max(shm, sizeof(T) * size_t(s.n_ph) * 64 + part);
    const unsigned long long blocks = (unsigned long long)a.b_dr + a.b_th + (unsigned long long)a.bx_ph * n_fields;
    if (blocks >= (1ull << 31)) return hipErrorNotSupported;
    hipLaunchKernelGGL((k_derivs3<T, O>), dim3((unsigned)blocks), dim3(64 * nw), shm, st, in, out_r, out_th, out_ph,
                       s.Drb, Hsb, Wph, a);
    return hipGetLastError();
}

hipError_t launch_derivs3(const KShell& s, const AxisOp& dph, const double* in, double* out, int n_fields,
                          hipStream_t st) {
    const long long cnt = (long long)s.npts * n_fields;
    return derivs3_t<double, double>(s, dph, dph.Wb, s.Hsb, in, out, out + cnt, out + 2 * cnt, n_fields, st);
}

hipError_t launch_derivs3_mixed(const KShell& s, const AxisOp& dph, const double* in, double* dr, float* dang,
                                int n_fields, hipStream_t st) {
    const long long cnt = (long long)s.npts * n_fields;
    return derivs3_t<float, float>(s, dph, dph.Wb_f, s.Hsb_f, in, dr, dang, dang + cnt, n_fields, st);
}

hipError_t launch_chain(const KShell& s, double* du, int n_fields, hipStream_t st) {
    const unsigned blocks = (unsigned)((s.npts + 255) / 256);
    hipLaunchKernelGGL(k_chain, dim3(blocks), dim3(256), 0, st, s, du, n_fields);
    return hipGetLastError();
}

}  // namespace sg
