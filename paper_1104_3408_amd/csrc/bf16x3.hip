// BF16x3 angular derivatives on the matrix cores (SG_PREC_BF16X3).
//
// The theta and phi contractions of Sec. 2.4 (eqs. D2, D3) are products of a
// small dense operator W (N_out x N_in) with a tile of 64 columns of the
// state.  Here they run as v_mfma_f32_32x32x16_bf16 with every operand split
// into two bfloat16 parts, x = x_hi + x_lo (x_hi = bf16(x), x_lo =
// bf16(x - x_hi)), and W x accumulated in FP32 as
//   W_hi x_hi + W_hi x_lo + W_lo x_hi
// (the W_lo x_lo term, about 2^-16 of |W||x|, is dropped).  The column means
// are removed in FP64 before the split, as in the FP32 path, and d_r, the rhs
// and the RK state stay FP64.
//
// Tiles: a workgroup of 4 waves stages 64 columns in LDS, transposed so that
// the 8 consecutive input rows one lane feeds to the MFMA are 16 contiguous
// bytes ([column][K + 8], the 8 padding values keep the 64 lanes' 16-byte
// reads on distinct banks); each wave produces 32 x 32 output blocks.  The
// operators are stored split and zero-padded on the host, [M][K] with M, K
// rounded up to 32 and 16, so the blocks need no bounds checks on K.
//
// MFMA 32x32x16 bf16 operand layout (checked on the device): lane l holds
// A[m = l % 32][k = 8 (l / 32) + i] and B[k = 8 (l / 32) + i][n = l % 32],
// i < 8; the 16 results are D[8 (i / 4) + 4 (l / 32) + i % 4][l % 32].
#include <algorithm>

#include "internal.h"
#include "tile_dr.h"

namespace sg {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kBfPad = 8;      // row padding of the transposed LDS tiles (bf16 values)
constexpr int kBfMaxIn = 128;  // largest contraction length (N_phi <= 128)

__device__ __forceinline__ void split_bf16(double x, __bf16& hi, __bf16& lo) {
    const float xf = (float)x;
    hi = (__bf16)xf;
    lo = (__bf16)(xf - (float)hi);
}

__device__ __forceinline__ bf16x8 lds8(const __bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }
__device__ __forceinline__ bf16x8 gld8(const __bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }

// acc += W (rows 32 mb.., split hi/lo, [M][K]) x tile (columns 32 nb.., split)
__device__ __forceinline__ floatx16 mfma3(floatx16 acc, const __bf16* __restrict__ Whi,
                                          const __bf16* __restrict__ Wlo, const __bf16* xhi, const __bf16* xlo,
                                          int K, int ldx, int mb, int nb, int lane) {
    const int m = 32 * mb + (lane & 31), n = 32 * nb + (lane & 31), k8 = 8 * (lane >> 5);
    const __bf16* wh = Whi + (long long)m * K + k8;
    const __bf16* wl = Wlo + (long long)m * K + k8;
    const __bf16* bh = xhi + n * ldx + k8;
    const __bf16* bl = xlo + n * ldx + k8;
    for (int kk = 0; kk < K; kk += 16) {
        const bf16x8 ah = gld8(wh + kk), al = gld8(wl + kk);
        const bf16x8 xh = lds8(bh + kk), xl = lds8(bl + kk);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, xh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, xl, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, xh, acc, 0, 0, 0);
    }
    return acc;
}

// out[f][q][c] = sum_r W[q][r] (in[f][r][c] - m_c) for the 64 columns of
// tile `tile` of field f, NW waves.  CENTER: m_c is the mean of column c
// over r (the d_phi contraction with the phi-circle mean removed, FP64
// input); otherwise m_c = 0 (the phi analysis and synthesis of the filter's
// FP32 difference columns).
template <int NW, typename I = double, bool CENTER = true>
__device__ __forceinline__ void bf3_axis_tile(long long tile, int f, const I* __restrict__ in,
                                              float* __restrict__ out, const __bf16* __restrict__ Whi,
                                              const __bf16* __restrict__ Wlo, int n_in, int n_out, int K, int M,
                                              long long ncol, double* __restrict__ smd) {
    // smd: partial sums [NW][64] FP64, then hi, lo tiles [64][K + kBfPad]
    double* spart = smd;
    const int ldx = K + kBfPad;
    __bf16* xhi = reinterpret_cast<__bf16*>(smd + NW * 64);
    __bf16* xlo = xhi + 64 * ldx;
    const long long c0 = tile * 64;
    const int nc = (int)min((long long)64, ncol - c0);
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lc = lane < nc ? lane : 0;
    const I* src = in + (long long)f * n_in * ncol + c0 + lc;
    constexpr int kPer = kBfMaxIn / NW;
    double v[kPer];
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        const int r = w + NW * t;
        v[t] = (r < n_in) ? (double)src[(long long)r * ncol] : 0.0;
    }
    double mc = 0.0;
    if (CENTER) {
        double part = 0.0;
#pragma unroll
        for (int t = 0; t < kPer; ++t) part += v[t];
        spart[w * 64 + lane] = part;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NW; ++q) mc += spart[q * 64 + lane];
        mc /= n_in;
    }
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        const int r = w + NW * t;
        if (r < K) {
            __bf16 h = (__bf16)0.0f, l = (__bf16)0.0f;
            if (r < n_in) split_bf16(v[t] - mc, h, l);
            xhi[lane * ldx + r] = h;
            xlo[lane * ldx + r] = l;
        }
    }
    __syncthreads();
    const int blocks = (M / 32) * 2;
    float* dst = out + (long long)f * n_out * ncol + c0;
    for (int b = w; b < blocks; b += NW) {
        const int mb = b >> 1, nb = b & 1;
        floatx16 acc;
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
        acc = mfma3(acc, Whi, Wlo, xhi, xlo, K, ldx, mb, nb, lane);
        const int col = 32 * nb + (lane & 31);
        if (col < nc) {
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int q = 32 * mb + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
                if (q < n_out) dst[(long long)q * ncol + col] = acc[i];
            }
        }
    }
}

// d_theta on meridian pairs (even/odd form of k_dtheta): column c =
// (f * half + jp) * n_r + k, S = f(phi_j) + f(phi_j + pi) with its circle
// mean removed, A = f(phi_j) - f(phi_j + pi); d f(phi_j) = (Hs S + Ha A) / 2,
// d f(phi_j + pi) = (Hs S - Ha A) / 2.  Column tile `tile`, NW waves.
template <int NW>
__device__ __forceinline__ void bf3_theta_tile(long long tile, const double* __restrict__ in, float* __restrict__ out,
                                               const __bf16* __restrict__ Shi, const __bf16* __restrict__ Slo,
                                               const __bf16* __restrict__ Ahi, const __bf16* __restrict__ Alo,
                                               int n_r, int n_th, int n_ph, int K, int M, long long n_cols,
                                               double* __restrict__ smd) {
    // smd: partial sums [NW][64], then S hi, S lo, A hi, A lo tiles [64][K + kBfPad]
    double* spart = smd;
    const int ldx = K + kBfPad;
    __bf16* shi = reinterpret_cast<__bf16*>(smd + NW * 64);
    __bf16* slo = shi + 64 * ldx;
    __bf16* ahi = slo + 64 * ldx;
    __bf16* alo = ahi + 64 * ldx;
    const int half = n_ph / 2;
    const long long plane = (long long)n_th * n_r;
    const long long c0 = tile * 64;
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    auto decode = [&](long long c, long long& fo, int& jp, int& k) {
        const long long fj = c / n_r;
        k = (int)(c - fj * n_r);
        fo = fj / half;
        jp = (int)(fj - fo * half);
    };
    const long long c = c0 + lane;
    const bool cok = c < n_cols;
    long long f = 0;
    int jp = 0, k = 0;
    if (cok) decode(c, f, jp, k);
    const double* base = in + f * n_ph * plane + (long long)jp * plane + k;
    constexpr int kPer = 64 / NW;   // N_theta <= 64
    double sv[kPer], av[kPer];
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        const int ip = w + NW * t;
        double a = 0.0, b = 0.0;
        if (ip < n_th) {
            a = base[(long long)ip * n_r];
            b = base[half * plane + (long long)ip * n_r];
        }
        sv[t] = cok ? a + b : 0.0;
        av[t] = cok ? a - b : 0.0;
    }
    double part = 0.0;
#pragma unroll
    for (int t = 0; t < kPer; ++t) part += sv[t];
    spart[w * 64 + lane] = part;
    __syncthreads();
    double mc = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) mc += spart[q * 64 + lane];
    mc /= n_th;
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        const int ip = w + NW * t;
        if (ip < K) {
            __bf16 h = (__bf16)0.0f, l = (__bf16)0.0f, h2 = (__bf16)0.0f, l2 = (__bf16)0.0f;
            if (ip < n_th) {
                split_bf16(sv[t] - mc, h, l);
                split_bf16(av[t], h2, l2);
            }
            shi[lane * ldx + ip] = h;
            slo[lane * ldx + ip] = l;
            ahi[lane * ldx + ip] = h2;
            alo[lane * ldx + ip] = l2;
        }
    }
    __syncthreads();
    const int blocks = (M / 32) * 2;
    for (int b = w; b < blocks; b += NW) {
        const int mb = b >> 1, nb = b & 1;
        floatx16 aS, aA;
#pragma unroll
        for (int i = 0; i < 16; ++i) aS[i] = aA[i] = 0.0f;
        aS = mfma3(aS, Shi, Slo, shi, slo, K, ldx, mb, nb, lane);
        aA = mfma3(aA, Ahi, Alo, ahi, alo, K, ldx, mb, nb, lane);
        const long long cc = c0 + 32 * nb + (lane & 31);
        if (cc < n_cols) {
            long long fo;
            int jo, ko;
            decode(cc, fo, jo, ko);
            float* o = out + fo * n_ph * plane + (long long)jo * plane + ko;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int q = 32 * mb + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
                if (q < n_th) {
                    o[(long long)q * n_r] = 0.5f * (aS[i] + aA[i]);
                    o[half * plane + (long long)q * n_r] = 0.5f * (aS[i] - aA[i]);
                }
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_bf3_axis(const double* __restrict__ in, float* __restrict__ out,
                                                  const __bf16* __restrict__ Whi, const __bf16* __restrict__ Wlo,
                                                  int n_in, int n_out, int K, int M, long long ncol) {
    extern __shared__ double smd[];
    bf3_axis_tile<4>(blockIdx.x, blockIdx.y, in, out, Whi, Wlo, n_in, n_out, K, M, ncol, smd);
}

// Fourier analysis / synthesis along phi of the filter's FP32 difference
// columns (Sec. 3.1), dense split operator: analysis K x N_phi, synthesis
// N_phi x K.
__global__ __launch_bounds__(256) void k_bf3_axis_ff(const float* __restrict__ in, float* __restrict__ out,
                                                     const __bf16* __restrict__ Whi, const __bf16* __restrict__ Wlo,
                                                     int n_in, int n_out, int K, int M, long long ncol) {
    extern __shared__ double smd[];
    bf3_axis_tile<4, float, false>(blockIdx.x, blockIdx.y, in, out, Whi, Wlo, n_in, n_out, K, M, ncol, smd);
}

__global__ __launch_bounds__(256) void k_bf3_theta(const double* __restrict__ in, float* __restrict__ out,
                                                   const __bf16* __restrict__ Shi, const __bf16* __restrict__ Slo,
                                                   const __bf16* __restrict__ Ahi, const __bf16* __restrict__ Alo,
                                                   int n_r, int n_th, int n_ph, int K, int M, long long n_cols) {
    extern __shared__ double smd[];
    bf3_theta_tile<4>(xcd_block(blockIdx.x, gridDim.x), in, out, Shi, Slo, Ahi, Alo, n_r, n_th, n_ph, K, M, n_cols,
                      smd);
}

// Theta filter of the split filter's FP32 spectral columns on the matrix
// cores (SG_PREC_BF16X3).  Same workgroups and combinations as k_ftheta
// (filter.hip): a column tile of one column set at order m; for a complex
// group at m > 0 two passes, P = F_+ (a^x + b^y), M = F_- (a^x - b^y) and
// P = F_- (a^y + b^x), M = F_+ (a^y - b^x), with F_- = J F_+ J applied as F_+
// on theta-reversed vectors (J reverses theta).  The two vectors of a pass
// are staged split (hi, lo bfloat16) and transposed, [column][K + pad], F is
// F^{|n|}_m split and zero-padded to [M][K]; four waves form the 32 x 32
// blocks of F v0 and F v1, which go through LDS (FP32) for the reversal on
// the way out.
__global__ __launch_bounds__(256) void k_ftheta_bf3(int n_r, int n_th, int m_keep, int n_cols_state,
                                                    const float* __restrict__ spec, float* __restrict__ spec2,
                                                    const __bf16* __restrict__ Fhi, const __bf16* __restrict__ Flo,
                                                    int K, int M, const FiltGroup* __restrict__ groups,
                                                    const FiltSet* __restrict__ sets, int n_sets) {
    extern __shared__ double smd[];
    const int ldx = K + kBfPad;
    __bf16* x0h = reinterpret_cast<__bf16*>(smd);   // [64][ldx] each
    __bf16* x0l = x0h + 64 * ldx;
    __bf16* x1h = x0l + 64 * ldx;
    __bf16* x1l = x1h + 64 * ldx;
    float* res = reinterpret_cast<float*>(x1l + 64 * ldx);   // [2][n_th][64]
    // (column tile, 2 m + pass, set x shell), tiles of one range on one XCD; the
    // two passes of a complex group at m > 0 read and write disjoint columns,
    // so they are separate workgroups (the second exits for every other set)
    const Blk3 b = xcd_block3();
    const int m = b.y >> 1, pass_sel = b.y & 1;
    const FiltSet fs = sets[b.z % n_sets];
    const int shell = b.z / n_sets;
    const long long per_m = (long long)n_th * n_r;
    const long long col = (long long)(2 * m_keep + 1) * per_m;   // one storage column
    {
        const long long so = (long long)shell * n_cols_state * col;
        spec += so;
        spec2 += so;
    }
    const long long c0 = (long long)b.x * 64;
    if (c0 >= (long long)fs.count * n_r) return;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    constexpr int NW = 4, kPer = 64 / NW;   // theta rows one thread stages (N_theta <= 64)
    const long long c = c0 + lane;
    const bool ok = c < (long long)fs.count * n_r;
    const int gi = ok ? (int)(c / n_r) : 0;
    const int k = ok ? (int)(c - (long long)gi * n_r) : 0;
    const FiltGroup G = groups[fs.first + gi];
    const int qa = (m == 0) ? 0 : 2 * m - 1, qb = 2 * m;
    const long long fo = (long long)(fs.mat * (m_keep + 1) + m) * M * K;
    const __bf16* Wh = Fhi + fo;
    const __bf16* Wl = Flo + fo;
    const bool mix = fs.cplx && m > 0;   // block-uniform
    const bool neg = G.sign < 0;          // F_+ = J F J for a negative spin
    if (pass_sel && !mix) return;
    for (int pass = pass_sel; pass <= pass_sel; ++pass) {
        const float* xa;
        const float* xb = nullptr;
        bool rev0 = false, rev1 = false;
        if (!fs.cplx) {
            xa = spec + G.re * col + qa * per_m + k;
            if (m > 0) xb = spec + G.re * col + qb * per_m + k;
        } else if (m == 0) {
            xa = spec + G.re * col + k;
            xb = spec + G.im * col + k;
        } else if (pass == 0) {
            xa = spec + G.re * col + qa * per_m + k;
            xb = spec + G.im * col + qb * per_m + k;
            rev0 = neg;
            rev1 = !neg;
        } else {
            xa = spec + G.im * col + qa * per_m + k;
            xb = spec + G.re * col + qb * per_m + k;
            rev0 = !neg;
            rev1 = neg;
        }
        float la[kPer], lb[kPer];
#pragma unroll
        for (int t = 0; t < kPer; ++t) {
            const int ip = w + NW * t;
            la[t] = (ip < n_th) ? xa[ip * (long long)n_r] : 0.0f;
            lb[t] = (ip < n_th && xb) ? xb[ip * (long long)n_r] : 0.0f;
        }
#pragma unroll
        for (int t = 0; t < kPer; ++t) {
            const int ip = w + NW * t;
            if (ip < K) {   // rows n_th .. K - 1 are zero padding of the contraction
                __bf16 h0 = (__bf16)0.0f, l0 = (__bf16)0.0f, h1 = (__bf16)0.0f, l1 = (__bf16)0.0f;
                int r0 = ip, r1 = ip;
                if (ip < n_th) {
                    const float va = ok ? la[t] : 0.0f, vb = ok ? lb[t] : 0.0f;
                    split_bf16(mix ? va + vb : va, h0, l0);
                    split_bf16(mix ? va - vb : vb, h1, l1);
                    r0 = rev0 ? n_th - 1 - ip : ip;
                    r1 = rev1 ? n_th - 1 - ip : ip;
                }
                x0h[lane * ldx + r0] = h0;
                x0l[lane * ldx + r0] = l0;
                x1h[lane * ldx + r1] = h1;
                x1l[lane * ldx + r1] = l1;
            }
        }
        __syncthreads();
        const int blocks = (M / 32) * 2 * 2;   // row blocks x column blocks x (v0, v1)
        for (int b = w; b < blocks; b += NW) {
            const int vec = b & 1, nb = (b >> 1) & 1, mb = b >> 2;
            floatx16 acc;
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
            acc = mfma3(acc, Wh, Wl, vec ? x1h : x0h, vec ? x1l : x0l, K, ldx, mb, nb, lane);
            const int cc = 32 * nb + (lane & 31);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int q = 32 * mb + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
                if (q < n_th) res[(vec * n_th + q) * 64 + cc] = acc[i];
            }
        }
        __syncthreads();
        if (!ok) continue;
        for (int i = w; i < n_th; i += NW) {
            const float p0 = res[(rev0 ? n_th - 1 - i : i) * 64 + lane];
            const float p1 = res[(n_th + (rev1 ? n_th - 1 - i : i)) * 64 + lane];
            const long long o = (long long)i * n_r + k;
            if (!fs.cplx) {
                spec2[G.re * col + qa * per_m + o] = p0;
                if (m > 0) spec2[G.re * col + qb * per_m + o] = p1;
            } else if (m == 0) {
                spec2[G.re * col + o] = p0;
                spec2[G.im * col + o] = p1;
            } else if (pass == 0) {
                spec2[G.re * col + qa * per_m + o] = 0.5f * (p0 + p1);   // a^x'
                spec2[G.im * col + qb * per_m + o] = 0.5f * (p0 - p1);   // b^y'
            } else {
                spec2[G.im * col + qa * per_m + o] = 0.5f * (p0 + p1);   // a^y'
                spec2[G.re * col + qb * per_m + o] = 0.5f * (p0 - p1);   // b^x'
            }
        }
    }
}

// One launch for a stage's three contractions in SG_PREC_BF16X3 (the FP64
// d_r tiles and the two matrix-core tiles interleaved over the grid as in the
// FP64 form; kMinWaves waves per workgroup).  Pointers are separate
// __restrict__ arguments (the FP64 d_r operator then stays in scalar loads).
struct B3Dims {
    long long n_lines, n_cols_th, ncol_ph;
    unsigned b_dr, b_th, bx_ph;
    int nf, R_dr, n_r, n_th, n_ph, K_th, M_th, K_ph, M_ph;
};

__global__ __launch_bounds__(64 * kMinWaves) void k_derivs3_bf3(
    const double* __restrict__ in, double* __restrict__ out_r, float* __restrict__ out_th,
    float* __restrict__ out_ph, const double* __restrict__ Drb, const __bf16* __restrict__ Shi,
    const __bf16* __restrict__ Slo, const __bf16* __restrict__ Ahi, const __bf16* __restrict__ Alo,
    const __bf16* __restrict__ Phi, const __bf16* __restrict__ Plo, B3Dims a) {
    extern __shared__ double smd[];
    const unsigned long long B = (unsigned long long)a.b_dr + a.b_th + (unsigned long long)a.bx_ph * a.nf;
    const unsigned long long bb = blockIdx.x;
    const unsigned long long d0 = bb * a.b_dr / B, d1 = (bb + 1) * a.b_dr / B;
    const unsigned long long o = bb - d0, n_o = B - a.b_dr;
    const unsigned long long t0 = n_o ? o * a.b_th / n_o : 0, t1 = n_o ? (o + 1) * a.b_th / n_o : 0;
    if (d1 > d0) {
        switch (a.R_dr) {
#define X(R) case R: dr_tile<R>(d0, in, out_r, Drb, a.n_r, a.n_lines, smd); break;
            X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9)
#undef X
        }
        return;
    }
    if (t1 > t0) {
        bf3_theta_tile<kMinWaves>(t0, in, out_th, Shi, Slo, Ahi, Alo, a.n_r, a.n_th, a.n_ph, a.K_th, a.M_th,
                                  a.n_cols_th, smd);
        return;
    }
    const unsigned long long p = o - t0;
    bf3_axis_tile<kMinWaves>((long long)(p % a.bx_ph), (int)(p / a.bx_ph), in, out_ph, Phi, Plo, a.n_ph, a.n_ph,
                             a.K_ph, a.M_ph, a.ncol_ph, smd);
}

}  // namespace

size_t bf3_axis_shm(int K, int nw = 4) { return nw * 64 * sizeof(double) + 2 * size_t(64) * (K + kBfPad) * sizeof(__bf16); }
size_t bf3_theta_shm(int K, int nw = 4) { return nw * 64 * sizeof(double) + 4 * size_t(64) * (K + kBfPad) * sizeof(__bf16); }

hipError_t launch_derivs3_bf3(const KShell& s, const Bf3Op& dph, const Bf3Op& hs, const Bf3Op& ha, const double* in,
                              double* dr, float* dang, int n_fields, hipStream_t st) {
    if (s.Dr_nw != kMinWaves || s.Dr_R > 9) return hipErrorNotSupported;
    if (s.n_th > 64 || hs.K != ha.K || hs.M != ha.M || hs.K < s.n_th || hs.K % 16 || hs.M % 32 || hs.M > 64 ||
        dph.n_in > kBfMaxIn || dph.K < dph.n_in || dph.K % 16 || dph.M % 32 || dph.M > 128)
        return hipErrorInvalidValue;
    B3Dims a;
    a.n_lines = (long long)n_fields * s.npts / s.n_r;
    a.n_cols_th = (long long)n_fields * (s.n_ph / 2) * s.n_r;
    a.ncol_ph = (long long)s.n_th * s.n_r;
    a.b_dr = (unsigned)((a.n_lines + 63) / 64);
    a.b_th = (unsigned)((a.n_cols_th + 63) / 64);
    a.bx_ph = (unsigned)((a.ncol_ph + 63) / 64);
    a.nf = n_fields;
    a.R_dr = s.Dr_R;
    a.n_r = s.n_r;
    a.n_th = s.n_th;
    a.n_ph = s.n_ph;
    a.K_th = hs.K;
    a.M_th = hs.M;
    a.K_ph = dph.K;
    a.M_ph = dph.M;
    size_t shm = sizeof(double) * size_t(s.n_r) * kDrStride;
    shm = std::max(shm, bf3_theta_shm(hs.K, kMinWaves));
    shm = std::max(shm, bf3_axis_shm(dph.K, kMinWaves));
    const unsigned long long blocks = (unsigned long long)a.b_dr + a.b_th + (unsigned long long)a.bx_ph * n_fields;
    if (blocks >= (1ull << 31)) return hipErrorNotSupported;
    const long long cnt = (long long)s.npts * n_fields;
    hipLaunchKernelGGL(k_derivs3_bf3, dim3((unsigned)blocks), dim3(64 * kMinWaves), shm, st, in, dr, dang,
                       dang + cnt, s.Drb, reinterpret_cast<const __bf16*>(hs.hi),
                       reinterpret_cast<const __bf16*>(hs.lo), reinterpret_cast<const __bf16*>(ha.hi),
                       reinterpret_cast<const __bf16*>(ha.lo), reinterpret_cast<const __bf16*>(dph.hi),
                       reinterpret_cast<const __bf16*>(dph.lo), a);
    return hipGetLastError();
}

hipError_t launch_bf3_dphi(const KShell& s, const Bf3Op& op, const double* in, float* out, int n_fields,
                           hipStream_t st) {
    const long long ncol = (long long)s.n_th * s.n_r;
    if (op.n_in > kBfMaxIn || op.K < op.n_in || op.K % 16 || op.M % 32 || op.M < op.n_out || op.M > 128)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bf3_axis, dim3((unsigned)((ncol + 63) / 64), (unsigned)n_fields), dim3(256),
                       bf3_axis_shm(op.K), st, in, out, reinterpret_cast<const __bf16*>(op.hi),
                       reinterpret_cast<const __bf16*>(op.lo), op.n_in, op.n_out, op.K, op.M, ncol);
    return hipGetLastError();
}

hipError_t launch_ftheta_bf3(const KShell& s, int count, const float* spec, float* spec2, const Bf3Op& F,
                             const FiltPlan& fp, int n_cols, int m_keep, hipStream_t st) {
    if (s.n_th > 64 || F.K < s.n_th || F.K % 16 || F.M % 32 || F.M < s.n_th || F.M > 64) return hipErrorInvalidValue;
    const long long cols = (long long)fp.max_groups * s.n_r;
    const dim3 grid((unsigned)((cols + 63) / 64), (unsigned)(2 * (m_keep + 1)), (unsigned)(fp.n_sets * count));
    const size_t shm = 4 * size_t(64) * (F.K + kBfPad) * sizeof(__bf16) + 2 * size_t(s.n_th) * 64 * sizeof(float);
    hipLaunchKernelGGL(k_ftheta_bf3, grid, dim3(256), shm, st, s.n_r, s.n_th, m_keep, n_cols, spec, spec2,
                       reinterpret_cast<const __bf16*>(F.hi), reinterpret_cast<const __bf16*>(F.lo), F.K, F.M,
                       fp.groups, fp.sets, fp.n_sets);
    return hipGetLastError();
}

hipError_t launch_bf3_axis_ff(const Bf3Op& op, const float* in, float* out, long long ncol, int n_fields,
                              hipStream_t st) {
    if (op.n_in > kBfMaxIn || op.K < op.n_in || op.K % 16 || op.M % 32 || op.M < op.n_out || op.M > 128)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bf3_axis_ff, dim3((unsigned)((ncol + 63) / 64), (unsigned)n_fields), dim3(256),
                       bf3_axis_shm(op.K), st, in, out, reinterpret_cast<const __bf16*>(op.hi),
                       reinterpret_cast<const __bf16*>(op.lo), op.n_in, op.n_out, op.K, op.M, ncol);
    return hipGetLastError();
}

hipError_t launch_bf3_dtheta(const KShell& s, const Bf3Op& hs, const Bf3Op& ha, const double* in, float* out,
                             int n_fields, hipStream_t st) {
    const long long n_cols = (long long)n_fields * (s.n_ph / 2) * s.n_r;
    if (s.n_th > 64 || hs.K != ha.K || hs.M != ha.M || hs.K < s.n_th || hs.K % 16 || hs.M % 32 || hs.M > 64)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bf3_theta, dim3((unsigned)((n_cols + 63) / 64)), dim3(256), bf3_theta_shm(hs.K), st, in,
                       out, reinterpret_cast<const __bf16*>(hs.hi), reinterpret_cast<const __bf16*>(hs.lo),
                       reinterpret_cast<const __bf16*>(ha.hi), reinterpret_cast<const __bf16*>(ha.lo), s.n_r,
                       s.n_th, s.n_ph, hs.K, hs.M, n_cols);
    return hipGetLastError();
}

}  // namespace sg
