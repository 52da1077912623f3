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
#include "internal.h"

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

// out[f][q][c] = sum_r W[q][r] (in[f][r][c] - m_c), m_c the mean of column c
// over r (the d_phi contraction with the phi-circle mean removed).
// grid (ceil(ncol / 64), n_fields), 256 threads.
__global__ __launch_bounds__(256) void k_bf3_axis(const double* __restrict__ in, float* __restrict__ out,
                                                  const __bf16* __restrict__ Whi, const __bf16* __restrict__ Wlo,
                                                  int n_in, int n_out, int K, int M, long long ncol) {
    extern __shared__ double smd[];   // partial sums [4][64] FP64, then hi, lo tiles [64][K + kBfPad]
    double* spart = smd;
    const int ldx = K + kBfPad;
    __bf16* xhi = reinterpret_cast<__bf16*>(smd + 4 * 64);
    __bf16* xlo = xhi + 64 * ldx;
    const long long c0 = (long long)blockIdx.x * 64;
    const int nc = (int)min((long long)64, ncol - c0);
    const int f = blockIdx.y;
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lc = lane < nc ? lane : 0;
    const double* src = in + (long long)f * n_in * ncol + c0 + lc;
    constexpr int kPer = kBfMaxIn / 4;
    double v[kPer];
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        const int r = w + 4 * t;
        v[t] = (r < n_in) ? src[(long long)r * ncol] : 0.0;
    }
    double part = 0.0;
#pragma unroll
    for (int t = 0; t < kPer; ++t) part += v[t];
    spart[w * 64 + lane] = part;
    __syncthreads();
    const double mc = (spart[lane] + spart[64 + lane] + spart[128 + lane] + spart[192 + lane]) / n_in;
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        const int r = w + 4 * t;
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
    for (int b = w; b < blocks; b += 4) {
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
// d f(phi_j + pi) = (Hs S - Ha A) / 2.  grid ceil(n_cols / 64), 256 threads.
__global__ __launch_bounds__(256) void k_bf3_theta(const double* __restrict__ in, float* __restrict__ out,
                                                   const __bf16* __restrict__ Shi, const __bf16* __restrict__ Slo,
                                                   const __bf16* __restrict__ Ahi, const __bf16* __restrict__ Alo,
                                                   int n_r, int n_th, int n_ph, int K, int M, long long n_cols) {
    extern __shared__ double smd[];   // partial sums [4][64], then S hi, S lo, A hi, A lo tiles [64][K + kBfPad]
    double* spart = smd;
    const int ldx = K + kBfPad;
    __bf16* shi = reinterpret_cast<__bf16*>(smd + 4 * 64);
    __bf16* slo = shi + 64 * ldx;
    __bf16* ahi = slo + 64 * ldx;
    __bf16* alo = ahi + 64 * ldx;
    const int half = n_ph / 2;
    const long long plane = (long long)n_th * n_r;
    const long long c0 = (long long)blockIdx.x * 64;
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
    constexpr int kPer = 64 / 4;   // N_theta <= 64
    double sv[kPer], av[kPer];
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        const int ip = w + 4 * t;
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
    const double mc = (spart[lane] + spart[64 + lane] + spart[128 + lane] + spart[192 + lane]) / n_th;
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        const int ip = w + 4 * t;
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
    for (int b = w; b < blocks; b += 4) {
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

}  // namespace

size_t bf3_axis_shm(int K) { return 4 * 64 * sizeof(double) + 2 * size_t(64) * (K + kBfPad) * sizeof(__bf16); }
size_t bf3_theta_shm(int K) { return 4 * 64 * sizeof(double) + 4 * size_t(64) * (K + kBfPad) * sizeof(__bf16); }

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
