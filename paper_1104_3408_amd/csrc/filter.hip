// Tensor Yn filter (Sec. 3.5) on the field-major layout.
//
// Pipeline per shell: (1) decompose every tensor on the complex tetrad
// (t, r, m, mbar) of Sec. 3.4 into real storage columns; (2) real Fourier
// analysis in phi (Sec. 3.1) on the shared phi-axis kernel; (3) the theta
// filters F^n_m per Fourier order m (this file); (4) Fourier synthesis;
// (5) recombination into Cartesian components (eq. tensorexpansion).
//
// Real form of the theta step.  A complex component f = x + i y of spin n has
// real Fourier coefficients (a^x, b^x) and (a^y, b^y) for every order m > 0.
// The orders +m and -m are filtered with F_+ = F^n_m and F_- = F^n_{-m} =
// F^{-n}_m; with S = (F_+ + F_-)/2 and D = (F_+ - F_-)/2 this becomes
//   a^x' = S a^x + D b^y     a^y' = S a^y - D b^x
//   b^x' = S b^x - D a^y     b^y' = S b^y + D a^x,
// and a' = S a at m = 0 (D vanishes there).  Real spin-0 columns use S only.
//
// Storage columns of the tetrad array (spin label n = #m - #mbar):
//   g, Pi (10 each): tt tr rr (m mbar) real; tm rm (n=1), mm (n=2) complex.
//   Phi (30): r-row as g; m-row complex: tt tr rr (m mbar) (n=1), tm rm (n=2),
//             t mbar, r mbar (n=0), mm (n=3), mbar mbar (n=-1).
//   H_a, Q_a (4 each, 58 fields): t r real, m (n=1) complex.
#include "internal.h"


namespace sg {

namespace {

struct cx {
    double re, im;
};
__device__ __forceinline__ cx operator+(cx a, cx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cx operator*(cx a, cx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cx operator*(double s, cx a) { return {s * a.re, s * a.im}; }
__device__ __forceinline__ cx conj(cx a) { return {a.re, -a.im}; }

__device__ __forceinline__ int pr(int a, int b) {
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    return lo == 0 ? hi : (lo == 1 ? 3 + hi : (lo == 2 ? 5 + hi : 9));
}

struct Tetrad {
    double r[3], th[3], ph[3];
    cx m[3], mb[3];
};

__device__ __forceinline__ Tetrad make_tetrad(const KShell& s, int i, int j) {
    Tetrad T;
    const double st = s.sth[i], ct = s.cth[i], sp = s.sph[j], cp = s.cph[j];
    const double h = 0.70710678118654752440;
    T.r[0] = st * cp; T.r[1] = st * sp; T.r[2] = ct;
    T.th[0] = ct * cp; T.th[1] = ct * sp; T.th[2] = -st;
    T.ph[0] = -sp; T.ph[1] = cp; T.ph[2] = 0.0;
    for (int x = 0; x < 3; ++x) {
        T.m[x] = {h * T.th[x], h * T.ph[x]};
        T.mb[x] = {h * T.th[x], -h * T.ph[x]};
    }
    return T;
}

// The seven independent tetrad components of a real symmetric 4-tensor.
struct Sym2 {
    double tt, tr, rr, mmb;
    cx tm, rm, mm;
};

__device__ __forceinline__ Sym2 decomp2(const double T[4][4], const Tetrad& e) {
    Sym2 c;
    c.tt = T[0][0];
    c.tr = 0.0;
    c.tm = {0.0, 0.0};
    double Sr[3] = {0, 0, 0};
    cx Sm[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int x = 0; x < 3; ++x) {
        c.tr += e.r[x] * T[0][x + 1];
        c.tm = c.tm + T[0][x + 1] * e.m[x];
        for (int y = 0; y < 3; ++y) {
            Sr[x] += T[x + 1][y + 1] * e.r[y];
            Sm[x] = Sm[x] + T[x + 1][y + 1] * e.m[y];
        }
    }
    c.rr = 0.0;
    c.rm = {0, 0};
    c.mm = {0, 0};
    double tt2 = 0.0;
    for (int x = 0; x < 3; ++x) {
        c.rr += e.r[x] * Sr[x];
        c.rm = c.rm + e.r[x] * Sm[x];
        c.mm = c.mm + e.m[x] * Sm[x];
        double Sth = 0.0, Sph = 0.0;
        for (int y = 0; y < 3; ++y) {
            Sth += T[x + 1][y + 1] * e.th[y];
            Sph += T[x + 1][y + 1] * e.ph[y];
        }
        tt2 += e.th[x] * Sth + e.ph[x] * Sph;
    }
    c.mmb = 0.5 * tt2;   // m^i mbar^j T_ij
    return c;
}

// Complex symmetric 4-tensor from the ten components c_{AB}, A, B in
// {t, r, m, mbar}, with the dual vectors t -> t, r -> r, m -> mbar, mbar -> m.
struct Cx10 {
    cx tt, tr, tm, tmb, rr, rm, rmb, mm, mbmb, mmb;
};

__device__ __forceinline__ void recomp_cx(const Cx10& c, const Tetrad& e, cx M[4][4]) {
    M[0][0] = c.tt;
    for (int x = 0; x < 3; ++x) {
        M[0][x + 1] = c.tr * cx{e.r[x], 0} + c.tm * e.mb[x] + c.tmb * e.m[x];
        M[x + 1][0] = M[0][x + 1];
        for (int y = 0; y < 3; ++y) {
            const double thth = e.th[x] * e.th[y] + e.ph[x] * e.ph[y];   // mbar_x m_y + m_x mbar_y
            M[x + 1][y + 1] = (e.r[x] * e.r[y]) * c.rr
                              + c.rm * (e.r[x] * e.mb[y] + e.r[y] * e.mb[x])
                              + c.rmb * (e.r[x] * e.m[y] + e.r[y] * e.m[x])
                              + c.mm * (e.mb[x] * e.mb[y]) + c.mbmb * (e.m[x] * e.m[y]) + thth * c.mmb;
        }
    }
}

__device__ __forceinline__ Cx10 sym2_to_cx10(const Sym2& c) {
    return {{c.tt, 0}, {c.tr, 0}, c.tm, conj(c.tm), {c.rr, 0}, c.rm, conj(c.rm), c.mm, conj(c.mm), {c.mmb, 0}};
}

// Three waves share 64 points: wave 0 decomposes g and Pi (and H_a, Q_a for
// 58 fields), waves 1 and 2 both decompose the three Phi_x tensors and write
// the r-row and the m-row of the rank-3 components respectively (their
// duplicate reads of the 30 Phi fields hit the CU's cache).  Each wave loads
// all of its fields into registers before any arithmetic, so its loads are
// in flight together.  Against one thread per point doing everything this
// triples the waves in flight, which a kernel with one thread per grid point
// lacks at the metric's size (measured: FP64 decompose 15.7 -> 14.6 us at
// 33x32x64, 0.87 -> 0.75 ms at 8 x 65x64x128; the same split of k_recompose,
// four waves each recomputing the rank-3 recombination, measured slower).
constexpr int kDecParts = 3;

// With uref the columns of u - uref are formed (in FP64, rounded once to TO).
template <typename TO, bool REF>
__global__ __launch_bounds__(64 * kDecParts) void k_decompose(KShell s, const double* __restrict__ u_,
                                                             const double* __restrict__ uref, TO* __restrict__ t) {
    const long long np = s.npts;
    const long long so = (long long)blockIdx.y * s.n_v * np;   // shell of a run
    const double* u0 = u_ + so;
    const double* ur = REF ? uref + so : nullptr;
    t += so;
    const int part = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const long long p = (long long)blockIdx.x * 64 + (threadIdx.x & 63);
    if (p >= np) return;
    const int i = (int)((p / s.n_r) % s.n_th);
    const int j = (int)(p / ((long long)s.n_r * s.n_th));
    auto put = [&](int c, double v) { t[(long long)c * np + p] = (TO)v; };
    auto putc = [&](int c, cx v) { put(c, v.re); put(c + 1, v.im); };
    if (part == 0) {
        double uv[20];
#pragma unroll
        for (int f = 0; f < 20; ++f) uv[f] = u0[(long long)f * np + p];
        double hq[8];
        if (s.n_v == 58) {
#pragma unroll
            for (int f = 0; f < 8; ++f) hq[f] = u0[(long long)(50 + f) * np + p];
        }
        if constexpr (REF) {
            double rv[20];
#pragma unroll
            for (int f = 0; f < 20; ++f) rv[f] = ur[(long long)f * np + p];
#pragma unroll
            for (int f = 0; f < 20; ++f) uv[f] -= rv[f];
            if (s.n_v == 58) {
#pragma unroll
                for (int f = 0; f < 8; ++f) hq[f] -= ur[(long long)(50 + f) * np + p];
            }
        }
        const Tetrad e = make_tetrad(s, i, j);
#pragma unroll
        for (int blk = 0; blk < 2; ++blk) {          // g, Pi
            double T[4][4];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = a; b < 4; ++b) T[a][b] = T[b][a] = uv[10 * blk + pr(a, b)];
            const Sym2 c = decomp2(T, e);
            const int o = 10 * blk;
            put(o + 0, c.tt); put(o + 1, c.tr); put(o + 2, c.rr); put(o + 3, c.mmb);
            putc(o + 4, c.tm); putc(o + 6, c.rm); putc(o + 8, c.mm);
        }
        if (s.n_v == 58) {
#pragma unroll
            for (int blk = 0; blk < 2; ++blk) {      // H_a, Q_a
                const int o = 50 + 4 * blk;
                const double v0 = hq[4 * blk];
                double vr = 0.0;
                cx vm{0, 0};
#pragma unroll
                for (int x = 0; x < 3; ++x) {
                    const double vx = hq[4 * blk + 1 + x];
                    vr += e.r[x] * vx;
                    vm = vm + vx * e.m[x];
                }
                put(o, v0); put(o + 1, vr); putc(o + 2, vm);
            }
        }
        return;
    }
    double uv[30];
#pragma unroll
    for (int f = 0; f < 30; ++f) uv[f] = u0[(long long)(20 + f) * np + p];
    if constexpr (REF) {
        double rv[30];
#pragma unroll
        for (int f = 0; f < 30; ++f) rv[f] = ur[(long long)(20 + f) * np + p];
#pragma unroll
        for (int f = 0; f < 30; ++f) uv[f] -= rv[f];
    }
    const Tetrad e = make_tetrad(s, i, j);
    Sym2 d[3];
#pragma unroll
    for (int x = 0; x < 3; ++x) {
        double T[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = a; b < 4; ++b) T[a][b] = T[b][a] = uv[10 * x + pr(a, b)];
        d[x] = decomp2(T, e);
    }
    if (part == 1) {   // r-row: real-tensor components contracted with rhat
        double tt = 0, tr = 0, rr = 0, mmb = 0;
        cx tm{0, 0}, rm{0, 0}, mm{0, 0};
        for (int x = 0; x < 3; ++x) {
            tt += e.r[x] * d[x].tt; tr += e.r[x] * d[x].tr; rr += e.r[x] * d[x].rr; mmb += e.r[x] * d[x].mmb;
            tm = tm + e.r[x] * d[x].tm; rm = rm + e.r[x] * d[x].rm; mm = mm + e.r[x] * d[x].mm;
        }
        put(20, tt); put(21, tr); put(22, rr); put(23, mmb);
        putc(24, tm); putc(26, rm); putc(28, mm);
    } else {           // m-row
        cx tt{0, 0}, tr{0, 0}, tm{0, 0}, tmb{0, 0}, rr{0, 0}, rm{0, 0}, rmb{0, 0}, mm{0, 0}, mmb{0, 0}, mbmb{0, 0};
        for (int x = 0; x < 3; ++x) {
            const cx m = e.m[x];
            tt = tt + d[x].tt * m; tr = tr + d[x].tr * m; rr = rr + d[x].rr * m; mmb = mmb + d[x].mmb * m;
            tm = tm + m * d[x].tm; tmb = tmb + m * conj(d[x].tm);
            rm = rm + m * d[x].rm; rmb = rmb + m * conj(d[x].rm);
            mm = mm + m * d[x].mm; mbmb = mbmb + m * conj(d[x].mm);
        }
        putc(30, tt); putc(32, tr); putc(34, tm); putc(36, tmb); putc(38, rr);
        putc(40, rm); putc(42, rmb); putc(44, mm); putc(46, mmb); putc(48, mbmb);
    }
}

// With base, u = base + (recomposed columns) (base: the filtered reference).
// Each block of fields (g and Pi, then Phi) is recombined into registers
// first; then the block's base values are loaded together and the sums
// stored, so a store does not wait on its own base load one at a time.
template <typename TI>
__global__ __launch_bounds__(256) void k_recompose(KShell s, const TI* __restrict__ t, const double* __restrict__ base,
                                                   double* __restrict__ u_) {
    const long long np = s.npts;
    const long long so = (long long)blockIdx.y * s.n_v * np;   // shell of a run
    t += so;
    double* __restrict__ u = u_ + so;
    const double* __restrict__ bs = base ? base + so : nullptr;
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int i = (int)((p / s.n_r) % s.n_th);
    const int j = (int)(p / ((long long)s.n_r * s.n_th));
    const Tetrad e = make_tetrad(s, i, j);
    auto get = [&](int c) { return (double)t[(long long)c * np + p]; };
    auto getc = [&](int c) { return cx{get(c), get(c + 1)}; };
    // store fields first .. first + n - 1 from vo, adding the base when present
    auto flush = [&](const double* vo, int first, int n) {
        if (bs) {
            double vb[30];
#pragma unroll
            for (int f = 0; f < 30; ++f)
                if (f < n) vb[f] = bs[(long long)(first + f) * np + p];
#pragma unroll
            for (int f = 0; f < 30; ++f)
                if (f < n) u[(long long)(first + f) * np + p] = vb[f] + vo[f];
        } else {
#pragma unroll
            for (int f = 0; f < 30; ++f)
                if (f < n) u[(long long)(first + f) * np + p] = vo[f];
        }
    };
    {
        double vo[20];
#pragma unroll
        for (int blk = 0; blk < 2; ++blk) {
            const int o = 10 * blk;
            Sym2 c;
            c.tt = get(o); c.tr = get(o + 1); c.rr = get(o + 2); c.mmb = get(o + 3);
            c.tm = getc(o + 4); c.rm = getc(o + 6); c.mm = getc(o + 8);
            cx M[4][4];
            recomp_cx(sym2_to_cx10(c), e, M);
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = a; b < 4; ++b) vo[o + pr(a, b)] = M[a][b].re;
        }
        flush(vo, 0, 20);
    }
    {
        double vo[30];
        Sym2 cr;
        cr.tt = get(20); cr.tr = get(21); cr.rr = get(22); cr.mmb = get(23);
        cr.tm = getc(24); cr.rm = getc(26); cr.mm = getc(28);
        cx R[4][4], M[4][4];
        recomp_cx(sym2_to_cx10(cr), e, R);
        Cx10 cm{getc(30), getc(32), getc(34), getc(36), getc(38), getc(40), getc(42), getc(44), getc(48), getc(46)};
        recomp_cx(cm, e, M);
#pragma unroll
        for (int x = 0; x < 3; ++x)
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = a; b < 4; ++b) {
                    // Phi_x = rhat_x R + mbar_x M + m_x conj(M)
                    const cx v = e.mb[x] * M[a][b];
                    vo[10 * x + pr(a, b)] = e.r[x] * R[a][b].re + 2.0 * v.re;
                }
        flush(vo, 20, 30);
    }
    if (s.n_v == 58) {
        double vo[8];
#pragma unroll
        for (int blk = 0; blk < 2; ++blk) {
            const int o = 4 * blk;
            const double v0 = get(50 + o), vr = get(51 + o);
            const cx vm = getc(52 + o);
            vo[o] = v0;
#pragma unroll
            for (int x = 0; x < 3; ++x) vo[o + 1 + x] = vr * e.r[x] + 2.0 * (vm * e.mb[x]).re;
        }
        flush(vo, 50, 8);
    }
}

// theta filter, spec[c][q][i][k] -> spec2 (q = 0: a_0; 2m-1: a_m; 2m: b_m).
// Workgroup (column tile, m, column set, shell of the run): the columns of a
// set are (group, r_k) pairs, one per lane, all real or all complex and all
// filtered with the same F = F^{|n|}_m; wave w of nw forms theta rows w R + r,
// with the rows of F wave-uniform (scalar operands, wave-blocked copy Fb).
//
// With F_+ = F^n_m and F_- = F^{-n}_m = J F^{|n|}_m J (J reverses theta; the
// staggered theta grid is symmetric about the equator), the S/D form of the
// file header is, for a complex group at m > 0,
//   P1 = F_+ (a^x + b^y), M1 = F_- (a^x - b^y):  a^x' = (P1 + M1)/2, b^y' = (P1 - M1)/2
//   P2 = F_- (a^y + b^x), M2 = F_+ (a^y - b^x):  a^y' = (P2 + M2)/2, b^x' = (P2 - M2)/2,
// two passes of two vectors and half the products of S and D.  Real groups
// filter a and b with F; at m = 0 a complex group filters a^x and a^y with F
// (F^n_0 = F^{-n}_0).  J F J v is F applied to v reversed, read back reversed.
template <int R, typename T, int NW>
__global__ __launch_bounds__(64 * NW) void k_ftheta(int n_r, int n_th, int m_keep, int n_cols_state,
                                                const T* __restrict__ spec, T* __restrict__ spec2,
                                                const T* __restrict__ Fb, const FiltGroup* __restrict__ groups,
                                                const FiltSet* __restrict__ sets, int n_sets) {
    extern __shared__ double smd[];   // v0, v1: [n_th][64] in T
    T* sm = reinterpret_cast<T*>(smd);
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
    constexpr int nw = NW;
    constexpr int kFtPer = 64 / NW;   // theta rows one thread stages (N_theta <= 64)
    const long long c = c0 + lane;
    const bool ok = c < (long long)fs.count * n_r;
    const int gi = ok ? (int)(c / n_r) : 0;
    const int k = ok ? (int)(c - (long long)gi * n_r) : 0;
    const FiltGroup G = groups[fs.first + gi];
    const int qa = (m == 0) ? 0 : 2 * m - 1, qb = 2 * m;
    const T* Fw = Fb + ((long long)(fs.mat * (m_keep + 1) + m) * nw + w) * n_th * R;
    T* v0 = sm;
    T* v1 = sm + n_th * 64;
    const bool mix = fs.cplx && m > 0;   // block-uniform
    const bool neg = G.sign < 0;          // F_+ = J F J for a negative spin
    if (pass_sel && !mix) return;
    for (int pass = pass_sel; pass <= pass_sel; ++pass) {
        const T* x0;
        const T* x1 = nullptr;
        bool rev0 = false, rev1 = false;
        if (!fs.cplx) {
            x0 = spec + G.re * col + qa * per_m + k;
            if (m > 0) x1 = spec + G.re * col + qb * per_m + k;
        } else if (m == 0) {
            x0 = spec + G.re * col + k;
            x1 = spec + G.im * col + k;
        } else if (pass == 0) {   // a^x, b^y -> P1 (F_+), M1 (F_-)
            x0 = spec + G.re * col + qa * per_m + k;
            x1 = spec + G.im * col + qb * per_m + k;
            rev0 = neg;
            rev1 = !neg;
        } else {                  // a^y, b^x -> P2 (F_-), M2 (F_+)
            x0 = spec + G.im * col + qa * per_m + k;
            x1 = spec + G.re * col + qb * per_m + k;
            rev0 = !neg;
            rev1 = neg;
        }
        // all loads of this thread's rows first (x0, x1 point into the
        // state for every lane; lanes past the end store zeros)
        T la[kFtPer], lb[kFtPer];
#pragma unroll
        for (int t = 0; t < kFtPer; ++t) {
            const int ip = w + nw * t;
            la[t] = (ip < n_th) ? x0[ip * (long long)n_r] : (T)0;
            lb[t] = (ip < n_th && x1) ? x1[ip * (long long)n_r] : (T)0;
        }
#pragma unroll
        for (int t = 0; t < kFtPer; ++t) {
            const int ip = w + nw * t;
            if (ip < n_th) {
                const T va = ok ? la[t] : (T)0, vb = ok ? lb[t] : (T)0;
                v0[(rev0 ? n_th - 1 - ip : ip) * 64 + lane] = mix ? va + vb : va;
                v1[(rev1 ? n_th - 1 - ip : ip) * 64 + lane] = mix ? va - vb : vb;
            }
        }
        __syncthreads();
        T acc0[R], acc1[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc0[r] = acc1[r] = (T)0;
        #pragma unroll 4   // operator loads run ahead of the FMAs (measured against 1, 2, default)
        for (int ip = 0; ip < n_th; ++ip) {
            const T a = v0[ip * 64 + lane], b = v1[ip * 64 + lane];
            const T* f = Fw + ip * R;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                acc0[r] = fma(f[r], a, acc0[r]);
                acc1[r] = fma(f[r], b, acc1[r]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = w * R + r;
            if (i < n_th) {
                v0[i * 64 + lane] = acc0[r];
                v1[i * 64 + lane] = acc1[r];
            }
        }
        __syncthreads();
        if (!ok) continue;
        for (int i = w; i < n_th; i += nw) {
            const T p0 = v0[(rev0 ? n_th - 1 - i : i) * 64 + lane];
            const T p1 = v1[(rev1 ? n_th - 1 - i : i) * 64 + lane];
            const long long o = (long long)i * n_r + k;
            if (!fs.cplx) {
                spec2[G.re * col + qa * per_m + o] = p0;
                if (m > 0) spec2[G.re * col + qb * per_m + o] = p1;
            } else if (m == 0) {
                spec2[G.re * col + o] = p0;
                spec2[G.im * col + o] = p1;
            } else if (pass == 0) {
                spec2[G.re * col + qa * per_m + o] = (T)0.5 * (p0 + p1);   // a^x'
                spec2[G.im * col + qb * per_m + o] = (T)0.5 * (p0 - p1);   // b^y'
            } else {
                spec2[G.im * col + qa * per_m + o] = (T)0.5 * (p0 + p1);   // a^y'
                spec2[G.re * col + qb * per_m + o] = (T)0.5 * (p0 - p1);   // b^x'
            }
        }
    }
}

}  // namespace

// Scalar filters (no tetrad): the columns are the Cartesian components.
__global__ __launch_bounds__(256) void k_delta_f32(const double* __restrict__ u, const double* __restrict__ uref,
                                                   float* __restrict__ t, long long n) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e < n) t[e] = (float)(u[e] - uref[e]);
}

__global__ __launch_bounds__(256) void k_add_base(const float* __restrict__ t, const double* __restrict__ base,
                                                  double* __restrict__ u, long long n) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e < n) u[e] = base[e] + (double)t[e];
}

hipError_t launch_delta_f32(const double* u, const double* uref, float* t, long long n, hipStream_t st) {
    hipLaunchKernelGGL(k_delta_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, u, uref, t, n);
    return hipGetLastError();
}

hipError_t launch_add_base(const float* t, const double* base, double* u, long long n, hipStream_t st) {
    hipLaunchKernelGGL(k_add_base, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, t, base, u, n);
    return hipGetLastError();
}

hipError_t launch_decompose(const KShell& s, int count, const double* u, double* t, hipStream_t st) {
    const dim3 grid((unsigned)((s.npts + 63) / 64), (unsigned)count);
    hipLaunchKernelGGL((k_decompose<double, false>), grid, dim3(64 * kDecParts), 0, st, s, u, (const double*)nullptr, t);
    return hipGetLastError();
}

hipError_t launch_decompose_delta(const KShell& s, int count, const double* u, const double* uref, float* t,
                                  hipStream_t st) {
    const dim3 grid((unsigned)((s.npts + 63) / 64), (unsigned)count);
    hipLaunchKernelGGL((k_decompose<float, true>), grid, dim3(64 * kDecParts), 0, st, s, u, uref, t);
    return hipGetLastError();
}

hipError_t launch_recompose(const KShell& s, int count, const double* t, double* u, hipStream_t st) {
    const dim3 grid((unsigned)((s.npts + 255) / 256), (unsigned)count);
    hipLaunchKernelGGL(k_recompose<double>, grid, dim3(256), 0, st, s, t, (const double*)nullptr, u);
    return hipGetLastError();
}

hipError_t launch_recompose_base(const KShell& s, int count, const float* t, const double* base, double* u,
                                 hipStream_t st) {
    const dim3 grid((unsigned)((s.npts + 255) / 256), (unsigned)count);
    hipLaunchKernelGGL(k_recompose<float>, grid, dim3(256), 0, st, s, t, base, u);
    return hipGetLastError();
}

template <typename T>
static hipError_t ftheta_t(const KShell& s, int count, const T* spec, T* spec2, const T* Fb, const FiltPlan& fp,
                           int n_cols, int m_keep, hipStream_t st) {
    if (fp.R < 1 || fp.nw * fp.R < s.n_th || s.n_th > 64) return hipErrorInvalidValue;
    const long long cols = (long long)fp.max_groups * s.n_r;
    const dim3 grid((unsigned)((cols + 63) / 64), (unsigned)(2 * (m_keep + 1)), (unsigned)(fp.n_sets * count));
    const size_t shm = sizeof(T) * 2 * size_t(s.n_th) * 64;
#define X(W_, R_)                                                                                               \
    if (fp.nw == W_ && fp.R == R_) {                                                                            \
        hipLaunchKernelGGL((k_ftheta<R_, T, W_>), grid, dim3(64 * W_), shm, st, s.n_r, s.n_th, m_keep, n_cols, \
                           spec, spec2, Fb, fp.groups, fp.sets, fp.n_sets);                                     \
        return hipGetLastError();                                                                               \
    }
    X(4, 1) X(4, 2) X(4, 3) X(4, 4) X(4, 5) X(4, 6) X(4, 7) X(4, 8) X(4, 9) X(4, 10) X(4, 11) X(4, 12) X(4, 13)
    X(4, 14) X(4, 15) X(4, 16)
    X(8, 1) X(8, 2) X(8, 3) X(8, 4) X(8, 5) X(8, 6) X(8, 7) X(8, 8)
    X(16, 1) X(16, 2) X(16, 3) X(16, 4)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_ftheta(const KShell& s, int count, const double* spec, double* spec2, const FiltPlan& fp,
                         int n_cols, int m_keep, hipStream_t st) {
    return ftheta_t<double>(s, count, spec, spec2, fp.Fb, fp, n_cols, m_keep, st);
}

hipError_t launch_ftheta_f32(const KShell& s, int count, const float* spec, float* spec2, const FiltPlan& fp,
                             int n_cols, int m_keep, hipStream_t st) {
    return ftheta_t<float>(s, count, spec, spec2, fp.Fb_f, fp, n_cols, m_keep, st);
}

}  // namespace sg
