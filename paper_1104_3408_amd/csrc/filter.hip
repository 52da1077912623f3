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

__global__ __launch_bounds__(256) void k_decompose(KShell s, const double* __restrict__ u, double* __restrict__ t) {
    const long long np = s.npts;
    u += (long long)blockIdx.y * s.n_v * np;   // shell of a run
    t += (long long)blockIdx.y * s.n_v * np;
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int i = (int)((p / s.n_r) % s.n_th);
    const int j = (int)(p / ((long long)s.n_r * s.n_th));
    const Tetrad e = make_tetrad(s, i, j);
    auto put = [&](int c, double v) { t[(long long)c * np + p] = v; };
    auto putc = [&](int c, cx v) { put(c, v.re); put(c + 1, v.im); };
    for (int blk = 0; blk < 2; ++blk) {          // g, Pi
        double T[4][4];
        for (int a = 0; a < 4; ++a)
            for (int b = a; b < 4; ++b) T[a][b] = T[b][a] = u[(long long)(10 * blk + pr(a, b)) * np + p];
        const Sym2 c = decomp2(T, e);
        const int o = 10 * blk;
        put(o + 0, c.tt); put(o + 1, c.tr); put(o + 2, c.rr); put(o + 3, c.mmb);
        putc(o + 4, c.tm); putc(o + 6, c.rm); putc(o + 8, c.mm);
    }
    Sym2 d[3];
    for (int x = 0; x < 3; ++x) {
        double T[4][4];
        for (int a = 0; a < 4; ++a)
            for (int b = a; b < 4; ++b) T[a][b] = T[b][a] = u[(long long)(20 + 10 * x + pr(a, b)) * np + p];
        d[x] = decomp2(T, e);
    }
    // r-row: real-tensor components contracted with rhat
    {
        double tt = 0, tr = 0, rr = 0, mmb = 0;
        cx tm{0, 0}, rm{0, 0}, mm{0, 0};
        for (int x = 0; x < 3; ++x) {
            tt += e.r[x] * d[x].tt; tr += e.r[x] * d[x].tr; rr += e.r[x] * d[x].rr; mmb += e.r[x] * d[x].mmb;
            tm = tm + e.r[x] * d[x].tm; rm = rm + e.r[x] * d[x].rm; mm = mm + e.r[x] * d[x].mm;
        }
        put(20, tt); put(21, tr); put(22, rr); put(23, mmb);
        putc(24, tm); putc(26, rm); putc(28, mm);
    }
    // m-row
    {
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
    if (s.n_v == 58) {
        for (int blk = 0; blk < 2; ++blk) {      // H_a, Q_a
            const int o = 50 + 4 * blk;
            const double v0 = u[(long long)o * np + p];
            double vr = 0.0;
            cx vm{0, 0};
            for (int x = 0; x < 3; ++x) {
                const double vx = u[(long long)(o + 1 + x) * np + p];
                vr += e.r[x] * vx;
                vm = vm + vx * e.m[x];
            }
            put(o, v0); put(o + 1, vr); putc(o + 2, vm);
        }
    }
}

__global__ __launch_bounds__(256) void k_recompose(KShell s, const double* __restrict__ t, double* __restrict__ u) {
    const long long np = s.npts;
    u += (long long)blockIdx.y * s.n_v * np;   // shell of a run
    t += (long long)blockIdx.y * s.n_v * np;
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int i = (int)((p / s.n_r) % s.n_th);
    const int j = (int)(p / ((long long)s.n_r * s.n_th));
    const Tetrad e = make_tetrad(s, i, j);
    auto get = [&](int c) { return t[(long long)c * np + p]; };
    auto getc = [&](int c) { return cx{get(c), get(c + 1)}; };
    for (int blk = 0; blk < 2; ++blk) {
        const int o = 10 * blk;
        Sym2 c;
        c.tt = get(o); c.tr = get(o + 1); c.rr = get(o + 2); c.mmb = get(o + 3);
        c.tm = getc(o + 4); c.rm = getc(o + 6); c.mm = getc(o + 8);
        cx M[4][4];
        recomp_cx(sym2_to_cx10(c), e, M);
        for (int a = 0; a < 4; ++a)
            for (int b = a; b < 4; ++b) u[(long long)(o + pr(a, b)) * np + p] = M[a][b].re;
    }
    Sym2 cr;
    cr.tt = get(20); cr.tr = get(21); cr.rr = get(22); cr.mmb = get(23);
    cr.tm = getc(24); cr.rm = getc(26); cr.mm = getc(28);
    cx R[4][4], M[4][4];
    recomp_cx(sym2_to_cx10(cr), e, R);
    Cx10 cm{getc(30), getc(32), getc(34), getc(36), getc(38), getc(40), getc(42), getc(44), getc(48), getc(46)};
    recomp_cx(cm, e, M);
    for (int x = 0; x < 3; ++x)
        for (int a = 0; a < 4; ++a)
            for (int b = a; b < 4; ++b) {
                // Phi_x = rhat_x R + mbar_x M + m_x conj(M)
                const cx v = e.mb[x] * M[a][b];
                u[(long long)(20 + 10 * x + pr(a, b)) * np + p] = e.r[x] * R[a][b].re + 2.0 * v.re;
            }
    if (s.n_v == 58) {
        for (int blk = 0; blk < 2; ++blk) {
            const int o = 50 + 4 * blk;
            const double v0 = get(o), vr = get(o + 1);
            const cx vm = getc(o + 2);
            u[(long long)o * np + p] = v0;
            for (int x = 0; x < 3; ++x) u[(long long)(o + 1 + x) * np + p] = vr * e.r[x] + 2.0 * (vm * e.mb[x]).re;
        }
    }
}

// spec[c][q][i][k] -> spec2, q = 0 (a_0), 2m-1 (a_m), 2m (b_m).
// Thread per (group, m, i, k), k fastest.
__global__ __launch_bounds__(256) void k_ftheta(int n_r, int n_th, int m_keep, int n_groups, int n_cols,
                                                const double* __restrict__ spec, double* __restrict__ spec2,
                                                const double* __restrict__ fmat,
                                                const FiltGroup* __restrict__ groups) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long per_m = (long long)n_th * n_r;
    {   // shell of a run
        const long long so = (long long)blockIdx.y * n_cols * (2 * m_keep + 1) * per_m;
        spec += so;
        spec2 += so;
    }
    const long long total = per_m * (m_keep + 1) * n_groups;
    if (e >= total) return;
    const int k = (int)(e % n_r);
    const int i = (int)((e / n_r) % n_th);
    const int m = (int)((e / per_m) % (m_keep + 1));
    const int gi = (int)(e / (per_m * (m_keep + 1)));
    const FiltGroup G = groups[gi];
    const int K = 2 * m_keep + 1;
    const long long NN = (long long)n_th * n_th;
    const double* S = fmat + ((long long)(G.set * (m_keep + 1) + m) * 2) * NN + (long long)i * n_th;
    const double* D = S + NN;
    const long long col = (long long)K * per_m;   // one storage column
    const int qa = (m == 0) ? 0 : 2 * m - 1, qb = 2 * m;
    const double* ax = spec + G.re * col + qa * per_m + k;
    const double* bx = spec + G.re * col + qb * per_m + k;
    double* oax = spec2 + G.re * col + qa * per_m + i * (long long)n_r + k;
    double* obx = spec2 + G.re * col + qb * per_m + i * (long long)n_r + k;
    if (G.im < 0) {
        double sa = 0.0, sb = 0.0;
        for (int ip = 0; ip < n_th; ++ip) {
            sa = fma(S[ip], ax[ip * n_r], sa);
            if (m > 0) sb = fma(S[ip], bx[ip * n_r], sb);
        }
        *oax = sa;
        if (m > 0) *obx = sb;
        return;
    }
    const double* ay = spec + G.im * col + qa * per_m + k;
    const double* by = spec + G.im * col + qb * per_m + k;
    double* oay = spec2 + G.im * col + qa * per_m + i * (long long)n_r + k;
    double* oby = spec2 + G.im * col + qb * per_m + i * (long long)n_r + k;
    const double sg = (double)G.sign;
    if (m == 0) {
        double sx = 0.0, sy = 0.0;
        for (int ip = 0; ip < n_th; ++ip) {
            sx = fma(S[ip], ax[ip * n_r], sx);
            sy = fma(S[ip], ay[ip * n_r], sy);
        }
        *oax = sx;
        *oay = sy;
        return;
    }
    double rax = 0, ray = 0, rbx = 0, rby = 0;
    for (int ip = 0; ip < n_th; ++ip) {
        const double s_ = S[ip], d_ = sg * D[ip];
        const double vax = ax[ip * n_r], vay = ay[ip * n_r], vbx = bx[ip * n_r], vby = by[ip * n_r];
        rax += s_ * vax + d_ * vby;
        ray += s_ * vay - d_ * vbx;
        rbx += s_ * vbx - d_ * vay;
        rby += s_ * vby + d_ * vax;
    }
    *oax = rax;
    *oay = ray;
    *obx = rbx;
    *oby = rby;
}

}  // namespace

hipError_t launch_decompose(const KShell& s, int count, const double* u, double* t, hipStream_t st) {
    const dim3 grid((unsigned)((s.npts + 255) / 256), (unsigned)count);
    hipLaunchKernelGGL(k_decompose, grid, dim3(256), 0, st, s, u, t);
    return hipGetLastError();
}

hipError_t launch_recompose(const KShell& s, int count, const double* t, double* u, hipStream_t st) {
    const dim3 grid((unsigned)((s.npts + 255) / 256), (unsigned)count);
    hipLaunchKernelGGL(k_recompose, grid, dim3(256), 0, st, s, t, u);
    return hipGetLastError();
}

hipError_t launch_ftheta(const KShell& s, int count, const double* spec, double* spec2, const double* fmat,
                         const FiltGroup* groups, int n_groups, int n_cols, int m_keep, hipStream_t st) {
    const long long total = (long long)s.n_th * s.n_r * (m_keep + 1) * n_groups;
    const dim3 grid((unsigned)((total + 255) / 256), (unsigned)count);
    hipLaunchKernelGGL(k_ftheta, grid, dim3(256), 0, st, s.n_r, s.n_th, m_keep, n_groups, n_cols, spec, spec2,
                       fmat, groups);
    return hipGetLastError();
}

}  // namespace sg
