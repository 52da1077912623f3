// Host-side construction of the operator matrices (run once per grid).
//
// Collocation points (Sec. 2.1), differentiation matrices (Sec. 2.3), real
// Fourier analysis/synthesis matrices (Sec. 3.1) and the spin-weighted
// projection-filter matrices F^n_m = P^n_m diag(f) (P^n_m)^+ (Sec. 3.2, 3.3,
// 3.5 eq. FasPfQ).  The spin-n Legendre functions come from the two-term
// recursion in n of Sec. 3.3 (eqs. Yninc, Yncoeffs) started from normalized
// associated Legendre functions; the pseudo-inverse of the full-column-rank
// synthesis matrix is taken through a Householder QR factorisation.
#include "host_math.h"

#include <cmath>
#include <vector>

namespace sg {

static const double kPi = 3.14159265358979323846;
static const long double kPiL = 3.141592653589793238462643383279502884L;

std::vector<double> radial_points(int n_r, double r_min, double r_max) {
    std::vector<double> r(n_r);
    for (int k = 0; k < n_r; ++k)
        r[k] = 0.5 * (r_max + r_min) - 0.5 * (r_max - r_min) * std::cos(kPi * k / (n_r - 1));
    return r;
}

std::vector<double> theta_points(int n_th) {
    std::vector<double> t(n_th);
    for (int i = 0; i < n_th; ++i) t[i] = kPi * (i + 0.5) / n_th;
    return t;
}

std::vector<double> phi_points(int n_ph) {
    std::vector<double> p(n_ph);
    for (int j = 0; j < n_ph; ++j) p[j] = 2.0 * kPi * j / n_ph;
    return p;
}

// Chebyshev extrema-grid matrix with the negative-sum diagonal (eq. CDhat),
// rescaled by 2/(r_max - r_min); row-major n x n.
std::vector<double> cheb_matrix(int n, double r_min, double r_max) {
    std::vector<double> x(n), c(n, 1.0), D(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i) x[i] = -std::cos(kPi * i / (n - 1));
    c[0] = c[n - 1] = 2.0;
    for (int i = 0; i < n; ++i) {
        double rowsum = 0.0;
        for (int j = 0; j < n; ++j) {
            if (i == j) continue;
            double sgn = ((i + j) & 1) ? -1.0 : 1.0;
            double v = (c[i] / c[j]) * sgn / (x[i] - x[j]);
            D[size_t(i) * n + j] = v;
            rowsum += v;
        }
        D[size_t(i) * n + i] = -rowsum;
    }
    const double s = 2.0 / (r_max - r_min);
    for (auto& v : D) v *= s;
    return D;
}

// First column fd[d] = FD[d][0] of the periodic Fourier differentiation
// matrix for n (even) points: FD[i][j] = fd[(i - j) mod n] with
// fd[d] = (-1)^d / (2 tan(pi d / n)), fd[0] = 0 (Sec. 2.3).
std::vector<double> fourier_column(int n) {
    std::vector<double> fd(n, 0.0);
    for (int d = 1; d < n; ++d) {
        double sgn = (d & 1) ? -1.0 : 1.0;
        fd[d] = sgn / (2.0 * std::tan(kPi * d / n));
    }
    return fd;
}

// Folded theta matrix (N x 2N): columns 0..N-1 act on f(theta_i', phi_j),
// columns N..2N-1 on f(theta_i', phi_j + pi); the second half-circle of the
// double cover holds f(theta_{N-1-i'}, phi_j + pi) (Sec. 2.1).
std::vector<double> theta_half_matrix(int n_th) {
    const int n2 = 2 * n_th;
    std::vector<double> fd = fourier_column(n2);
    std::vector<double> H(size_t(n_th) * n2);
    for (int i = 0; i < n_th; ++i)
        for (int ip = 0; ip < n_th; ++ip) {
            H[size_t(i) * n2 + ip] = fd[((i - ip) % n2 + n2) % n2];
            const int circ = n2 - 1 - ip;  // circle index of f(theta_ip, phi + pi)
            H[size_t(i) * n2 + n_th + ip] = fd[((i - circ) % n2 + n2) % n2];
        }
    return H;
}

// Orthonormal associated Legendre functions with the Condon-Shortley phase,
// Phat^m_l(cos theta) for 0 <= m <= l <= L, stored at [l][m]:
// Phat^0_0 = 1/sqrt(4 pi), Phat^m_m = -sqrt((2m+1)/(2m)) sin(theta) Phat^{m-1}_{m-1},
// Phat^m_{m+1} = sqrt(2m+3) cos(theta) Phat^m_m,
// Phat^m_l = a (cos(theta) Phat^m_{l-1} - b Phat^m_{l-2}),
// a = sqrt((4l^2-1)/(l^2-m^2)), b = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)).
// Evaluated in extended precision (x87 long double): the recursion in n
// below divides by sin(theta) and cancels near the poles, which costs about
// four decimal digits for |n| = 3 at the first staggered angle.
typedef long double xf;
static std::vector<xf> legendre_table(int L, xf theta) {
    const xf x = std::cos(theta), s = std::sin(theta);
    std::vector<xf> P(size_t(L + 1) * (L + 1), 0.0L);
    auto at = [&](int l, int m) -> xf& { return P[size_t(l) * (L + 1) + m]; };
    at(0, 0) = 1.0L / std::sqrt(4.0L * (xf)kPiL);
    for (int m = 1; m <= L; ++m) at(m, m) = -std::sqrt((2.0L * m + 1.0L) / (2.0L * m)) * s * at(m - 1, m - 1);
    for (int m = 0; m < L; ++m) at(m + 1, m) = std::sqrt(2.0L * m + 3.0L) * x * at(m, m);
    for (int m = 0; m <= L; ++m)
        for (int l = m + 2; l <= L; ++l) {
            const xf a = std::sqrt((4.0L * l * l - 1.0L) / ((xf)l * l - (xf)m * m));
            const xf b = std::sqrt(((l - 1.0L) * (l - 1.0L) - (xf)m * m) / (4.0L * (l - 1.0L) * (l - 1.0L) - 1.0L));
            at(l, m) = a * (x * at(l - 1, m) - b * at(l - 2, m));
        }
    return P;
}

// Spin-weighted associated Legendre functions Phat^n_{lm}(theta) for
// n = 0..3, -L <= m <= L, 0 <= l <= L, at one angle: spin 0 from the table
// above (Phat^0_{l,-m} = (-1)^m Phat^0_{lm}); spin n from spin n-1 by
// eq. Yninc: Y^n_lm = alpha_nl (m/l - cos)/sin Y^{n-1}_lm + beta_nlm / sin Y^{n-1}_{l-1,m},
// alpha_nl = sqrt((l-n+1)/(l+n)),
// beta_nlm = sqrt((2l+1)/(2l-1) (l+n-1)(l^2-m^2)/(l+n)) / l.
// Result indexed [n][l][m + L].
static std::vector<xf> spin_table(int L, xf theta) {
    const int W = 2 * L + 1;
    auto idx = [&](int n, int l, int m) { return (size_t(n) * (L + 1) + l) * W + (m + L); };
    std::vector<xf> Y(size_t(4) * (L + 1) * W, 0.0L);
    std::vector<xf> P = legendre_table(L, theta);
    for (int l = 0; l <= L; ++l)
        for (int m = 0; m <= l; ++m) {
            const xf v = P[size_t(l) * (L + 1) + m];
            Y[idx(0, l, m)] = v;
            Y[idx(0, l, -m)] = (m & 1) ? -v : v;
        }
    const xf c = std::cos(theta), s = std::sin(theta);
    for (int n = 1; n <= 3; ++n)
        for (int l = n; l <= L; ++l)
            for (int m = -l; m <= l; ++m) {
                const xf al = std::sqrt((l - n + 1.0L) / (l + n));
                const xf be = std::sqrt((2.0L * l + 1.0L) / (2.0L * l - 1.0L) * (l + n - 1.0L) *
                                        ((xf)l * l - (xf)m * m) / (l + n)) / l;
                xf v = al * ((xf)m / l - c) / s * Y[idx(n - 1, l, m)];
                if (l - 1 >= std::abs(m) && l - 1 >= n - 1) v += be / s * Y[idx(n - 1, l - 1, m)];
                Y[idx(n, l, m)] = v;
            }
    return Y;
}

// Spin-n synthesis matrix columns l = max(|m|,|n|)..L at the staggered
// angles, N x K row-major; negative n by Phat^{-n}_{lm} = (-1)^{n+m} Phat^n_{l,-m}.
std::vector<double> spin_synthesis(int n, int m, int n_th, int& K) {
    const int L = n_th - 1;
    const int l0 = std::max(std::abs(m), std::abs(n));
    K = std::max(0, L - l0 + 1);
    std::vector<double> P(size_t(n_th) * std::max(K, 1), 0.0);
    if (K == 0) return P;
    const int an = std::abs(n);
    const int mm = (n < 0) ? -m : m;
    const double sgn = (n < 0 && ((an + std::abs(m)) & 1)) ? -1.0 : 1.0;
    const int W = 2 * L + 1;
    for (int i = 0; i < n_th; ++i) {
        std::vector<xf> Y = spin_table(L, kPiL * ((xf)i + 0.5L) / n_th);
        for (int c = 0; c < K; ++c) {
            const int l = l0 + c;
            P[size_t(i) * K + c] = (double)(sgn * Y[(size_t(an) * (L + 1) + l) * W + (mm + L)]);
        }
    }
    return P;
}

// F = P diag(f) P^+, f_l = 1 for l <= L - n_f.  P (N x K, K <= N, full column
// rank) = Q R by Householder reflections; P^+ = R^-1 Q^T.
std::vector<double> filter_matrix(int n, int m, int n_th, int n_f) {
    const int N = n_th, L = n_th - 1;
    std::vector<double> F(size_t(N) * N, 0.0);
    int K = 0;
    std::vector<double> P = spin_synthesis(n, m, n_th, K);
    if (K == 0) return F;
    const int l0 = std::max(std::abs(m), std::abs(n));
    // Householder QR of a copy; reflectors stored in A below the diagonal.
    std::vector<double> A = P;
    std::vector<double> R(size_t(K) * K, 0.0), vbeta(K);
    std::vector<std::vector<double>> V(K);
    for (int c = 0; c < K; ++c) {
        double nrm = 0.0;
        for (int i = c; i < N; ++i) nrm += A[size_t(i) * K + c] * A[size_t(i) * K + c];
        nrm = std::sqrt(nrm);
        const double a0 = A[size_t(c) * K + c];
        const double alpha = (a0 > 0) ? -nrm : nrm;
        std::vector<double> v(N - c);
        for (int i = c; i < N; ++i) v[i - c] = A[size_t(i) * K + c];
        v[0] -= alpha;
        double vv = 0.0;
        for (double t : v) vv += t * t;
        V[c] = v;
        vbeta[c] = (vv > 0) ? 2.0 / vv : 0.0;
        for (int cc = c; cc < K; ++cc) {
            double d = 0.0;
            for (int i = c; i < N; ++i) d += v[i - c] * A[size_t(i) * K + cc];
            d *= vbeta[c];
            for (int i = c; i < N; ++i) A[size_t(i) * K + cc] -= d * v[i - c];
        }
    }
    for (int r = 0; r < K; ++r)
        for (int c = r; c < K; ++c) R[size_t(r) * K + c] = A[size_t(r) * K + c];
    // Q^T (K x N): apply the reflectors to the identity, keep the first K rows.
    std::vector<double> QT(size_t(N) * N, 0.0);
    for (int i = 0; i < N; ++i) QT[size_t(i) * N + i] = 1.0;
    for (int c = 0; c < K; ++c)
        for (int col = 0; col < N; ++col) {
            double d = 0.0;
            for (int i = c; i < N; ++i) d += V[c][i - c] * QT[size_t(i) * N + col];
            d *= vbeta[c];
            for (int i = c; i < N; ++i) QT[size_t(i) * N + col] -= d * V[c][i - c];
        }
    // X = R^-1 (Q^T)[0:K, :] by back substitution.
    std::vector<double> X(size_t(K) * N, 0.0);
    for (int col = 0; col < N; ++col)
        for (int r = K - 1; r >= 0; --r) {
            double s = QT[size_t(r) * N + col];
            for (int c = r + 1; c < K; ++c) s -= R[size_t(r) * K + c] * X[size_t(c) * N + col];
            X[size_t(r) * N + col] = s / R[size_t(r) * K + r];
        }
    for (int i = 0; i < N; ++i)
        for (int col = 0; col < N; ++col) {
            double s = 0.0;
            for (int c = 0; c < K; ++c)
                if (l0 + c <= L - n_f) s += P[size_t(i) * K + c] * X[size_t(c) * N + col];
            F[size_t(i) * N + col] = s;
        }
    return F;
}

}  // namespace sg
