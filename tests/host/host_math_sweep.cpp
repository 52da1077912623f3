// Host-only sweep of the library's operator builders (host_math.cpp) for the
// sanitizer test: every builder over N_r = 4..80 and N_theta from 4 to 64
// (odd and even), spins |n| <= 3, the first, middle and last orders and
// several cutoffs; all values must be finite.
#include "host_math.h"
#include <cmath>
#include <cstdio>
using namespace sg;
int main() {
    double acc = 0;
    for (int n = 4; n <= 80; ++n) {
        for (double v : cheb_matrix(n, 1.8, 11.8)) acc += std::fabs(v);
        for (double v : radial_points(n, 1.8, 11.8)) acc += v;
    }
    for (int nt : {4, 5, 9, 12, 16, 17, 24, 32, 48, 64}) {
        for (double v : theta_points(nt)) acc += v;
        for (double v : phi_points(2 * nt)) acc += v;
        for (double v : fourier_column(2 * nt)) acc += v;
        for (double v : theta_half_matrix(nt)) acc += v;
        const bool big = nt >= 32;
        for (int s = -3; s <= 3; s += big ? 3 : 1)
            for (int m : {0, 1, nt / 2, nt - 5, nt - 1}) {
                if (m < 0 || m >= nt || (big && m != 0 && m != nt - 5)) continue;
                int K = 0;
                for (double v : spin_synthesis(s, m, nt, K)) acc += v;
                for (int nf : {0, 1, 4}) {
                    if (nf >= nt || (big && nf != 4)) continue;
                    auto F = filter_matrix(s, m, nt, nf);
                    for (double v : F) if (!std::isfinite(v)) { std::printf("nonfinite %d %d %d %d\n", s, m, nt, nf); return 1; }
                    for (double v : F) acc += v;
                }
            }
    }
    std::printf("ok %g\n", acc);
    return 0;
}
