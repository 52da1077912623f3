// Host-side operator construction (see host_math.cpp).
#pragma once
#include <algorithm>
#include <vector>

namespace sg {
std::vector<double> radial_points(int n_r, double r_min, double r_max);
std::vector<double> theta_points(int n_th);
std::vector<double> phi_points(int n_ph);
std::vector<double> cheb_matrix(int n, double r_min, double r_max);
std::vector<double> fourier_column(int n);
std::vector<double> theta_half_matrix(int n_th);
std::vector<double> spin_synthesis(int n, int m, int n_th, int& K);
std::vector<double> filter_matrix(int n, int m, int n_th, int n_f);
}  // namespace sg
