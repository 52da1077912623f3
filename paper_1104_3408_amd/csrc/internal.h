// Internal definitions shared by the HIP translation units of libshellspec.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "shellspec.h"

namespace sg {

// Kernel-side view of one shell (passed by value).
struct KShell {
    int n_r, n_th, n_ph, n_v;
    long long npts;           // N_r N_theta N_phi
    const double* Drb;        // Chebyshev D_r, wave-blocked (see block_operator)
    const double* Hsb;        // theta operator in the equator-parity form of dtheta_tile, wave-blocked
    int Dr_R, Hth_R;          // rows per wave of the blocked d_r / d_theta operators
    int Dr_nw, Hth_nw;        // waves per workgroup of k_dr / k_dtheta
    int th_plane;             // FP64 d_theta on whole meridian plane pairs (k_dtheta_plane)
    const float* Hsb_f;       // FP32 copy for the mixed-precision path
    const double* rk;         // radii
    const double* sth; const double* cth;   // sin, cos theta_i
    const double* sph; const double* cph;   // sin, cos phi_j
    const double* H;          // static gauge H_a, [4][npts]
    const double* dH;         // Cartesian d_i H_b, [3][4][npts]
    // nested shells (SG_NESTED): the right-hand side at the outer (inner)
    // sphere, before any boundary treatment, is also stored here,
    // [n_v][N_theta N_phi]; an outer sphere with kraw_out gets no boundary
    // operator (the interface kernel couples it)
    double* kraw_out;
    double* kraw_in;
};

// One group of filter columns: a real column (im < 0) or the real and
// imaginary storage columns of a complex tetrad component.
struct FiltGroup {
    int re, im, set, sign;
};

// Groups [first, first + count) of the sorted group list: all real or all
// complex (cplx) and filtered with matrix set mat.
struct FiltSet {
    int first, count, mat, cplx;
};

// Device view of the theta filter of one shell.
struct FiltPlan {
    const double* Fb;           // [mat][m][wave][N_theta][R], F^{|n|}_m rows wave-blocked
    const float* Fb_f;          // FP32 copy (mixed-precision filter)
    const FiltGroup* groups;
    const FiltSet* sets;
    int n_sets, max_groups, R, nw;   // R rows per wave, nw waves per workgroup
};

// A matrix applied along the phi axis (n_out x n_in), wave-blocked.
struct AxisOp {
    double* Wb = nullptr;
    float* Wb_f = nullptr;          // FP32 copy for the mixed-precision path
    int n_in = 0, n_out = 0, R = 0, passes = 0;
    // circ: W is circulant, W[q][c] = v[(q - c) mod n], and Wb holds the
    // doubled vector dv[t] = v[(t - n) mod n] (zero-padded for padding rows),
    // so the R weights of a wave for input c are dv[n + q0 - c .. + R - 1]
    int circ = 0;
    // par: the real Fourier analysis (1) or synthesis (2) in the parity form
    // of axis_par_tile (derivs.hip), keeping orders m <= m_keep; R and passes
    // then block the row pairs (a_m, b_m), resp. (A_j, B_j), j <= N_phi / 2
    int par = 0, m_keep = 0;
    // mfma: the FP64 circulant d_phi on the matrix cores (k_dphi_mfma; N a
    // multiple of 16, at most 128)
    int mfma = 0;
};

// Largest number of output rows one wave accumulates, and of waves in one
// workgroup of the derivative kernels (4 kMaxWaves rows cover n <= 320).
constexpr int kMaxRows = 20;
constexpr int kMaxWaves = 16, kMinWaves = 8;
constexpr size_t kMaxLdsBytes = 160 * 1024;   // LDS of one workgroup on gfx950

// The 8 XCDs of the chip take the workgroups of a launch round-robin by linear
// id, each with its own L2.  xcd_block(b, n) renumbers the n workgroups so
// that XCD x runs one contiguous range of tiles: neighbouring tiles whose
// HBM rows share cache lines at their edges then meet in the same L2 instead
// of fetching the shared lines once per XCD.  A bijection of [0, n).
constexpr unsigned kXcds = 8;
__device__ __forceinline__ unsigned long long xcd_block(unsigned long long b, unsigned long long n) {
    const unsigned long long x = b % kXcds, per = n / kXcds, rem = n % kXcds;
    return x * per + (x < rem ? x : rem) + b / kXcds;
}

// (x, y, z) of this workgroup in a 3-d grid after xcd_block on its linear id.
struct Blk3 {
    unsigned x, y, z;
};
__device__ __forceinline__ Blk3 xcd_block3() {
    const unsigned long long n = (unsigned long long)gridDim.x * gridDim.y * gridDim.z;
    const unsigned long long L = xcd_block(
        blockIdx.x + (unsigned long long)gridDim.x * (blockIdx.y + (unsigned long long)gridDim.y * blockIdx.z), n);
    const unsigned long long t = L / gridDim.x;
    return Blk3{(unsigned)(L % gridDim.x), (unsigned)(t % gridDim.y), (unsigned)(t / gridDim.y)};
}
// Tile shapes of one shell size: target output rows per wave of the d_r,
// d_theta, d_phi, phi-analysis and phi-synthesis contractions (fewer rows
// means more waves on one staged tile, see blocked_shape) and waves per
// workgroup of the theta filter (4, 8 or 16).  The defaults are the shapes
// measured best on the 33 x 32 x 64 shell; a table written by the project's
// autotuner (paper_1104_3408_amd/tune.py) gives them per (N_r, N_theta,
// n_fields, precision), read by shell_grid_create (tuning.cpp).
struct Tune {
    int dr_rows = 9, th_rows = 4, dph_rows = 8, ana_rows = 8, syn_rows = 8, filt_waves = 8;
    int dph_par = -1;   // d_phi form: 0 circulant window, 1 parity; -1: parity in FP32 modes only
    int th_plane = 0;   // FP64 d_theta tile: 0 64 columns, 1 a meridian plane pair
    int fuse = 1;       // the three derivative contractions as one launch where the shapes allow
    int dph_mfma = 0;   // FP64 circulant d_phi on the matrix cores (N_phi a multiple of 16)
};
// The table entry for this shell size, or the defaults; *source names where
// it came from (the table's path, or "defaults").
Tune lookup_tuning(int n_r, int n_theta, int n_fields, int precision, std::string* source);

// A contraction operator split into two bfloat16 parts (raw bits), W = hi +
// lo, zero-padded to [M][K] (M a multiple of 32, K of 16) for the matrix
// cores (SG_PREC_BF16X3).
struct Bf3Op {
    uint16_t* hi = nullptr;
    uint16_t* lo = nullptr;
    int n_in = 0, n_out = 0, K = 0, M = 0;
};

struct ShellHost {
    sg_shell_desc d;
    size_t off = 0, count = 0, npts = 0;
    double dt = 0;
    int m_keep = 0, K = 0;
    double *Drb = nullptr, *Hsb = nullptr;
    float *Hsb_f = nullptr;
    int Dr_R = 0, Hth_R = 0, Dr_nw = 0, Hth_nw = 0;
    int th_plane = 0;
    AxisOp dph, ana, syn;                    // d_phi, Fourier analysis, Fourier synthesis
    Bf3Op bf_dph, bf_hs, bf_ha;              // split d_phi, H_L + H_R, H_L - H_R (BF16X3 only)
    Bf3Op bf_ana, bf_syn;                    // split phi analysis / synthesis of the filter (BF16X3 only)
    Bf3Op bf_F;                              // split theta filters F^{|n|}_m, [set][m][M][K] (BF16X3 only)
    double *rk = nullptr, *sth = nullptr, *cth = nullptr, *sph = nullptr, *cph = nullptr;
    double *Fb = nullptr;                    // theta filter matrices, FiltPlan layout
    float *Fb_f = nullptr;                   // FP32 copy
    int F_R = 0, F_nw = 0;                   // theta rows per wave and waves per workgroup of Fb
    Tune tune;                               // tile shapes of this shell size
    double *H = nullptr, *dH = nullptr;      // static gauge
    double *kraw_out = nullptr, *kraw_in = nullptr;   // interface right-hand sides (SG_NESTED)
    bool owns_ops = true;                    // false: operators belong to an earlier identical shell
    std::vector<double> r_host, th_host, ph_host;
    KShell view(int n_v) const;
};

// One captured filtered RK4 step (all shells), replayed per step.
// Consecutive shells with identical grids: one launch per kernel covers them.
struct Run {
    int first = 0, count = 0;
};

// A sphere shared by shell a (its outer sphere) and shell a + 1 (its inner).
struct Interface {
    int a = 0;
    double* kraw = nullptr;   // [2][n_v][N_theta N_phi]: raw rhs of shell a, then of shell a + 1
};

// Steps per replay of the longer step graph: consecutive replays of one graph
// leave a gap of several microseconds on the device between the last kernel
// of one replay and the first of the next, which a graph of several steps
// pays once per replay.
constexpr int kGraphSteps = 8;

// Mixed precision: steps between refreshes of the split filter's reference
// state (the FP32 part of the filter rounds relative to the change of the
// state since the last refresh; a refresh costs one FP64 filter).
constexpr int kRefSteps = 64;

struct StepGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const double* u = nullptr;
    std::vector<double> dt;
};

struct Timing {
    bool on = false;
    std::vector<hipEvent_t> ev;   // pairs (start, stop)
    std::vector<int> cls;
    double ms[SG_K_COUNT] = {};
    int cnt[SG_K_COUNT] = {};
};

}  // namespace sg

struct sg_grid {
    sg_options opt{};
    std::vector<sg::ShellHost> sh;
    std::vector<sg::Run> runs;
    double *Hall = nullptr, *dHall = nullptr;   // static gauge of all shells (4, 12 fields per point)
    size_t total = 0;                 // state size in doubles
    int n_sets = 0;
    std::vector<sg::FiltGroup> groups;   // sorted by column set
    sg::FiltGroup* d_groups = nullptr;
    std::vector<sg::FiltSet> fsets;
    sg::FiltSet* d_fsets = nullptr;
    int max_groups = 0;               // largest column set
    int n_cols = 0;                   // filter storage columns (= n_fields)
    bool tetrad = false;              // Yn: decompose on the tetrad
    double *us = nullptr, *acc = nullptr, *dbuf = nullptr;   // RK and derivative workspaces
    double *tcol = nullptr, *spec = nullptr, *spec2 = nullptr;  // filter workspaces
    size_t spec_size = 0, tcol_size = 0;   // doubles in spec (and spec2), in tcol
    int* d_flag = nullptr;
    double* cpart = nullptr;          // constraint-norm partials, 4 per 256 points of the largest shell
    // mixed-precision filter (SG_PREC_FP32): reference state, its FP64 filter,
    // FP32 column and spectral workspaces
    double *uref = nullptr, *furef = nullptr;
    float *tcol32 = nullptr, *spec32 = nullptr, *spec2_32 = nullptr;
    sg::Timing tm;
    hipStream_t cap = nullptr;        // capture stream for the step graph
    hipStream_t side[2] = {nullptr, nullptr};   // forked branches of the captured step
    hipEvent_t fork_ev[3] = {nullptr, nullptr, nullptr};
    sg::StepGraph sgraph;            // one filtered step
    sg::StepGraph sgraph_k;          // kGraphSteps filtered steps
    std::vector<sg::Interface> ifaces;   // nested-shell interfaces (SG_NESTED)
};

namespace sg {
// Record msg as the calling thread's last error (sg_last_error) and return st.
sg_status set_error(sg_status st, const std::string& msg);

// Launchers (stream-ordered; return a HIP error code).
hipError_t launch_dr(const KShell& s, const double* in, double* out, int n_fields, hipStream_t st);
hipError_t launch_dtheta(const KShell& s, const double* in, double* out, int n_fields, hipStream_t st);
// d_r, d_theta, d_phi of n_fields variables in one launch (out: three blocks
// of n_fields npts); hipErrorNotSupported when the blocked shapes of the
// three operators differ in waves per workgroup (nothing is launched then).
hipError_t launch_derivs3(const KShell& s, const AxisOp& dph, const double* in, double* out, int n_fields,
                          hipStream_t st);
hipError_t launch_derivs3_mixed(const KShell& s, const AxisOp& dph, const double* in, double* dr, float* dang,
                                int n_fields, hipStream_t st);
hipError_t launch_dtheta_f32(const KShell& s, const double* in, float* out, int n_fields, hipStream_t st);
hipError_t launch_axis_f32(const AxisOp& op, const double* in, float* out, long long ncol, int n_fields, int center,
                           hipStream_t st);
hipError_t launch_axis(const AxisOp& op, const double* in, double* out, long long ncol, int n_fields, int center,
                       hipStream_t st);
std::vector<double> block_operator(const std::vector<double>& W, int n_out, int n_in, int R, int passes);
// Rows per wave R and 4-wave groups `passes` (nw = 4 passes waves) for an
// operator of n_out rows; -1 if R would exceed kMaxRows.
int blocked_shape(int n_out, int target, int& R, int& passes);
hipError_t launch_bf3_dphi(const KShell& s, const Bf3Op& op, const double* in, float* out, int n_fields,
                           hipStream_t st);
// Theta filter of FP32 spectral columns on the matrix cores (F: the split
// filter matrices of every column set and order m).
hipError_t launch_ftheta_bf3(const KShell& s, int count, const float* spec, float* spec2, const Bf3Op& F,
                             const FiltPlan& fp, int n_cols, int m_keep, hipStream_t st);
// Fourier analysis / synthesis of FP32 columns along phi on the matrix cores
// (dense split operator, n_fields blocks of ncol columns).
hipError_t launch_bf3_axis_ff(const Bf3Op& op, const float* in, float* out, long long ncol, int n_fields,
                              hipStream_t st);
hipError_t launch_bf3_dtheta(const KShell& s, const Bf3Op& hs, const Bf3Op& ha, const double* in, float* out,
                             int n_fields, hipStream_t st);
// d_r (FP64, into dr) and the BF16x3 d_theta, d_phi (FP32, into dang) in one
// launch; hipErrorNotSupported (nothing launched) unless d_r uses kMinWaves.
hipError_t launch_derivs3_bf3(const KShell& s, const Bf3Op& dph, const Bf3Op& hs, const Bf3Op& ha, const double* in,
                              double* dr, float* dang, int n_fields, hipStream_t st);
hipError_t launch_chain(const KShell& s, double* du, int n_fields, hipStream_t st);
// Kernels taking `count` process a run of `count` identical shells stored one
// after the other (shell index in blockIdx.y).
hipError_t launch_rhs(const KShell& s, int count, const double* u, const double* du, bool cart, double* out,
                      const double* ubase, double* acc, double dt, int stage, hipStream_t st);
hipError_t launch_rhs_mixed(const KShell& s, int count, const double* u, const double* dr, const float* dang,
                            double* out, const double* ubase, double* acc, double dt, int stage, hipStream_t st);
hipError_t launch_decompose(const KShell& s, int count, const double* u, double* t, hipStream_t st);
// Mixed-precision filter by reference splitting: columns of u - uref in FP32,
// and u = base + recomposed FP32 columns (base = the FP64-filtered reference).
hipError_t launch_decompose_delta(const KShell& s, int count, const double* u, const double* uref, float* t,
                                  hipStream_t st);
hipError_t launch_recompose_base(const KShell& s, int count, const float* t, const double* base, double* u,
                                 hipStream_t st);
hipError_t launch_delta_f32(const double* u, const double* uref, float* t, long long n, hipStream_t st);
hipError_t launch_add_base(const float* t, const double* base, double* u, long long n, hipStream_t st);
hipError_t launch_ftheta_f32(const KShell& s, int count, const float* spec, float* spec2, const FiltPlan& fp,
                             int n_cols, int m_keep, hipStream_t st);
hipError_t launch_axis_ff(const AxisOp& op, const float* in, float* out, long long ncol, int n_fields,
                          hipStream_t st);
hipError_t launch_recompose(const KShell& s, int count, const double* t, double* u, hipStream_t st);
hipError_t launch_ftheta(const KShell& s, int count, const double* spec, double* spec2, const FiltPlan& fp,
                         int n_cols, int m_keep, hipStream_t st);
hipError_t launch_initial(const KShell& s, const double* g10, const double* dg, double* u,
                          double* H, hipStream_t st);
hipError_t launch_finite_check(const double* u, size_t n, int* flag, hipStream_t st);
// Interface of nested shells a (inside) and b (outside): the common
// right-hand side of the two copies of the shared sphere from the raw ones
// (ka, kb: [n_v][N_theta N_phi]), ua the stage input state of shell a; the
// copies' stage outputs (and RK accumulators, stages 1-3) are corrected by
// the difference to the raw right-hand side with the stage's coefficients
// (stage 0: out is the right-hand side itself).
hipError_t launch_patch(const KShell& a, const KShell& b, const double* ua, const double* ka, const double* kb,
                        double* out_a, double* acc_a, double* out_b, double* acc_b, double dt, int stage,
                        hipStream_t st);
// dg: Cartesian derivatives of the ten g_ab, block x at dg + x * dblk;
// part: ceil(npts/256) * 4 doubles of workspace; norms: 4 doubles.
hipError_t launch_constraints(const KShell& s, const double* u, const double* dg, long long dblk, double* part,
                              double* norms, hipStream_t st);
// norms (4 doubles) from the constraint partials of one shell.
hipError_t launch_constraint_norms(const KShell& s, const double* part, double* norms, hipStream_t st);
}  // namespace sg
