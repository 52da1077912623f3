// C-ABI entry points of libshellspec (declared in include/shellspec.h).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "host_math.h"
#include "internal.h"

using namespace sg;

namespace {

thread_local std::string g_err;

sg_status fail(sg_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(SG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
    } while (0)

template <class T>
hipError_t upload(T** dst, const std::vector<T>& v) {
    hipError_t e = hipMalloc((void**)dst, sizeof(T) * std::max<size_t>(v.size(), 1));
    if (e != hipSuccess) return e;
    return hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice);
}

// Spatial-index count d(u^mu) of the Cartesian components (Sec. 3.5), used
// by the graded filter.
int spatial_degree(int mu) {
    static const int d2[10] = {0, 1, 1, 1, 2, 2, 2, 2, 2, 2};
    if (mu < 20) return d2[mu % 10];
    if (mu < 50) return 1 + d2[(mu - 20) % 10];
    return ((mu - 50) % 4 == 0) ? 0 : 1;
}

void build_groups(sg_grid* g) {
    auto& G = g->groups;
    G.clear();
    const int nv = g->opt.n_fields;
    if (g->opt.filter_kind == SG_FILTER_YN) {
        for (int o : {0, 10}) {
            for (int c = 0; c < 4; ++c) G.push_back({o + c, -1, 0, 1});
            G.push_back({o + 4, o + 5, 1, 1});
            G.push_back({o + 6, o + 7, 1, 1});
            G.push_back({o + 8, o + 9, 2, 1});
        }
        for (int c = 20; c < 24; ++c) G.push_back({c, -1, 0, 1});
        G.push_back({24, 25, 1, 1});
        G.push_back({26, 27, 1, 1});
        G.push_back({28, 29, 2, 1});
        // m-row: tt tr tm tmb rr rm rmb mm mmb mbmb
        const int spin[10] = {1, 1, 2, 0, 1, 2, 0, 3, 1, -1};
        for (int t = 0; t < 10; ++t) G.push_back({30 + 2 * t, 31 + 2 * t, std::abs(spin[t]), spin[t] < 0 ? -1 : 1});
        if (nv == 58)
            for (int o : {50, 54}) {
                G.push_back({o, -1, 0, 1});
                G.push_back({o + 1, -1, 0, 1});
                G.push_back({o + 2, o + 3, 1, 1});
            }
    } else {
        const bool graded = g->opt.filter_kind == SG_FILTER_YG;
        for (int mu = 0; mu < nv; ++mu) G.push_back({mu, -1, graded ? spatial_degree(mu) : 0, 1});
    }
    // column sets of the theta filter: one per (matrix set, real/complex)
    std::stable_sort(G.begin(), G.end(), [](const FiltGroup& a, const FiltGroup& b) {
        return a.set != b.set ? a.set < b.set : (a.im >= 0) < (b.im >= 0);
    });
    g->fsets.clear();
    g->max_groups = 0;
    for (size_t i = 0; i < G.size();) {
        size_t j = i;
        while (j < G.size() && G[j].set == G[i].set && (G[j].im >= 0) == (G[i].im >= 0)) ++j;
        g->fsets.push_back({int(i), int(j - i), G[i].set, G[i].im >= 0 ? 1 : 0});
        g->max_groups = std::max(g->max_groups, int(j - i));
        i = j;
    }
}

// n_f of filter matrix set s: Yn sets are spins |n| = s with the global n_f;
// Y has one spin-0 set; Yg sets are spin 0 with n_f - s (Sec. 3.5 eq. nfofmu).
int set_spin(const sg_grid* g, int s) { return g->opt.filter_kind == SG_FILTER_YN ? s : 0; }
int set_nf(const sg_grid* g, int s) { return g->opt.filter_kind == SG_FILTER_YG ? g->opt.n_f - s : g->opt.n_f; }

sg_status check_opts(const sg_shell_desc* shells, int n_shells, const sg_options* opt) {
    if (!shells || n_shells <= 0 || !opt) return fail(SG_EINVAL, "shells/options missing");
    if (opt->n_fields != 50 && opt->n_fields != 58) return fail(SG_EINVAL, "n_fields must be 50 or 58");
    if (opt->filter_kind < 0 || opt->filter_kind > 3) return fail(SG_EINVAL, "unknown filter_kind");
    if (opt->n_f < 0) return fail(SG_EINVAL, "n_f must be >= 0");
    if (opt->precision != SG_PREC_FP64 && opt->precision != SG_PREC_FP32 && opt->precision != SG_PREC_BF16X3)
        return fail(SG_EUNSUPPORTED, "precision must be SG_PREC_FP64, SG_PREC_FP32 or SG_PREC_BF16X3");
    if (!(opt->courant > 0)) return fail(SG_EINVAL, "courant must be > 0");
    for (int s = 0; s < n_shells; ++s) {
        const auto& d = shells[s];
        if (d.n_r < 4 || d.n_r > 80) return fail(SG_ESHAPE, "N_r must be in [4, 80]");
        if (d.n_theta < 4 || d.n_theta > 64) return fail(SG_ESHAPE, "N_theta must be in [4, 64]");
        if (d.n_phi != 2 * d.n_theta) return fail(SG_ESHAPE, "N_phi must equal 2 N_theta");
        if (!(d.r_min > 0 && d.r_max > d.r_min)) return fail(SG_EINVAL, "need 0 < r_min < r_max");
    }
    return SG_OK;
}

void free_shell(ShellHost& s) {
    if (!s.owns_ops) return;   // operators shared with an earlier identical shell
    for (double* p : {s.Drb, s.Hsb, s.dph.Wb, s.ana.Wb, s.syn.Wb, s.rk, s.sth, s.cth, s.sph, s.cph, s.Fb})
        if (p) (void)hipFree(p);
    for (float* p : {s.Hsb_f, s.dph.Wb_f, s.ana.Wb_f, s.syn.Wb_f, s.Fb_f})
        if (p) (void)hipFree(p);
    for (uint16_t* p : {s.bf_dph.hi, s.bf_dph.lo, s.bf_hs.hi, s.bf_hs.lo, s.bf_ha.hi, s.bf_ha.lo, s.bf_ana.hi,
                        s.bf_ana.lo, s.bf_syn.hi, s.bf_syn.lo, s.bf_F.hi, s.bf_F.lo})
        if (p) (void)hipFree(p);
}

// bfloat16 of a float, round to nearest even (raw bits; finite inputs).
static uint16_t bf16_bits(float x) {
    uint32_t b;
    std::memcpy(&b, &x, 4);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}
static float bf16_value(uint16_t h) {
    const uint32_t b = (uint32_t)h << 16;
    float x;
    std::memcpy(&x, &b, 4);
    return x;
}

// W (count matrices of n_out x n_in, row-major, one after the other) split as
// W = hi + lo in bfloat16 and zero-padded to [count][M][K] for the
// matrix-core kernels.
static hipError_t make_bf3(Bf3Op& op, const std::vector<double>& W, int n_out, int n_in, int count = 1) {
    op.n_in = n_in;
    op.n_out = n_out;
    op.K = (n_in + 15) / 16 * 16;
    op.M = (n_out + 31) / 32 * 32;
    const size_t per = size_t(op.M) * op.K;
    std::vector<uint16_t> hi(per * count, 0), lo(per * count, 0);
    for (int t = 0; t < count; ++t)
        for (int q = 0; q < n_out; ++q)
            for (int r = 0; r < n_in; ++r) {
                const float w = (float)W[(size_t(t) * n_out + q) * n_in + r];
                const uint16_t h = bf16_bits(w);
                hi[per * t + size_t(q) * op.K + r] = h;
                lo[per * t + size_t(q) * op.K + r] = bf16_bits(w - bf16_value(h));
            }
    hipError_t e = upload(&op.hi, hi);
    if (e != hipSuccess) return e;
    return upload(&op.lo, lo);
}

struct TimeScope {
    sg_grid* g;
    int cls;
    hipStream_t st;
    hipEvent_t e1 = nullptr;
    TimeScope(sg_grid* g_, int c, hipStream_t s) : g(g_), cls(c), st(s) {
        if (!g->tm.on) return;
        hipEvent_t e0;
        (void)hipEventCreate(&e0);
        (void)hipEventCreate(&e1);
        (void)hipEventRecord(e0, st);
        g->tm.ev.push_back(e0);
    }
    ~TimeScope() {
        if (!g->tm.on) return;
        (void)hipEventRecord(e1, st);
        g->tm.ev.push_back(e1);
        g->tm.cls.push_back(cls);
    }
};

size_t layout_offset(const sg_grid* g, int shell, int nfield) {
    size_t o = 0;
    for (int s = 0; s < shell; ++s) o += g->sh[s].npts * nfield;
    return o;
}

// The three derivative contractions are independent.  They run as one
// launch (launch_derivs3) whenever their blocked shapes agree on the waves
// per workgroup, the tuning table does not ask for separate launches (fuse
// 0) and the timing mode is off; otherwise, with fork (graph capture only),
// d_theta and d_phi run on the two side streams beside d_r and the stream
// waits for both, so the captured graph holds three parallel nodes.
static hipError_t fork_begin(sg_grid* g, hipStream_t st) {
    hipError_t e;
    if ((e = hipEventRecord(g->fork_ev[0], st)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(g->side[0], g->fork_ev[0], 0)) != hipSuccess) return e;
    return hipStreamWaitEvent(g->side[1], g->fork_ev[0], 0);
}

static hipError_t fork_end(sg_grid* g, hipStream_t st) {
    hipError_t e;
    if ((e = hipEventRecord(g->fork_ev[1], g->side[0])) != hipSuccess) return e;
    if ((e = hipEventRecord(g->fork_ev[2], g->side[1])) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(st, g->fork_ev[1], 0)) != hipSuccess) return e;
    return hipStreamWaitEvent(st, g->fork_ev[2], 0);
}

// The three separate contractions; with fork, d_theta and d_phi go to the
// two side streams, and the side streams are joined back to st whatever
// happens after the fork (an error from a launch leaves no side stream
// joined to a capture that the caller then ends).
template <class F1, class F2, class F3>
static hipError_t three_launches(sg_grid* g, hipStream_t st, bool fork, F1 l_dr, F2 l_th, F3 l_ph) {
    hipError_t e;
    if (fork && (e = fork_begin(g, st)) != hipSuccess) return e;
    const hipStream_t s1 = fork ? g->side[0] : st, s2 = fork ? g->side[1] : st;
    {
        TimeScope ts(g, SG_K_DR, st);
        e = l_dr(st);
    }
    if (e == hipSuccess) {
        TimeScope ts(g, SG_K_DTHETA, s1);
        e = l_th(s1);
    }
    if (e == hipSuccess) {
        TimeScope ts(g, SG_K_DPHI, s2);
        e = l_ph(s2);
    }
    if (fork) {
        const hipError_t e2 = fork_end(g, st);
        if (e == hipSuccess) e = e2;
    }
    return e;
}

// Coordinate (or Cartesian) derivatives of n_fields variables of one shell.
hipError_t derivs_shell(sg_grid* g, int s, const double* in, double* out, int nfield, bool cart, hipStream_t st,
                        bool fork = false) {
    const ShellHost& S = g->sh[s];
    const KShell v = S.view(nfield);
    const long long cnt = (long long)S.npts * nfield;
    hipError_t e;
    if (!g->tm.on && S.tune.fuse) {   // one launch for the three (the timing mode keeps them apart)
        e = launch_derivs3(v, S.dph, in, out, nfield, st);
        if (e == hipSuccess) return cart ? launch_chain(v, out, nfield, st) : hipSuccess;
        if (e != hipErrorNotSupported) return e;
    }
    e = three_launches(
        g, st, fork, [&](hipStream_t q) { return launch_dr(v, in, out, nfield, q); },
        [&](hipStream_t q) { return launch_dtheta(v, in, out + cnt, nfield, q); },
        [&](hipStream_t q) {
            return launch_axis(S.dph, in, out + 2 * cnt, (long long)S.d.n_theta * S.d.n_r, nfield, 1, q);
        });
    if (e != hipSuccess) return e;
    return cart ? launch_chain(v, out, nfield, st) : hipSuccess;
}

// Mixed precision: d_r in FP64 into dr; d_theta, d_phi in FP32 into dang
// (two blocks of n_fields * npts floats).
hipError_t derivs_shell_mixed(sg_grid* g, int s, const double* in, double* dr, float* dang, int nfield,
                              hipStream_t st, bool fork = false) {
    const ShellHost& S = g->sh[s];
    const KShell v = S.view(nfield);
    const long long cnt = (long long)S.npts * nfield;
    hipError_t e;
    auto l_dr = [&](hipStream_t q) { return launch_dr(v, in, dr, nfield, q); };
    if (g->opt.precision == SG_PREC_BF16X3) {   // angular contractions on the matrix cores
        if (!g->tm.on && S.tune.fuse) {
            e = launch_derivs3_bf3(v, S.bf_dph, S.bf_hs, S.bf_ha, in, dr, dang, nfield, st);
            if (e != hipErrorNotSupported) return e;
        }
        return three_launches(
            g, st, fork, l_dr, [&](hipStream_t q) { return launch_bf3_dtheta(v, S.bf_hs, S.bf_ha, in, dang, nfield, q); },
            [&](hipStream_t q) { return launch_bf3_dphi(v, S.bf_dph, in, dang + cnt, nfield, q); });
    }
    if (!g->tm.on && S.tune.fuse) {
        e = launch_derivs3_mixed(v, S.dph, in, dr, dang, nfield, st);
        if (e != hipErrorNotSupported) return e;
    }
    return three_launches(
        g, st, fork, l_dr, [&](hipStream_t q) { return launch_dtheta_f32(v, in, dang, nfield, q); },
        [&](hipStream_t q) {
            return launch_axis_f32(S.dph, in, dang + cnt, (long long)S.d.n_theta * S.d.n_r, nfield, 1, q);
        });
}

// Filter of a run of identical shells (state of the run at u).
hipError_t filter_run(sg_grid* g, const Run& R, double* u, hipStream_t st) {
    const ShellHost& S = g->sh[R.first];
    const KShell v = S.view(g->opt.n_fields);
    const long long ncol = (long long)S.d.n_theta * S.d.n_r;
    hipError_t e;
    double* cols = u;
    if (g->tetrad) {
        TimeScope ts(g, SG_K_DECOMP, st);
        if ((e = launch_decompose(v, R.count, u, g->tcol, st)) != hipSuccess) return e;
        cols = g->tcol;
    }
    {
        TimeScope ts(g, SG_K_FANA, st);
        if ((e = launch_axis(S.ana, cols, g->spec, ncol, g->n_cols * R.count, 0, st)) != hipSuccess) return e;
    }
    {
        TimeScope ts(g, SG_K_FTHETA, st);
        const FiltPlan fp{S.Fb, S.Fb_f, g->d_groups, g->d_fsets, (int)g->fsets.size(), g->max_groups, S.F_R, S.F_nw};
        if ((e = launch_ftheta(v, R.count, g->spec, g->spec2, fp, g->n_cols, S.m_keep, st)) != hipSuccess)
            return e;
    }
    {
        TimeScope ts(g, SG_K_FSYN, st);
        if ((e = launch_axis(S.syn, g->spec2, cols, ncol, g->n_cols * R.count, 0, st)) != hipSuccess) return e;
    }
    if (g->tetrad) {
        TimeScope ts(g, SG_K_RECOMP, st);
        return launch_recompose(v, R.count, g->tcol, u, st);
    }
    return hipSuccess;
}

// Mixed-precision filter of a run by reference splitting: the filter is
// linear, so F(u) = F(uref) + F(u - uref) with F(uref) formed in FP64 (furef)
// at the start of every rk_step call and every kRefSteps steps after, and
// F(u - uref) in FP32 (the difference is small, so its FP32 rounding is small
// in absolute terms).
hipError_t filter_run_split(sg_grid* g, const Run& R, double* u, hipStream_t st) {
    const ShellHost& S = g->sh[R.first];
    const KShell v = S.view(g->opt.n_fields);
    const long long ncol = (long long)S.d.n_theta * S.d.n_r;
    float* tcol = g->tcol32;           // workspaces shared by the runs (they run in order)
    float* spec = g->spec32;
    float* spec2 = g->spec2_32;
    const double* uref = g->uref + S.off;
    const double* base = g->furef + S.off;
    hipError_t e;
    const long long n = (long long)S.count * R.count;
    {
        TimeScope ts(g, SG_K_DECOMP, st);
        e = g->tetrad ? launch_decompose_delta(v, R.count, u, uref, tcol, st) : launch_delta_f32(u, uref, tcol, n, st);
        if (e != hipSuccess) return e;
    }
    const bool bf3 = g->opt.precision == SG_PREC_BF16X3;   // phi contractions on the matrix cores
    {
        TimeScope ts(g, SG_K_FANA, st);
        e = bf3 ? launch_bf3_axis_ff(S.bf_ana, tcol, spec, ncol, g->n_cols * R.count, st)
                : launch_axis_ff(S.ana, tcol, spec, ncol, g->n_cols * R.count, st);
        if (e != hipSuccess) return e;
    }
    {
        TimeScope ts(g, SG_K_FTHETA, st);
        const FiltPlan fp{S.Fb, S.Fb_f, g->d_groups, g->d_fsets, (int)g->fsets.size(), g->max_groups, S.F_R, S.F_nw};
        e = bf3 ? launch_ftheta_bf3(v, R.count, spec, spec2, S.bf_F, fp, g->n_cols, S.m_keep, st)
                : launch_ftheta_f32(v, R.count, spec, spec2, fp, g->n_cols, S.m_keep, st);
        if (e != hipSuccess) return e;
    }
    {
        TimeScope ts(g, SG_K_FSYN, st);
        e = bf3 ? launch_bf3_axis_ff(S.bf_syn, spec2, tcol, ncol, g->n_cols * R.count, st)
                : launch_axis_ff(S.syn, spec2, tcol, ncol, g->n_cols * R.count, st);
        if (e != hipSuccess) return e;
    }
    TimeScope ts(g, SG_K_RECOMP, st);
    return g->tetrad ? launch_recompose_base(v, R.count, tcol, base, u, st) : launch_add_base(tcol, base, u, n, st);
}

// Runs of consecutive shells with identical grids (and, for a step, equal dt).
std::vector<Run> make_runs(const sg_grid* g, const double* dts) {
    std::vector<Run> runs;
    for (int s = 0; s < (int)g->sh.size(); ++s) {
        const sg_shell_desc& d = g->sh[s].d;
        bool join = false;
        if (!runs.empty()) {
            const int f = runs.back().first;
            const sg_shell_desc& e = g->sh[f].d;
            // shells at an interface of nested shells run alone (their kernels
            // store the interface's raw right-hand sides)
            join = d.n_r == e.n_r && d.n_theta == e.n_theta && d.n_phi == e.n_phi && d.r_min == e.r_min &&
                   d.r_max == e.r_max && (!dts || dts[s] == dts[f]) && !g->sh[s].kraw_out && !g->sh[s].kraw_in &&
                   !g->sh[f].kraw_out && !g->sh[f].kraw_in;
        }
        if (join)
            runs.back().count++;
        else
            runs.push_back({s, 1});
    }
    return runs;
}

}  // namespace

sg_status sg::set_error(sg_status st, const std::string& msg) { return fail(st, msg); }

KShell ShellHost::view(int n_v) const {
    KShell k;
    k.n_r = d.n_r;
    k.n_th = d.n_theta;
    k.n_ph = d.n_phi;
    k.n_v = n_v;
    k.npts = (long long)npts;
    k.Drb = Drb;
    k.Hsb = Hsb;
    k.Dr_R = Dr_R;
    k.Hth_R = Hth_R;
    k.Dr_nw = Dr_nw;
    k.Hth_nw = Hth_nw;
    k.th_plane = th_plane;
    k.Hsb_f = Hsb_f;
    k.rk = rk;
    k.sth = sth;
    k.cth = cth;
    k.sph = sph;
    k.cph = cph;
    k.H = H;
    k.dH = dH;
    k.kraw_out = kraw_out;
    k.kraw_in = kraw_in;
    return k;
}

extern "C" {

const char* sg_last_error(void) { return g_err.c_str(); }

sg_status shell_grid_create(const sg_shell_desc* shells, int n_shells, const sg_options* opt, const double* gauge_H,
                            sg_grid** out) {
    if (!out) return fail(SG_EINVAL, "out is NULL");
    *out = nullptr;
    sg_status st = check_opts(shells, n_shells, opt);
    if (st != SG_OK) return st;
    if (gauge_H && opt->n_fields == 58) return fail(SG_EINVAL, "gauge_H is only used by the 50-field system");
    sg_grid* g = new sg_grid();
    g->opt = *opt;
    g->tetrad = opt->filter_kind == SG_FILTER_YN;
    g->n_cols = opt->n_fields;
    g->n_sets = opt->filter_kind == SG_FILTER_YN ? 4 : (opt->filter_kind == SG_FILTER_YG ? 4 : 1);
    build_groups(g);
    size_t off = 0, spec = 0;
    auto cleanup = [&](sg_status s, const std::string& m) {
        shell_grid_destroy(g);
        return fail(s, m);
    };
    for (int s = 0; s < n_shells; ++s) {
        ShellHost S;
        S.d = shells[s];
        S.tune = lookup_tuning(S.d.n_r, S.d.n_theta, opt->n_fields, opt->precision, nullptr);
        const int nr = S.d.n_r, nt = S.d.n_theta, np_ = S.d.n_phi, L = nt - 1;
        S.npts = size_t(nr) * nt * np_;
        S.count = S.npts * opt->n_fields;
        S.off = off;
        off += S.count;
        S.r_host = radial_points(nr, S.d.r_min, S.d.r_max);
        S.th_host = theta_points(nt);
        S.ph_host = phi_points(np_);
        const double dr = S.r_host[1] - S.r_host[0];
        const double chord = 2.0 * S.r_host[0] * std::sin(S.th_host[0]) * std::sin(M_PI / np_);
        S.dt = opt->courant * std::min(dr, chord);
        int min_nf = 1 << 20;
        for (int k = 0; k < g->n_sets; ++k) min_nf = std::min(min_nf, set_nf(g, k));
        S.m_keep = std::max(0, std::min(L, L - min_nf));
        S.K = 2 * S.m_keep + 1;
        spec = std::max(spec, size_t(g->n_cols) * S.K * nt * nr);
        // identical shells share their (read-only) device operators
        int twin = -1;
        for (int t = 0; t < s && twin < 0; ++t) {
            const sg_shell_desc& e = g->sh[t].d;
            if (e.n_r == nr && e.n_theta == nt && e.n_phi == np_ && e.r_min == S.d.r_min && e.r_max == S.d.r_max)
                twin = t;
        }
        if (twin >= 0) {
            const ShellHost& T = g->sh[twin];
            S.Drb = T.Drb; S.Hsb = T.Hsb; S.Hsb_f = T.Hsb_f;
            S.Dr_R = T.Dr_R; S.Hth_R = T.Hth_R; S.Dr_nw = T.Dr_nw; S.Hth_nw = T.Hth_nw;
            S.th_plane = T.th_plane;
            S.dph = T.dph; S.ana = T.ana; S.syn = T.syn;
            S.bf_dph = T.bf_dph; S.bf_hs = T.bf_hs; S.bf_ha = T.bf_ha; S.bf_ana = T.bf_ana; S.bf_syn = T.bf_syn; S.bf_F = T.bf_F;
            S.rk = T.rk; S.sth = T.sth; S.cth = T.cth; S.sph = T.sph; S.cph = T.cph;
            S.Fb = T.Fb; S.Fb_f = T.Fb_f; S.F_R = T.F_R; S.F_nw = T.F_nw;
            S.owns_ops = false;
            g->sh.push_back(S);
            continue;
        }
        g->sh.push_back(S);
        ShellHost& H = g->sh.back();
        std::vector<double> sth(nt), cth(nt), sph(np_), cph(np_);
        for (int i = 0; i < nt; ++i) { sth[i] = std::sin(H.th_host[i]); cth[i] = std::cos(H.th_host[i]); }
        for (int j = 0; j < np_; ++j) { sph[j] = std::sin(H.ph_host[j]); cph[j] = std::cos(H.ph_host[j]); }
        const std::vector<double> fd = fourier_column(np_);
        // theta filters F^{|n|}_m, rows blocked over the waves of k_ftheta
        H.F_nw = H.tune.filt_waves;
        H.F_R = (nt + H.F_nw - 1) / H.F_nw;
        const size_t per_mat = size_t(H.F_nw) * nt * H.F_R;
        std::vector<double> fm(size_t(g->n_sets) * (H.m_keep + 1) * per_mat, 0.0);
        const bool bf3 = opt->precision == SG_PREC_BF16X3;
        std::vector<double> fdense(bf3 ? size_t(g->n_sets) * (H.m_keep + 1) * nt * nt : 0);
        for (int k = 0; k < g->n_sets; ++k) {
            const int n = set_spin(g, k), nf = set_nf(g, k);
            for (int m = 0; m <= H.m_keep; ++m) {
                const std::vector<double> F = filter_matrix(n, m, nt, nf);
                if (bf3)
                    std::copy(F.begin(), F.end(), fdense.begin() + (size_t(k) * (H.m_keep + 1) + m) * nt * nt);
                double* Fb = fm.data() + (size_t(k) * (H.m_keep + 1) + m) * per_mat;
                for (int w = 0; w < H.F_nw; ++w)
                    for (int ip = 0; ip < nt; ++ip)
                        for (int r = 0; r < H.F_R; ++r) {
                            const int i = w * H.F_R + r;
                            Fb[(size_t(w) * nt + ip) * H.F_R + r] = i < nt ? F[size_t(i) * nt + ip] : 0.0;
                        }
            }
        }
        std::vector<double> Hth = theta_half_matrix(nt), Hs(size_t(nt) * nt), Ha(size_t(nt) * nt);
        for (int a = 0; a < nt; ++a)
            for (int b = 0; b < nt; ++b) {
                const double hl = Hth[size_t(a) * 2 * nt + b], hr = Hth[size_t(a) * 2 * nt + nt + b];
                Hs[size_t(a) * nt + b] = hl + hr;
                Ha[size_t(a) * nt + b] = hl - hr;
            }
        int passes = 0, passes_th = 0;
        const int hh = (nt + 1) / 2;   // theta rows of the equator-parity form
        if (blocked_shape(nr, H.tune.dr_rows, H.Dr_R, passes) != 0 ||
            blocked_shape(hh, H.tune.th_rows, H.Hth_R, passes_th) != 0)
            return cleanup(SG_ESHAPE, "radial or theta operator too large for one workgroup");
        H.Dr_nw = 4 * passes;
        H.Hth_nw = 4 * passes_th;
        // the plane tile stages two N_theta x N_r planes: within the LDS of one workgroup
        H.th_plane = H.tune.th_plane && opt->precision == SG_PREC_FP64 &&
                     sizeof(double) * (2 * size_t(nt) * nr + size_t(H.Hth_nw) * nr) <= kMaxLdsBytes;
        std::vector<double> Drb = block_operator(cheb_matrix(nr, H.d.r_min, H.d.r_max), nr, nr, H.Dr_R, passes);
        // equator-parity form of Hs and Ha (dtheta_tile): for rows i < hh and
        // inputs i' < hh, Q = (M_ii' + M_i,N-1-i') / 2 and P = (M_ii' - M_i,N-1-i') / 2
        // (the middle input of an odd N_theta: Q = M_ii', P = 0), blocked
        // [wave][i'][Qs (R), Ps (R), Qa (R), Pa (R)]
        std::vector<double> Hsb(size_t(H.Hth_nw) * hh * 4 * H.Hth_R, 0.0);
        for (int w = 0; w < H.Hth_nw; ++w)
            for (int ip = 0; ip < hh; ++ip)
                for (int r = 0; r < H.Hth_R; ++r) {
                    const int i = w * H.Hth_R + r, im = nt - 1 - ip;
                    if (i >= hh) continue;
                    double* blk = Hsb.data() + (size_t(w) * hh + ip) * 4 * H.Hth_R;
                    const double* M2[2] = {Hs.data() + size_t(i) * nt, Ha.data() + size_t(i) * nt};
                    for (int op = 0; op < 2; ++op) {
                        const double q = im == ip ? M2[op][ip] : 0.5 * (M2[op][ip] + M2[op][im]);
                        const double pp = im == ip ? 0.0 : 0.5 * (M2[op][ip] - M2[op][im]);
                        blk[(2 * op) * H.Hth_R + r] = q;
                        blk[(2 * op + 1) * H.Hth_R + r] = pp;
                    }
                }
        auto to_f = [](const std::vector<double>& v) { return std::vector<float>(v.begin(), v.end()); };
        // d_phi in the parity form measured faster in FP32, the circulant
        // window in FP64 (one per shell size: spec_derivs runs FP64 in every mode)
        const bool dph_par = H.tune.dph_par >= 0 ? H.tune.dph_par == 1 : opt->precision == SG_PREC_FP32;
        // the Fourier derivative along phi is circulant: upload the doubled
        // column vector, padded for the rows past n of the last wave (the
        // waves read their rows as a sliding window of it, which stays in the
        // scalar cache)
        auto make_circ = [&](AxisOp& op, const std::vector<double>& col, int n, int rows) {
            op.n_in = n;
            op.n_out = n;
            op.circ = 1;
            op.mfma = H.tune.dph_mfma && n % 16 == 0 && n <= 128;   // FP64 launches on the matrix cores
            if (blocked_shape(n, rows, op.R, op.passes) != 0) return hipErrorInvalidValue;
            std::vector<double> dv(size_t(2 * n + 4 * op.R * op.passes), 0.0);
            for (int t = 0; t < 2 * n; ++t) dv[t] = col[((t - n) % n + n) % n];
            hipError_t e = upload(&op.Wb, dv);
            if (e != hipSuccess) return e;
            return upload(&op.Wb_f, to_f(dv));
        };
        // phi contractions in the parity form of axis_par_tile: real Fourier
        // analysis (kind 1), synthesis (kind 2) and the Fourier derivative
        // (kind 3, FD[q][c] = fd[(q - c) mod N]); rows m (analysis) or
        // j, q <= N/2, blocked [wave][input][C (R), S (R)]; Fourier angles
        // from the integer j m mod N
        auto make_axis_par = [&](AxisOp& op, int kind, int rows_target) {
            const int n = np_, half = n / 2, mk = H.m_keep;
            op.par = kind;
            op.m_keep = kind == 3 ? 0 : mk;
            op.n_in = kind == 2 ? 2 * mk + 1 : n;
            op.n_out = kind == 1 ? 2 * mk + 1 : n;
            const int rows = kind == 1 ? mk + 1 : half + 1, n_loop = kind == 2 ? mk + 1 : half + 1;
            if (blocked_shape(rows, rows_target, op.R, op.passes) != 0) return hipErrorInvalidValue;
            const int nw = 4 * op.passes, R = op.R;
            auto v = [&](int d) { return fd[((d % n) + n) % n]; };
            std::vector<double> Wb(size_t(nw) * n_loop * 2 * R, 0.0);
            for (int w = 0; w < nw; ++w)
                for (int jj = 0; jj < n_loop; ++jj)
                    for (int r = 0; r < R; ++r) {
                        const int q = w * R + r;
                        if (q >= rows) continue;
                        double c, sn;
                        if (kind == 3) {   // e_jj and o_jj weights of row q
                            const bool edge = jj == 0 || jj == half;
                            c = edge ? v(q - jj) : 0.5 * (v(q - jj) + v(q + jj));
                            sn = edge ? 0.0 : 0.5 * (v(q - jj) - v(q + jj));
                        } else {
                            const int j = kind == 1 ? jj : q, m = kind == 1 ? q : jj;
                            const double ang = 2.0 * M_PI * (double)((long long)j * m % n) / n;
                            c = std::cos(ang);
                            sn = (m == 0 || j == 0 || j == half) ? 0.0 : std::sin(ang);
                            if (kind == 1) {   // a_0 = (1/N) sum f, a_m, b_m = (2/N) sum (cos, sin) f
                                c *= (m == 0 ? 1.0 : 2.0) / n;
                                sn *= 2.0 / n;
                            }
                        }
                        double* blk = Wb.data() + (size_t(w) * n_loop + jj) * 2 * R;
                        blk[r] = c;
                        blk[R + r] = sn;
                    }
            hipError_t e = upload(&op.Wb, Wb);
            if (e != hipSuccess) return e;
            return upload(&op.Wb_f, to_f(Wb));
        };
        if (upload(&H.Drb, Drb) != hipSuccess || upload(&H.Hsb, Hsb) != hipSuccess ||
            upload(&H.Hsb_f, to_f(Hsb)) != hipSuccess || (dph_par ? make_axis_par(H.dph, 3, H.tune.dph_rows) : make_circ(H.dph, fd, np_, H.tune.dph_rows)) != hipSuccess ||
            make_axis_par(H.ana, 1, H.tune.ana_rows) != hipSuccess ||
            make_axis_par(H.syn, 2, H.tune.syn_rows) != hipSuccess ||
            upload(&H.rk, H.r_host) != hipSuccess || upload(&H.sth, sth) != hipSuccess ||
            upload(&H.cth, cth) != hipSuccess || upload(&H.sph, sph) != hipSuccess ||
            upload(&H.cph, cph) != hipSuccess || upload(&H.Fb, fm) != hipSuccess ||
            upload(&H.Fb_f, to_f(fm)) != hipSuccess)
            return cleanup(SG_ENOMEM, "device allocation/upload of operator matrices failed");
        if (opt->precision == SG_PREC_BF16X3) {
            std::vector<double> Wph(size_t(np_) * np_);
            for (int q = 0; q < np_; ++q)
                for (int c = 0; c < np_; ++c) Wph[size_t(q) * np_ + c] = fd[((q - c) % np_ + np_) % np_];
            // dense real Fourier analysis (K x N_phi) and synthesis (N_phi x K) of
            // the filter, rows a_0, a_1, b_1, ... (Sec. 3.1)
            std::vector<double> ana(size_t(H.K) * np_), syn(size_t(np_) * H.K);
            for (int j = 0; j < np_; ++j)
                for (int m = 0; m <= H.m_keep; ++m) {
                    const double ang = 2.0 * M_PI * (double)((long long)j * m % np_) / np_;
                    const double c = std::cos(ang), sn = std::sin(ang);
                    if (m == 0) {
                        ana[j] = 1.0 / np_;
                        syn[size_t(j) * H.K] = 1.0;
                        continue;
                    }
                    ana[size_t(2 * m - 1) * np_ + j] = 2.0 * c / np_;
                    ana[size_t(2 * m) * np_ + j] = 2.0 * sn / np_;
                    syn[size_t(j) * H.K + 2 * m - 1] = c;
                    syn[size_t(j) * H.K + 2 * m] = sn;
                }
            if (make_bf3(H.bf_dph, Wph, np_, np_) != hipSuccess || make_bf3(H.bf_hs, Hs, nt, nt) != hipSuccess ||
                make_bf3(H.bf_ha, Ha, nt, nt) != hipSuccess || make_bf3(H.bf_ana, ana, H.K, np_) != hipSuccess ||
                make_bf3(H.bf_syn, syn, np_, H.K) != hipSuccess ||
                make_bf3(H.bf_F, fdense, nt, nt, g->n_sets * (H.m_keep + 1)) != hipSuccess)
                return cleanup(SG_ENOMEM, "upload of the split bfloat16 operators failed");
        }
    }
    g->total = off;
    if (opt->flags & SG_NESTED) {   // shells coupled at shared spheres (reading of Sec. 1 / Sec. 5)
        for (int s = 0; s + 1 < n_shells; ++s) {
            ShellHost &A = g->sh[s], &B = g->sh[s + 1];
            if (A.d.r_max != B.d.r_min) continue;
            if (A.d.n_theta != B.d.n_theta || A.d.n_phi != B.d.n_phi)
                return cleanup(SG_ESHAPE, "nested shells must share the angular grid of their common sphere");
            Interface I;
            I.a = s;
            const size_t n = size_t(opt->n_fields) * A.d.n_theta * A.d.n_phi;
            if (hipMalloc((void**)&I.kraw, sizeof(double) * 2 * n) != hipSuccess)
                return cleanup(SG_ENOMEM, "interface workspace allocation failed");
            g->ifaces.push_back(I);
            A.kraw_out = I.kraw;
            B.kraw_in = I.kraw + n;
        }
        // one time step for every chain of coupled shells: the smallest
        for (size_t c = 0; c < g->sh.size();) {
            size_t e = c;
            double m = g->sh[c].dt;
            while (e + 1 < g->sh.size() && g->sh[e].kraw_out) m = std::min(m, g->sh[++e].dt);
            for (size_t t = c; t <= e; ++t) g->sh[t].dt = m;
            c = e + 1;
        }
    }
    g->runs = make_runs(g, nullptr);
    size_t maxc = 0;
    spec = 0;
    for (const Run& R : g->runs) {
        const ShellHost& S = g->sh[R.first];
        maxc = std::max(maxc, S.count * R.count);
        spec = std::max(spec, size_t(R.count) * g->n_cols * S.K * S.d.n_theta * S.d.n_r);
    }
    g->spec_size = spec;
    g->tcol_size = maxc;
    size_t max_cblocks = 1;
    for (const ShellHost& S : g->sh) max_cblocks = std::max(max_cblocks, (S.npts + 255) / 256);
    if (opt->n_fields == 50) {
        size_t pts = 0;
        for (auto& S : g->sh) pts += S.npts;
        if (hipMalloc((void**)&g->Hall, sizeof(double) * 4 * pts) != hipSuccess ||
            hipMalloc((void**)&g->dHall, sizeof(double) * 12 * pts) != hipSuccess)
            return cleanup(SG_ENOMEM, "gauge allocation failed");
        (void)hipMemset(g->Hall, 0, sizeof(double) * 4 * pts);
        (void)hipMemset(g->dHall, 0, sizeof(double) * 12 * pts);
        size_t po = 0;
        for (auto& S : g->sh) {
            S.H = g->Hall + 4 * po;
            S.dH = g->dHall + 12 * po;
            po += S.npts;
        }
    }
    if (hipMalloc((void**)&g->us, sizeof(double) * 2 * g->total) != hipSuccess ||
        hipMalloc((void**)&g->acc, sizeof(double) * g->total) != hipSuccess ||
        hipMalloc((void**)&g->dbuf, sizeof(double) * 3 * g->total) != hipSuccess ||
        hipMalloc((void**)&g->tcol, sizeof(double) * maxc) != hipSuccess ||
        hipMalloc((void**)&g->spec, sizeof(double) * spec) != hipSuccess ||
        hipMalloc((void**)&g->spec2, sizeof(double) * spec) != hipSuccess ||
        hipMalloc((void**)&g->d_flag, sizeof(int)) != hipSuccess ||
        hipMalloc((void**)&g->cpart, sizeof(double) * 4 * max_cblocks) != hipSuccess)
        return cleanup(SG_ENOMEM, "workspace allocation failed");
    if (upload(&g->d_groups, g->groups) != hipSuccess || upload(&g->d_fsets, g->fsets) != hipSuccess)
        return cleanup(SG_ENOMEM, "group upload failed");
    if (opt->precision != SG_PREC_FP64 && opt->filter_kind != SG_FILTER_NONE) {
        if (hipMalloc((void**)&g->uref, sizeof(double) * g->total) != hipSuccess ||
            hipMalloc((void**)&g->furef, sizeof(double) * g->total) != hipSuccess ||
            hipMalloc((void**)&g->tcol32, sizeof(float) * g->total) != hipSuccess ||
            hipMalloc((void**)&g->spec32, sizeof(float) * spec) != hipSuccess ||
            hipMalloc((void**)&g->spec2_32, sizeof(float) * spec) != hipSuccess)
            return cleanup(SG_ENOMEM, "mixed-precision filter workspace allocation failed");
        if (hipMemset(g->spec2_32, 0, sizeof(float) * spec) != hipSuccess) return cleanup(SG_EHIP, "memset failed");
    }
    if (hipMemset(g->spec2, 0, sizeof(double) * spec) != hipSuccess) return cleanup(SG_EHIP, "memset failed");
    if (gauge_H) {
        sg_status s2 = sg_set_gauge(g, gauge_H, nullptr);
        if (s2 != SG_OK) {
            std::string m = g_err;
            return cleanup(s2, m);
        }
        if (hipDeviceSynchronize() != hipSuccess) return cleanup(SG_EHIP, "gauge setup failed");
    }
    *out = g;
    return SG_OK;
}

static void drop_graph(sg_grid* g);

void shell_grid_destroy(sg_grid* g) {
    if (!g) return;
    drop_graph(g);
    for (auto& I : g->ifaces)
        if (I.kraw) (void)hipFree(I.kraw);
    if (g->cap) (void)hipStreamDestroy(g->cap);
    for (auto sd : g->side)
        if (sd) (void)hipStreamDestroy(sd);
    for (auto ev : g->fork_ev)
        if (ev) (void)hipEventDestroy(ev);
    for (auto& s : g->sh) free_shell(s);
    for (void* p : {(void*)g->us, (void*)g->acc, (void*)g->dbuf, (void*)g->tcol, (void*)g->spec, (void*)g->spec2,
                    (void*)g->d_flag, (void*)g->d_groups, (void*)g->d_fsets, (void*)g->Hall, (void*)g->dHall,
                    (void*)g->cpart, (void*)g->uref, (void*)g->furef, (void*)g->tcol32, (void*)g->spec32,
                    (void*)g->spec2_32})
        if (p) (void)hipFree(p);
    for (auto e : g->tm.ev) (void)hipEventDestroy(e);
    delete g;
}

sg_status shell_grid_info(const sg_grid* g, int shell, size_t* offset, size_t* count, double* dt) {
    if (!g) return fail(SG_EINVAL, "grid is NULL");
    if (shell == -1) {
        double m = 1e300;
        for (auto& s : g->sh) m = std::min(m, s.dt);
        if (offset) *offset = 0;
        if (count) *count = g->total;
        if (dt) *dt = m;
        return SG_OK;
    }
    if (shell < 0 || shell >= (int)g->sh.size()) return fail(SG_EINVAL, "shell index out of range");
    if (offset) *offset = g->sh[shell].off;
    if (count) *count = g->sh[shell].count;
    if (dt) *dt = g->sh[shell].dt;
    return SG_OK;
}

sg_status shell_grid_coords(const sg_grid* g, int shell, double* r, double* theta, double* phi) {
    if (!g) return fail(SG_EINVAL, "grid is NULL");
    if (shell < 0 || shell >= (int)g->sh.size()) return fail(SG_EINVAL, "shell index out of range");
    const ShellHost& S = g->sh[shell];
    if (r) std::memcpy(r, S.r_host.data(), sizeof(double) * S.r_host.size());
    if (theta) std::memcpy(theta, S.th_host.data(), sizeof(double) * S.th_host.size());
    if (phi) std::memcpy(phi, S.ph_host.data(), sizeof(double) * S.ph_host.size());
    return SG_OK;
}

sg_status sg_set_gauge(sg_grid* g, const double* H, sg_stream_t stream) {
    if (!g || !H) return fail(SG_EINVAL, "grid or H is NULL");
    if (g->opt.n_fields != 50) return fail(SG_EINVAL, "the 58-field system evolves its gauge source");
    hipStream_t st = (hipStream_t)stream;
    for (int s = 0; s < (int)g->sh.size(); ++s) {
        ShellHost& S = g->sh[s];
        const double* src = H + layout_offset(g, s, 4);
        HIP_TRY(hipMemcpyAsync(S.H, src, sizeof(double) * 4 * S.npts, hipMemcpyDeviceToDevice, st));
        HIP_TRY(derivs_shell(g, s, S.H, g->dbuf, 4, true, st));
        HIP_TRY(hipMemcpyAsync(S.dH, g->dbuf, sizeof(double) * 12 * S.npts, hipMemcpyDeviceToDevice, st));
    }
    return SG_OK;
}

sg_status spec_derivs(sg_grid* g, const double* u, double* du, int mode, sg_stream_t stream) {
    if (!g || !u || !du) return fail(SG_EINVAL, "NULL argument");
    if (mode != SG_COORD && mode != SG_CART) return fail(SG_EINVAL, "mode must be SG_COORD or SG_CART");
    if ((const double*)du == u) return fail(SG_EINVAL, "du must not alias u");
    hipStream_t st = (hipStream_t)stream;
    for (int s = 0; s < (int)g->sh.size(); ++s) {
        const ShellHost& S = g->sh[s];
        HIP_TRY(derivs_shell(g, s, u + S.off, du + 3 * S.off, g->opt.n_fields, mode == SG_CART, st));
    }
    return SG_OK;
}

sg_status swsh_filter(sg_grid* g, double* u, sg_stream_t stream) {
    if (!g || !u) return fail(SG_EINVAL, "NULL argument");
    if (g->opt.filter_kind == SG_FILTER_NONE) return SG_OK;
    hipStream_t st = (hipStream_t)stream;
    for (const Run& R : g->runs) HIP_TRY(filter_run(g, R, u + g->sh[R.first].off, st));
    return SG_OK;
}

sg_status ghg_constraints(sg_grid* g, const double* u, double* norms, sg_stream_t stream) {
    if (!g || !u || !norms) return fail(SG_EINVAL, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    for (int s = 0; s < (int)g->sh.size(); ++s) {
        const ShellHost& S = g->sh[s];
        const KShell v = S.view(g->opt.n_fields);
        // Cartesian derivatives of the ten g_ab of this shell into the workspace
        HIP_TRY(derivs_shell(g, s, u + S.off, g->dbuf, 10, true, st));
        HIP_TRY(launch_constraints(v, u + S.off, g->dbuf, 10LL * (long long)S.npts, g->cpart, norms + 4 * s, st));
    }
    return SG_OK;
}

static hipError_t patch_interface(sg_grid* g, const Interface& I, double* u, double* out, double dt, int stage,
                                  hipStream_t st);

sg_status ghg_rhs(sg_grid* g, const double* u, const double* du_cart, double* rhs, sg_stream_t stream) {
    if (!g || !u || !rhs) return fail(SG_EINVAL, "NULL argument");
    if ((const double*)rhs == u) return fail(SG_EINVAL, "rhs must not alias u");
    hipStream_t st = (hipStream_t)stream;
    for (int s = 0; s < (int)g->sh.size(); ++s) {
        const ShellHost& S = g->sh[s];
        const KShell v = S.view(g->opt.n_fields);
        const double* d = du_cart ? du_cart + 3 * S.off : g->dbuf;
        if (!du_cart) HIP_TRY(derivs_shell(g, s, u + S.off, g->dbuf, g->opt.n_fields, false, st));
        TimeScope ts(g, SG_K_RHS, st);
        HIP_TRY(launch_rhs(v, 1, u + S.off, d, du_cart != nullptr, rhs + S.off, nullptr, nullptr, 0.0, 0, st));
    }
    for (const Interface& I : g->ifaces) HIP_TRY(patch_interface(g, I, const_cast<double*>(u), rhs, 0.0, 0, st));
    return SG_OK;
}

// Host-side check that a run's slices of the state and of every workspace the
// step uses lie inside the grid's allocations (the run's shells are
// consecutive and identical, so they occupy S.count * R.count doubles).
static bool run_fits(const sg_grid* g, const Run& R) {
    if (R.first < 0 || R.count < 1 || R.first + R.count > (int)g->sh.size()) return false;
    const ShellHost& S = g->sh[R.first];
    const size_t n = S.count * size_t(R.count);
    const size_t spec = size_t(R.count) * g->n_cols * S.K * S.d.n_theta * S.d.n_r;
    return S.off + n <= g->total && n <= g->tcol_size && spec <= g->spec_size;
}

// Stage `stage` (1..4) of one run of shells (Sec. 2.5): stage inputs u -> a ->
// b -> a, the fourth stage writes u.
static hipError_t run_stage(sg_grid* g, const Run& R, double* u, const double* dt, int stage, hipStream_t st,
                            bool fork) {
    const int nv = g->opt.n_fields;
    const ShellHost& S = g->sh[R.first];
    const KShell v = S.view(nv);
    const double h = dt[R.first];
    const int nvr = nv * R.count;                 // variables of the whole run
    double* u0 = u + S.off;
    double* a = g->us + S.off;
    double* b = g->us + g->total + S.off;
    double* ac = g->acc + S.off;
    const double* in[4] = {u0, a, b, a};
    double* outp[4] = {a, b, a, u0};
    hipError_t e;
    if (g->opt.precision != SG_PREC_FP64) {
        float* dang = reinterpret_cast<float*>(g->dbuf + S.count * R.count);
        if ((e = derivs_shell_mixed(g, R.first, in[stage - 1], g->dbuf, dang, nvr, st, fork)) != hipSuccess) return e;
        TimeScope ts(g, SG_K_RHS, st);
        return launch_rhs_mixed(v, R.count, in[stage - 1], g->dbuf, dang, outp[stage - 1], u0, ac, h, stage, st);
    }
    if ((e = derivs_shell(g, R.first, in[stage - 1], g->dbuf, nvr, false, st, fork)) != hipSuccess) return e;
    TimeScope ts(g, SG_K_RHS, st);
    return launch_rhs(v, R.count, in[stage - 1], g->dbuf, false, outp[stage - 1], u0, ac, h, stage, st);
}

// Interface I of nested shells after stage `stage` (1..4) of rk_step on the
// state u: the common right-hand side of the two copies of the shared sphere
// replaces the raw ones in the copies' stage outputs and accumulators.
// Stage 0 (ghg_rhs): u is the state and out the right-hand side array.
static hipError_t patch_interface(sg_grid* g, const Interface& I, double* u, double* out, double dt, int stage,
                                  hipStream_t st) {
    const ShellHost &A = g->sh[I.a], &B = g->sh[I.a + 1];
    const int nv = g->opt.n_fields;
    const size_t n = size_t(nv) * A.d.n_theta * A.d.n_phi;
    const double* in_s = u;
    double* out_s = out;
    if (stage > 0) {   // the stage inputs and outputs of run_stage
        double* a = g->us;
        double* b = g->us + g->total;
        const double* ins[4] = {u, a, b, a};
        double* outs[4] = {a, b, a, u};
        in_s = ins[stage - 1];
        out_s = outs[stage - 1];
    }
    double* acc = (stage >= 1 && stage <= 3) ? g->acc : nullptr;
    return launch_patch(A.view(nv), B.view(nv), in_s + A.off, I.kraw, I.kraw + n, out_s + A.off,
                        acc ? acc + A.off : nullptr, out_s + B.off, acc ? acc + B.off : nullptr, dt, stage, st);
}

// One filtered RK4 step of every shell (Sec. 2.5), then the filter.  Runs go
// one after the other; with nested shells every stage of all runs comes
// before the next stage, with the interfaces coupled after each stage.
static hipError_t step_launches(sg_grid* g, double* u, const double* dt, hipStream_t st, bool fork) {
    hipError_t e;
    const std::vector<Run> runs = make_runs(g, dt);
    for (const Run& R : runs)
        if (!run_fits(g, R)) return hipErrorInvalidValue;
    const bool mixed = g->opt.precision != SG_PREC_FP64;
    auto filt = [&](const Run& R) -> hipError_t {
        if (g->opt.filter_kind == SG_FILTER_NONE) return hipSuccess;
        double* u0 = u + g->sh[R.first].off;
        return mixed ? filter_run_split(g, R, u0, st) : filter_run(g, R, u0, st);
    };
    if (g->ifaces.empty()) {
        for (const Run& R : runs) {
            for (int stage = 1; stage <= 4; ++stage)
                if ((e = run_stage(g, R, u, dt, stage, st, fork)) != hipSuccess) return e;
            if ((e = filt(R)) != hipSuccess) return e;
        }
        return hipSuccess;
    }
    for (int stage = 1; stage <= 4; ++stage) {
        for (const Run& R : runs)
            if ((e = run_stage(g, R, u, dt, stage, st, fork)) != hipSuccess) return e;
        for (const Interface& I : g->ifaces)
            if ((e = patch_interface(g, I, u, nullptr, dt[I.a], stage, st)) != hipSuccess) return e;
    }
    for (const Run& R : runs)
        if ((e = filt(R)) != hipSuccess) return e;
    return hipSuccess;
}

static void drop_graph(StepGraph& sg) {
    if (sg.exec) (void)hipGraphExecDestroy(sg.exec);
    if (sg.graph) (void)hipGraphDestroy(sg.graph);
    sg = StepGraph();
}

static void drop_graph(sg_grid* g) {
    drop_graph(g->sgraph);
    drop_graph(g->sgraph_k);
}

// Capture n_steps filtered steps of the state u into sg (private stream; the
// three derivative contractions as one launch or forked, see derivs_shell).
static sg_status capture_steps(sg_grid* g, StepGraph& sg, int n_steps, double* u, const std::vector<double>& dts) {
    drop_graph(sg);
    if (!g->cap) HIP_TRY(hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking));
    for (auto& sd : g->side)
        if (!sd) HIP_TRY(hipStreamCreateWithFlags(&sd, hipStreamNonBlocking));
    for (auto& ev : g->fork_ev)
        if (!ev) HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIP_TRY(hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int n = 0; n < n_steps && e == hipSuccess; ++n) e = step_launches(g, u, dts.data(), g->cap, true);
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(g->cap, &graph);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(SG_EHIP, std::string("step capture failed: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t e3 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e3 != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return fail(SG_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e3));
    }
    sg.graph = graph;
    sg.exec = exec;
    sg.u = u;
    sg.dt = dts;
    return SG_OK;
}

sg_status rk_step(sg_grid* g, double* u, const double* dt, int n_steps, sg_stream_t stream) {
    if (!g || !u) return fail(SG_EINVAL, "NULL argument");
    if (n_steps < 0) return fail(SG_EINVAL, "n_steps must be >= 0");
    hipStream_t st = (hipStream_t)stream;
    if (g->tm.on) {
        for (auto e : g->tm.ev) (void)hipEventDestroy(e);
        g->tm.ev.clear();
        g->tm.cls.clear();
    }
    std::vector<double> dts(g->sh.size());
    for (size_t s = 0; s < g->sh.size(); ++s) {
        dts[s] = dt ? dt[s] : g->sh[s].dt;
        if (!(dts[s] > 0.0) || !std::isfinite(dts[s])) return fail(SG_EINVAL, "dt must be finite and positive");
    }
    for (const Interface& I : g->ifaces)
        if (dts[I.a] != dts[I.a + 1]) return fail(SG_EINVAL, "nested shells coupled at a sphere need one time step");
    // mixed precision: the split filter's reference u_ref is the state at the
    // start of this call, refreshed every kRefSteps steps (F(u_ref) in FP64),
    // so the FP32 part always rounds relative to the change of the state over
    // at most kRefSteps steps, whatever the caller wrote into u before
    auto refresh_ref = [&]() -> sg_status {
        HIP_TRY(hipMemcpyAsync(g->uref, u, sizeof(double) * g->total, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(g->furef, u, sizeof(double) * g->total, hipMemcpyDeviceToDevice, st));
        for (const Run& R : g->runs) HIP_TRY(filter_run(g, R, g->furef + g->sh[R.first].off, st));
        return SG_OK;
    };
    const bool graph = !g->tm.on && !(g->opt.flags & SG_NO_GRAPH) && n_steps > 0;
    auto stale = [&](const StepGraph& sg) { return !sg.exec || sg.u != u || sg.dt != dts; };
    for (int done = 0; done < n_steps;) {
        int n = n_steps - done;
        if (g->uref) {
            n = std::min(n, kRefSteps);
            sg_status s2 = refresh_ref();
            if (s2 != SG_OK) return s2;
        }
        done += n;
        if (!graph) {
            for (; n > 0; --n) HIP_TRY(step_launches(g, u, dts.data(), st, false));
            continue;
        }
        if (n >= kGraphSteps) {
            if (stale(g->sgraph_k)) {
                sg_status s2 = capture_steps(g, g->sgraph_k, kGraphSteps, u, dts);
                if (s2 != SG_OK) return s2;
            }
            for (; n >= kGraphSteps; n -= kGraphSteps) HIP_TRY(hipGraphLaunch(g->sgraph_k.exec, st));
        }
        if (n > 0) {
            if (stale(g->sgraph)) {
                sg_status s2 = capture_steps(g, g->sgraph, 1, u, dts);
                if (s2 != SG_OK) return s2;
            }
            for (; n > 0; --n) HIP_TRY(hipGraphLaunch(g->sgraph.exec, st));
        }
    }
    if (g->opt.flags & SG_CHECK_FINITE) {
        HIP_TRY(hipMemsetAsync(g->d_flag, 0, sizeof(int), st));
        HIP_TRY(launch_finite_check(u, g->total, g->d_flag, st));
        int flag = 0;
        HIP_TRY(hipMemcpyAsync(&flag, g->d_flag, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (flag) return fail(SG_ENONFINITE, "state contains NaN or Inf");
    }
    return SG_OK;
}

sg_status sg_kerr_schild_data(sg_grid* g, const double* g10, const double* extra8, double* u, double* H_out,
                              sg_stream_t stream) {
    if (!g || !g10 || !u) return fail(SG_EINVAL, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    const int nv = g->opt.n_fields;
    for (int s = 0; s < (int)g->sh.size(); ++s) {
        ShellHost& S = g->sh[s];
        const KShell v = S.view(nv);
        const double* gs = g10 + layout_offset(g, s, 10);
        double* us = u + S.off;
        if (nv == 58) {
            if (extra8)
                HIP_TRY(hipMemcpyAsync(us + 50 * S.npts, extra8 + layout_offset(g, s, 8), sizeof(double) * 8 * S.npts,
                                       hipMemcpyDeviceToDevice, st));
            else
                HIP_TRY(hipMemsetAsync(us + 50 * S.npts, 0, sizeof(double) * 8 * S.npts, st));
        }
        HIP_TRY(derivs_shell(g, s, gs, g->dbuf, 10, true, st));
        HIP_TRY(launch_initial(v, gs, g->dbuf, us, nv == 50 ? S.H : nullptr, st));
        if (nv == 50) {
            HIP_TRY(derivs_shell(g, s, S.H, g->dbuf, 4, true, st));
            HIP_TRY(hipMemcpyAsync(S.dH, g->dbuf, sizeof(double) * 12 * S.npts, hipMemcpyDeviceToDevice, st));
            if (H_out)
                HIP_TRY(hipMemcpyAsync(H_out + layout_offset(g, s, 4), S.H, sizeof(double) * 4 * S.npts,
                                       hipMemcpyDeviceToDevice, st));
        }
    }
    return SG_OK;
}

sg_status sg_enable_timing(sg_grid* g, int on) {
    if (!g) return fail(SG_EINVAL, "grid is NULL");
    g->tm.on = on != 0;
    return SG_OK;
}

sg_status sg_kernel_times(sg_grid* g, double* ms, int* counts, int n_classes) {
    if (!g || !ms) return fail(SG_EINVAL, "NULL argument");
    for (int c = 0; c < SG_K_COUNT; ++c) {
        g->tm.ms[c] = 0;
        g->tm.cnt[c] = 0;
    }
    if (!g->tm.ev.empty()) HIP_TRY(hipEventSynchronize(g->tm.ev.back()));
    for (size_t k = 0; k < g->tm.cls.size(); ++k) {
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, g->tm.ev[2 * k], g->tm.ev[2 * k + 1]));
        g->tm.ms[g->tm.cls[k]] += t;
        g->tm.cnt[g->tm.cls[k]] += 1;
    }
    for (int c = 0; c < n_classes && c < SG_K_COUNT; ++c) {
        ms[c] = g->tm.ms[c];
        if (counts) counts[c] = g->tm.cnt[c];
    }
    return SG_OK;
}

// Host-only helpers (no device work): the operator matrices the library
// builds, for comparison against an independent construction.
int sg_host_filter_matrix(int n, int m, int n_theta, int n_f, double* out) {
    if (!out || n_theta < 2 || n_theta > 96 || n < -3 || n > 3) return SG_EINVAL;
    std::vector<double> F = filter_matrix(n, m, n_theta, n_f);
    std::memcpy(out, F.data(), sizeof(double) * F.size());
    return SG_OK;
}

int sg_host_cheb_matrix(int n_r, double r_min, double r_max, double* out) {
    if (!out || n_r < 2) return SG_EINVAL;
    std::vector<double> D = cheb_matrix(n_r, r_min, r_max);
    std::memcpy(out, D.data(), sizeof(double) * D.size());
    return SG_OK;
}

int sg_host_theta_matrix(int n_theta, double* out) {
    if (!out || n_theta < 2) return SG_EINVAL;
    std::vector<double> H = theta_half_matrix(n_theta);
    std::memcpy(out, H.data(), sizeof(double) * H.size());
    return SG_OK;
}

}  // extern "C"
