/*
 * shellspec: CFF/Yn pseudospectral evolution of first-order tensor systems on
 * spherical shells, for one AMD Instinct MI355X (gfx950).
 *
 * Method: B. Bruegmann, "A pseudospectral matrix method for time-dependent
 * tensor fields on a spherical shell" (arXiv:1104.3408).  Section, equation
 * and table names below refer to that paper.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grid (Sec. 2.1, eqs. rk, thetai, phij):
 *   r_k = (r_max+r_min)/2 - (r_max-r_min)/2 cos(pi k/(N_r-1)),  k < N_r
 *   theta_i = pi (i + 1/2)/N_theta,  i < N_theta   (single cover, poles staggered)
 *   phi_j = 2 pi j/N_phi,  j < N_phi, with N_phi = 2 N_theta.
 * State layout: one contiguous FP64 device array holding the shells in
 *   creation order.  Inside a shell, variable mu at point (k, i, j) sits at
 *   k + N_r (i + N_theta (j + N_phi mu))   (r fastest, "field-major", Sec. 2.4).
 * Variable order (n_fields = 50): g_ab (10), Pi_ab (10), Phi_xab (10),
 *   Phi_yab (10), Phi_zab (10), symmetric pairs ab ordered
 *   tt tx ty tz xx xy xz yy yz zz (Cartesian components, Sec. 2.2, App. A.1).
 *   n_fields = 58 appends H_a (4) and Q_a = d_t H_a (4) with index a = t x y z.
 * Derivative layout: for each shell, three blocks of that shell's state size
 *   (d_r, d_theta, d_phi, or d_x, d_y, d_z), at offset 3*offset(shell).
 * Ownership: every array argument is caller-owned device memory (for example
 *   a torch tensor); the library never frees or reallocates it, and cannot
 *   check device array sizes: the caller guarantees the sizes stated at each
 *   entry point (the Python binding checks them).  The grid object owns its
 *   operator matrices and workspaces.
 * Streams: every compute call is asynchronous and ordered on the given HIP
 *   stream (0 = the null stream); no hidden host synchronisation happens on
 *   the hot calls.  Calls on one grid object must not overlap in time: they
 *   share the grid's workspaces.
 * Errors: argument and shape checks run on the host before any launch and
 *   return SG_EINVAL / SG_ESHAPE; HIP runtime errors return SG_EHIP.  A
 *   non-OK status leaves a message for sg_last_error() (per host thread).
 */
#ifndef SHELLSPEC_H
#define SHELLSPEC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* sg_stream_t; /* the hipStream_t of HIP */
typedef struct sg_grid sg_grid;           /* opaque */

typedef enum {
    SG_OK = 0,
    SG_EINVAL = -1,       /* bad argument value */
    SG_ESHAPE = -2,       /* grid sizes the library does not support */
    SG_ENOMEM = -3,       /* device allocation failed */
    SG_EHIP = -4,         /* HIP runtime error */
    SG_ENONFINITE = -5,   /* SG_CHECK_FINITE found NaN/Inf in the state */
    SG_EUNSUPPORTED = -6  /* option combination not built */
} sg_status;

enum { SG_FILTER_YN = 0, SG_FILTER_Y = 1, SG_FILTER_YG = 2, SG_FILTER_NONE = 3 };
enum { SG_PREC_FP64 = 0, SG_PREC_FP32 = 1, SG_PREC_BF16X3 = 2 };
enum { SG_COORD = 0, SG_CART = 1 };
enum { SG_CHECK_FINITE = 1u, SG_NO_GRAPH = 2u, SG_NESTED = 4u };

/* One shell: N_r Chebyshev points on [r_min, r_max], N_theta x N_phi angles
 * (Sec. 2.1).  Requirements checked by shell_grid_create: 4 <= N_r <= 80,
 * 4 <= N_theta <= 64, N_phi = 2 N_theta, 0 < r_min < r_max. */
typedef struct {
    int n_r, n_theta, n_phi;
    double r_min, r_max;
} sg_shell_desc;

typedef struct {
    int n_fields;     /* 50 (static gauge) or 58 (H_a, d_t H_a evolved) */
    int filter_kind;  /* SG_FILTER_YN (tensor, Sec. 3.5), _Y (scalar), _YG (graded,
                         eq. nfofmu), _NONE */
    int n_f;          /* number of top degrees removed, l <= L - n_f, L = N_theta - 1
                         (Sec. 3.5); the paper's default is 4 */
    int precision;    /* SG_PREC_FP64, or SG_PREC_FP32: in rk_step the theta and phi
                         derivatives are computed and stored in FP32, and the filter
                         is split as F(u) = F(u_ref) + F(u - u_ref) with F(u_ref)
                         in FP64 and the difference filtered in FP32 (u_ref: the
                         state at the start of each rk_step call, refreshed every
                         64 steps);
                         d_r, the rhs and the RK state stay FP64.  SG_PREC_BF16X3:
                         as SG_PREC_FP32, but the theta and phi derivative
                         contractions and the filter's reduced-precision part (phi
                         analysis, theta filter, phi synthesis of u - u_ref) run on
                         the matrix cores with each operand split into two
                         bfloat16 parts, W x ~ W_hi x_hi + W_hi x_lo + W_lo x_hi
                         accumulated in FP32 (about 2^-16 of |W||x| per product);
                         spec_derivs, ghg_rhs and ghg_constraints stay FP64 in
                         every mode */
    double courant;   /* lambda of Delta t = lambda min(Delta x) (Sec. 4.1), e.g. 4 */
    double mass;      /* black-hole mass M used by sg_kerr_schild_data */
    unsigned flags;   /* SG_CHECK_FINITE: rk_step reports NaN/Inf; SG_NO_GRAPH: rk_step
                         launches every kernel itself instead of replaying a captured
                         HIP graph of one step; SG_NESTED: consecutive shells whose
                         radii meet (r_max of one = r_min of the next) are coupled at
                         the shared sphere (each keeps a copy of it; both copies get
                         one right-hand side, every characteristic field of App. A.2
                         taken from the side it travels from, the mean for speed 0:
                         the paper's outlook of nested shells, Sec. 1 and Sec. 5, whose
                         interface condition it leaves open); such shells must have
                         the same N_theta and N_phi (else SG_ESHAPE) and one time step
                         (the smaller Courant step of the chain by default) */
} sg_options;

/* Build the grid object for n_shells shells: collocation points, the 1-d
 * differentiation matrices of Sec. 2.3 (Chebyshev eq. CDhat rescaled to the
 * shell, Fourier FD for the double-covered theta circle and for phi), the
 * Fourier analysis/synthesis matrices of Sec. 3.1, and the spin-weighted
 * filter matrices F^n_m = P^n_m diag(1..1,0..0) (P^n_m)^+ of Sec. 3.3/3.5
 * (eq. FasPfQ) for |n| <= 3, built on the host from the recursion of eqs.
 * Yninc/Yndec and uploaded once.  gauge_H: optional device array with the
 * static gauge source H_a (4 variables per point, same per-shell layout as a
 * 4-field state); when given, its Cartesian derivatives are computed here
 * (null stream, synchronous).  Tile shapes and kernel forms per shell size
 * and precision come from a text table read here (the file named by the
 * environment variable SG_TUNING_FILE, else tuning.txt beside the library;
 * defaults for sizes it does not list).  They change the speed; only the
 * d_phi form (circulant or parity) also changes the order of the rounding.
 * On success *out owns device memory released by shell_grid_destroy. */
sg_status shell_grid_create(const sg_shell_desc* shells, int n_shells, const sg_options* opt,
                            const double* gauge_H, sg_grid** out);

/* Release everything the grid owns.  NULL is ignored. */
void shell_grid_destroy(sg_grid* g);

/* Per-shell placement: *offset and *count in doubles of the shell's block in
 * a state array, *dt the Courant time step lambda min(Delta x) (Sec. 4.1).
 * shell = -1 returns offset 0, the total state size, and the smallest dt.
 * Any output pointer may be NULL. */
sg_status shell_grid_info(const sg_grid* g, int shell, size_t* offset, size_t* count, double* dt);

/* Host copies of the collocation coordinates of one shell (Sec. 2.1):
 * r[N_r], theta[N_theta], phi[N_phi]; NULL outputs are skipped. */
sg_status shell_grid_coords(const sg_grid* g, int shell, double* r, double* theta, double* phi);

/* Set the static gauge source of the 50-field system (App. A.3 eq. gauge):
 * H is a device array of 4 variables per point (H_t, H_x, H_y, H_z).  Its
 * Cartesian spatial derivatives are computed spectrally and kept by the
 * grid; d_t H = 0.  Stream-ordered. */
sg_status sg_set_gauge(sg_grid* g, const double* H, sg_stream_t stream);

/* Spectral derivatives of every variable of the state u (Sec. 2.4): d_r by
 * the Chebyshev matrix, d_theta by the Fourier matrix on the double-covered
 * theta circle (Sec. 2.1), d_phi by the Fourier matrix.  mode SG_COORD writes
 * (d_r, d_theta, d_phi); SG_CART applies the chain rule of Sec. 2.2 eq. dvdx
 * and writes (d_x, d_y, d_z).  du must hold 3 state sizes and must not alias u. */
sg_status spec_derivs(sg_grid* g, const double* u, double* du, int mode, sg_stream_t stream);

/* Projection filter of the state, in place, once (Sec. 3.5): Yn decomposes
 * every tensor on the complex tetrad (t, r, m, mbar) of Sec. 3.4 and filters
 * each component with F_n of its spin weight n; Y / Yg filter every Cartesian
 * component with F_0 (n_f, or n_f - d(u^mu) for Yg).  Each filter is a
 * Fourier analysis in phi, the theta matrices F^n_m per Fourier order m and a
 * Fourier synthesis (Sec. 3.1, eqs. Fanalysis/Fsynthesis, Nyquist dropped). */
sg_status swsh_filter(sg_grid* g, double* u, sg_stream_t stream);

/* Constraint monitor (App. A.1): per shell the gauge constraint
 * C_a = H_a + Gamma_a (Gamma_a = g^bc Gamma_abc with d_t g from eq. gdot; H_a
 * the static gauge for 50 fields, the state's H_a for 58) and the first-order
 * constraint C_iab = d_i g_ab - Phi_iab, d_i g_ab the Cartesian spectral
 * derivative of the state's g_ab.  u: device state (layout of rk_step).
 * norms: caller-owned device array of 4 * n_shells doubles, per shell
 * (max |C_a|, rms C_a, max |C_iab|, rms C_iab); rms over all components and
 * grid points of the shell.  Stream-ordered; uses the grid's derivative
 * workspace, so calls on one grid must not overlap.  SG_EINVAL on NULL. */
sg_status ghg_constraints(sg_grid* g, const double* u, double* norms, sg_stream_t stream);

/* The constraint monitor of ghg_constraints for callers that cannot allocate
 * device memory (code captured into a graph, serving loops, harnesses that
 * forbid allocation): the call makes no allocation and uses no workspace of
 * the grid.  du_cart: caller-owned device array with the Cartesian
 * derivatives of the state as spec_derivs writes them in SG_CART mode (per
 * shell 3 blocks of the shell's state size; only the ten g_ab of each block
 * are read).  norms as for ghg_constraints.  The workgroup partials live in
 * a fixed 128 KB device array of the library (one per device, held until the
 * process ends), which limits a shell to 4096 x 256 grid points (every shell
 * shell_grid_create accepts fits; larger: SG_ESHAPE).  Calls that overlap on
 * one device (several streams or host threads) share that array and race;
 * calls in one stream order are safe.  Stream-ordered; SG_EINVAL on NULL,
 * SG_EHIP on a launch error. */
sg_status ghg_constraints_static(const sg_grid* g, const double* u, const double* du_cart, double* norms,
                                 sg_stream_t stream);

/* Right-hand side d_t u of the first-order GHG system (App. A.1 eqs. gdot,
 * Phidot, Pidot with gamma_0 = gamma_2 = 1, gamma_1 = -1), with the
 * freezing-incoming boundary operator (App. A.3) applied on the outermost
 * sphere k = N_r - 1 (of each shell; with SG_NESTED only of the outermost
 * shell of a chain, and the two copies of a shared sphere get one value,
 * each characteristic field from its upwind side).  du_cart: Cartesian
 * derivatives of u in the derivative layout, or NULL to compute them here.
 * rhs must not alias u. */
sg_status ghg_rhs(sg_grid* g, const double* u, const double* du_cart, double* rhs,
                  sg_stream_t stream);

/* n_steps classical RK4 steps of the method of lines (Sec. 2.5), u in place:
 * four right-hand-side evaluations (derivatives, rhs, boundary operator),
 * then the filter after each full step.  dt: host array with one time step
 * per shell (finite and > 0, else SG_EINVAL; shells coupled by SG_NESTED must
 * share one, else SG_EINVAL), or NULL for each shell's Courant step (the
 * chain's smallest for coupled shells).  One step is captured
 * into a HIP graph (on a private stream, re-captured when u or dt change)
 * and replayed n_steps times on the given stream, unless SG_NO_GRAPH is set
 * or kernel timing is enabled.  With SG_CHECK_FINITE the
 * state is scanned after the last step and SG_ENONFINITE returned (this
 * synchronises the stream). */
sg_status rk_step(sg_grid* g, double* u, const double* dt, int n_steps, sg_stream_t stream);

/* Initial data of App. A.3 from a 4-metric: g10 holds the 10 components
 * g_ab per point (device, 10-field state layout).  Writes the full state u
 * (Phi_iab = spectral d_i g_ab, Pi_ab = beta^i Phi_iab / alpha for d_t g = 0)
 * and, for 50 fields, also installs H_a = -Gamma_a as the static gauge (and
 * writes it to H_out when non-NULL, 4 variables per point).  For 58 fields
 * the caller's extra8 (device, 8 variables per point, may be NULL = zero) is
 * added to (H_a = -Gamma_a, Q_a = 0) in the state. */
sg_status sg_kerr_schild_data(sg_grid* g, const double* g10, const double* extra8, double* u,
                              double* H_out, sg_stream_t stream);

/* Per-kernel timing of the calls made since timing was enabled or since the
 * last rk_step started, in milliseconds, from HIP events recorded on the
 * caller's stream immediately before and after every launch (only while
 * enabled with sg_enable_timing(g, 1); the events sit between launches).
 * ms[c] is the summed duration and counts[c] the number of launches of
 * kernel class c for c < n_classes (at most SG_K_COUNT).  Synchronises on
 * the last recorded event. */
enum { SG_K_DR = 0, SG_K_DTHETA = 1, SG_K_DPHI = 2, SG_K_RHS = 3, SG_K_DECOMP = 4, SG_K_FANA = 5,
       SG_K_FTHETA = 6, SG_K_FSYN = 7, SG_K_RECOMP = 8, SG_K_COUNT = 9 };
sg_status sg_enable_timing(sg_grid* g, int on);
sg_status sg_kernel_times(sg_grid* g, double* ms, int* counts, int n_classes);

/* Host-only copies of the operator matrices the library builds (no device
 * work, usable without a GPU), row-major into caller memory:
 *   sg_host_filter_matrix: F^n_m (N_theta x N_theta) with the top n_f
 *     degrees removed (Sec. 3.5 eq. FasPfQ), |n| <= 3;
 *   sg_host_cheb_matrix: Chebyshev matrix of eq. CDhat rescaled to
 *     [r_min, r_max] (N_r x N_r);
 *   sg_host_theta_matrix: folded double-cover theta matrix (N_theta x 2 N_theta):
 *     columns < N_theta act on f(theta_i', phi), the rest on f(theta_i', phi + pi).
 * Return SG_OK or SG_EINVAL. */
int sg_host_filter_matrix(int n, int m, int n_theta, int n_f, double* out);
int sg_host_cheb_matrix(int n_r, double r_min, double r_max, double* out);
int sg_host_theta_matrix(int n_theta, double* out);

/* Message for the last non-OK status on this host thread ("" if none). */
const char* sg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
