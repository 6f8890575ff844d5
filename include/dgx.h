/*
 * dgx.h -- C ABI of the MI355X (gfx950) DGSEM compressible-Euler right-hand side.
 *
 * The method is the semidiscretisation of Trixi.jl (arXiv 2108.06476): the
 * conservation law of Eq. (1) for the ideal-gas Euler equations (no source term)
 * discretised by the nodal DGSEM on Legendre-Gauss-Lobatto nodes (Section 2.1)
 * on a uniform, periodic Cartesian quad/hex grid (the TreeMesh of Section 2.3.1
 * at uniform refinement), with
 *   - the flux-differencing volume integral with an entropy-conservative,
 *     kinetic-energy-preserving two-point flux, or a central volume flux
 *     (equal to the weak form, Section 3.1),
 *   - LLF / HLL / EC interface fluxes (Sections 2.3.1 and 3.1),
 *   - the surface lift and the Cartesian Jacobian 2/h,
 *   - the entropy-stable subcell shock capturing of Section 2.1
 *     (Hennemann-Gassner indicator, blended DG/FV volume integral),
 *   - the Carpenter-Kennedy five-stage fourth-order low-storage Runge-Kutta
 *     method with the adaptive CFL time step of Section 3.1.
 * Every step runs in hand-written HIP kernels on the GPU.
 *
 * Conventions for every call:
 *   - State layout: u[var][elem][node], float64, contiguous (structure of
 *     arrays); var = (rho, rho v_1 .. rho v_dim, rho E); node = i + n*(j + n*k)
 *     with n = N+1 and i along x; elem = ex + Kx*(ey + Ky*ez).  Element e spans
 *     [xmin + e h, xmin + (e+1) h] per direction; its node i sits at
 *     xmin + e h + (h/2)(1 + x_i), x_i the LGL nodes.
 *   - Every array argument is a caller-owned DEVICE pointer, borrowed only for
 *     the work enqueued by the call.  Host pointers are named as such.
 *   - All work is enqueued asynchronously on the handle's HIP stream; only
 *     dgx_check() and dgx_last_error() synchronise or read host state.  The
 *     library allocates device scratch at create time and frees it at destroy.
 *   - Calls return a dgx_status.  Argument errors are detected on the host and
 *     returned at once (nothing is enqueued); a non-physical state met by a
 *     kernel (rho <= 0, p <= 0 or NaN) raises a device flag read by dgx_check().
 *   - There is no global state: handles are independent (Section 2.3.3) and may
 *     be used from different host threads; one handle is not thread-safe.
 */
#ifndef DGX_H
#define DGX_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DGX_OK = 0,
  DGX_EINVAL = 1,        /* bad argument or configuration */
  DGX_EHIP = 2,          /* a HIP runtime call failed (see dgx_last_error) */
  DGX_ENOMEM = 3,        /* device allocation failed */
  DGX_ENONPHYS = 4,      /* a kernel met a non-physical state */
  DGX_EUNSUPPORTED = 5   /* valid but not built (e.g. polydeg outside the compiled set) */
} dgx_status;

typedef enum {
  DGX_VOL_EC = 0,          /* flux differencing, entropy-conservative two-point flux */
  DGX_VOL_CENTRAL = 1,     /* flux differencing, central flux (= weak form) */
  DGX_VOL_SHOCKCAP_HG = 2, /* blended: (1-alpha) EC flux differencing + alpha FV */
  DGX_VOL_WEAK = 3,        /* weak form: (2/h) sum_m Dhat_im f(u_m), Dhat_im = (w_m/w_i) D_mi
                              (Section 3.1, the paper's other measured DG solver); FP64 */
  DGX_VOL_NONE = 4,        /* no volume term (testing: surface terms only) */
  DGX_VOL_WEAK_MFMA = 5    /* the weak form with its line contractions on the matrix cores
                              (v_mfma_f64_4x4x4f64); 3D, polydeg 3 only, else
                              DGX_EUNSUPPORTED */
} dgx_volume;

typedef enum {
  DGX_SURF_LLF = 0,
  DGX_SURF_HLL = 1,
  DGX_SURF_EC = 2,
  DGX_SURF_NONE = 3        /* no surface term (testing: volume term only) */
} dgx_surface;

typedef enum {
  DGX_FP64 = 0,            /* every operation in float64 */
  DGX_MIXED = 1            /* volume two-point fluxes and volume sums in float32;
                              near-equal-state log means, interface fluxes, RK
                              accumulation and reductions in float64 */
} dgx_precision;

typedef struct {
  int32_t dim;            /* 2 or 3 */
  int32_t polydeg;        /* N; compiled for 1..7 (3D) and 1..7 (2D) */
  int32_t cells[3];       /* elements per direction, periodic; cells[2] = 1 in 2D */
  double  xmin[3], xmax[3];
  double  gamma;          /* ratio of specific heats, > 1 */
  int32_t volume;         /* dgx_volume */
  int32_t surface;        /* dgx_surface */
  int32_t fv_flux;        /* DGX_SURF_LLF or DGX_SURF_HLL: subcell FV flux */
  double  alpha_max;      /* shock capturing: upper clip of alpha (e.g. 0.5) */
  double  alpha_min;      /* alpha < alpha_min -> 0, alpha > 1 - alpha_min -> 1 (e.g. 0.001) */
  int32_t alpha_smooth;   /* 1: alpha_e = max(alpha_e, max_neighbours alpha_nb / 2) */
  int32_t precision;      /* dgx_precision */
} dgx_config;

typedef struct dgx_solver *dgx_handle;

/* Create a solver for cfg (host pointer, copied) whose work goes to hip_stream
 * (a hipStream_t; NULL = the null stream).  Allocates the device scratch (two state-sized
 * arrays, u2 and k, plus per-element buffers).  Size: fewer than 2^30 elements (the kernels
 * use 64-bit offsets, so a state may fill most of the device memory); DGX_EUNSUPPORTED
 * beyond, DGX_ENOMEM when the device memory runs out. */
dgx_status dgx_create(const dgx_config *cfg, void *hip_stream, dgx_handle *out);
dgx_status dgx_destroy(dgx_handle h);
/* Re-target the handle's work to another stream (e.g. the caller's current one). */
dgx_status dgx_set_stream(dgx_handle h, void *hip_stream);

/* E * (N+1)^dim: nodes per variable. */
int64_t dgx_num_nodes(dgx_handle h);
int64_t dgx_num_elements(dgx_handle h);

/* Node coordinates, device xyz[dim][E][n^dim] (the layout above). */
dgx_status dgx_node_coords(dgx_handle h, double *xyz);

/* du = R(u): the semidiscrete right-hand side du/dt (Eq. (1) discretised).  u, du
 * are device [nvar][E][n^dim] and must not overlap.  For DGX_VOL_SHOCKCAP_HG the
 * indicator is evaluated from u first.  t: the time of a source term (curvilinear handles
 * with DGX_SOURCE_MMS; unused otherwise). */
dgx_status dgx_rhs(dgx_handle h, const double *u, double *du, double t);

/* Hennemann-Gassner indicator of u: alpha[E] (device), clipped and, when
 * cfg.alpha_smooth, smoothed.  alpha_raw (device, may be NULL) receives the
 * unsmoothed clipped values; energy (device, may be NULL) the modal energy ratio. */
dgx_status dgx_indicator(dgx_handle h, const double *u, double *alpha, double *alpha_raw,
                         double *energy);

/* du = R(u) with the blending factors alpha[E] (device) given instead of computed
 * (DGX_VOL_SHOCKCAP_HG only). */
dgx_status dgx_rhs_alpha(dgx_handle h, const double *u, const double *alpha, double *du);

/* dt = cfl * 2 / ((N+1) max_e sum_d (2/h_d) max_nodes(|v_d| + c)), written to the
 * device scalar *dt (Section 3.1: local wave speed, relative grid size, CFL). */
dgx_status dgx_max_dt(dgx_handle h, const double *u, double cfl, double *dt);

/* dgx_max_dt without any device allocation, for callers that cannot allocate (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same result
 * as dgx_max_dt (bitwise: the same kernels in the same order), with the per-element
 * partials in a static device array of the library, 2^20 float64 (8 MiB) per device, which
 * each device that the library runs on keeps until the process ends.  The call allocates
 * nothing and frees nothing; the handle (created beforehand, on the current device) and
 * the arguments are as for dgx_max_dt.  DGX_EINVAL when the handle has more than 2^20
 * elements or the current device is not the handle's.  Every call on one device shares
 * that array: calls that overlap on one device (other streams, other host threads, other
 * handles) race and must be ordered by the caller. */
dgx_status dgx_max_dt_noalloc(dgx_handle h, const double *u, double cfl, double *dt);

/* Advance u in place by nsteps Carpenter-Kennedy 5-stage 4th-order 2N-storage
 * steps: per step dt from u at its start (cfl > 0) or dt_fixed (cfl <= 0), then
 * for s = 1..5: k <- A_s k + dt R(u), u <- u + B_s k.  t (device scalar, may be
 * NULL) is advanced by every dt.  Ownership differs from a 2N-storage call in which the
 * caller passes k: the handle owns k and a second state buffer (two state-sized arrays,
 * 168 MB at 32^3 elements, N = 3), because every stage reads the face neighbours of its
 * input state while it writes the updated state, so it writes into the other buffer; ten
 * stages (two steps) bring the result back to u, and an odd step count ends with one copy
 * into u.  Pairs of
 * steps are replayed from a hipGraph that the handle captures once per (u, t, cfl,
 * dt_fixed) and keeps; the result is bitwise that of launching every kernel (which the
 * handle does while profiling is enabled). */
dgx_status dgx_step(dgx_handle h, double *u, int32_t nsteps, double cfl, double dt_fixed,
                    double *t);

/* out7 (device, 7 doubles): [0..dim+1] = sum J w u_v, [5] = sum J w S(u) with
 * S = -rho s/(gamma-1), s = ln p - gamma ln rho, [6] = sum J w w(u).du (0 when du
 * is NULL), J = prod h_d/2.  Deterministic order. */
dgx_status dgx_integrals(dgx_handle h, const double *u, const double *du, double *out7);

/* Synchronise the stream and report (and clear) the non-physical-state flag:
 * *flag = 1 if any kernel since the last check met rho <= 0, p <= 0 or NaN. */
dgx_status dgx_check(dgx_handle h, int32_t *flag);

/* The handle's last error message (host string owned by the handle). */
const char *dgx_last_error(dgx_handle h);

/* ---- curvilinear mesh (the PID study's geometry, Section 3.1) ------------------------
 * The periodic box [-1,1]^3 with cells^3 hexahedra, warped by the mapping of Eq. (2)
 * (amplitude warp; 0.15 in the paper, 0 = Cartesian):
 *   y = eta + warp cos(1.5 pi xi) cos(0.5 pi eta) cos(0.5 pi zeta),
 *   x = xi  + warp cos(0.5 pi xi) cos(2 pi y)     cos(0.5 pi zeta),
 *   z = zeta + warp cos(0.5 pi x) cos(pi y)       cos(0.5 pi zeta).
 * The element nodes are the mapped LGL points; metric terms (J a^i)_n come from the
 * conservative curl form of the interpolated mapping (discrete metric identities hold, so a
 * constant state stays constant), J from the interpolant's derivatives.  The two-point
 * volume flux is contracted with the pair's averaged metric vector; interface fluxes pass
 * through the face's contravariant vector; du/dt = -(1/J)(...) + s(x, t).
 * source = DGX_SOURCE_MMS adds the source of the manufactured solution
 *   rho = 2 + 0.1 sin(pi (x + y + z) - 2 pi t), v = (1, 1, 1), rho E = rho^2
 * (the paper's Euler test is a manufactured solution with sine/cosine source terms, which
 * it does not print; this one is the library's reading).  Stage times t + c_s dt. */
typedef enum { DGX_SOURCE_NONE = 0, DGX_SOURCE_MMS = 1 } dgx_source;

typedef struct {
  int32_t polydeg;        /* N; compiled for 1..7 */
  int32_t cells;          /* elements per direction */
  double  warp;           /* Eq. (2) amplitude, 0 <= warp < 0.5 */
  double  gamma;          /* > 1 */
  int32_t volume;         /* DGX_VOL_EC, DGX_VOL_CENTRAL or DGX_VOL_NONE (else EUNSUPPORTED) */
  int32_t surface;        /* dgx_surface */
  int32_t source;         /* dgx_source */
} dgx_curv_config;

/* A solver on the curvilinear mesh (FP64).  The handle works with dgx_rhs (t is the time
 * of the source term), dgx_step (t required with a source: the stages use its value at the
 * start of each step), dgx_max_dt (dt from sum_i max (|v . Ja^i| + c |Ja^i|)/J),
 * dgx_node_coords (the mapped positions), dgx_check and the profiling calls;
 * dgx_indicator, dgx_rhs_alpha and dgx_integrals return DGX_EUNSUPPORTED on it.
 * Computes the geometry on the device (synchronises the stream once).  Size: 9 * nodes
 * below 2^31 (its kernels index the metric arrays in 32 bits), else DGX_EUNSUPPORTED. */
dgx_status dgx_create_curved(const dgx_curv_config *cfg, void *hip_stream, dgx_handle *out);

/* The geometry of a curvilinear handle: ja [3 (i)][3 (n)][E][n^3] = (J a^i)_n and
 * jac [E][n^3] = J (device; either may be NULL).  DGX_EINVAL on a Cartesian handle. */
dgx_status dgx_geometry(dgx_handle h, double *ja, double *jac);

/* ---- ideal MHD (the PID study's second system, Section 3.1) --------------------------
 * 8 variables u = (rho, rho v_1..3, E, B_1..3), mu_0 = 1, E = p/(gamma-1) + rho|v|^2/2 +
 * |B|^2/2, on the periodic Cartesian box [-1,1]^3 with cells^3 elements, the two solvers of
 * the paper's MHD comparison: volume = DGX_VOL_WEAK, the weak-form DGSEM with the HLL (or
 * LLF) interface flux; volume = DGX_VOL_EC, flux differencing with an entropy-conservative
 * two-point flux and Powell's non-conservative term phi(u) div B, phi = (0, B, v.B, v),
 * discretised as phi(u_i) {{B_d}} in the volume and on the faces (surface EC, LLF or HLL;
 * EC everywhere conserves the entropy exactly).  Fast magnetosonic wave speeds.  The handle works
 * with dgx_rhs, dgx_step (dt from sum_d (2/h) max (|v_d| + c_f,d)), dgx_max_dt,
 * dgx_node_coords, dgx_check and the profiling calls; states are [8][E][n^3].  Size:
 * 8 * nodes below 2^31 (32-bit state offsets), else DGX_EUNSUPPORTED. */
typedef struct {
  int32_t polydeg;        /* N; compiled for 1..7 */
  int32_t cells;          /* elements per direction */
  double  gamma;          /* > 1 */
  int32_t surface;        /* DGX_SURF_HLL or DGX_SURF_LLF; DGX_SURF_EC with DGX_VOL_EC */
  int32_t volume;         /* DGX_VOL_WEAK or DGX_VOL_EC */
} dgx_mhd_config;

dgx_status dgx_create_mhd(const dgx_mhd_config *cfg, void *hip_stream, dgx_handle *out);

/* Kernel timing for benchmarks: enables HIP-event timing of the dominant (stage) kernel on
 * the handle's stream.  One event pair brackets each run of back-to-back stage launches
 * (the five stages of an RK step; a single launch where indicator kernels sit between
 * stages, and for dgx_rhs), so the time includes the launch gaps inside a run. */
dgx_status dgx_profile_enable(dgx_handle h, int32_t on);
/* Average duration in milliseconds of the timed kernel's launches since enable, and
 * its name (host string). */
dgx_status dgx_profile_read(dgx_handle h, double *avg_ms, int64_t *launches, const char **name);

/* ----- ensembles: many independent solvers advanced together ----- */
typedef struct dgx_batch_s *dgx_batch;

/* nruns configurations (host array, copied); every run is 3D, DGX_VOL_EC, DGX_SURF_LLF or
 * HLL, polydeg 3..5, with its own grid, extent and gamma; all share one precision (the
 * many independent instances of Section 2.3.3).  Each RK stage of all runs is one launch
 * over (run, element tile) work items, runs of higher polydeg first.  The launch takes one
 * block per work item unless the tuner (or dgx_batch_set_shape) picks a persistent grid
 * whose blocks loop over the items; one block per item is the default and what the tuner
 * normally keeps, since the persistent loop holds more registers live.  A step (per-run
 * dt + 5 stages) is replayed from a captured hipGraph.  The library owns each run's second
 * state buffer and RK register (they are not passed in: a stage reads its input buffer's
 * face neighbours while it writes the other). */
dgx_status dgx_batch_create(const dgx_config *cfgs, int32_t nruns, void *hip_stream,
                            dgx_batch *out);
dgx_status dgx_batch_destroy(dgx_batch b);
/* number of nodes of run r (per variable) */
int64_t dgx_batch_num_nodes(dgx_batch b, int32_t r);
/* Advance every run in place by nsteps CK(5,4) steps, each with its own CFL dt from its
 * own state (cfl > 0).  u: host array of nruns device pointers, each [5][E_r][n_r^3]
 * (the dgx_step layout).  t: device [nruns] (may be NULL), advanced by each run's dt. */
dgx_status dgx_batch_step(dgx_batch b, double *const *u, int32_t nsteps, double cfl,
                          double *t);
/* du_r = R_r(u_r) for every run (host arrays of device pointers). */
dgx_status dgx_batch_rhs(dgx_batch b, const double *const *u, double *const *du);
/* Autotuner: time one right-hand side of every run (written into the library's RK
 * registers; the states u are only read) for each candidate tile shape (threads per block:
 * 256 or 512, i.e. elements per work item) and persistent grid (2, 4 or 8 blocks per CU,
 * or one block per work item) and keep the fastest.  budget_ms bounds the tuning time. */
dgx_status dgx_batch_tune(dgx_batch b, double *const *u, int32_t budget_ms);
/* Set the tile shape by hand: block = 256 or 512 threads; grid = 0 for one block per work
 * item, or a positive multiple of 8 (8 XCDs): a grid smaller than the number of work items
 * runs the persistent kernel, whose blocks loop over XCD-contiguous ranges of items.
 * DGX_EINVAL otherwise.  Synchronises the stream and drops the captured step graph. */
dgx_status dgx_batch_set_shape(dgx_batch b, int32_t block, int32_t grid);
/* The current tile shape: threads per block and persistent blocks. */
dgx_status dgx_batch_shape(dgx_batch b, int32_t *block, int32_t *grid);
/* Synchronise and report (and clear) the non-physical-state flag of any run. */
dgx_status dgx_batch_check(dgx_batch b, int32_t *flag);
const char *dgx_batch_last_error(dgx_batch b);

/* ---- measured peaks of the board (a measurement aid for rooflines, not a step of the
 * method; the paper reports throughput, Section 3.1, and the published MI355X peaks are
 * what a roofline divides by, these measured ones stand beside them) ---- */
enum {
  DGX_PEAK_HBM_COPY = 0,   /* GB/s read + written by a copy of a 2 GiB float64 buffer */
  DGX_PEAK_FP64_FMA = 1    /* TFLOP/s of independent FP64 vector FMA chains on every lane
                              (2 flops per FMA, 8 waves per SIMD) */
};
/* Runs the probe `kind` on HIP device `device` (best of 10 launches timed with HIP events,
 * after one warm-up launch) and writes the rate to the HOST double *value.  Unlike the
 * other calls it blocks: it allocates its buffers (4 GiB for the copy), creates its own
 * stream, synchronises and frees everything before it returns; no handle is needed.
 * DGX_EINVAL for a NULL value, an unknown kind or device; DGX_ENOMEM, DGX_EHIP. */
dgx_status dgx_measure_peak(int32_t device, int32_t kind, double *value);

#ifdef __cplusplus
}
#endif
#endif
