/*
 * orc.h -- plain FP64 CPU oracle for the DGSEM compressible-Euler right-hand side.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
 * its Python binding) may include, link or call this code; only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark do.  The oracle shares
 * no source with the HIP path.
 *
 * What it computes (paper: Trixi.jl, arXiv 2108.06476):
 *   - the semidiscretisation of the conservation law of Eq. (1) (Section 2)
 *     for the ideal-gas Euler equations, no source term, by the nodal DGSEM on
 *     Legendre-Gauss-Lobatto nodes (Section 2.1, "matrix-free DG methods"),
 *   - with the flux-differencing volume integral and an entropy-conservative,
 *     kinetic-energy-preserving two-point flux (Section 3.1), or a central
 *     volume flux, or the weak form (Section 3.1: central volume flux == weak
 *     form), or the Hennemann-Gassner blended DG/FV shock-capturing volume
 *     integral (Section 2.1, "entropy-stable sub-cell shock capturing"),
 *   - LLF / HLL / EC interface fluxes (Sections 2.3.1 and 3.1),
 *   - the Carpenter-Kennedy five-stage fourth-order low-storage Runge-Kutta
 *     method with the CFL time step of Section 3.1.
 * Every evaluation is straightforward FP64 loops, compiled without FMA
 * contraction (the appendix discusses contraction; the oracle keeps every
 * product and sum rounded separately).
 *
 * Layout of every state array: u[var][elem][node], FP64, var in
 * (rho, rho v_1 .. rho v_dim, rho E); node = i + n*(j + n*k) with n = N+1 and
 * i along x; elem = ex + Kx*(ey + Ky*ez).  All arrays are caller-owned host
 * memory.  Functions return ORC_OK (0) or a positive error code.
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_ENONPHYS = 4 };
enum { ORC_VOL_EC = 0, ORC_VOL_CENTRAL = 1, ORC_VOL_SHOCKCAP_HG = 2, ORC_VOL_WEAK = 3,
       ORC_VOL_NONE = 4 };
enum { ORC_SURF_LLF = 0, ORC_SURF_HLL = 1, ORC_SURF_EC = 2, ORC_SURF_NONE = 3 };

#define ORC_MAXN 15   /* polynomial degrees 3..15 as in the PID study (Section 3.1) */

typedef struct {
  int32_t dim;        /* 2 or 3 */
  int32_t polydeg;    /* N, 1 <= N <= ORC_MAXN */
  int32_t cells[3];   /* elements per direction, periodic; cells[2] = 1 in 2D */
  double  xmin[3], xmax[3];
  double  gamma;
  int32_t volume;     /* ORC_VOL_* */
  int32_t surface;    /* ORC_SURF_* */
  int32_t fv_flux;    /* ORC_SURF_LLF or ORC_SURF_HLL: subcell FV flux */
  double  alpha_max;  /* shock capturing: upper clip of alpha */
  double  alpha_min;  /* shock capturing: alpha below this -> 0, above 1-this -> 1 */
  int32_t alpha_smooth; /* 1: neighbour smoothing of alpha */
} orc_config;

/* LGL nodes x[N+1], weights w[N+1], differentiation matrix D[(N+1)*(N+1)] (row-major,
 * D[i*(N+1)+j] = l_j'(x_i)). */
int orc_lgl(int N, double *x, double *w, double *D);
/* Inverse of the orthonormal-Legendre Vandermonde matrix V_ia = Lt_a(x_i). */
int orc_legendre_vinv(int N, double *Vinv);

/* Pointwise physics (direction d in 0..dim-1).  u, fL/fR/f have dim+2 entries. */
double orc_ln_mean(double x, double y);
int orc_flux_phys(const double *u, int d, int dim, double gamma, double *f);
int orc_flux_ec(const double *uL, const double *uR, int d, int dim, double gamma, double *f);
int orc_flux_central(const double *uL, const double *uR, int d, int dim, double gamma, double *f);
int orc_flux_llf(const double *uL, const double *uR, int d, int dim, double gamma, double *f);
int orc_flux_hll(const double *uL, const double *uR, int d, int dim, double gamma, double *f);
/* entropy S(u) and entropy variables w(u) */
double orc_entropy(const double *u, int dim, double gamma);
int orc_entropy_vars(const double *u, int dim, double gamma, double *w);

int64_t orc_num_nodes(const orc_config *cfg);
int orc_node_coords(const orc_config *cfg, double *xyz);            /* [dim][E][n^dim] */
int orc_rhs(const orc_config *cfg, const double *u, double *du);
int orc_indicator(const orc_config *cfg, const double *u, double *alpha_raw, double *alpha);
int orc_indicator_energy(const orc_config *cfg, const double *u, double *energy); /* [E] */
int orc_rhs_alpha(const orc_config *cfg, const double *u, const double *alpha, double *du);
int orc_max_dt(const orc_config *cfg, const double *u, double cfl, double *dt);
int orc_lsrk_coeffs(double *A, double *B, double *c);
int orc_step(const orc_config *cfg, double *u, int32_t nsteps, double cfl, double dt_fixed,
             double *t);
int orc_integrals(const orc_config *cfg, const double *u, const double *du, double *out7);
int orc_num_threads(void);
int orc_set_num_threads(int n);   /* returns the previous number */

/* Curvilinear mesh of the PID study (Section 3.1): the periodic box [-1,1]^3 with cells^3
 * elements, mapped by Eq. (2) with amplitude warp (0.15 in the paper; 0 gives the Cartesian
 * grid).  Reference-element node positions are mapped; metric terms (J a^i)_n come from the
 * conservative curl form of the interpolated mapping, J from the interpolant's derivatives.
 * Volume: flux differencing with the two-point flux contracted with the averaged metric
 * vector; surface: the interface flux through the face's contravariant vector.
 * source = ORC_SRC_MMS adds the manufactured solution's source term (orc_curv_mms). */
enum { ORC_SRC_NONE = 0, ORC_SRC_MMS = 1 };
typedef struct {
  int32_t polydeg;
  int32_t cells;      /* elements per direction */
  double  warp;       /* amplitude of the Eq. (2) mapping */
  double  gamma;
  int32_t volume;     /* ORC_VOL_EC, ORC_VOL_CENTRAL or ORC_VOL_NONE */
  int32_t surface;    /* ORC_SURF_* */
  int32_t source;     /* ORC_SRC_* */
} orc_curv_config;

int orc_curv_map(double warp, const double *xi, double *x);               /* Eq. (2) */
/* the manufactured solution u(x, t) and its source s(x, t) (either may be NULL) */
int orc_curv_mms(double gamma, const double *x, double t, double *u, double *s);
int64_t orc_curv_num_nodes(const orc_curv_config *cfg);
/* xyz [3][E][n^3], Ja [3 (i)][3 (n)][E][n^3] = (J a^i)_n, J [E][n^3]; any may be NULL */
int orc_curv_geometry(const orc_curv_config *cfg, double *xyz, double *Ja, double *J);
int orc_curv_initial(const orc_curv_config *cfg, double t, double *u);   /* MMS at nodes */
int orc_curv_rhs(const orc_curv_config *cfg, const double *u, double t, double *du);
int orc_curv_max_dt(const orc_curv_config *cfg, const double *u, double cfl, double *dt);
int orc_curv_step(const orc_curv_config *cfg, double *u, int32_t nsteps, double cfl,
                  double dt_fixed, double *t);

/* Ideal MHD (the PID study's second system, Section 3.1): 8 variables
 * u = (rho, rho v_1..3, E, B_1..3), mu_0 = 1, E = p/(gamma-1) + rho|v|^2/2 + |B|^2/2, on the
 * periodic Cartesian box [-1,1]^3 with cells^3 elements; weak-form DGSEM with the HLL (or
 * LLF) interface flux, or flux differencing with an entropy-conservative two-point flux and
 * Powell's non-conservative term (Section 3.1: the paper's MHD flux-differencing solver is
 * entropy conservative and needs non-conservative terms); fast magnetosonic wave speeds;
 * CK(5,4) with the CFL step. */
typedef struct {
  int32_t polydeg;
  int32_t cells;
  double  gamma;
  int32_t surface;    /* ORC_SURF_HLL, ORC_SURF_LLF; ORC_SURF_EC with flux differencing */
  int32_t volume;     /* ORC_VOL_WEAK, or ORC_VOL_EC: flux differencing with the
                         entropy-conservative flux and Powell's non-conservative term */
} orc_mhd_config;

int orc_mhd_ec_flux(const double *uL, const double *uR, int d, double gamma, double *f);
double orc_mhd_entropy(const double *u, double gamma);
int orc_mhd_entropy_vars(const double *u, double gamma, double *w);

int orc_mhd_flux(const double *u, int d, double gamma, double *f);          /* f^d(u), 8 */
int orc_mhd_surface_flux(int kind, const double *uL, const double *uR, int d, double gamma,
                         double *f);
double orc_mhd_fast_speed(const double *u, int d, double gamma);
int64_t orc_mhd_num_nodes(const orc_mhd_config *cfg);
int orc_mhd_rhs(const orc_mhd_config *cfg, const double *u, double *du);   /* [8][E][n^3] */
int orc_mhd_max_dt(const orc_mhd_config *cfg, const double *u, double cfl, double *dt);
int orc_mhd_step(const orc_mhd_config *cfg, double *u, int32_t nsteps, double cfl,
                 double dt_fixed, double *t);
/* the circularly polarised Alfven wave (an exact solution) at one point */
int orc_mhd_alfven(double gamma, const double *x, double t, double *u);

#ifdef __cplusplus
}
#endif
#endif
