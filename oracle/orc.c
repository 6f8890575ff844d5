/*
 * orc.c -- plain FP64 CPU oracle for the DGSEM compressible-Euler right-hand side.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the benchmark's
 * CPU-baseline leg, never by the product path.  Shares no code with the HIP
 * library.  Built with -O2 -fopenmp -ffp-contract=off (no FMA contraction).
 *
 * Everything here is written from the mathematics the paper names (Trixi.jl,
 * arXiv 2108.06476) and the textbook DGSEM it cites for its DG methods
 * (Section 2.1).  The paper names the ingredients but does not print their
 * formulas; each function states the formula it evaluates and the reading of
 * the paper it follows.
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NMAX (ORC_MAXN + 1)

/* ------------------------------------------------------------------------- */
/* Legendre-Gauss-Lobatto operator (nodal DGSEM on LGL nodes, Section 2.1).   */
/* ------------------------------------------------------------------------- */

/* P_N(x) and P_N'(x) by the three-term recurrence
 * (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1} and P'_{k+1} = P'_{k-1} + (2k+1) P_k. */
static void legendre(int N, double x, double *P, double *dP)
{
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  if (N == 0) { *P = 1.0; *dP = 0.0; return; }
  for (int k = 1; k < N; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    double d2 = d0 + (2.0 * k + 1.0) * p1;
    p0 = p1; p1 = p2;
    d0 = d1; d1 = d2;
  }
  *P = p1;
  *dP = d1;
}

/* Nodes: -1, the N-1 roots of P_N', +1 (Newton on P_N' with P_N'' taken from
 * Legendre's equation).  Weights w_i = 2 / (N (N+1) P_N(x_i)^2).
 * D_ij = l_j'(x_i) from barycentric weights lambda_j = 1/prod_{k!=j}(x_j - x_k):
 * D_ij = (lambda_j/lambda_i)/(x_i - x_j), D_ii = -sum_{j!=i} D_ij. */
int orc_lgl(int N, double *x, double *w, double *D)
{
  if (N < 1 || N > ORC_MAXN) return ORC_EINVAL;
  const int n = N + 1;
  x[0] = -1.0;
  x[N] = 1.0;
  for (int i = 1; i < N; ++i) {
    double xi = -cos(M_PI * i / N);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(N, xi, &P, &dP);
      double ddP = (2.0 * xi * dP - N * (N + 1.0) * P) / (1.0 - xi * xi);
      double dx = dP / ddP;
      xi = xi - dx;
      if (fabs(dx) < 1e-17) break;
    }
    x[i] = xi;
  }
  for (int i = 0; i < n; ++i) {
    double P, dP;
    legendre(N, x[i], &P, &dP);
    w[i] = 2.0 / (N * (N + 1.0) * P * P);
  }
  double lam[NMAX];
  for (int j = 0; j < n; ++j) {
    double prod = 1.0;
    for (int k = 0; k < n; ++k)
      if (k != j) prod = prod * (x[j] - x[k]);
    lam[j] = 1.0 / prod;
  }
  for (int i = 0; i < n; ++i) {
    double diag = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      D[i * n + j] = (lam[j] / lam[i]) / (x[i] - x[j]);
      diag = diag - D[i * n + j];
    }
    D[i * n + i] = diag;
  }
  return ORC_OK;
}

/* Orthonormal Legendre Vandermonde V_ia = sqrt((2a+1)/2) P_a(x_i) on the LGL
 * nodes, inverted by Gauss-Jordan elimination with partial pivoting.
 * Vinv[a*n + i]. */
int orc_legendre_vinv(int N, double *Vinv)
{
  if (N < 1 || N > ORC_MAXN) return ORC_EINVAL;
  const int n = N + 1;
  double x[NMAX], w[NMAX], D[NMAX * NMAX];
  orc_lgl(N, x, w, D);
  double A[NMAX][2 * NMAX];
  for (int i = 0; i < n; ++i) {
    for (int a = 0; a < n; ++a) {
      double P, dP;
      legendre(a, x[i], &P, &dP);
      A[i][a] = sqrt((2.0 * a + 1.0) / 2.0) * P;
      A[i][n + a] = (i == a) ? 1.0 : 0.0;
    }
  }
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
    if (A[piv][col] == 0.0) return ORC_EINVAL;
    if (piv != col)
      for (int c = 0; c < 2 * n; ++c) { double t = A[col][c]; A[col][c] = A[piv][c]; A[piv][c] = t; }
    double inv = 1.0 / A[col][col];
    for (int c = 0; c < 2 * n; ++c) A[col][c] = A[col][c] * inv;
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      double f = A[r][col];
      for (int c = 0; c < 2 * n; ++c) A[r][c] = A[r][c] - f * A[col][c];
    }
  }
  /* A = V^{-1} V after elimination: the right half holds V^{-1}, indexed [row a][col i]. */
  for (int a = 0; a < n; ++a)
    for (int i = 0; i < n; ++i) Vinv[a * n + i] = A[a][n + i];
  return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Pointwise physics: ideal-gas Euler, Eq. (1) with s = 0.                    */
/* u = (rho, rho v_1..rho v_dim, rho E), p = (gamma-1)(rho E - rho |v|^2 / 2). */
/* ------------------------------------------------------------------------- */

typedef struct { double rho, v[3], p, c; } prim_t;

/* Returns 0 for a physical state (rho > 0, p > 0, both finite), 1 otherwise. */
static int to_prim(const double *u, int dim, double gamma, prim_t *q)
{
  double v2 = 0.0;
  q->rho = u[0];
  for (int k = 0; k < 3; ++k) q->v[k] = 0.0;
  for (int k = 0; k < dim; ++k) {
    q->v[k] = u[1 + k] / u[0];
    v2 = v2 + q->v[k] * q->v[k];
  }
  q->p = (gamma - 1.0) * (u[dim + 1] - 0.5 * u[0] * v2);
  q->c = sqrt(gamma * q->p / q->rho);
  if (!(q->rho > 0.0) || !(q->p > 0.0) || !isfinite(q->rho) || !isfinite(q->p)) return 1;
  return 0;
}

/* f^d(u) = (rho v_d, rho v_d v + p e_d, v_d (rho E + p)). */
static void phys_flux(const double *u, const prim_t *q, int d, int dim, double *f)
{
  f[0] = u[1 + d];
  for (int k = 0; k < dim; ++k) f[1 + k] = u[1 + d] * q->v[k] + (k == d ? q->p : 0.0);
  f[dim + 1] = q->v[d] * (u[dim + 1] + q->p);
}

/* Logarithmic mean (y - x)/(ln y - ln x), with the stable evaluation of the
 * efficiency reference the paper cites for its flux kernels (Section 3.2):
 * f2 = ((x-y)/(x+y))^2 written as (x(x-2y)+y^2)/(x(x+2y)+y^2); for f2 < 1e-4
 * the truncated series of ln(y/x) = 2 artanh((y-x)/(y+x)) gives
 * (x+y)/(2 + f2(2/3 + f2(2/5 + f2 2/7))); otherwise (y-x)/ln(y/x). */
double orc_ln_mean(double x, double y)
{
  double f2 = (x * (x - 2.0 * y) + y * y) / (x * (x + 2.0 * y) + y * y);
  if (f2 < 1.0e-4)
    return (x + y) / (2.0 + f2 * (2.0 / 3.0 + f2 * (2.0 / 5.0 + f2 * (2.0 / 7.0))));
  return (y - x) / log(y / x);
}

/* Entropy-conservative and kinetic-energy-preserving two-point flux for the
 * Euler equations (the EC flux of Section 3.1), direction d:
 *   f_rho  = {{rho}}_ln {{v_d}}
 *   f_rhov = f_rho {{v}} + {{p}} e_d
 *   f_rhoE = f_rho ( 1/((gamma-1) {{rho/p}}_ln) + v_L.v_R/2 ) + (p_L v_dR + p_R v_dL)/2
 * with {{a}} = (a_L + a_R)/2 and {{.}}_ln the logarithmic mean. */
static void ec_flux(const prim_t *L, const prim_t *R, int d, int dim, double gamma, double *f)
{
  double rho_ln = orc_ln_mean(L->rho, R->rho);
  double beta_ln = orc_ln_mean(L->rho / L->p, R->rho / R->p);
  double vavg[3] = {0.0, 0.0, 0.0}, vLvR = 0.0;
  for (int k = 0; k < dim; ++k) {
    vavg[k] = 0.5 * (L->v[k] + R->v[k]);
    vLvR = vLvR + L->v[k] * R->v[k];
  }
  double pavg = 0.5 * (L->p + R->p);
  double frho = rho_ln * vavg[d];
  f[0] = frho;
  for (int k = 0; k < dim; ++k) f[1 + k] = frho * vavg[k] + (k == d ? pavg : 0.0);
  f[dim + 1] = frho * (1.0 / ((gamma - 1.0) * beta_ln) + 0.5 * vLvR)
               + 0.5 * (L->p * R->v[d] + R->p * L->v[d]);
}

/* Central volume flux (f(u_L) + f(u_R))/2: flux differencing with it equals the
 * weak form (Section 3.1). */
static void central_flux(const double *uL, const prim_t *L, const double *uR, const prim_t *R,
                         int d, int dim, double *f)
{
  double fL[5], fR[5];
  phys_flux(uL, L, d, dim, fL);
  phys_flux(uR, R, d, dim, fR);
  for (int v = 0; v < dim + 2; ++v) f[v] = 0.5 * (fL[v] + fR[v]);
}

/* Local Lax-Friedrichs (Rusanov): (f_L + f_R)/2 - lambda (u_R - u_L)/2 with
 * lambda = max(|v_dL| + c_L, |v_dR| + c_R). */
static void llf_flux(const double *uL, const prim_t *L, const double *uR, const prim_t *R,
                     int d, int dim, double *f)
{
  double fL[5], fR[5];
  phys_flux(uL, L, d, dim, fL);
  phys_flux(uR, R, d, dim, fR);
  double lL = fabs(L->v[d]) + L->c, lR = fabs(R->v[d]) + R->c;
  double lam = lL > lR ? lL : lR;
  for (int v = 0; v < dim + 2; ++v) f[v] = 0.5 * (fL[v] + fR[v]) - 0.5 * lam * (uR[v] - uL[v]);
}

/* HLL with the two-state wave-speed estimates
 * s_L = min(v_dL - c_L, v_dR - c_R), s_R = max(v_dL + c_L, v_dR + c_R). */
static void hll_flux(const double *uL, const prim_t *L, const double *uR, const prim_t *R,
                     int d, int dim, double *f)
{
  double fL[5], fR[5];
  phys_flux(uL, L, d, dim, fL);
  phys_flux(uR, R, d, dim, fR);
  double a = L->v[d] - L->c, b = R->v[d] - R->c;
  double sL = a < b ? a : b;
  a = L->v[d] + L->c; b = R->v[d] + R->c;
  double sR = a > b ? a : b;
  for (int v = 0; v < dim + 2; ++v) {
    if (sL >= 0.0) f[v] = fL[v];
    else if (sR <= 0.0) f[v] = fR[v];
    else f[v] = (sR * fL[v] - sL * fR[v] + sL * sR * (uR[v] - uL[v])) / (sR - sL);
  }
}

static void surface_flux(int kind, const double *uL, const prim_t *L, const double *uR,
                         const prim_t *R, int d, int dim, double gamma, double *f)
{
  if (kind == ORC_SURF_LLF) llf_flux(uL, L, uR, R, d, dim, f);
  else if (kind == ORC_SURF_HLL) hll_flux(uL, L, uR, R, d, dim, f);
  else ec_flux(L, R, d, dim, gamma, f);
}

/* pointwise exports (used by the pinning tests) */
int orc_flux_phys(const double *u, int d, int dim, double gamma, double *f)
{
  prim_t q;
  int bad = to_prim(u, dim, gamma, &q);
  phys_flux(u, &q, d, dim, f);
  return bad ? ORC_ENONPHYS : ORC_OK;
}
int orc_flux_ec(const double *uL, const double *uR, int d, int dim, double gamma, double *f)
{
  prim_t L, R;
  int bad = to_prim(uL, dim, gamma, &L) | to_prim(uR, dim, gamma, &R);
  ec_flux(&L, &R, d, dim, gamma, f);
  return bad ? ORC_ENONPHYS : ORC_OK;
}
int orc_flux_central(const double *uL, const double *uR, int d, int dim, double gamma, double *f)
{
  prim_t L, R;
  int bad = to_prim(uL, dim, gamma, &L) | to_prim(uR, dim, gamma, &R);
  central_flux(uL, &L, uR, &R, d, dim, f);
  return bad ? ORC_ENONPHYS : ORC_OK;
}
int orc_flux_llf(const double *uL, const double *uR, int d, int dim, double gamma, double *f)
{
  prim_t L, R;
  int bad = to_prim(uL, dim, gamma, &L) | to_prim(uR, dim, gamma, &R);
  llf_flux(uL, &L, uR, &R, d, dim, f);
  return bad ? ORC_ENONPHYS : ORC_OK;
}
int orc_flux_hll(const double *uL, const double *uR, int d, int dim, double gamma, double *f)
{
  prim_t L, R;
  int bad = to_prim(uL, dim, gamma, &L) | to_prim(uR, dim, gamma, &R);
  hll_flux(uL, &L, uR, &R, d, dim, f);
  return bad ? ORC_ENONPHYS : ORC_OK;
}

/* S(u) = -rho s/(gamma-1), s = ln p - gamma ln rho. */
double orc_entropy(const double *u, int dim, double gamma)
{
  prim_t q;
  to_prim(u, dim, gamma, &q);
  double s = log(q.p) - gamma * log(q.rho);
  return -q.rho * s / (gamma - 1.0);
}

/* w(u) = ((gamma - s)/(gamma-1) - rho|v|^2/(2p), rho v/p, -rho/p). */
int orc_entropy_vars(const double *u, int dim, double gamma, double *w)
{
  prim_t q;
  int bad = to_prim(u, dim, gamma, &q);
  double s = log(q.p) - gamma * log(q.rho);
  double v2 = 0.0;
  for (int k = 0; k < dim; ++k) v2 = v2 + q.v[k] * q.v[k];
  w[0] = (gamma - s) / (gamma - 1.0) - q.rho * v2 / (2.0 * q.p);
  for (int k = 0; k < dim; ++k) w[1 + k] = q.rho * q.v[k] / q.p;
  w[dim + 1] = -q.rho / q.p;
  return bad ? ORC_ENONPHYS : ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Mesh: uniform periodic Cartesian grid (the TreeMesh of Section 2.3.1, at a  */
/* uniform refinement; elements in lexicographic order).                      */
/* ------------------------------------------------------------------------- */

typedef struct {
  int dim, N, n, NN, nvar;
  int K[3];
  int64_t E;
  double h[3];
  double x[NMAX], w[NMAX], D[NMAX * NMAX];
  double S[NMAX * NMAX];     /* S = 2D - M^{-1}B, diagonal zero */
  double Dhat[NMAX * NMAX];  /* weak-form matrix Dhat_im = (w_m/w_i) D_mi */
} mesh_t;

static int setup(const orc_config *cfg, mesh_t *m)
{
  if (!cfg) return ORC_EINVAL;
  if (cfg->dim != 2 && cfg->dim != 3) return ORC_EINVAL;
  if (cfg->polydeg < 1 || cfg->polydeg > ORC_MAXN) return ORC_EINVAL;
  if (!(cfg->gamma > 1.0)) return ORC_EINVAL;
  m->dim = cfg->dim;
  m->N = cfg->polydeg;
  m->n = m->N + 1;
  m->nvar = m->dim + 2;
  m->NN = m->dim == 3 ? m->n * m->n * m->n : m->n * m->n;
  m->E = 1;
  for (int d = 0; d < 3; ++d) {
    m->K[d] = d < m->dim ? cfg->cells[d] : 1;
    if (m->K[d] < 1) return ORC_EINVAL;
    m->E *= m->K[d];
    if (d < m->dim) {
      if (!(cfg->xmax[d] > cfg->xmin[d])) return ORC_EINVAL;
      m->h[d] = (cfg->xmax[d] - cfg->xmin[d]) / m->K[d];
    } else {
      m->h[d] = 1.0;
    }
  }
  orc_lgl(m->N, m->x, m->w, m->D);
  const int n = m->n;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double B = 0.0;
      if (i == j && i == 0) B = -1.0;
      if (i == j && i == m->N) B = 1.0;
      m->S[i * n + j] = 2.0 * m->D[i * n + j] - B / m->w[i];
      m->Dhat[i * n + j] = (m->w[j] / m->w[i]) * m->D[j * n + i];
    }
  return ORC_OK;
}

static void elem_coords(const mesh_t *m, int64_t e, int c[3])
{
  c[0] = (int)(e % m->K[0]);
  c[1] = (int)((e / m->K[0]) % m->K[1]);
  c[2] = (int)(e / ((int64_t)m->K[0] * m->K[1]));
}

/* periodic face neighbour of element e in direction d, side s = -1 or +1 */
static int64_t neighbour(const mesh_t *m, int64_t e, int d, int s)
{
  int c[3];
  elem_coords(m, e, c);
  c[d] = (c[d] + s + m->K[d]) % m->K[d];
  return c[0] + (int64_t)m->K[0] * (c[1] + (int64_t)m->K[1] * c[2]);
}

static void node_idx(const mesh_t *m, int node, int idx[3])
{
  idx[0] = node % m->n;
  idx[1] = (node / m->n) % m->n;
  idx[2] = m->dim == 3 ? node / (m->n * m->n) : 0;
}

static int node_of(const mesh_t *m, const int idx[3])
{
  return idx[0] + m->n * (idx[1] + m->n * idx[2]);
}

static void load_node(const mesh_t *m, const double *u, int64_t e, int node, double *un)
{
  for (int v = 0; v < m->nvar; ++v) un[v] = u[((int64_t)v * m->E + e) * m->NN + node];
}

int64_t orc_num_nodes(const orc_config *cfg)
{
  mesh_t m;
  if (setup(cfg, &m)) return -1;
  return m.E * m.NN;
}

/* node i of element e sits at xmin + e h + (h/2)(1 + x_i) in each direction */
int orc_node_coords(const orc_config *cfg, double *xyz)
{
  mesh_t m;
  int st = setup(cfg, &m);
  if (st) return st;
  for (int64_t e = 0; e < m.E; ++e) {
    int c[3];
    elem_coords(&m, e, c);
    for (int node = 0; node < m.NN; ++node) {
      int idx[3];
      node_idx(&m, node, idx);
      for (int d = 0; d < m.dim; ++d)
        xyz[((int64_t)d * m.E + e) * m.NN + node] =
            cfg->xmin[d] + c[d] * m.h[d] + 0.5 * m.h[d] * (1.0 + m.x[idx[d]]);
    }
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Hennemann-Gassner indicator (sub-cell shock capturing, Section 2.1).       */
/* ------------------------------------------------------------------------- */

/* Per element: q = rho p at the nodes; modal coefficients qhat = (Vinv x Vinv [x Vinv]) q
 * in the orthonormal Legendre basis; energies over index cubes
 * E_tot = sum_{[0,N]^d} qhat^2, E_1 = sum_{[0,N-1]^d}, E_2 = sum_{[0,N-2]^d};
 * energy = max((E_tot-E_1)/E_tot, (E_1-E_2)/E_1), a ratio with a zero
 * denominator counting as 0. */
static double energy_of(const mesh_t *m, const double *u, int64_t e, const double *Vinv,
                        double gamma)
{
  const int n = m->n, NN = m->NN, N = m->N;
  double q[NMAX * NMAX * NMAX];
  for (int node = 0; node < NN; ++node) {
    double un[5];
    prim_t p;
    load_node(m, u, e, node, un);
    to_prim(un, m->dim, gamma, &p);
    q[node] = p.rho * p.p;
  }
  double Etot = 0.0, E1 = 0.0, E2 = 0.0;
  const int nc = m->dim == 3 ? n : 1;
  for (int c = 0; c < nc; ++c)
    for (int b = 0; b < n; ++b)
      for (int a = 0; a < n; ++a) {
        double qh = 0.0;
        for (int k = 0; k < nc; ++k)
          for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
              double coef = Vinv[a * n + i] * Vinv[b * n + j];
              if (m->dim == 3) coef = coef * Vinv[c * n + k];
              qh = qh + coef * q[i + n * (j + n * k)];
            }
        double e2 = qh * qh;
        int mx = a > b ? a : b;
        if (c > mx) mx = c;
        Etot = Etot + e2;
        if (mx <= N - 1) E1 = E1 + e2;
        if (mx <= N - 2) E2 = E2 + e2;
      }
  double r1 = Etot != 0.0 ? (Etot - E1) / Etot : 0.0;
  double r2 = E1 != 0.0 ? (E1 - E2) / E1 : 0.0;
  return r1 > r2 ? r1 : r2;
}

/* alpha = 1/(1 + exp(-(s/T)(energy - T))), T = 0.5 10^(-1.8 (N+1)^(1/4)),
 * s = ln((1 - 1e-4)/1e-4); alpha < alpha_min -> 0, alpha > 1 - alpha_min -> 1;
 * alpha = min(alpha, alpha_max). */
static double alpha_of(double energy, int N, double alpha_min, double alpha_max)
{
  double T = 0.5 * pow(10.0, -1.8 * pow(N + 1.0, 0.25));
  double s = log((1.0 - 0.0001) / 0.0001);
  double a = 1.0 / (1.0 + exp(-(s / T) * (energy - T)));
  if (a < alpha_min) a = 0.0;
  else if (a > 1.0 - alpha_min) a = 1.0;
  if (a > alpha_max) a = alpha_max;
  return a;
}

int orc_indicator_energy(const orc_config *cfg, const double *u, double *energy)
{
  mesh_t m;
  int st = setup(cfg, &m);
  if (st) return st;
  double Vinv[NMAX * NMAX];
  orc_legendre_vinv(m.N, Vinv);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m.E; ++e) energy[e] = energy_of(&m, u, e, Vinv, cfg->gamma);
  return ORC_OK;
}

/* alpha_raw: the clipped per-element alpha; alpha: after the smoothing
 * alpha_e = max(alpha_e, max over face neighbours of alpha_nb / 2), taken from
 * the unsmoothed values.  Either output pointer may be NULL. */
int orc_indicator(const orc_config *cfg, const double *u, double *alpha_raw, double *alpha)
{
  mesh_t m;
  int st = setup(cfg, &m);
  if (st) return st;
  double *en = (double *)malloc(sizeof(double) * m.E);
  double *ar = (double *)malloc(sizeof(double) * m.E);
  if (!en || !ar) { free(en); free(ar); return ORC_EINVAL; }
  orc_indicator_energy(cfg, u, en);
  for (int64_t e = 0; e < m.E; ++e) ar[e] = alpha_of(en[e], m.N, cfg->alpha_min, cfg->alpha_max);
  if (alpha_raw)
    for (int64_t e = 0; e < m.E; ++e) alpha_raw[e] = ar[e];
  if (alpha) {
    for (int64_t e = 0; e < m.E; ++e) {
      double a = ar[e];
      if (cfg->alpha_smooth)
        for (int d = 0; d < m.dim; ++d)
          for (int s = -1; s <= 1; s += 2) {
            double nb = 0.5 * ar[neighbour(&m, e, d, s)];
            if (nb > a) a = nb;
          }
      alpha[e] = a;
    }
  }
  free(en);
  free(ar);
  return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Right-hand side.                                                          */
/* ------------------------------------------------------------------------- */

/* For node (i,j,k) of element e (drop k in 2D), per direction d with 1D index i_d:
 *   V_d    = sum_{m != i_d} S_{i_d m} fvol_d(u_node, u_partner(m))       (EC/central)
 *          = - sum_m Dhat_{i_d m} f^d(u_partner(m))                        (weak form)
 *   V_d    = (1 - alpha) V_d + alpha V^FV_d                                (shock capturing)
 *   V^FV_d = (F_{i+1/2} - F_{i-1/2}) / w_i, F_{i+1/2} = f_fv(u_i, u_{i+1}) for i < N, 0 at both ends
 *   Surf_d = ( [i_d == N] f*(u_node, u_{e+d}(0)) - [i_d == 0] f*(u_{e-d}(N), u_node) ) / w_0
 *   du     = - sum_d (2/h_d) (V_d + Surf_d).                                                  */
static int rhs_core(const orc_config *cfg, const mesh_t *m, const double *u, const double *alpha,
                    double *du)
{
  const int dim = m->dim, n = m->n, N = m->N, NN = m->NN, nvar = m->nvar;
  const double gamma = cfg->gamma;
  const int vol = cfg->volume, surf = cfg->surface;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t e = 0; e < m->E; ++e) {
    double ue[NMAX * NMAX * NMAX][5];
    prim_t qe[NMAX * NMAX * NMAX];
    for (int node = 0; node < NN; ++node) {
      load_node(m, u, e, node, ue[node]);
      bad |= to_prim(ue[node], dim, gamma, &qe[node]);
    }
    const double a = (vol == ORC_VOL_SHOCKCAP_HG) ? alpha[e] : 0.0;
    for (int node = 0; node < NN; ++node) {
      int idx[3];
      node_idx(m, node, idx);
      double acc[5] = {0, 0, 0, 0, 0};
      for (int d = 0; d < dim; ++d) {
        const int id = idx[d];
        double V[5] = {0, 0, 0, 0, 0}, Sf[5] = {0, 0, 0, 0, 0}, f[5];
        int pidx[3] = {idx[0], idx[1], idx[2]};
        if (vol == ORC_VOL_EC || vol == ORC_VOL_CENTRAL || vol == ORC_VOL_SHOCKCAP_HG) {
          for (int mm = 0; mm < n; ++mm) {
            if (mm == id) continue;
            pidx[d] = mm;
            int pn = node_of(m, pidx);
            if (vol == ORC_VOL_CENTRAL) central_flux(ue[node], &qe[node], ue[pn], &qe[pn], d, dim, f);
            else ec_flux(&qe[node], &qe[pn], d, dim, gamma, f);
            for (int v = 0; v < nvar; ++v) V[v] = V[v] + m->S[id * n + mm] * f[v];
          }
        } else if (vol == ORC_VOL_WEAK) {
          for (int mm = 0; mm < n; ++mm) {
            pidx[d] = mm;
            int pn = node_of(m, pidx);
            phys_flux(ue[pn], &qe[pn], d, dim, f);
            for (int v = 0; v < nvar; ++v) V[v] = V[v] - m->Dhat[id * n + mm] * f[v];
          }
        }
        if (vol == ORC_VOL_SHOCKCAP_HG) {
          double Fp[5] = {0, 0, 0, 0, 0}, Fm[5] = {0, 0, 0, 0, 0};
          if (id < N) {
            pidx[d] = id + 1;
            int pn = node_of(m, pidx);
            surface_flux(cfg->fv_flux, ue[node], &qe[node], ue[pn], &qe[pn], d, dim, gamma, Fp);
          }
          if (id > 0) {
            pidx[d] = id - 1;
            int pn = node_of(m, pidx);
            surface_flux(cfg->fv_flux, ue[pn], &qe[pn], ue[node], &qe[node], d, dim, gamma, Fm);
          }
          for (int v = 0; v < nvar; ++v) {
            double vfv = (Fp[v] - Fm[v]) / m->w[id];
            V[v] = (1.0 - a) * V[v] + a * vfv;
          }
        }
        if (surf != ORC_SURF_NONE) {
          double un[5];
          prim_t qn;
          pidx[0] = idx[0]; pidx[1] = idx[1]; pidx[2] = idx[2];
          if (id == N) {
            pidx[d] = 0;
            load_node(m, u, neighbour(m, e, d, +1), node_of(m, pidx), un);
            bad |= to_prim(un, dim, gamma, &qn);
            surface_flux(surf, ue[node], &qe[node], un, &qn, d, dim, gamma, f);
            for (int v = 0; v < nvar; ++v) Sf[v] = Sf[v] + f[v] / m->w[N];
          }
          if (id == 0) {
            pidx[d] = N;
            load_node(m, u, neighbour(m, e, d, -1), node_of(m, pidx), un);
            bad |= to_prim(un, dim, gamma, &qn);
            surface_flux(surf, un, &qn, ue[node], &qe[node], d, dim, gamma, f);
            for (int v = 0; v < nvar; ++v) Sf[v] = Sf[v] - f[v] / m->w[0];
          }
        }
        for (int v = 0; v < nvar; ++v) acc[v] = acc[v] + (2.0 / m->h[d]) * (V[v] + Sf[v]);
      }
      for (int v = 0; v < nvar; ++v) du[((int64_t)v * m->E + e) * NN + node] = -acc[v];
    }
  }
  return bad ? ORC_ENONPHYS : ORC_OK;
}

int orc_rhs_alpha(const orc_config *cfg, const double *u, const double *alpha, double *du)
{
  mesh_t m;
  int st = setup(cfg, &m);
  if (st) return st;
  if (cfg->volume == ORC_VOL_SHOCKCAP_HG && !alpha) return ORC_EINVAL;
  return rhs_core(cfg, &m, u, alpha, du);
}

/* The indicator is evaluated from the RHS input at every evaluation. */
int orc_rhs(const orc_config *cfg, const double *u, double *du)
{
  mesh_t m;
  int st = setup(cfg, &m);
  if (st) return st;
  if (cfg->volume != ORC_VOL_SHOCKCAP_HG) return rhs_core(cfg, &m, u, NULL, du);
  double *alpha = (double *)malloc(sizeof(double) * m.E);
  if (!alpha) return ORC_EINVAL;
  orc_indicator(cfg, u, NULL, alpha);
  st = rhs_core(cfg, &m, u, alpha, du);
  free(alpha);
  return st;
}

/* ------------------------------------------------------------------------- */
/* Time step and low-storage Runge-Kutta (Section 3.1).                       */
/* ------------------------------------------------------------------------- */

/* dt = CFL * 2 / ((N+1) * max_e [ sum_d (2/h_d) max_{nodes of e} (|v_d| + c) ]):
 * local maximum wave speed, relative grid size and the CFL coefficient. */
int orc_max_dt(const orc_config *cfg, const double *u, double cfl, double *dt)
{
  mesh_t m;
  int st = setup(cfg, &m);
  if (st) return st;
  double lam_max = 0.0;
  int bad = 0;
  for (int64_t e = 0; e < m.E; ++e) {
    double lam = 0.0;
    for (int d = 0; d < m.dim; ++d) {
      double mx = 0.0;
      for (int node = 0; node < m.NN; ++node) {
        double un[5];
        prim_t q;
        load_node(&m, u, e, node, un);
        bad |= to_prim(un, m.dim, cfg->gamma, &q);
        double s = fabs(q.v[d]) + q.c;
        if (s > mx) mx = s;
      }
      lam = lam + (2.0 / m.h[d]) * mx;
    }
    if (lam > lam_max) lam_max = lam;
  }
  *dt = cfl * 2.0 / ((m.N + 1.0) * lam_max);
  return bad ? ORC_ENONPHYS : ORC_OK;
}

/* Carpenter-Kennedy (1994) five-stage fourth-order 2N-storage coefficients. */
int orc_lsrk_coeffs(double *A, double *B, double *c)
{
  static const double a[5] = {0.0, -567301805773.0 / 1357537059087.0,
                              -2404267990393.0 / 2016746695238.0,
                              -3550918686646.0 / 2091501179385.0,
                              -1275806237668.0 / 842570457699.0};
  static const double b[5] = {1432997174477.0 / 9575080441755.0,
                              5161836677717.0 / 13612068292357.0,
                              1720146321549.0 / 2090206949498.0,
                              3134564353537.0 / 4481467310338.0,
                              2277821191437.0 / 14882151754819.0};
  static const double cc[5] = {0.0, 1432997174477.0 / 9575080441755.0,
                               2526269341429.0 / 6820363183890.0,
                               2006345519317.0 / 3224310063776.0,
                               2802321613138.0 / 2924317926251.0};
  for (int s = 0; s < 5; ++s) {
    if (A) A[s] = a[s];
    if (B) B[s] = b[s];
    if (c) c[s] = cc[s];
  }
  return ORC_OK;
}

/* Per step: dt from the state at the start of the step (cfl > 0) or dt_fixed;
 * then for s = 1..5: k <- A_s k + dt R(u); u <- u + B_s k; finally t += dt.
 * Stops at the first RHS that meets a non-physical state. */
int orc_step(const orc_config *cfg, double *u, int32_t nsteps, double cfl, double dt_fixed,
             double *t)
{
  mesh_t m;
  int st = setup(cfg, &m);
  if (st) return st;
  const int64_t len = (int64_t)m.nvar * m.E * m.NN;
  double *k = (double *)calloc(len, sizeof(double));
  double *du = (double *)malloc(sizeof(double) * len);
  if (!k || !du) { free(k); free(du); return ORC_EINVAL; }
  double A[5], B[5];
  orc_lsrk_coeffs(A, B, NULL);
  for (int step = 0; step < nsteps && st == ORC_OK; ++step) {
    double dt = dt_fixed;
    if (cfl > 0.0) st = orc_max_dt(cfg, u, cfl, &dt);
    for (int s = 0; s < 5 && st == ORC_OK; ++s) {
      st = orc_rhs(cfg, u, du);
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < len; ++i) {
        k[i] = A[s] * k[i] + dt * du[i];
        u[i] = u[i] + B[s] * k[i];
      }
    }
    if (t) *t = *t + dt;
  }
  free(k);
  free(du);
  return st;
}

/* out7[v] = sum J w_node u_v (v < dim+2, rest 0); out7[5] = sum J w S(u);
 * out7[6] = sum J w w(u).du (0 if du == NULL); J = prod_d h_d/2, w_node = prod_d w_{i_d}. */
int orc_integrals(const orc_config *cfg, const double *u, const double *du, double *out7)
{
  mesh_t m;
  int st = setup(cfg, &m);
  if (st) return st;
  double J = 1.0;
  for (int d = 0; d < m.dim; ++d) J = J * (0.5 * m.h[d]);
  for (int i = 0; i < 7; ++i) out7[i] = 0.0;
  int bad = 0;
  for (int64_t e = 0; e < m.E; ++e) {
    for (int node = 0; node < m.NN; ++node) {
      int idx[3];
      node_idx(&m, node, idx);
      double wn = 1.0;
      for (int d = 0; d < m.dim; ++d) wn = wn * m.w[idx[d]];
      double un[5], w[5];
      load_node(&m, u, e, node, un);
      for (int v = 0; v < m.nvar; ++v) out7[v] = out7[v] + J * wn * un[v];
      out7[5] = out7[5] + J * wn * orc_entropy(un, m.dim, cfg->gamma);
      bad |= orc_entropy_vars(un, m.dim, cfg->gamma, w) != ORC_OK;
      if (du) {
        double dot = 0.0;
        for (int v = 0; v < m.nvar; ++v) dot = dot + w[v] * du[((int64_t)v * m.E + e) * m.NN + node];
        out7[6] = out7[6] + J * wn * dot;
      }
    }
  }
  return bad ? ORC_ENONPHYS : ORC_OK;
}

/* Number of OpenMP threads of the following calls; returns the previous number. */
int orc_set_num_threads(int n)
{
#ifdef _OPENMP
  const int prev = omp_get_max_threads();
  if (n > 0) omp_set_num_threads(n);
  return prev;
#else
  (void)n;
  return 1;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ========================================================================= */
/* Curvilinear hexahedral mesh (Section 3.1): the periodic box [-1,1]^3 with   */
/* K^3 elements, warped by the mapping of Eq. (2); a manufactured solution of  */
/* the Euler equations with its source term (the PID study's Euler problem;    */
/* the paper names it without printing it, the one below is this oracle's      */
/* reading).                                                                   */
/* ========================================================================= */

/* Eq. (2): y first, then x (uses y), then z (uses x and y); a = warp amplitude. */
int orc_curv_map(double a, const double *xi, double *X)
{
  const double pi = 3.14159265358979323846;
  const double s = xi[0], e = xi[1], z = xi[2];
  const double y = e + a * (cos(1.5 * pi * s) * cos(0.5 * pi * e) * cos(0.5 * pi * z));
  const double x = s + a * (cos(0.5 * pi * s) * cos(2.0 * pi * y) * cos(0.5 * pi * z));
  const double w = z + a * (cos(0.5 * pi * x) * cos(pi * y) * cos(0.5 * pi * z));
  X[0] = x;
  X[1] = y;
  X[2] = w;
  return ORC_OK;
}

/* Manufactured solution (reading): rho = 2 + A sin(theta), theta = k (x + y + z) - om t,
 * v = (1, 1, 1), rho E = rho^2, with A = 0.1, k = pi, om = 2 pi; p = (gamma-1)(rho^2 - 1.5 rho).
 * Its source s = du/dt + div f(u), derived by hand (h = A cos theta):
 *   s_rho   = (3k - om) h
 *   s_rhov  = (3k - om) h + (gamma-1)(2 rho - 1.5) k h      (each component)
 *   s_rhoE  = -2 rho om h + 3 k (2 rho + (gamma-1)(2 rho - 1.5)) h                          */
int orc_curv_mms(double gamma, const double *x, double t, double *u, double *s)
{
  const double pi = 3.14159265358979323846;
  const double A = 0.1, k = pi, om = 2.0 * pi;
  const double th = k * (x[0] + x[1] + x[2]) - om * t;
  const double rho = 2.0 + A * sin(th);
  const double h = A * cos(th);
  if (u) {
    u[0] = rho;
    u[1] = rho;
    u[2] = rho;
    u[3] = rho;
    u[4] = rho * rho;
  }
  if (s) {
    const double dp = (gamma - 1.0) * (2.0 * rho - 1.5) * k * h;
    s[0] = (3.0 * k - om) * h;
    s[1] = s[0] + dp;
    s[2] = s[0] + dp;
    s[3] = s[0] + dp;
    s[4] = -2.0 * rho * om * h + 3.0 * k * (2.0 * rho + (gamma - 1.0) * (2.0 * rho - 1.5)) * h;
  }
  return ORC_OK;
}

typedef struct {
  mesh_t m;           /* 3D, n, S, w, D of the reference element; h unused */
  int K;
  double warp;
  double *xyz;        /* [3][E][NN] */
  double *Ja;         /* [3 (reference direction i)][3 (component n)][E][NN]: (J a^i)_n */
  double *J;          /* [E][NN] */
} curv_t;

static int curv_setup(const orc_curv_config *cfg, curv_t *c)
{
  if (!cfg || cfg->cells < 1 || cfg->polydeg < 1 || cfg->polydeg > ORC_MAXN) return ORC_EINVAL;
  if (!(cfg->gamma > 1.0)) return ORC_EINVAL;
  if (cfg->volume != ORC_VOL_EC && cfg->volume != ORC_VOL_CENTRAL && cfg->volume != ORC_VOL_NONE)
    return ORC_EINVAL;
  orc_config q;
  memset(&q, 0, sizeof(q));
  q.dim = 3;
  q.polydeg = cfg->polydeg;
  for (int d = 0; d < 3; ++d) {
    q.cells[d] = cfg->cells;
    q.xmin[d] = -1.0;
    q.xmax[d] = 1.0;
  }
  q.gamma = cfg->gamma;
  int st = setup(&q, &c->m);
  if (st) return st;
  c->K = cfg->cells;
  c->warp = cfg->warp;
  const int64_t len = c->m.E * c->m.NN;
  c->xyz = malloc(sizeof(double) * 3 * len);
  c->Ja = malloc(sizeof(double) * 9 * len);
  c->J = malloc(sizeof(double) * len);
  if (!c->xyz || !c->Ja || !c->J) return ORC_EINVAL;
  const mesh_t *m = &c->m;
  const int n = m->n, NN = m->NN;
  const double hr = 2.0 / c->K;   /* element width in the reference box */
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m->E; ++e) {
    int ec[3];
    elem_coords(m, e, ec);
    double X[3][NMAX * NMAX * NMAX], dX[3][3][NMAX * NMAX * NMAX], V[3][NMAX * NMAX * NMAX];
    /* node positions: the mapping of the reference-box point of each LGL node */
    for (int node = 0; node < NN; ++node) {
      int idx[3];
      node_idx(m, node, idx);
      double xi[3], P[3];
      for (int d = 0; d < 3; ++d) xi[d] = -1.0 + hr * (ec[d] + 0.5 * (1.0 + m->x[idx[d]]));
      orc_curv_map(c->warp, xi, P);
      for (int d = 0; d < 3; ++d) X[d][node] = P[d];
    }
    /* dX[j][comp][node] = derivative of the interpolant of X_comp along element direction j */
    for (int j = 0; j < 3; ++j)
      for (int comp = 0; comp < 3; ++comp)
        for (int node = 0; node < NN; ++node) {
          int idx[3], pidx[3];
          node_idx(m, node, idx);
          double sum = 0.0;
          for (int mm = 0; mm < n; ++mm) {
            pidx[0] = idx[0]; pidx[1] = idx[1]; pidx[2] = idx[2];
            pidx[j] = mm;
            sum = sum + m->D[idx[j] * n + mm] * X[comp][node_of(m, pidx)];
          }
          dX[j][comp][node] = sum;
        }
    for (int node = 0; node < NN; ++node) {
      double c0 = dX[1][1][node] * dX[2][2][node] - dX[1][2][node] * dX[2][1][node];
      double c1 = dX[1][2][node] * dX[2][0][node] - dX[1][0][node] * dX[2][2][node];
      double c2 = dX[1][0][node] * dX[2][1][node] - dX[1][1][node] * dX[2][0][node];
      c->J[e * NN + node] = dX[0][0][node] * c0 + dX[0][1][node] * c1 + dX[0][2][node] * c2;
    }
    /* conservative curl form: (J a^i)_nc = -[curl_s (X_l grad_s X_m)]_i, (nc, m, l) cyclic */
    for (int nc = 0; nc < 3; ++nc) {
      const int mm_ = (nc + 1) % 3, l = (nc + 2) % 3;
      for (int j = 0; j < 3; ++j)
        for (int node = 0; node < NN; ++node) V[j][node] = X[l][node] * dX[j][mm_][node];
      for (int node = 0; node < NN; ++node) {
        int idx[3];
        node_idx(m, node, idx);
        /* dV[j][k] = derivative of V_k along direction j at this node */
        double dV[3][3];
        for (int j = 0; j < 3; ++j)
          for (int k = 0; k < 3; ++k) {
            double sum = 0.0;
            for (int q2 = 0; q2 < n; ++q2) {
              int pidx[3] = {idx[0], idx[1], idx[2]};
              pidx[j] = q2;
              sum = sum + m->D[idx[j] * n + q2] * V[k][node_of(m, pidx)];
            }
            dV[j][k] = sum;
          }
        const double curl[3] = {dV[1][2] - dV[2][1], dV[2][0] - dV[0][2], dV[0][1] - dV[1][0]};
        for (int i = 0; i < 3; ++i) c->Ja[((int64_t)(i * 3 + nc) * m->E + e) * NN + node] = -curl[i];
      }
    }
    for (int d = 0; d < 3; ++d)
      for (int node = 0; node < NN; ++node) c->xyz[((int64_t)d * m->E + e) * NN + node] = X[d][node];
  }
  return ORC_OK;
}

static void curv_free(curv_t *c)
{
  free(c->xyz);
  free(c->Ja);
  free(c->J);
}

int64_t orc_curv_num_nodes(const orc_curv_config *cfg)
{
  if (!cfg || cfg->cells < 1 || cfg->polydeg < 1 || cfg->polydeg > ORC_MAXN) return -1;
  const int64_t n = cfg->polydeg + 1;
  return (int64_t)cfg->cells * cfg->cells * cfg->cells * n * n * n;
}

int orc_curv_geometry(const orc_curv_config *cfg, double *xyz, double *Ja, double *J)
{
  curv_t c;
  memset(&c, 0, sizeof(c));
  int st = curv_setup(cfg, &c);
  if (st == ORC_OK) {
    const int64_t len = c.m.E * c.m.NN;
    if (xyz) memcpy(xyz, c.xyz, sizeof(double) * 3 * len);
    if (Ja) memcpy(Ja, c.Ja, sizeof(double) * 9 * len);
    if (J) memcpy(J, c.J, sizeof(double) * len);
  }
  curv_free(&c);
  return st;
}

/* Physical flux along a (not necessarily unit) vector nv: sum_k nv_k f^k(u). */
static void flux_along(const double *u, const prim_t *q, const double *nv, double *f)
{
  double fk[5];
  for (int v = 0; v < 5; ++v) f[v] = 0.0;
  for (int k = 0; k < 3; ++k) {
    phys_flux(u, q, k, 3, fk);
    for (int v = 0; v < 5; ++v) f[v] = f[v] + nv[k] * fk[v];
  }
}

/* Two-point volume flux contracted with the averaged metric vector a:
 * sum_n a_n f#_n(L, R) (EC or central f#). */
static void vol_flux_curv(int vol, const double *uL, const prim_t *L, const double *uR,
                          const prim_t *R, const double *a, double gamma, double *f)
{
  double fn[5];
  for (int v = 0; v < 5; ++v) f[v] = 0.0;
  for (int nc = 0; nc < 3; ++nc) {
    if (vol == ORC_VOL_CENTRAL) central_flux(uL, L, uR, R, nc, 3, fn);
    else ec_flux(L, R, nc, 3, gamma, fn);
    for (int v = 0; v < 5; ++v) f[v] = f[v] + a[nc] * fn[v];
  }
}

/* Interface flux through a face whose contravariant vector is nv (pointing from L to R):
 * |nv| f*(uL, uR; nv/|nv|) for LLF and HLL (the Cartesian formulas with v_d -> v.n),
 * sum_n nv_n f#_n(L, R) for the EC flux. */
static void surf_flux_curv(int kind, const double *uL, const prim_t *L, const double *uR,
                           const prim_t *R, const double *nv, double gamma, double *f)
{
  if (kind == ORC_SURF_EC) {
    vol_flux_curv(ORC_VOL_EC, uL, L, uR, R, nv, gamma, f);
    return;
  }
  const double len = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
  const double nh[3] = {nv[0] / len, nv[1] / len, nv[2] / len};
  double fL[5], fR[5];
  flux_along(uL, L, nh, fL);
  flux_along(uR, R, nh, fR);
  const double vnL = L->v[0] * nh[0] + L->v[1] * nh[1] + L->v[2] * nh[2];
  const double vnR = R->v[0] * nh[0] + R->v[1] * nh[1] + R->v[2] * nh[2];
  if (kind == ORC_SURF_LLF) {
    double lL = fabs(vnL) + L->c, lR = fabs(vnR) + R->c;
    double lam = lL > lR ? lL : lR;
    for (int v = 0; v < 5; ++v) f[v] = len * (0.5 * (fL[v] + fR[v]) - 0.5 * lam * (uR[v] - uL[v]));
  } else {
    double a = vnL - L->c, b = vnR - R->c;
    double sL = a < b ? a : b;
    a = vnL + L->c; b = vnR + R->c;
    double sR = a > b ? a : b;
    for (int v = 0; v < 5; ++v) {
      double g;
      if (sL >= 0.0) g = fL[v];
      else if (sR <= 0.0) g = fR[v];
      else g = (sR * fL[v] - sL * fR[v] + sL * sR * (uR[v] - uL[v])) / (sR - sL);
      f[v] = len * g;
    }
  }
}

static void curv_ja(const curv_t *c, int i, int64_t e, int node, double *a)
{
  for (int nc = 0; nc < 3; ++nc) a[nc] = c->Ja[((int64_t)(i * 3 + nc) * c->m.E + e) * c->m.NN + node];
}

/* du = -(1/J) sum_i [ sum_{m != i_i} S_{i_i m} f~#_i(u_node, u_m)
 *                     + ([i_i == N] F~*_{i+} - [i_i == 0] F~*_{i-}) / w_0 ]  + s(x, t)
 * with f~#_i(A, B) = sum_n (Ja^i_n(A) + Ja^i_n(B))/2 f#_n(A, B), F~* the interface flux
 * through the face's contravariant vector Ja^i (the same on both sides of the face). */
static int curv_rhs_core(const orc_curv_config *cfg, const curv_t *c, const double *u, double t,
                         double *du)
{
  const mesh_t *m = &c->m;
  const int n = m->n, N = m->N, NN = m->NN;
  const double gamma = cfg->gamma;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t e = 0; e < m->E; ++e) {
    double ue[NMAX * NMAX * NMAX][5];
    prim_t qe[NMAX * NMAX * NMAX];
    for (int node = 0; node < NN; ++node) {
      load_node(m, u, e, node, ue[node]);
      bad |= to_prim(ue[node], 3, gamma, &qe[node]);
    }
    for (int node = 0; node < NN; ++node) {
      int idx[3];
      node_idx(m, node, idx);
      double acc[5] = {0, 0, 0, 0, 0}, f[5];
      for (int i = 0; i < 3; ++i) {
        const int id = idx[i];
        double ai[3];
        curv_ja(c, i, e, node, ai);
        if (cfg->volume != ORC_VOL_NONE) {
          for (int mm = 0; mm < n; ++mm) {
            if (mm == id) continue;
            int pidx[3] = {idx[0], idx[1], idx[2]};
            pidx[i] = mm;
            const int pn = node_of(m, pidx);
            double ap[3], abar[3];
            curv_ja(c, i, e, pn, ap);
            for (int k = 0; k < 3; ++k) abar[k] = 0.5 * (ai[k] + ap[k]);
            vol_flux_curv(cfg->volume, ue[node], &qe[node], ue[pn], &qe[pn], abar, gamma, f);
            for (int v = 0; v < 5; ++v) acc[v] = acc[v] + m->S[id * n + mm] * f[v];
          }
        }
        if (cfg->surface != ORC_SURF_NONE && (id == 0 || id == N)) {
          int pidx[3] = {idx[0], idx[1], idx[2]};
          double un[5];
          prim_t qn;
          if (id == N) {
            pidx[i] = 0;
            load_node(m, u, neighbour(m, e, i, +1), node_of(m, pidx), un);
            bad |= to_prim(un, 3, gamma, &qn);
            surf_flux_curv(cfg->surface, ue[node], &qe[node], un, &qn, ai, gamma, f);
            for (int v = 0; v < 5; ++v) acc[v] = acc[v] + f[v] / m->w[N];
          }
          if (id == 0) {
            pidx[i] = N;
            load_node(m, u, neighbour(m, e, i, -1), node_of(m, pidx), un);
            bad |= to_prim(un, 3, gamma, &qn);
            surf_flux_curv(cfg->surface, un, &qn, ue[node], &qe[node], ai, gamma, f);
            for (int v = 0; v < 5; ++v) acc[v] = acc[v] - f[v] / m->w[0];
          }
        }
      }
      const double Jn = c->J[e * NN + node];
      double s[5] = {0, 0, 0, 0, 0};
      if (cfg->source == ORC_SRC_MMS) {
        double x[3];
        for (int d = 0; d < 3; ++d) x[d] = c->xyz[((int64_t)d * m->E + e) * NN + node];
        orc_curv_mms(gamma, x, t, NULL, s);
      }
      for (int v = 0; v < 5; ++v) du[((int64_t)v * m->E + e) * NN + node] = -acc[v] / Jn + s[v];
    }
  }
  return bad ? ORC_ENONPHYS : ORC_OK;
}

int orc_curv_rhs(const orc_curv_config *cfg, const double *u, double t, double *du)
{
  curv_t c;
  memset(&c, 0, sizeof(c));
  int st = curv_setup(cfg, &c);
  if (st == ORC_OK) st = curv_rhs_core(cfg, &c, u, t, du);
  curv_free(&c);
  return st;
}

int orc_curv_initial(const orc_curv_config *cfg, double t, double *u)
{
  curv_t c;
  memset(&c, 0, sizeof(c));
  int st = curv_setup(cfg, &c);
  if (st == ORC_OK) {
    const int64_t len = c.m.E * c.m.NN;
    for (int64_t i = 0; i < len; ++i) {
      double x[3] = {c.xyz[i], c.xyz[len + i], c.xyz[2 * len + i]}, un[5];
      orc_curv_mms(cfg->gamma, x, t, un, NULL);
      for (int v = 0; v < 5; ++v) u[v * len + i] = un[v];
    }
  }
  curv_free(&c);
  return st;
}

/* dt = cfl 2 / ((N+1) max_e sum_i max_{nodes} (|Ja^i . v| + c |Ja^i|) / J): the Cartesian
 * rule with 2/h_d (|v_d| + c) replaced by its contravariant counterpart. */
static int curv_max_dt_core(const orc_curv_config *cfg, const curv_t *c, const double *u,
                            double cfl, double *dt)
{
  const mesh_t *m = &c->m;
  const int NN = m->NN;
  double lmax = 0.0;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(max : lmax) reduction(| : bad)
  for (int64_t e = 0; e < m->E; ++e) {
    double lam = 0.0;
    for (int i = 0; i < 3; ++i) {
      double mx = 0.0;
      for (int node = 0; node < NN; ++node) {
        double un[5], a[3];
        prim_t q;
        load_node(m, u, e, node, un);
        bad |= to_prim(un, 3, cfg->gamma, &q);
        curv_ja(c, i, e, node, a);
        const double an = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
        const double va = q.v[0] * a[0] + q.v[1] * a[1] + q.v[2] * a[2];
        const double l = (fabs(va) + q.c * an) / c->J[e * NN + node];
        if (l > mx) mx = l;
      }
      lam = lam + mx;
    }
    if (lam > lmax) lmax = lam;
  }
  *dt = cfl * 2.0 / ((m->N + 1) * lmax);
  return bad ? ORC_ENONPHYS : ORC_OK;
}

int orc_curv_max_dt(const orc_curv_config *cfg, const double *u, double cfl, double *dt)
{
  curv_t c;
  memset(&c, 0, sizeof(c));
  int st = curv_setup(cfg, &c);
  if (st == ORC_OK) st = curv_max_dt_core(cfg, &c, u, cfl, dt);
  curv_free(&c);
  return st;
}

/* CK(5,4) with stage times t + c_s dt for the time-dependent source. */
int orc_curv_step(const orc_curv_config *cfg, double *u, int32_t nsteps, double cfl,
                  double dt_fixed, double *t)
{
  curv_t c;
  memset(&c, 0, sizeof(c));
  int st = curv_setup(cfg, &c);
  if (st) {
    curv_free(&c);
    return st;
  }
  const int64_t len = 5 * c.m.E * c.m.NN;
  double *k = calloc(len, sizeof(double)), *du = malloc(sizeof(double) * len);
  double A[5], B[5], cs[5];
  orc_lsrk_coeffs(A, B, cs);
  double tt = t ? *t : 0.0;
  for (int step = 0; step < nsteps && st == ORC_OK; ++step) {
    double dt = dt_fixed;
    if (cfl > 0.0) st = curv_max_dt_core(cfg, &c, u, cfl, &dt);
    for (int s = 0; s < 5 && st == ORC_OK; ++s) {
      st = curv_rhs_core(cfg, &c, u, tt + cs[s] * dt, du);
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < len; ++i) {
        k[i] = A[s] * k[i] + dt * du[i];
        u[i] = u[i] + B[s] * k[i];
      }
    }
    tt = tt + dt;
  }
  if (t) *t = tt;
  free(k);
  free(du);
  curv_free(&c);
  return st;
}

/* ========================================================================= */
/* Ideal MHD (the PID study's second system, Section 3.1): weak-form DGSEM     */
/* with the HLL interface flux on the periodic Cartesian box, 8 variables      */
/* u = (rho, rho v, E, B), mu_0 = 1, no divergence cleaning.                   */
/* ========================================================================= */

typedef struct { double rho, v[3], p, B[3], pt, c2, b2; } mhd_prim_t;

/* p = (gamma-1)(E - rho |v|^2/2 - |B|^2/2), total pressure pt = p + |B|^2/2. */
static int mhd_to_prim(const double *u, double gamma, mhd_prim_t *q)
{
  q->rho = u[0];
  double v2 = 0.0, B2 = 0.0;
  for (int k = 0; k < 3; ++k) {
    q->v[k] = u[1 + k] / u[0];
    q->B[k] = u[5 + k];
    v2 = v2 + q->v[k] * q->v[k];
    B2 = B2 + q->B[k] * q->B[k];
  }
  q->p = (gamma - 1.0) * (u[4] - 0.5 * u[0] * v2 - 0.5 * B2);
  q->pt = q->p + 0.5 * B2;
  q->c2 = gamma * q->p / q->rho;   /* sound speed squared */
  q->b2 = B2 / q->rho;             /* Alfven speed squared (|B|^2 / rho) */
  if (!(q->rho > 0.0) || !(q->p > 0.0) || !isfinite(q->rho) || !isfinite(q->p)) return 1;
  return 0;
}

/* f^d(u) = (rho v_d, rho v_d v + pt e_d - B_d B, v_d (E + pt) - B_d (v.B), v_d B - B_d v). */
static void mhd_flux(const double *u, const mhd_prim_t *q, int d, double *f)
{
  const double vB = q->v[0] * q->B[0] + q->v[1] * q->B[1] + q->v[2] * q->B[2];
  f[0] = u[1 + d];
  for (int k = 0; k < 3; ++k) f[1 + k] = u[1 + d] * q->v[k] + (k == d ? q->pt : 0.0) - q->B[d] * q->B[k];
  f[4] = q->v[d] * (u[4] + q->pt) - q->B[d] * vB;
  for (int k = 0; k < 3; ++k) f[5 + k] = q->v[d] * q->B[k] - q->B[d] * q->v[k];
}

/* fast magnetosonic speed along d: c_f^2 = (a^2 + b^2 + sqrt((a^2 + b^2)^2 - 4 a^2 b_d^2))/2
 * with a^2 = gamma p / rho, b^2 = |B|^2 / rho, b_d^2 = B_d^2 / rho. */
static double mhd_cf(const mhd_prim_t *q, int d)
{
  const double s = q->c2 + q->b2, bd2 = q->B[d] * q->B[d] / q->rho;
  double disc = s * s - 4.0 * q->c2 * bd2;
  if (disc < 0.0) disc = 0.0;
  return sqrt(0.5 * (s + sqrt(disc)));
}

/* HLL with s_L = min(v_dL - c_fL, v_dR - c_fR), s_R = max(v_dL + c_fL, v_dR + c_fR). */
static void mhd_hll(const double *uL, const mhd_prim_t *L, const double *uR, const mhd_prim_t *R,
                    int d, double *f)
{
  double fL[8], fR[8];
  mhd_flux(uL, L, d, fL);
  mhd_flux(uR, R, d, fR);
  const double cL = mhd_cf(L, d), cR = mhd_cf(R, d);
  double a = L->v[d] - cL, b = R->v[d] - cR;
  const double sL = a < b ? a : b;
  a = L->v[d] + cL; b = R->v[d] + cR;
  const double sR = a > b ? a : b;
  for (int v = 0; v < 8; ++v) {
    if (sL >= 0.0) f[v] = fL[v];
    else if (sR <= 0.0) f[v] = fR[v];
    else f[v] = (sR * fL[v] - sL * fR[v] + sL * sR * (uR[v] - uL[v])) / (sR - sL);
  }
}

/* LLF with lambda = max(|v_dL| + c_fL, |v_dR| + c_fR). */
static void mhd_llf(const double *uL, const mhd_prim_t *L, const double *uR, const mhd_prim_t *R,
                    int d, double *f)
{
  double fL[8], fR[8];
  mhd_flux(uL, L, d, fL);
  mhd_flux(uR, R, d, fR);
  const double lL = fabs(L->v[d]) + mhd_cf(L, d), lR = fabs(R->v[d]) + mhd_cf(R, d);
  const double lam = lL > lR ? lL : lR;
  for (int v = 0; v < 8; ++v) f[v] = 0.5 * (fL[v] + fR[v]) - 0.5 * lam * (uR[v] - uL[v]);
}

/* Entropy-conservative two-point flux of ideal MHD along d, with the Powell term
 * phi(u) = (0, B, v.B, v) discretised as phi(u_i) {{B_d}}:  with beta = rho/(2p) the
 * entropy condition  [[w]].f* + {{B_d}} [[w.phi]] = [[rho v_d + beta v_d |B|^2]]  and the
 * discrete product rules give (averages {{a}} = (a_L + a_R)/2, log means of rho and beta)
 *   f_rho = rho_ln {{v_d}}
 *   f_rhov = f_rho {{v}} - {{B_d}} {{B}} + e_d ({{rho}}/(2 {{beta}}) + {{|B|^2}}/2)
 *   f_B   = ({{beta v_d}}/{{beta}}) {{B}} - {{B_d}} {{v}}
 *   f_E   = f_rho (1/(2(gamma-1) beta_ln) - {{|v|^2}}/2) + {{v}}.f_rhov + {{B}}.f_B
 *           + {{B_d}} {{v.B}} - {{|B|^2}} {{v_d}}/2. */
static void mhd_ec_flux(const mhd_prim_t *L, const mhd_prim_t *R, int d, double gamma, double *f)
{
  const double bL = L->rho / (2.0 * L->p), bR = R->rho / (2.0 * R->p);
  const double rho_ln = orc_ln_mean(L->rho, R->rho), beta_ln = orc_ln_mean(bL, bR);
  const double rho_a = 0.5 * (L->rho + R->rho), beta_a = 0.5 * (bL + bR);
  double va[3], Ba[3], v2L = 0.0, v2R = 0.0, B2L = 0.0, B2R = 0.0, vBL = 0.0, vBR = 0.0;
  for (int k = 0; k < 3; ++k) {
    va[k] = 0.5 * (L->v[k] + R->v[k]);
    Ba[k] = 0.5 * (L->B[k] + R->B[k]);
    v2L = v2L + L->v[k] * L->v[k];
    v2R = v2R + R->v[k] * R->v[k];
    B2L = B2L + L->B[k] * L->B[k];
    B2R = B2R + R->B[k] * R->B[k];
    vBL = vBL + L->v[k] * L->B[k];
    vBR = vBR + R->v[k] * R->B[k];
  }
  const double v2a = 0.5 * (v2L + v2R), B2a = 0.5 * (B2L + B2R), vBa = 0.5 * (vBL + vBR);
  const double bva = 0.5 * (bL * L->v[d] + bR * R->v[d]);
  const double fr = rho_ln * va[d];
  const double pt = rho_a / (2.0 * beta_a) + 0.5 * B2a;
  f[0] = fr;
  for (int k = 0; k < 3; ++k) {
    f[1 + k] = fr * va[k] - Ba[d] * Ba[k] + (k == d ? pt : 0.0);
    f[5 + k] = (bva / beta_a) * Ba[k] - Ba[d] * va[k];
  }
  double e = fr * (1.0 / (2.0 * (gamma - 1.0) * beta_ln) - 0.5 * v2a);
  for (int k = 0; k < 3; ++k) e = e + va[k] * f[1 + k] + Ba[k] * f[5 + k];
  f[4] = e + Ba[d] * vBa - 0.5 * B2a * va[d];
}

/* Powell's non-conservative term's coefficient phi(u) = (0, B, v.B, v). */
static void mhd_phi(const mhd_prim_t *q, double *phi)
{
  phi[0] = 0.0;
  double vB = 0.0;
  for (int k = 0; k < 3; ++k) {
    phi[1 + k] = q->B[k];
    phi[5 + k] = q->v[k];
    vB = vB + q->v[k] * q->B[k];
  }
  phi[4] = vB;
}

static void mhd_face_flux(int kind, const double *uL, const mhd_prim_t *L, const double *uR,
                          const mhd_prim_t *R, int d, double gamma, double *f)
{
  if (kind == ORC_SURF_HLL) mhd_hll(uL, L, uR, R, d, f);
  else if (kind == ORC_SURF_LLF) mhd_llf(uL, L, uR, R, d, f);
  else mhd_ec_flux(L, R, d, gamma, f);
}

/* S(u) = -rho s/(gamma-1), s = ln p - gamma ln rho; w = dS/du =
 * ((gamma - s)/(gamma-1) - beta |v|^2, 2 beta v, -2 beta, 2 beta B), beta = rho/(2p). */
double orc_mhd_entropy(const double *u, double gamma)
{
  mhd_prim_t q;
  mhd_to_prim(u, gamma, &q);
  return -q.rho * (log(q.p) - gamma * log(q.rho)) / (gamma - 1.0);
}

int orc_mhd_entropy_vars(const double *u, double gamma, double *w)
{
  mhd_prim_t q;
  int bad = mhd_to_prim(u, gamma, &q);
  const double s = log(q.p) - gamma * log(q.rho), beta = q.rho / (2.0 * q.p);
  double v2 = 0.0;
  for (int k = 0; k < 3; ++k) v2 = v2 + q.v[k] * q.v[k];
  w[0] = (gamma - s) / (gamma - 1.0) - beta * v2;
  for (int k = 0; k < 3; ++k) {
    w[1 + k] = 2.0 * beta * q.v[k];
    w[5 + k] = 2.0 * beta * q.B[k];
  }
  w[4] = -2.0 * beta;
  return bad ? ORC_ENONPHYS : ORC_OK;
}

int orc_mhd_ec_flux(const double *uL, const double *uR, int d, double gamma, double *f)
{
  mhd_prim_t L, R;
  int bad = mhd_to_prim(uL, gamma, &L) | mhd_to_prim(uR, gamma, &R);
  mhd_ec_flux(&L, &R, d, gamma, f);
  return bad ? ORC_ENONPHYS : ORC_OK;
}

int orc_mhd_flux(const double *u, int d, double gamma, double *f)
{
  mhd_prim_t q;
  int bad = mhd_to_prim(u, gamma, &q);
  mhd_flux(u, &q, d, f);
  return bad ? ORC_ENONPHYS : ORC_OK;
}

int orc_mhd_surface_flux(int kind, const double *uL, const double *uR, int d, double gamma,
                         double *f)
{
  mhd_prim_t L, R;
  int bad = mhd_to_prim(uL, gamma, &L) | mhd_to_prim(uR, gamma, &R);
  mhd_face_flux(kind, uL, &L, uR, &R, d, gamma, f);
  return bad ? ORC_ENONPHYS : ORC_OK;
}

double orc_mhd_fast_speed(const double *u, int d, double gamma)
{
  mhd_prim_t q;
  mhd_to_prim(u, gamma, &q);
  return mhd_cf(&q, d);
}

static int mhd_setup(const orc_mhd_config *cfg, mesh_t *m)
{
  if (!cfg || cfg->cells < 1) return ORC_EINVAL;
  if (cfg->volume != ORC_VOL_WEAK && cfg->volume != ORC_VOL_EC) return ORC_EINVAL;
  if (cfg->surface != ORC_SURF_HLL && cfg->surface != ORC_SURF_LLF &&
      !(cfg->surface == ORC_SURF_EC && cfg->volume == ORC_VOL_EC))
    return ORC_EINVAL;
  orc_config q;
  memset(&q, 0, sizeof(q));
  q.dim = 3;
  q.polydeg = cfg->polydeg;
  for (int d = 0; d < 3; ++d) {
    q.cells[d] = cfg->cells;
    q.xmin[d] = -1.0;
    q.xmax[d] = 1.0;
  }
  q.gamma = cfg->gamma;
  return setup(&q, m);
}

int64_t orc_mhd_num_nodes(const orc_mhd_config *cfg)
{
  mesh_t m;
  if (mhd_setup(cfg, &m)) return -1;
  return m.E * m.NN;
}

/* Weak form: du = (2/h) sum_d [ sum_m Dhat_{i_d m} f^d(u_m)
 *                              - ([i_d == N] f*_{d+} - [i_d == 0] f*_{d-}) / w_0 ];
 * flux differencing (volume ORC_VOL_EC): du = -(2/h) sum_d [ sum_{m != i_d} S_{i_d m}
 *   (f*(u, u_m) + phi(u) {{B_d}}) + ([i_d == N] g_{d+} - [i_d == 0] g_{d-}) / w_0 ] with the
 *   face terms g = F*(u_L, u_R) + phi(u) {{B_d}} (phi of the node's own state);
 * u laid out [8][E][NN] on the Cartesian box [-1,1]^3 (cells^3 elements). */
int orc_mhd_rhs(const orc_mhd_config *cfg, const double *u, double *du)
{
  mesh_t m;
  int st = mhd_setup(cfg, &m);
  if (st) return st;
  const int n = m.n, N = m.N, NN = m.NN;
  const double gamma = cfg->gamma;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t e = 0; e < m.E; ++e) {
    double ue[NMAX * NMAX * NMAX][8];
    mhd_prim_t qe[NMAX * NMAX * NMAX];
    for (int node = 0; node < NN; ++node) {
      for (int v = 0; v < 8; ++v) ue[node][v] = u[((int64_t)v * m.E + e) * NN + node];
      bad |= mhd_to_prim(ue[node], gamma, &qe[node]);
    }
    for (int node = 0; node < NN; ++node) {
      int idx[3];
      node_idx(&m, node, idx);
      double R[8] = {0, 0, 0, 0, 0, 0, 0, 0}, f[8];
      for (int d = 0; d < 3; ++d) {
        const int id = idx[d];
        double V[8] = {0, 0, 0, 0, 0, 0, 0, 0}, phi[8];
        mhd_phi(&qe[node], phi);
        for (int mm = 0; mm < n; ++mm) {
          int pidx[3] = {idx[0], idx[1], idx[2]};
          pidx[d] = mm;
          const int pn = node_of(&m, pidx);
          if (cfg->volume == ORC_VOL_WEAK) {
            mhd_flux(ue[pn], &qe[pn], d, f);
            for (int v = 0; v < 8; ++v) V[v] = V[v] + m.Dhat[id * n + mm] * f[v];
          } else if (mm != id) {
            /* flux differencing: -(S_im (f*(u_i, u_m) + phi(u_i) {{B_d}})) */
            mhd_ec_flux(&qe[node], &qe[pn], d, gamma, f);
            const double Bm = 0.5 * (qe[node].B[d] + qe[pn].B[d]);
            for (int v = 0; v < 8; ++v) V[v] = V[v] - m.S[id * n + mm] * (f[v] + phi[v] * Bm);
          }
        }
        double Sf[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (id == N || id == 0) {
          int pidx[3] = {idx[0], idx[1], idx[2]};
          pidx[d] = (id == N) ? 0 : N;
          const int64_t nb = neighbour(&m, e, d, id == N ? +1 : -1);
          const int pn = node_of(&m, pidx);
          double un[8];
          mhd_prim_t qn;
          for (int v = 0; v < 8; ++v) un[v] = u[((int64_t)v * m.E + nb) * NN + pn];
          bad |= mhd_to_prim(un, gamma, &qn);
          /* flux differencing adds the non-conservative face term phi(u_i) {{B_d}} */
          const double Bf = cfg->volume == ORC_VOL_EC ? 0.5 * (qe[node].B[d] + qn.B[d]) : 0.0;
          if (id == N) {
            mhd_face_flux(cfg->surface, ue[node], &qe[node], un, &qn, d, gamma, f);
            for (int v = 0; v < 8; ++v) Sf[v] = Sf[v] + (f[v] + phi[v] * Bf) / m.w[N];
          }
          if (id == 0) {
            mhd_face_flux(cfg->surface, un, &qn, ue[node], &qe[node], d, gamma, f);
            for (int v = 0; v < 8; ++v) Sf[v] = Sf[v] - (f[v] + phi[v] * Bf) / m.w[0];
          }
        }
        for (int v = 0; v < 8; ++v) R[v] = R[v] + (2.0 / m.h[d]) * (V[v] - Sf[v]);
      }
      for (int v = 0; v < 8; ++v) du[((int64_t)v * m.E + e) * NN + node] = R[v];
    }
  }
  return bad ? ORC_ENONPHYS : ORC_OK;
}

/* dt = cfl 2 / ((N+1) max_e sum_d (2/h) max_nodes (|v_d| + c_f,d)). */
int orc_mhd_max_dt(const orc_mhd_config *cfg, const double *u, double cfl, double *dt)
{
  mesh_t m;
  int st = mhd_setup(cfg, &m);
  if (st) return st;
  const int NN = m.NN;
  double lmax = 0.0;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(max : lmax) reduction(| : bad)
  for (int64_t e = 0; e < m.E; ++e) {
    double lam = 0.0;
    for (int d = 0; d < 3; ++d) {
      double mx = 0.0;
      for (int node = 0; node < NN; ++node) {
        double un[8];
        mhd_prim_t q;
        for (int v = 0; v < 8; ++v) un[v] = u[((int64_t)v * m.E + e) * NN + node];
        bad |= mhd_to_prim(un, cfg->gamma, &q);
        const double l = fabs(q.v[d]) + mhd_cf(&q, d);
        if (l > mx) mx = l;
      }
      lam = lam + (2.0 / m.h[d]) * mx;
    }
    if (lam > lmax) lmax = lam;
  }
  *dt = cfl * 2.0 / ((m.N + 1) * lmax);
  return bad ? ORC_ENONPHYS : ORC_OK;
}

int orc_mhd_step(const orc_mhd_config *cfg, double *u, int32_t nsteps, double cfl,
                 double dt_fixed, double *t)
{
  const int64_t nodes = orc_mhd_num_nodes(cfg);
  if (nodes < 0) return ORC_EINVAL;
  const int64_t len = 8 * nodes;
  double *k = calloc(len, sizeof(double)), *du = malloc(sizeof(double) * len);
  double A[5], B[5];
  orc_lsrk_coeffs(A, B, NULL);
  int st = ORC_OK;
  for (int step = 0; step < nsteps && st == ORC_OK; ++step) {
    double dt = dt_fixed;
    if (cfl > 0.0) st = orc_mhd_max_dt(cfg, u, cfl, &dt);
    for (int s = 0; s < 5 && st == ORC_OK; ++s) {
      st = orc_mhd_rhs(cfg, u, du);
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < len; ++i) {
        k[i] = A[s] * k[i] + dt * du[i];
        u[i] = u[i] + B[s] * k[i];
      }
    }
    if (t) *t = *t + dt;
  }
  free(k);
  free(du);
  return st;
}

/* Circularly polarised Alfven wave along e1 = (1,1,1)/sqrt 3 with wave vector k = pi (1,1,1)
 * (period 2 in every direction): rho = 1, p = 0.1, B = B0 e1 + eps (cos phi e2 + sin phi e3),
 * v = -(eps / sqrt rho)(cos phi e2 + sin phi e3), phi = k.x - |k| c_a t, c_a = B0/sqrt(rho),
 * B0 = 1, eps = 0.1; e2 = (1,-1,0)/sqrt 2, e3 = e1 x e2.  An exact solution of ideal MHD. */
int orc_mhd_alfven(double gamma, const double *x, double t, double *u)
{
  const double pi = 3.14159265358979323846;
  const double rho = 1.0, p = 0.1, B0 = 1.0, eps = 0.1;
  const double r3 = sqrt(3.0), r2 = sqrt(2.0), r6 = sqrt(6.0);
  const double e1[3] = {1.0 / r3, 1.0 / r3, 1.0 / r3};
  const double e2[3] = {1.0 / r2, -1.0 / r2, 0.0};
  const double e3[3] = {1.0 / r6, 1.0 / r6, -2.0 / r6};   /* e1 x e2 */
  const double ca = B0 / sqrt(rho);
  const double phi = pi * (x[0] + x[1] + x[2]) - pi * r3 * ca * t;
  const double c = cos(phi), s = sin(phi);
  double v[3], B[3], v2 = 0.0, B2 = 0.0;
  for (int k = 0; k < 3; ++k) {
    B[k] = B0 * e1[k] + eps * (c * e2[k] + s * e3[k]);
    v[k] = -(eps / sqrt(rho)) * (c * e2[k] + s * e3[k]);
    v2 = v2 + v[k] * v[k];
    B2 = B2 + B[k] * B[k];
  }
  u[0] = rho;
  for (int k = 0; k < 3; ++k) u[1 + k] = rho * v[k];
  u[4] = p / (gamma - 1.0) + 0.5 * rho * v2 + 0.5 * B2;
  for (int k = 0; k < 3; ++k) u[5 + k] = B[k];
  return ORC_OK;
}
