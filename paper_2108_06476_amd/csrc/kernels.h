// kernels.h -- gfx950 kernels of the DGSEM right-hand side, templated on the space
// dimension and the polynomial degree.  Included by the per-dimension translation
// units, which instantiate them and register host launchers.
//
// Data in HBM (float64, structure of arrays):
//   u[var][elem][node]              state, node = i + n (j + n k)
//   F[dir][var][elem][face node]    interface flux on the minus face of elem
//   tab                             per-handle operator tables (layout: TAB_* below)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "physics.h"

namespace dgx {

// Table layout (doubles), fixed strides for polydeg <= 7 (8 nodes per direction).
constexpr int TMAX = 8;
constexpr int TAB_S = 0;                           // [3][8][8]  -(2/h_d) S_im, S = 2D - M^-1 B
constexpr int TAB_LIFT = TAB_S + 3 * TMAX * TMAX;  // [3][2]     +(2/h_d)/w_0, -(2/h_d)/w_N
constexpr int TAB_FV = TAB_LIFT + 6;               // [3][8]     -(2/h_d)/w_i
constexpr int TAB_VINV = TAB_FV + 3 * TMAX;        // [8][8]     orthonormal-Legendre V^-1
constexpr int TAB_W = TAB_VINV + TMAX * TMAX;      // [8]        LGL weights
constexpr int TAB_X = TAB_W + TMAX;                // [8]        LGL nodes
constexpr int TAB_JAC = TAB_X + TMAX;              // [3]        2/h_d
constexpr int TAB_SIZE = TAB_JAC + 3;

enum { VOL_EC = 0, VOL_CENTRAL = 1, VOL_SHOCKCAP = 2, VOL_NONE = 4 };
enum { EPI_RHS = 0, EPI_RK = 1 };

template <int DIM, int N>
struct Shape {
  static constexpr int n = N + 1;
  static constexpr int NN = DIM == 3 ? n * n * n : n * n;  // nodes per element
  static constexpr int NF = DIM == 3 ? n * n : n;          // nodes per face
  static constexpr int NV = DIM + 2;
  static constexpr int NE = NN >= 256 ? 1 : 256 / NN;      // elements per block
  static constexpr int THREADS = ((NE * NN + 63) / 64) * 64;
};

template <int D, int n>
struct Stride {
  static constexpr int value = D == 0 ? 1 : (D == 1 ? n : n * n);
};

struct Geom {
  int64_t E;
  int K[3];
  double gamma;
  const double* tab;
  int* flag;   // set to 1 when a non-physical state is met
};

__device__ __forceinline__ int64_t neighbour(const Geom& g, int64_t e, int d, int s) {
  int c0 = (int)(e % g.K[0]);
  int64_t r = e / g.K[0];
  int c1 = (int)(r % g.K[1]);
  int c2 = (int)(r / g.K[1]);
  if (d == 0) c0 = (c0 + s + g.K[0]) % g.K[0];
  else if (d == 1) c1 = (c1 + s + g.K[1]) % g.K[1];
  else c2 = (c2 + s + g.K[2]) % g.K[2];
  return c0 + (int64_t)g.K[0] * (c1 + (int64_t)g.K[1] * c2);
}

template <int n, int D>
__device__ __forceinline__ int face_index(int node) {
  constexpr int st = Stride<D, n>::value;
  return (node % st) + (node / (st * n)) * st;
}

// --------------------------------------------------------------------------------------
// Interface flux: one thread per (direction, element, face node).  F[d][v][e][f] is the
// numerical flux between the minus neighbour e-d (left) and e (right).
// --------------------------------------------------------------------------------------
template <int DIM, int N, int SURF, int D>
__device__ __forceinline__ void surface_one(const double* __restrict__ u, double* __restrict__ F,
                                            const Geom& g, int64_t e, int f) {
  using S = Shape<DIM, N>;
  constexpr int n = S::n, st = Stride<D, n>::value;
  const int64_t eL = neighbour(g, e, D, -1);
  // node with index_D = 0 and face index f, and its partner with index_D = N
  const int nodeR = (f % st) + (f / st) * st * n;
  const int nodeL = nodeR + N * st;
  const int64_t ENN = g.E * S::NN;
  double uL[DIM + 2], uR[DIM + 2];
#pragma unroll
  for (int v = 0; v < DIM + 2; ++v) {
    uL[v] = u[v * ENN + eL * S::NN + nodeL];
    uR[v] = u[v * ENN + e * S::NN + nodeR];
  }
  Prim<double> L, R;
  const bool okL = cons_to_prim<DIM>(uL, g.gamma, L);
  const bool okR = cons_to_prim<DIM>(uR, g.gamma, R);
  if (!(okL && okR)) *g.flag = 1;
  double fs[DIM + 2];
  surface_flux<DIM, D, SURF>(uL, L, uR, R, g.gamma, fs);
  const int64_t EF = g.E * S::NF;
#pragma unroll
  for (int v = 0; v < DIM + 2; ++v) F[((int64_t)D * (DIM + 2) + v) * EF + e * S::NF + f] = fs[v];
}

template <int DIM, int N, int SURF>
__global__ __launch_bounds__(256) void k_surface(const double* __restrict__ u,
                                                 double* __restrict__ F, Geom g) {
  using S = Shape<DIM, N>;
  const int64_t EF = g.E * S::NF;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= DIM * EF) return;
  const int d = (int)(gid / EF);
  const int64_t r = gid - d * EF;
  const int64_t e = r / S::NF;
  const int f = (int)(r - e * S::NF);
  if (d == 0) surface_one<DIM, N, SURF, 0>(u, F, g, e, f);
  else if (d == 1) surface_one<DIM, N, SURF, 1>(u, F, g, e, f);
  else if constexpr (DIM == 3) surface_one<DIM, N, SURF, 2>(u, F, g, e, f);
}

// --------------------------------------------------------------------------------------
// Volume term + surface lift + Jacobian (+ low-storage RK stage), one thread per node,
// Shape::NE elements per block staged in LDS.
//
//   R = sum_d [ -(2/h_d) sum_{m != i_d} S_{i_d m} f#(u, u_m) ]                (DG part)
//   R = (1 - alpha) R_DG + alpha sum_d [ -(2/h_d) (F_{i+1/2} - F_{i-1/2}) / w_i ]
//       + (2/h_d)/w_0 F_minus [i_d == 0] - (2/h_d)/w_N F_plus [i_d == N]       (lift)
// Epilogue: RHS: du = R.  RK: k = A k + dt R; u = u + B k (u read and written by the
// same thread; the interface fluxes were computed from u beforehand).
// --------------------------------------------------------------------------------------
template <typename RT, int DIM, int NE_NN, bool CONS>
struct VolLds {
  RT rho[NE_NN], v[DIM][NE_NN], p[NE_NN], beta[NE_NN];
  double u[CONS ? DIM + 2 : 1][CONS ? NE_NN : 1];
};

template <int DIM, int N, int D, int VOL, typename RT, typename L>
__device__ __forceinline__ void volume_dir(const L& s, int base, int node, const Prim<RT>& me,
                                           const double (&ume)[DIM + 2], const double* sS,
                                           RT inv_gm1, RT (&acc)[DIM + 2]) {
  constexpr int n = N + 1, st = Stride<D, n>::value;
  const int id = (node / st) % n;
  const int nb = base + node - id * st;
#pragma unroll
  for (int sft = 1; sft <= N; ++sft) {
    int m = id + sft;
    if (m >= n) m -= n;
    const int pn = nb + m * st;
    Prim<RT> q;
    q.rho = s.rho[pn];
#pragma unroll
    for (int k = 0; k < DIM; ++k) q.v[k] = s.v[k][pn];
    q.p = s.p[pn];
    q.beta = s.beta[pn];
    RT f[DIM + 2];
    if constexpr (VOL == VOL_CENTRAL) {
      double uq[DIM + 2], fd[DIM + 2];
      Prim<double> qd;
#pragma unroll
      for (int v = 0; v < DIM + 2; ++v) uq[v] = s.u[v][pn];
      qd.rho = q.rho;
#pragma unroll
      for (int k = 0; k < 3; ++k) qd.v[k] = k < DIM ? (double)q.v[k] : 0.0;
      qd.p = q.p;
      Prim<double> med;
      med.rho = me.rho;
#pragma unroll
      for (int k = 0; k < 3; ++k) med.v[k] = k < DIM ? (double)me.v[k] : 0.0;
      med.p = me.p;
      central_flux<DIM, D>(ume, med, uq, qd, fd);
#pragma unroll
      for (int v = 0; v < DIM + 2; ++v) f[v] = (RT)fd[v];
    } else {
      ec_flux<DIM, D, RT>(me, q, inv_gm1, f);
    }
    const RT c = (RT)sS[(D * TMAX + id) * TMAX + m];
#pragma unroll
    for (int v = 0; v < DIM + 2; ++v) acc[v] += c * f[v];
  }
}

// First-order FV on the LGL subcells in direction D with the fv flux (LLF or HLL):
// acc += -(2/h_d)/w_i (F_{i+1/2} - F_{i-1/2}), element-boundary subcell fluxes zero.
template <int DIM, int N, int D, int FVF, typename L>
__device__ __forceinline__ void fv_dir(const L& s, int base, int node, const Prim<double>& me,
                                       const double (&ume)[DIM + 2], const double* sFV,
                                       double gamma, double (&acc)[DIM + 2]) {
  constexpr int n = N + 1, st = Stride<D, n>::value;
  const int id = (node / st) % n;
  double Fp[DIM + 2], Fm[DIM + 2];
#pragma unroll
  for (int v = 0; v < DIM + 2; ++v) { Fp[v] = 0.0; Fm[v] = 0.0; }
  auto load = [&](int pn, double (&uq)[DIM + 2], Prim<double>& q) {
#pragma unroll
    for (int v = 0; v < DIM + 2; ++v) uq[v] = s.u[v][pn];
    q.rho = s.rho[pn];
    q.v[0] = q.v[1] = q.v[2] = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) q.v[k] = s.v[k][pn];
    q.p = s.p[pn];
    q.beta = s.beta[pn];
  };
  if (id < N) {
    double uq[DIM + 2];
    Prim<double> q;
    load(base + node + st, uq, q);
    surface_flux<DIM, D, FVF>(ume, me, uq, q, gamma, Fp);
  }
  if (id > 0) {
    double uq[DIM + 2];
    Prim<double> q;
    load(base + node - st, uq, q);
    surface_flux<DIM, D, FVF>(uq, q, ume, me, gamma, Fm);
  }
  const double c = sFV[D * TMAX + id];
#pragma unroll
  for (int v = 0; v < DIM + 2; ++v) acc[v] += c * (Fp[v] - Fm[v]);
}

template <int DIM, int N, int D>
__device__ __forceinline__ void lift_dir(const double* __restrict__ F, const Geom& g, int64_t e,
                                         int node, const double* sL, double (&R)[DIM + 2]) {
  using S = Shape<DIM, N>;
  constexpr int n = S::n, st = Stride<D, n>::value;
  const int id = (node / st) % n;
  const int64_t EF = g.E * S::NF;
  const int f = face_index<n, D>(node);
  if (id == 0) {
    const double c = sL[D * 2 + 0];
#pragma unroll
    for (int v = 0; v < DIM + 2; ++v) R[v] += c * F[((int64_t)D * (DIM + 2) + v) * EF + e * S::NF + f];
  }
  if (id == N) {
    const double c = sL[D * 2 + 1];
    const int64_t ep = neighbour(g, e, D, +1);
#pragma unroll
    for (int v = 0; v < DIM + 2; ++v) R[v] += c * F[((int64_t)D * (DIM + 2) + v) * EF + ep * S::NF + f];
  }
}

struct VolArgs {
  const double* u;       // stage input
  double* out;           // RHS: du; RK: u (in place)
  double* k;             // RK register
  const double* F;       // interface fluxes (nullptr: no surface term)
  const double* alpha;   // blending factors (shock capturing)
  const double* dt;      // device dt (RK)
  double A, B;           // RK stage coefficients
};

template <int DIM, int N, int VOL, int EPI, int FVF, typename RT>
__global__ __launch_bounds__((Shape<DIM, N>::THREADS)) void k_volume(VolArgs a, Geom g) {
  using S = Shape<DIM, N>;
  constexpr int NV = S::NV, NN = S::NN;
  constexpr bool CONS = (VOL == VOL_CENTRAL || VOL == VOL_SHOCKCAP);
  __shared__ VolLds<RT, DIM, S::NE * NN, CONS> s;
  __shared__ double sT[TAB_JAC];
  for (int i = threadIdx.x; i < TAB_JAC; i += blockDim.x) sT[i] = g.tab[i];

  const int le = threadIdx.x / NN;
  const int node = threadIdx.x - le * NN;
  const int64_t e = (int64_t)blockIdx.x * S::NE + le;
  const bool active = (le < S::NE) && (e < g.E);
  const int base = le * NN;
  const int64_t ENN = g.E * NN;

  double um[NV];
  Prim<double> qd;
  if (active) {
#pragma unroll
    for (int v = 0; v < NV; ++v) um[v] = a.u[v * ENN + e * NN + node];
    if (!cons_to_prim<DIM>(um, g.gamma, qd)) *g.flag = 1;
    const int li = base + node;
    s.rho[li] = (RT)qd.rho;
#pragma unroll
    for (int k = 0; k < DIM; ++k) s.v[k][li] = (RT)qd.v[k];
    s.p[li] = (RT)qd.p;
    s.beta[li] = (RT)qd.beta;
    if constexpr (CONS) {
#pragma unroll
      for (int v = 0; v < NV; ++v) s.u[v][li] = um[v];
    }
  }
  __syncthreads();
  if (!active) return;

  double R[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) R[v] = 0.0;

  if constexpr (VOL != VOL_NONE) {
    Prim<RT> me;
    me.rho = (RT)qd.rho;
#pragma unroll
    for (int k = 0; k < 3; ++k) me.v[k] = (RT)qd.v[k];
    me.p = (RT)qd.p;
    me.beta = (RT)qd.beta;
    const RT inv_gm1 = (RT)(1.0 / (g.gamma - 1.0));
    RT acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = RT(0);
    volume_dir<DIM, N, 0, VOL, RT>(s, base, node, me, um, sT + TAB_S, inv_gm1, acc);
    volume_dir<DIM, N, 1, VOL, RT>(s, base, node, me, um, sT + TAB_S, inv_gm1, acc);
    if constexpr (DIM == 3) volume_dir<DIM, N, 2, VOL, RT>(s, base, node, me, um, sT + TAB_S, inv_gm1, acc);
    if constexpr (VOL == VOL_SHOCKCAP) {
      const double al = a.alpha[e];
      if (al != 0.0) {
        double fv[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) fv[v] = 0.0;
        fv_dir<DIM, N, 0, FVF>(s, base, node, qd, um, sT + TAB_FV, g.gamma, fv);
        fv_dir<DIM, N, 1, FVF>(s, base, node, qd, um, sT + TAB_FV, g.gamma, fv);
        if constexpr (DIM == 3) fv_dir<DIM, N, 2, FVF>(s, base, node, qd, um, sT + TAB_FV, g.gamma, fv);
#pragma unroll
        for (int v = 0; v < NV; ++v) R[v] = (1.0 - al) * (double)acc[v] + al * fv[v];
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) R[v] = (double)acc[v];
      }
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) R[v] = (double)acc[v];
    }
  }

  if (a.F != nullptr) {
    lift_dir<DIM, N, 0>(a.F, g, e, node, sT + TAB_LIFT, R);
    lift_dir<DIM, N, 1>(a.F, g, e, node, sT + TAB_LIFT, R);
    if constexpr (DIM == 3) lift_dir<DIM, N, 2>(a.F, g, e, node, sT + TAB_LIFT, R);
  }

  if constexpr (EPI == EPI_RHS) {
#pragma unroll
    for (int v = 0; v < NV; ++v) a.out[v * ENN + e * NN + node] = R[v];
  } else {
    const double dt = *a.dt;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int64_t ix = v * ENN + e * NN + node;
      const double kv = (a.A == 0.0) ? dt * R[v] : a.A * a.k[ix] + dt * R[v];
      a.k[ix] = kv;
      a.out[ix] = um[v] + a.B * kv;
    }
  }
}

// --------------------------------------------------------------------------------------
// Hennemann-Gassner indicator: q = rho p; modal coefficients by the orthonormal-Legendre
// V^-1 applied along each direction; energy = max((E_tot - E_1)/E_tot, (E_1 - E_2)/E_1)
// over the index cubes [0,N]^d, [0,N-1]^d, [0,N-2]^d; alpha = logistic(energy) with
// threshold T = 0.5 10^(-1.8 (N+1)^(1/4)) and sharpness ln(9999)/T; clip below
// alpha_min to 0, above 1 - alpha_min to 1, then to alpha_max.
// --------------------------------------------------------------------------------------
template <int DIM, int N>
__global__ __launch_bounds__((Shape<DIM, N>::THREADS)) void k_indicator(
    const double* __restrict__ u, double* __restrict__ alpha_raw, double* __restrict__ energy,
    Geom g, double alpha_min, double alpha_max) {
  using S = Shape<DIM, N>;
  constexpr int NN = S::NN, n = S::n;
  __shared__ double sa[S::NE * NN], sb[S::NE * NN];
  __shared__ double sV[TMAX * TMAX];
  for (int i = threadIdx.x; i < TMAX * TMAX; i += blockDim.x) sV[i] = g.tab[TAB_VINV + i];
  const int le = threadIdx.x / NN;
  const int node = threadIdx.x - le * NN;
  const int64_t e = (int64_t)blockIdx.x * S::NE + le;
  const bool active = (le < S::NE) && (e < g.E);
  const int base = le * NN;
  const int64_t ENN = g.E * NN;
  if (active) {
    double um[S::NV];
#pragma unroll
    for (int v = 0; v < S::NV; ++v) um[v] = u[v * ENN + e * NN + node];
    Prim<double> q;
    if (!cons_to_prim<DIM>(um, g.gamma, q)) *g.flag = 1;
    sa[base + node] = q.rho * q.p;
  }
  __syncthreads();
  double* in = sa;
  double* out = sb;
#pragma unroll
  for (int D = 0; D < DIM; ++D) {
    const int st = D == 0 ? 1 : (D == 1 ? n : n * n);
    if (active) {
      const int id = (node / st) % n;
      const int nb = base + node - id * st;
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < n; ++m) acc += sV[id * TMAX + m] * in[nb + m * st];
      out[base + node] = acc;
    }
    __syncthreads();
    double* t = in;
    in = out;
    out = t;
  }
  // in[] holds the modal coefficients; square them
  if (active) in[base + node] = in[base + node] * in[base + node];
  __syncthreads();
  if (active && node == 0) {
    double Et = 0.0, E1 = 0.0, E2 = 0.0;
    for (int nd = 0; nd < NN; ++nd) {
      const int i = nd % n, j = (nd / n) % n, k = DIM == 3 ? nd / (n * n) : 0;
      const int mx = max(i, max(j, k));
      const double c = in[base + nd];
      Et += c;
      if (mx <= N - 1) E1 += c;
      if (mx <= N - 2) E2 += c;
    }
    const double r1 = Et != 0.0 ? (Et - E1) / Et : 0.0;
    const double r2 = E1 != 0.0 ? (E1 - E2) / E1 : 0.0;
    const double en = fmax(r1, r2);
    const double T = 0.5 * pow(10.0, -1.8 * pow((double)(N + 1), 0.25));
    const double sg = log((1.0 - 0.0001) / 0.0001);
    double al = 1.0 / (1.0 + exp(-(sg / T) * (en - T)));
    if (al < alpha_min) al = 0.0;
    else if (al > 1.0 - alpha_min) al = 1.0;
    al = fmin(al, alpha_max);
    alpha_raw[e] = al;
    if (energy) energy[e] = en;
  }
}

// alpha_e = max(alpha_raw_e, max over face neighbours alpha_raw_nb / 2)
template <int DIM>
__global__ __launch_bounds__(256) void k_smooth(const double* __restrict__ ar,
                                                double* __restrict__ alpha, Geom g, int smooth) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.E) return;
  double a = ar[e];
  if (smooth) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      a = fmax(a, 0.5 * ar[neighbour(g, e, d, -1)]);
      a = fmax(a, 0.5 * ar[neighbour(g, e, d, +1)]);
    }
  }
  alpha[e] = a;
}

// --------------------------------------------------------------------------------------
// CFL time step, first pass: per block max over its elements of
// sum_d (2/h_d) max_nodes (|v_d| + c).
// --------------------------------------------------------------------------------------
template <int DIM, int N>
__global__ __launch_bounds__((Shape<DIM, N>::THREADS)) void k_maxspeed(const double* __restrict__ u,
                                                                     double* __restrict__ partial,
                                                                     Geom g) {
  using S = Shape<DIM, N>;
  constexpr int NN = S::NN;
  __shared__ double sm[DIM][S::NE * NN];
  const int le = threadIdx.x / NN;
  const int node = threadIdx.x - le * NN;
  const int64_t e = (int64_t)blockIdx.x * S::NE + le;
  const bool active = (le < S::NE) && (e < g.E);
  const int base = le * NN;
  const int64_t ENN = g.E * NN;
  if (active) {
    double um[S::NV];
#pragma unroll
    for (int v = 0; v < S::NV; ++v) um[v] = u[v * ENN + e * NN + node];
    Prim<double> q;
    if (!cons_to_prim<DIM>(um, g.gamma, q)) *g.flag = 1;
    const double c = sqrt(g.gamma * q.p / q.rho);
#pragma unroll
    for (int d = 0; d < DIM; ++d) sm[d][base + node] = fabs(q.v[d]) + c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double best = 0.0;
    for (int l = 0; l < S::NE; ++l) {
      if ((int64_t)blockIdx.x * S::NE + l >= g.E) break;
      double lam = 0.0;
      for (int d = 0; d < DIM; ++d) {
        double mx = 0.0;
        for (int nd = 0; nd < NN; ++nd) mx = fmax(mx, sm[d][l * NN + nd]);
        lam += g.tab[TAB_JAC + d] * mx;
      }
      best = fmax(best, lam);
    }
    partial[blockIdx.x] = best;
  }
}

// --------------------------------------------------------------------------------------
// Integrals, first pass: per block sums (fixed order) of J w u_v, J w S(u), J w w(u).du.
// --------------------------------------------------------------------------------------
template <int DIM, int N>
__global__ __launch_bounds__((Shape<DIM, N>::THREADS)) void k_integrals(
    const double* __restrict__ u, const double* __restrict__ du, double* __restrict__ partial,
    Geom g) {
  using S = Shape<DIM, N>;
  constexpr int NN = S::NN, n = S::n, NV = S::NV;
  __shared__ double red[7][S::THREADS];
  const int le = threadIdx.x / NN;
  const int node = threadIdx.x - le * NN;
  const int64_t e = (int64_t)blockIdx.x * S::NE + le;
  const bool active = (le < S::NE) && (e < g.E);
  const int64_t ENN = g.E * NN;
  double val[7] = {0, 0, 0, 0, 0, 0, 0};
  if (active) {
    double um[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) um[v] = u[v * ENN + e * NN + node];
    Prim<double> q;
    if (!cons_to_prim<DIM>(um, g.gamma, q)) *g.flag = 1;
    const int i = node % n, j = (node / n) % n, k = DIM == 3 ? node / (n * n) : 0;
    // J w_node = prod_d (h_d/2) w_{i_d} = prod_d w_{i_d} / (2/h_d)
    double wJ = g.tab[TAB_W + i] * g.tab[TAB_W + j] / (g.tab[TAB_JAC + 0] * g.tab[TAB_JAC + 1]);
    if (DIM == 3) wJ *= g.tab[TAB_W + k] / g.tab[TAB_JAC + 2];
    const double gm1 = g.gamma - 1.0;
    const double sp = log(q.p) - g.gamma * log(q.rho);
#pragma unroll
    for (int v = 0; v < NV; ++v) val[v] = wJ * um[v];
    val[5] = wJ * (-q.rho * sp / gm1);
    if (du) {
      double v2 = 0.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) v2 += q.v[d] * q.v[d];
      double w[NV];
      w[0] = (g.gamma - sp) / gm1 - q.rho * v2 / (2.0 * q.p);
#pragma unroll
      for (int d = 0; d < DIM; ++d) w[1 + d] = q.rho * q.v[d] / q.p;
      w[NV - 1] = -q.rho / q.p;
      double dot = 0.0;
#pragma unroll
      for (int v = 0; v < NV; ++v) dot += w[v] * du[v * ENN + e * NN + node];
      val[6] = wJ * dot;
    }
  }
#pragma unroll
  for (int c = 0; c < 7; ++c) red[c][threadIdx.x] = val[c];
  __syncthreads();
  // tree over the next power of two (the block size need not be one)
  constexpr int P2 = S::THREADS <= 256 ? 256 : (S::THREADS <= 512 ? 512 : 1024);
  for (int half = P2 / 2; half > 0; half >>= 1) {
    if ((int)threadIdx.x < half && (int)threadIdx.x + half < S::THREADS) {
#pragma unroll
      for (int c = 0; c < 7; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + half];
    }
    __syncthreads();
  }
  if (threadIdx.x < 7) partial[blockIdx.x * 7 + threadIdx.x] = red[threadIdx.x][0];
}

// node coordinates: x = xmin + c h + (h/2)(1 + x_i)
template <int DIM, int N>
__global__ __launch_bounds__(256) void k_coords(double* __restrict__ xyz, Geom g, double x0,
                                                double y0, double z0) {
  using S = Shape<DIM, N>;
  constexpr int NN = S::NN, n = S::n;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= g.E * NN) return;
  const int64_t e = gid / NN;
  const int node = (int)(gid - e * NN);
  int c[3];
  c[0] = (int)(e % g.K[0]);
  c[1] = (int)((e / g.K[0]) % g.K[1]);
  c[2] = (int)(e / ((int64_t)g.K[0] * g.K[1]));
  const int idx[3] = {node % n, (node / n) % n, DIM == 3 ? node / (n * n) : 0};
  const double lo[3] = {x0, y0, z0};
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const double h = 2.0 / g.tab[TAB_JAC + d];
    xyz[(int64_t)d * g.E * NN + gid] = lo[d] + c[d] * h + 0.5 * h * (1.0 + g.tab[TAB_X + idx[d]]);
  }
}

}  // namespace dgx
