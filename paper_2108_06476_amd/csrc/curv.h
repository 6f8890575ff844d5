// curv.h -- curvilinear hexahedral elements (the warped periodic box of the PID study,
// Section 3.1, Eq. (2)): geometry, the fused RK stage with metric terms and the
// manufactured solution's source term, and the CFL wave-speed pass.
//
// Geometry (per element, from the LGL nodes mapped by Eq. (2)): the interpolant's
// derivatives dX/ds_j by the differentiation matrix, J = dX/ds_0 . (dX/ds_1 x dX/ds_2), and
// the metric terms in the conservative curl form
//   (J a^i)_n = -[curl_s (X_l grad_s X_m)]_i,   (n, m, l) cyclic,
// which satisfy the discrete metric identities sum_i d/ds_i (J a^i) = 0 node by node (a
// constant state stays constant) and agree on both sides of every face.
// Semidiscretisation (reference element, no 2/h):
//   du/dt = -(1/J) sum_i [ sum_m S_im f~#_i(u, u_m) + (face terms with F~*)/w ] + s(x, t),
// f~#_i(A, B) = sum_n (Ja^i_n(A) + Ja^i_n(B))/2 f#_n(A, B), F~* through the face's Ja^i.
#pragma once
#include <hip/hip_runtime.h>
#include "kernels.h"

namespace dgx {

template <int NE_NN, int XB, bool CONS>
struct CurvLds {
  double rho[NE_NN], v[3][NE_NN], p[NE_NN], beta[NE_NN];
  double ja[9][NE_NN];                  // (J a^i)_n of every node, [i * 3 + n]
  double u[CONS ? 5 : 1][CONS ? NE_NN : 1];
  alignas(16) unsigned char xb[XB];     // per element: partner shares | wave speeds
};

template <int N, int VOL>
struct CurvLdsOf {
  using SS = StageShape<3, N, double, 256>;
  using type = CurvLds<SS::NENN, SS::XB, VOL == VOL_CENTRAL>;
};

template <typename L>
__device__ __forceinline__ void ja_of(const L& s, int i, int li, double (&a)[3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) a[k] = s.ja[i * 3 + k][li];
}

// Unique-pair rounds along reference direction D (as volume_dir) with the two-point flux
// contracted with the averaged metric vector of the pair.  Both fluxes are linear in that
// vector, so the rounds contract with the sum of the two nodes' vectors and the handle's
// table holds -S/2 (exact scalings: the same values).  The EC form reads the partner's
// velocity halved (hme: this node's halves).
template <int N, int D, int VOL, bool HALF, typename L>
__device__ __forceinline__ void volume_dir_curv(const L& s, double* __restrict__ x, bool on,
                                                int base, int node, const Prim<double>& me,
                                                const double (&hme)[3], const double (&ume)[5],
                                                const double* sS, double inv_gm1,
                                                double (&acc)[5]) {
  constexpr int n = N + 1, st = Stride<D, n>::value;
  constexpr int NN = Shape<3, N>::NN;
  constexpr int FULL = (n - 1) / 2;
  constexpr int ROUNDS = FULL + (HALF && n % 2 == 0 ? 1 : 0);
  const int id = (node / st) % n;
  const int nb = base + node - id * st;
  double am[3];
  ja_of(s, D, base + node, am);
#pragma unroll
  for (int r = 1; r <= ROUNDS; ++r) {
    const bool half = (r > FULL);
    int m = id + r;
    if (m >= n) m -= n;
    const int pn = nb + m * st;
    if (on && (!half || id < n / 2)) {
      Prim<double> q;
      q.rho = s.rho[pn];
#pragma unroll
      for (int k = 0; k < 3; ++k) q.v[k] = s.v[k][pn];
      q.p = s.p[pn];
      q.beta = s.beta[pn];
      double ap[3], ab[3], f[5];
      ja_of(s, D, pn, ap);
#pragma unroll
      for (int k = 0; k < 3; ++k) ab[k] = am[k] + ap[k];
      if constexpr (VOL == VOL_CENTRAL) {
        double uq[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) uq[v] = s.u[v][pn];
        central_flux_vec(ume, me, uq, q, ab, f);
      } else {
        ec_flux_vec_h(me, hme, q, ab, inv_gm1, f);
      }
      const double cme = sS[(D * TMAX + id) * TMAX + m];
      const double cpa = sS[(D * TMAX + m) * TMAX + id];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        acc[v] += cme * f[v];
        lds_add(&x[v * NN + pn - base], cpa * f[v]);
      }
    }
    if constexpr (!WaveElem<3, N>::value) __syncthreads();
  }
}

// The half rounds of the first two reference directions in one full round (even n): the
// pairing of the Cartesian kernels' packed round (a node whose x and y indices lie on the
// same side of n/2 takes its x pair, the others their y pair).  The contracted fluxes take
// the direction only through the metric vectors and the table row, so no components move.
template <int N, int VOL, typename L>
__device__ __forceinline__ void volume_xy_half_curv(const L& s, double* __restrict__ x, bool on,
                                                    int base, int node, const Prim<double>& me,
                                                    const double (&hme)[3],
                                                    const double (&ume)[5], const double* sS,
                                                    double inv_gm1, double (&acc)[5]) {
  constexpr int n = N + 1, h = n / 2;
  constexpr int NN = Shape<3, N>::NN;
  static_assert(n % 2 == 0, "packed half rounds need an even number of nodes per line");
  const int ix = node % n, iy = (node / n) % n;
  const bool dy = (ix < h) != (iy < h);
  const int D = dy ? 1 : 0;
  const int id = dy ? iy : ix;
  const int m = id < h ? id + h : id - h;
  const int pn = base + node + (m - id) * (dy ? n : 1);
  if (on) {
    Prim<double> q;
    q.rho = s.rho[pn];
#pragma unroll
    for (int k = 0; k < 3; ++k) q.v[k] = s.v[k][pn];
    q.p = s.p[pn];
    q.beta = s.beta[pn];
    double am[3], ap[3], ab[3], f[5];
    ja_of(s, D, base + node, am);
    ja_of(s, D, pn, ap);
#pragma unroll
    for (int k = 0; k < 3; ++k) ab[k] = am[k] + ap[k];
    if constexpr (VOL == VOL_CENTRAL) {
      double uq[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) uq[v] = s.u[v][pn];
      central_flux_vec(ume, me, uq, q, ab, f);
    } else {
      ec_flux_vec_h(me, hme, q, ab, inv_gm1, f);
    }
    const double cme = sS[(D * TMAX + id) * TMAX + m];
    const double cpa = sS[(D * TMAX + m) * TMAX + id];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      acc[v] += cme * f[v];
      lds_add(&x[v * NN + pn - base], cpa * f[v]);
    }
  }
  if constexpr (!WaveElem<3, N>::value) __syncthreads();
}

// Face term along reference direction D for a boundary node: the interface flux through the
// node's Ja^D (equal on both sides of the face), evaluated with the minus-side state first
// so that both elements evaluate the same expression (equal to rounding), lifted with -+1/w.
template <int N, int D, typename L>
__device__ __forceinline__ void surface_dir_curv(const L& s, const Geom& g, int surf, int node,
                                                 int li, const double (&um)[5],
                                                 const Prim<double>& qm, const double (&un)[5],
                                                 const double* sL, double (&R)[5]) {
  constexpr int n = N + 1, st = Stride<D, n>::value;
  const int id = (node / st) % n;
  if (id != 0 && id != N) return;
  const bool plus = (id == N);
  Prim<double> qn;
  if (!cons_to_prim<3, true>(un, g.gamma, qn)) *g.flag = 1;
  double a[3], uL[5], uR[5], F[5];
  ja_of(s, D, li, a);
  Prim<double> qL, qR;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    uL[v] = plus ? um[v] : un[v];
    uR[v] = plus ? un[v] : um[v];
  }
  qL.rho = plus ? qm.rho : qn.rho;
  qR.rho = plus ? qn.rho : qm.rho;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    qL.v[k] = plus ? qm.v[k] : qn.v[k];
    qR.v[k] = plus ? qn.v[k] : qm.v[k];
  }
  qL.p = plus ? qm.p : qn.p;
  qR.p = plus ? qn.p : qm.p;
  qL.beta = plus ? qm.beta : qn.beta;
  qR.beta = plus ? qn.beta : qm.beta;
  qL.c = plus ? qm.c : qn.c;
  qR.c = plus ? qn.c : qm.c;
  const double half = surface_flux_vec(surf, uL, qL, uR, qR, a, g.inv_gm1, F);
  const double c = half * (plus ? sL[2 * D + 1] : sL[2 * D]);
#pragma unroll
  for (int v = 0; v < 5; ++v) R[v] += c * F[v];
}

// One tile of curvilinear elements (3D, float64).  The tables hold -S and +-1/w (the
// reference element's own scale); the metric terms carry the geometry.
template <int N, int VOL, int EPI>
__device__ __forceinline__ void stage_tile_curv(typename CurvLdsOf<N, VOL>::type& s,
                                                const double* sT, const StageArgs& a,
                                                const Geom& g, int tile) {
  using S = Shape<3, N>;
  using SS = StageShape<3, N, double, 256>;
  constexpr int NV = 5, NN = S::NN;
  const int le = elem_slot<NN>();
  const int node = (int)(threadIdx.x % (unsigned)NN);
  const int e = tile * S::NE + le;
  const bool inb = le < S::NE;
  const bool active = inb && (e < g.E);
  const int base = le * NN;
  const int li = base + node;
  const unsigned ENN = (unsigned)g.E * NN;
  const unsigned own_ix = (unsigned)e * NN + node;

  double um[NV], unb[3][NV];
  Prim<double> qd;
  double ij = 1.0;   // 1/J of this node
  if (active) {
#pragma unroll
    for (int v = 0; v < NV; ++v) um[v] = (a.uin + (size_t)e * NN + (size_t)v * ENN)[(unsigned)node];
    if (a.surf != SURF_NONE) {
      int ec[3];
      elem_xyz(g, e, ec);
      face_load<3, N, 0>(a.uin, g, e, ec, node, unb[0]);
      face_load<3, N, 1>(a.uin, g, e, ec, node, unb[1]);
      face_load<3, N, 2>(a.uin, g, e, ec, node, unb[2]);
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) s.ja[q][li] = g.ja[q * ENN + own_ix];
    ij = rcp_nr(g.jac[own_ix]);
    if (!cons_to_prim<3>(um, g.gamma, qd)) *g.flag = 1;
    s.rho[li] = qd.rho;
#pragma unroll
    for (int k = 0; k < 3; ++k) s.v[k][li] = VOL == VOL_CENTRAL ? qd.v[k] : 0.5 * qd.v[k];
    s.p[li] = qd.p;
    s.beta[li] = qd.beta;
    if constexpr (VOL == VOL_CENTRAL) {
#pragma unroll
      for (int v = 0; v < NV; ++v) s.u[v][li] = um[v];
    }
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) um[v] = 1.0;
    qd.rho = qd.p = qd.beta = qd.c = 1.0;
    qd.v[0] = qd.v[1] = qd.v[2] = 0.0;
  }
  if (inb) {
    double* x = reinterpret_cast<double*>(s.xb + le * SS::SLOT);
#pragma unroll
    for (int v = 0; v < NV; ++v) x[v * NN + node] = 0.0;
  }
  double R[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) R[v] = 0.0;
  __syncthreads();

  if (a.surf != SURF_NONE && active) {
    surface_dir_curv<N, 0>(s, g, a.surf, node, li, um, qd, unb[0], sT + TAB_LIFT, R);
    surface_dir_curv<N, 1>(s, g, a.surf, node, li, um, qd, unb[1], sT + TAB_LIFT, R);
    surface_dir_curv<N, 2>(s, g, a.surf, node, li, um, qd, unb[2], sT + TAB_LIFT, R);
  }
  if constexpr (VOL != VOL_NONE) {
    double* x = reinterpret_cast<double*>(s.xb + (le < S::NE ? le : 0) * SS::SLOT);
    const double inv_gm1 = g.inv_gm1;
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = R[v];
    const double hme[3] = {0.5 * qd.v[0], 0.5 * qd.v[1], 0.5 * qd.v[2]};
    // even n: the x and y half rounds run as one packed round
    constexpr bool PACK = N % 2 == 1;
    volume_dir_curv<N, 0, VOL, !PACK>(s, x, active, base, node, qd, hme, um, sT + TAB_S, inv_gm1, acc);
    volume_dir_curv<N, 1, VOL, !PACK>(s, x, active, base, node, qd, hme, um, sT + TAB_S, inv_gm1, acc);
    if constexpr (PACK)
      volume_xy_half_curv<N, VOL>(s, x, active, base, node, qd, hme, um, sT + TAB_S, inv_gm1, acc);
    volume_dir_curv<N, 2, VOL, true>(s, x, active, base, node, qd, hme, um, sT + TAB_S, inv_gm1, acc);
    elem_sync<3, N>();
    if (active) {
#pragma unroll
      for (int v = 0; v < NV; ++v) R[v] = acc[v] + x[v * NN + node];
    }
  }
  if (active) {
#pragma unroll
    for (int v = 0; v < NV; ++v) R[v] *= ij;
    if (g.source) {
      const double ts = a.t0 ? (a.cs == 0.0 ? *a.t0 : *a.t0 + a.cs * *a.dt) : a.t;
      double src[NV];
      mms_source(g.gamma, g.xyz[own_ix], g.xyz[ENN + own_ix], g.xyz[2 * ENN + own_ix], ts, src);
#pragma unroll
      for (int v = 0; v < NV; ++v) R[v] += src[v];
    }
  }
  // next-step wave speed per reference direction: (|v . Ja^d| + c |Ja^d|) / J
  stage_epilogue<3, N, 5, EPI, 256>(
      s.xb, a, g, le, node, e, inb, active, ENN, own_ix, um, R,
      [&](const double (&un)[5], double (&ls)[3]) {
        Prim<double> q;
        const bool ok = cons_to_prim<3, false>(un, g.gamma, q);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          double ad[3];
          ja_of(s, d, li, ad);
          const double va = q.v[0] * ad[0] + q.v[1] * ad[1] + q.v[2] * ad[2];
          const double al = sqrt_pos(ad[0] * ad[0] + ad[1] * ad[1] + ad[2] * ad[2]);
          ls[d] = (fabs(va) + q.c * al) * ij;
        }
        return ok;
      });
}

template <int N, int VOL, int EPI>
__global__ __launch_bounds__((Shape<3, N>::THREADS)) void k_stage_curv(StageArgs a, Geom g) {
  __shared__ typename CurvLdsOf<N, VOL>::type s;
  __shared__ double sT[TAB_SIZE];
  for (int i = threadIdx.x; i < TAB_SIZE; i += blockDim.x) sT[i] = g.tab[i];
  stage_tile_curv<N, VOL, EPI>(s, sT, a, g, (int)xcd_tile(blockIdx.x, gridDim.x));
}

// Small curvilinear meshes: a stage of a few elements is a chain of single-wave latencies (the
// paper's 4^3 mesh has 64 elements for 1,024 SIMDs).  Here four waves share one element of
// 4^3 nodes (lane = node in every wave) and divide its work:
//   wave 0: x faces, x pair round;  wave 1: y faces, y pair round, source term;
//   wave 2: z faces, the packed x/y half round;  wave 3: z pair round and z half round.
// Before the block barrier the waves stage what the others read (wave d < 3: the metric
// vectors Ja^d and its faces' neighbour states; wave 3: the primitives).  Each wave adds its
// partner shares and then its own node's sum into its own LDS slot (one wave's LDS operations
// complete in issue order); wave 0 sums the four slots in a fixed order, scales by 1/J, adds
// the source and runs the epilogue.
template <int VOL>
struct CurvSplitLds {
  double rho[64], v[3][64], p[64], beta[64];
  double ja[9][64];
  double u[VOL == VOL_CENTRAL ? 5 : 1][VOL == VOL_CENTRAL ? 64 : 1];
  double x[4][5][64];   // per-wave accumulators
  double src[5][64];    // source term at the nodes
};

constexpr int CURV_SPLIT_MAX_E = 512;   // element count up to which the split kernel runs

template <int VOL, int EPI>
__global__ __launch_bounds__(256) void k_stage_curv_split(StageArgs a, Geom g) {
  constexpr int N = 3, NN = 64, NV = 5;
  __shared__ CurvSplitLds<VOL> s;
  __shared__ double sT[TAB_SIZE];
  for (int i = threadIdx.x; i < TAB_SIZE; i += blockDim.x) sT[i] = g.tab[i];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave (uniform)
  const int node = (int)(threadIdx.x & 63u);
  const int e = blockIdx.x;
  const unsigned ENN = (unsigned)g.E * NN;
  const unsigned own_ix = (unsigned)e * NN + node;
  double um[NV], un[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) um[v] = (a.uin + (size_t)e * NN + (size_t)v * ENN)[(unsigned)node];
  // wave 0 runs the epilogue: its RK register and dt are loaded now, their latency hidden
  // behind the stage (a few blocks leave the chip idle, so registers are not scarce here)
  double kp[NV], dtp = 0.0;
  if constexpr (EPI == EPI_RK) {
    if (w == 0) {
      dtp = a.dt_from ? stage_dt_from_partials(a) : *a.dt;
      if (a.A != 0.0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) kp[v] = (a.k + (size_t)e * NN + (size_t)v * ENN)[(unsigned)node];
      }
    }
  }
  if (w < 3) {
    if (a.surf != SURF_NONE) {
      int ec[3];
      elem_xyz(g, e, ec);
      if (w == 0) face_load<3, N, 0>(a.uin, g, e, ec, node, un);
      else if (w == 1) face_load<3, N, 1>(a.uin, g, e, ec, node, un);
      else face_load<3, N, 2>(a.uin, g, e, ec, node, un);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) s.ja[w * 3 + k][node] = g.ja[(w * 3 + k) * ENN + own_ix];
  }
  Prim<double> qd;
  if (!cons_to_prim<3>(um, g.gamma, qd)) *g.flag = 1;
  if (w == 3) {
    s.rho[node] = qd.rho;
#pragma unroll
    for (int k = 0; k < 3; ++k) s.v[k][node] = VOL == VOL_CENTRAL ? qd.v[k] : 0.5 * qd.v[k];
    s.p[node] = qd.p;
    s.beta[node] = qd.beta;
    if constexpr (VOL == VOL_CENTRAL) {
#pragma unroll
      for (int v = 0; v < NV; ++v) s.u[v][node] = um[v];
    }
  }
  double* x = &s.x[w][0][0];
#pragma unroll
  for (int v = 0; v < NV; ++v) x[v * NN + node] = 0.0;
  __syncthreads();   // tables, metric vectors, primitives and zeroed slots visible

  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  if (a.surf != SURF_NONE && w < 3) {
    if (w == 0) surface_dir_curv<N, 0>(s, g, a.surf, node, node, um, qd, un, sT + TAB_LIFT, acc);
    else if (w == 1) surface_dir_curv<N, 1>(s, g, a.surf, node, node, um, qd, un, sT + TAB_LIFT, acc);
    else surface_dir_curv<N, 2>(s, g, a.surf, node, node, um, qd, un, sT + TAB_LIFT, acc);
  }
  if constexpr (VOL != VOL_NONE) {
    const double hme[3] = {0.5 * qd.v[0], 0.5 * qd.v[1], 0.5 * qd.v[2]};
    const double* sS = sT + TAB_S;
    if (w == 0) volume_dir_curv<N, 0, VOL, false>(s, x, true, 0, node, qd, hme, um, sS, g.inv_gm1, acc);
    else if (w == 1) volume_dir_curv<N, 1, VOL, false>(s, x, true, 0, node, qd, hme, um, sS, g.inv_gm1, acc);
    else if (w == 2) volume_xy_half_curv<N, VOL>(s, x, true, 0, node, qd, hme, um, sS, g.inv_gm1, acc);
    else volume_dir_curv<N, 2, VOL, true>(s, x, true, 0, node, qd, hme, um, sS, g.inv_gm1, acc);
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) lds_add(&x[v * NN + node], acc[v]);
  if (w == 1) {
    double src[NV] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (g.source) {
      const double ts = a.t0 ? (a.cs == 0.0 ? *a.t0 : *a.t0 + a.cs * *a.dt) : a.t;
      mms_source(g.gamma, g.xyz[own_ix], g.xyz[ENN + own_ix], g.xyz[2 * ENN + own_ix], ts, src);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) s.src[v][node] = src[v];
  }
  __syncthreads();   // every wave's shares, own sums and the source have landed
  if (w != 0) return;
  const double ij = rcp_nr(g.jac[own_ix]);
  double R[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v)
    R[v] = (((s.x[0][v][node] + s.x[1][v][node]) + s.x[2][v][node]) + s.x[3][v][node]) * ij +
           s.src[v][node];
  // wave 0 alone: the epilogue's element-wide reductions are wave reductions
  stage_epilogue<3, N, 5, EPI, 256>(
      nullptr, a, g, 0, node, e, true, true, ENN, own_ix, um, R,
      [&](const double (&unew)[5], double (&ls)[3]) {
        Prim<double> q;
        const bool ok = cons_to_prim<3, false>(unew, g.gamma, q);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          double ad[3];
          ja_of(s, d, node, ad);
          const double va = q.v[0] * ad[0] + q.v[1] * ad[1] + q.v[2] * ad[2];
          const double al = sqrt_pos(ad[0] * ad[0] + ad[1] * ad[1] + ad[2] * ad[2]);
          ls[d] = (fabs(va) + q.c * al) * ij;
        }
        return ok;
      },
      nullptr, EPI == EPI_RK ? kp : nullptr, dtp);
  if constexpr (EPI == EPI_RK) {
    if (a.t_step && blockIdx.x == 0 && node == 0) stage_time_publish(a, dtp);
  }
}

// Geometry of one element per block (one thread per node): positions from Eq. (2) at the
// mapped LGL points of the reference box [-1,1]^3 (cells K per direction), J and the
// curl-form metric terms.  Dm: the LGL differentiation matrix [n][n].
template <int N>
__global__ __launch_bounds__(((N + 1) * (N + 1) * (N + 1))) void k_curv_geometry(
    Geom g, const double* __restrict__ Dm, double warp, double* __restrict__ xyz,
    double* __restrict__ ja, double* __restrict__ jac) {
  constexpr int n = N + 1, NN = n * n * n;
  __shared__ double X[3][NN], dX[9][NN], V[3][NN];
  __shared__ double sD[n * n];
  const int e = blockIdx.x;
  const int node = threadIdx.x;
  for (int i = node; i < n * n; i += NN) sD[i] = Dm[i];
  const int idx[3] = {node % n, (node / n) % n, node / (n * n)};
  int ec[3];
  elem_xyz(g, e, ec);
  const double* xl = g.tab + TAB_X;
  double xi[3];
#pragma unroll
  for (int d = 0; d < 3; ++d)
    xi[d] = -1.0 + (2.0 / g.K[d]) * (ec[d] + 0.5 * (1.0 + xl[idx[d]]));
  // Eq. (2): y first, then x (uses y), then z (uses x and y)
  constexpr double pi = 3.14159265358979323846;
  const double cz = cos(0.5 * pi * xi[2]);
  const double y = xi[1] + warp * (cos(1.5 * pi * xi[0]) * cos(0.5 * pi * xi[1]) * cz);
  const double x = xi[0] + warp * (cos(0.5 * pi * xi[0]) * cos(2.0 * pi * y) * cz);
  const double z = xi[2] + warp * (cos(0.5 * pi * x) * cos(pi * y) * cz);
  X[0][node] = x;
  X[1][node] = y;
  X[2][node] = z;
  __syncthreads();
  const int stride[3] = {1, n, n * n};
  auto deriv = [&](const double* f, int j) {   // d/ds_j of nodal data f at this node
    const int b = node - idx[j] * stride[j];
    double sum = 0.0;
    for (int m = 0; m < n; ++m) sum += sD[idx[j] * n + m] * f[b + m * stride[j]];
    return sum;
  };
  for (int j = 0; j < 3; ++j)
    for (int c = 0; c < 3; ++c) dX[j * 3 + c][node] = deriv(X[c], j);
  __syncthreads();
  const unsigned ENN = (unsigned)g.E * NN, own = (unsigned)e * NN + node;
  {
    const double c0 = dX[3 + 1][node] * dX[6 + 2][node] - dX[3 + 2][node] * dX[6 + 1][node];
    const double c1 = dX[3 + 2][node] * dX[6 + 0][node] - dX[3 + 0][node] * dX[6 + 2][node];
    const double c2 = dX[3 + 0][node] * dX[6 + 1][node] - dX[3 + 1][node] * dX[6 + 0][node];
    jac[own] = dX[0][node] * c0 + dX[1][node] * c1 + dX[2][node] * c2;
  }
  for (int nc = 0; nc < 3; ++nc) {
    const int mm = (nc + 1) % 3, l = (nc + 2) % 3;
#pragma unroll
    for (int j = 0; j < 3; ++j) V[j][node] = X[l][node] * dX[j * 3 + mm][node];
    __syncthreads();
    const double curl0 = deriv(V[2], 1) - deriv(V[1], 2);
    const double curl1 = deriv(V[0], 2) - deriv(V[2], 0);
    const double curl2 = deriv(V[1], 0) - deriv(V[0], 1);
    ja[(0 * 3 + nc) * ENN + own] = -curl0;
    ja[(1 * 3 + nc) * ENN + own] = -curl1;
    ja[(2 * 3 + nc) * ENN + own] = -curl2;
    __syncthreads();
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) xyz[d * ENN + own] = X[d][node];
}

// CFL partial per element: sum_d max_nodes (|v . Ja^d| + c |Ja^d|) / J.
template <int N>
__global__ __launch_bounds__((Shape<3, N>::THREADS)) void k_maxspeed_curv(
    const double* __restrict__ u, double* __restrict__ partial, Geom g) {
  using S = Shape<3, N>;
  constexpr int NN = S::NN;
  constexpr int P2 = NN <= 64 ? 64 : NN <= 128 ? 128 : NN <= 256 ? 256 : 512;
  __shared__ double sm[3][S::NE * NN];
  const int le = elem_slot<NN>();
  const int node = (int)(threadIdx.x % (unsigned)NN);
  const int64_t e = (int64_t)blockIdx.x * S::NE + le;
  const bool inb = le < S::NE;
  const bool active = inb && (e < g.E);
  const int base = le * NN;
  const unsigned ENN = (unsigned)g.E * NN;
  if (inb) {
    if (active) {
      const unsigned own = (unsigned)e * NN + node;
      double um[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) um[v] = u[v * ENN + own];
      Prim<double> q;
      if (!cons_to_prim<3, false>(um, g.gamma, q)) *g.flag = 1;
      const double ij = rcp_nr(g.jac[own]);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        double ad[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) ad[k] = g.ja[(d * 3 + k) * ENN + own];
        const double va = q.v[0] * ad[0] + q.v[1] * ad[1] + q.v[2] * ad[2];
        const double al = sqrt_pos(ad[0] * ad[0] + ad[1] * ad[1] + ad[2] * ad[2]);
        sm[d][base + node] = (fabs(va) + q.c * al) * ij;
      }
    } else {
#pragma unroll
      for (int d = 0; d < 3; ++d) sm[d][base + node] = 0.0;
    }
  }
  __syncthreads();
  for (int half = P2 / 2; half > 0; half >>= 1) {
    if (inb && node < half && node + half < NN) {
#pragma unroll
      for (int d = 0; d < 3; ++d) sm[d][base + node] = fmax(sm[d][base + node], sm[d][base + node + half]);
    }
    __syncthreads();
  }
  if (active && node == 0) partial[e] = sm[0][base] + sm[1][base] + sm[2][base];
}

}  // namespace dgx
