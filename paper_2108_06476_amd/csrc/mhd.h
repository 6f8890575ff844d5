// mhd.h -- ideal MHD (the PID study's second system, Section 3.1) on the periodic Cartesian
// box: the weak-form DGSEM with HLL or LLF interface fluxes in one fused RK stage kernel.
// Variables u = (rho, rho v_1..3, E, B_1..3), mu_0 = 1, E = p/(gamma-1) + rho|v|^2/2 + |B|^2/2:
//   f^d(u) = (rho v_d, rho v_d v + p_t e_d - B_d B, v_d (E + p_t) - B_d (v.B), v_d B - B_d v),
// p_t = p + |B|^2/2; wave speeds from the fast magnetosonic speed along d,
//   c_f^2 = (a^2 + b^2 + sqrt((a^2 + b^2)^2 - 4 a^2 b_d^2))/2,
// a^2 = gamma p/rho, b^2 = |B|^2/rho, b_d^2 = B_d^2/rho.
#pragma once
#include <hip/hip_runtime.h>
#include "kernels.h"

namespace dgx {

struct MhdPrim {
  double rho, v[3], p, B[3], pt, c2, b2;
};

__device__ __forceinline__ bool mhd_prim(const double (&u)[8], double gamma, MhdPrim& q) {
  q.rho = u[0];
  const double inv = rcp_nr(u[0]);
  double v2 = 0.0, B2 = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    q.v[k] = u[1 + k] * inv;
    q.B[k] = u[5 + k];
    v2 += q.v[k] * q.v[k];
    B2 += q.B[k] * q.B[k];
  }
  q.p = (gamma - 1.0) * (u[4] - 0.5 * u[0] * v2 - 0.5 * B2);
  q.pt = q.p + 0.5 * B2;
  q.c2 = gamma * q.p * inv;
  q.b2 = B2 * inv;
  return (q.rho > 0.0) && (q.p > 0.0) && (q.p < 1.0e300) && (q.rho < 1.0e300);
}

template <int D>
__device__ __forceinline__ void mhd_flux(const double (&u)[8], const MhdPrim& q, double (&f)[8]) {
  const double vB = q.v[0] * q.B[0] + q.v[1] * q.B[1] + q.v[2] * q.B[2];
  f[0] = u[1 + D];
#pragma unroll
  for (int k = 0; k < 3; ++k) f[1 + k] = u[1 + D] * q.v[k] + (k == D ? q.pt : 0.0) - q.B[D] * q.B[k];
  f[4] = q.v[D] * (u[4] + q.pt) - q.B[D] * vB;
#pragma unroll
  for (int k = 0; k < 3; ++k) f[5 + k] = q.v[D] * q.B[k] - q.B[D] * q.v[k];
}

template <int D>
__device__ __forceinline__ double mhd_cf(const MhdPrim& q) {
  const double s = q.c2 + q.b2;
  const double bd2 = q.B[D] * q.B[D] / q.rho;
  const double disc = fmax(s * s - 4.0 * q.c2 * bd2, 0.0);
  const double r = disc > 0.0 ? sqrt_pos(disc) : 0.0;
  return sqrt_pos(0.5 * (s + r));
}

// Interface flux along D from the minus-side state L to the plus side R (HLL or LLF).
template <int D>
__device__ __forceinline__ double mhd_surface_flux(int surf, const double (&uL)[8], const MhdPrim& L,
                                                   const double (&uR)[8], const MhdPrim& R,
                                                   double (&f)[8]) {
  double fL[8], fR[8];
  mhd_flux<D>(uL, L, fL);
  mhd_flux<D>(uR, R, fR);
  const double cL = mhd_cf<D>(L), cR = mhd_cf<D>(R);
  if (surf == SURF_LLF) {   // twice the flux: factor 1/2
    const double lam = fmax(fabs(L.v[D]) + cL, fabs(R.v[D]) + cR);
#pragma unroll
    for (int v = 0; v < 8; ++v) f[v] = (fL[v] + fR[v]) - lam * (uR[v] - uL[v]);
    return 0.5;
  }
  const double sL = fmin(L.v[D] - cL, R.v[D] - cR);
  const double sR = fmax(L.v[D] + cL, R.v[D] + cR);
  if (sL >= 0.0) {
#pragma unroll
    for (int v = 0; v < 8; ++v) f[v] = fL[v];
    return 1.0;
  }
  if (sR <= 0.0) {
#pragma unroll
    for (int v = 0; v < 8; ++v) f[v] = fR[v];
    return 1.0;
  }
#pragma unroll
  for (int v = 0; v < 8; ++v) f[v] = sR * fL[v] - sL * fR[v] + sL * sR * (uR[v] - uL[v]);
  return rcp_nr(sR - sL);   // the division, left to the caller's lift coefficient
}

template <int NE_NN, int XB>
struct MhdLds {
  double f[8][NE_NN];                  // one direction's physical fluxes of every node
  alignas(16) unsigned char xb[XB];    // per element: wave speeds (elements of several waves)
};

template <int N>
struct MhdLdsOf {
  using SS = StageShape<3, N, double, 256>;
  using type = MhdLds<SS::NENN, WaveElem<3, N>::value ? 16 : SS::XB>;
};

// Weak-form volume term and face term along D for one node: stage f^D of the element's
// nodes, contract R += (2/h_D) sum_m Dhat_{i m} f^D(u_m) along the line, and for a face node
// add the lifted interface flux (minus-side state first: both elements compute it alike).
template <int N, int D, typename L>
__device__ __forceinline__ void mhd_dir(L& s, const Geom& g, const StageArgs& a, const double* sT,
                                        bool active, int e, const int (&ec)[3], int base,
                                        int node, const double (&um)[8], const MhdPrim& qm,
                                        double (&R)[8]) {
  constexpr int n = N + 1, NN = Shape<3, N>::NN, st = Stride<D, n>::value;
  const int id = (node / st) % n;
  const int nb = base + node - id * st;
  double f[8];
  if (active) {
    mhd_flux<D>(um, qm, f);
#pragma unroll
    for (int v = 0; v < 8; ++v) s.f[v][base + node] = f[v];
  }
  elem_sync<3, N>();
  if (active) {
#pragma unroll
    for (int m = 0; m < n; ++m) {
      const double c = sT[TAB_S + (D * TMAX + id) * TMAX + m];
#pragma unroll
      for (int v = 0; v < 8; ++v) R[v] = fma(c, s.f[v][nb + m * st], R[v]);
    }
    if (a.surf != SURF_NONE && (id == 0 || id == N)) {
      const bool plus = (id == N);
      const int oth = plus ? node - N * st : node + N * st;
      const int enbp = elem_nb(g, e, ec, D, 1), enbm = elem_nb(g, e, ec, D, -1);
      const unsigned off = (unsigned)(plus ? enbp : enbm) * NN + (unsigned)oth;
      const unsigned ENN = (unsigned)g.E * NN;
      double un[8], uL[8], uR[8], F[8];
#pragma unroll
      for (int v = 0; v < 8; ++v) un[v] = (a.uin + (size_t)v * ENN)[off];
      MhdPrim qn;
      if (!mhd_prim(un, g.gamma, qn)) *g.flag = 1;
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        uL[v] = plus ? um[v] : un[v];
        uR[v] = plus ? un[v] : um[v];
      }
      const double cf = mhd_surface_flux<D>(a.surf, uL, plus ? qm : qn, uR, plus ? qn : qm, F);
      const double c = cf * (plus ? sT[TAB_LIFT + 2 * D + 1] : sT[TAB_LIFT + 2 * D]);
#pragma unroll
      for (int v = 0; v < 8; ++v) R[v] += c * F[v];
    }
  }
  elem_sync<3, N>();   // the staged fluxes are read before the next direction overwrites them
}

template <int N, int EPI>
__global__ __launch_bounds__((Shape<3, N>::THREADS)) void k_stage_mhd(StageArgs a, Geom g) {
  using S = Shape<3, N>;
  constexpr int NN = S::NN;
  __shared__ typename MhdLdsOf<N>::type s;
  __shared__ double sT[TAB_SIZE];
  for (int i = threadIdx.x; i < TAB_SIZE; i += blockDim.x) sT[i] = g.tab[i];
  const int tile = (int)xcd_tile(blockIdx.x, gridDim.x);
  const int le = elem_slot<NN>();
  const int node = (int)(threadIdx.x % (unsigned)NN);
  const int e = tile * S::NE + le;
  const bool inb = le < S::NE;
  const bool active = inb && (e < g.E);
  const int base = le * NN;
  const unsigned ENN = (unsigned)g.E * NN;
  const unsigned own_ix = (unsigned)e * NN + node;
  double um[8];
  MhdPrim qm;
  int ec[3] = {0, 0, 0};
  if (active) {
#pragma unroll
    for (int v = 0; v < 8; ++v) um[v] = (a.uin + (size_t)e * NN + (size_t)v * ENN)[(unsigned)node];
    if (!mhd_prim(um, g.gamma, qm)) *g.flag = 1;
    elem_xyz(g, e, ec);
  } else {
#pragma unroll
    for (int v = 0; v < 8; ++v) um[v] = 0.0;
    um[0] = 1.0;
    um[4] = 1.0;
    mhd_prim(um, g.gamma, qm);
  }
  double R[8];
#pragma unroll
  for (int v = 0; v < 8; ++v) R[v] = 0.0;
  __syncthreads();   // tables in LDS
  mhd_dir<N, 0>(s, g, a, sT, active, e, ec, base, node, um, qm, R);
  mhd_dir<N, 1>(s, g, a, sT, active, e, ec, base, node, um, qm, R);
  mhd_dir<N, 2>(s, g, a, sT, active, e, ec, base, node, um, qm, R);
  stage_epilogue<3, N, 8, EPI, 256>(
      s.xb, a, g, le, node, e, inb, active, ENN, own_ix, um, R,
      [&](const double (&un)[8], double (&ls)[3]) {
        MhdPrim q;
        const bool ok = mhd_prim(un, g.gamma, q);
        ls[0] = sT[TAB_JAC + 0] * (fabs(q.v[0]) + mhd_cf<0>(q));
        ls[1] = sT[TAB_JAC + 1] * (fabs(q.v[1]) + mhd_cf<1>(q));
        ls[2] = sT[TAB_JAC + 2] * (fabs(q.v[2]) + mhd_cf<2>(q));
        return ok;
      });
}

// ---- entropy-conservative flux differencing with Powell's non-conservative term ----------
// Node data of the pair flux: rho, v, beta = rho/(2p), B, and |v|^2, |B|^2, v.B.
struct MhdNode {
  double rho, v[3], beta, B[3], v2, B2, vB;
};

__device__ __forceinline__ MhdNode mhd_node(const MhdPrim& q) {
  MhdNode a;
  a.rho = q.rho;
  a.beta = 0.5 * q.rho * rcp_nr(q.p);
  a.v2 = a.B2 = a.vB = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    a.v[k] = q.v[k];
    a.B[k] = q.B[k];
    a.v2 += q.v[k] * q.v[k];
    a.B2 += q.B[k] * q.B[k];
    a.vB += q.v[k] * q.B[k];
  }
  return a;
}

// The two-point flux along D that makes flux differencing with phi(u_i) {{B_D}} entropy
// conservative: with beta = rho/(2p), the condition
//   [[w]].f* + {{B_D}} [[w.phi]] = [[rho v_D + beta v_D |B|^2]],  phi = (0, B, v.B, v),
// and the discrete product rules give
//   f_rho = rho_ln {{v_D}},  f_rhov = f_rho {{v}} - {{B_D}} {{B}} + e_D ({{rho}}/(2{{beta}}) + {{|B|^2}}/2),
//   f_B = ({{beta v_D}}/{{beta}}) {{B}} - {{B_D}} {{v}},
//   f_E = f_rho (1/(2(gamma-1) beta_ln) - {{|v|^2}}/2) + {{v}}.f_rhov + {{B}}.f_B
//         + {{B_D}} {{v.B}} - {{|B|^2}} {{v_D}}/2.
template <int D>
__device__ __forceinline__ void mhd_ec_flux(const MhdNode& L, const MhdNode& R, double inv_gm1,
                                            double (&f)[8]) {
  // the near-equal series and the logarithm only: this kernel is short of registers
  const double rho_ln = ln_mean<false>(L.rho, R.rho);
  const double ibeta = inv_ln_mean<false>(L.beta, R.beta);
  const double ba = 0.5 * (L.beta + R.beta);
  const double iba = rcp_nr(ba);
  double va[3], Ba[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    va[k] = 0.5 * (L.v[k] + R.v[k]);
    Ba[k] = 0.5 * (L.B[k] + R.B[k]);
  }
  const double v2a = 0.5 * (L.v2 + R.v2), B2a = 0.5 * (L.B2 + R.B2), vBa = 0.5 * (L.vB + R.vB);
  const double bva = 0.5 * (L.beta * L.v[D] + R.beta * R.v[D]);
  const double fr = rho_ln * va[D];
  const double pt = 0.25 * (L.rho + R.rho) * iba + 0.5 * B2a;
  const double cb = bva * iba;
  f[0] = fr;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    f[1 + k] = fr * va[k] - Ba[D] * Ba[k] + (k == D ? pt : 0.0);
    f[5 + k] = cb * Ba[k] - Ba[D] * va[k];
  }
  double e = fr * (0.5 * inv_gm1 * ibeta - 0.5 * v2a);
#pragma unroll
  for (int k = 0; k < 3; ++k) e += va[k] * f[1 + k] + Ba[k] * f[5 + k];
  f[4] = e + Ba[D] * vBa - 0.5 * B2a * va[D];
}

template <int NE_NN, int XB>
struct MhdEcLds {
  double rho[NE_NN], v[3][NE_NN], beta[NE_NN], B[3][NE_NN], v2[NE_NN], B2[NE_NN], vB[NE_NN];
  alignas(16) unsigned char xb[XB];   // per element: partner shares [8][NN] | wave speeds
};

template <int N>
struct MhdEcLdsOf {
  static constexpr int NN = Shape<3, N>::NN, NE = Shape<3, N>::NE;
  static constexpr int SLOT = 8 * 8 * NN;   // eight float64 partner shares per node
  using type = MhdEcLds<NE * NN, NE * SLOT>;
};

template <typename L>
__device__ __forceinline__ MhdNode mhd_node_lds(const L& s, int i) {
  MhdNode a;
  a.rho = s.rho[i];
  a.beta = s.beta[i];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    a.v[k] = s.v[k][i];
    a.B[k] = s.B[k][i];
  }
  a.v2 = s.v2[i];
  a.B2 = s.B2[i];
  a.vB = s.vB[i];
  return a;
}

// Unique-pair rounds along D (as volume_dir) with the MHD EC flux; then Powell's term as the
// node's phi times the contraction sum_{m != i} S_im {{B_D}}_im.
template <int N, int D, typename L>
__device__ __forceinline__ void mhd_ec_dir(const L& s, double* __restrict__ x, bool on, int base,
                                           int node, const MhdNode& me, const double (&phi)[8],
                                           const double* sS, double inv_gm1, double (&acc)[8]) {
  constexpr int n = N + 1, st = Stride<D, n>::value, NN = Shape<3, N>::NN;
  constexpr int FULL = (n - 1) / 2;
  constexpr int ROUNDS = FULL + (n % 2 == 0 ? 1 : 0);
  const int id = (node / st) % n;
  const int nb = base + node - id * st;
#pragma unroll
  for (int r = 1; r <= ROUNDS; ++r) {
    const bool half = (r > FULL);
    int m = id + r;
    if (m >= n) m -= n;
    const int pn = nb + m * st;
    if (on && (!half || id < n / 2)) {
      const MhdNode q = mhd_node_lds(s, pn);
      double f[8];
      mhd_ec_flux<D>(me, q, inv_gm1, f);
      const double cme = sS[(D * TMAX + id) * TMAX + m];
      const double cpa = sS[(D * TMAX + m) * TMAX + id];
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        acc[v] += cme * f[v];
        lds_add(&x[v * NN + pn - base], cpa * f[v]);
      }
    }
    if constexpr (!WaveElem<3, N>::value) __syncthreads();
  }
  if (on) {
    double c = 0.0;
#pragma unroll
    for (int m = 0; m < n; ++m)
      if (m != id) c += sS[(D * TMAX + id) * TMAX + m] * (0.5 * (me.B[D] + s.B[D][nb + m * st]));
#pragma unroll
    for (int v = 0; v < 8; ++v) acc[v] += phi[v] * c;
  }
}

// Face term along D for a boundary node: the interface flux (minus side first) plus the
// node's phi times {{B_D}} across the face, lifted with -+(2/h)/w.
template <int N, int D>
__device__ __forceinline__ void mhd_ec_face(const Geom& g, const StageArgs& a, const double* sT,
                                            int e, const int (&ec)[3], int node,
                                            const double (&um)[8], const MhdPrim& qm,
                                            const MhdNode& me, const double (&phi)[8],
                                            double (&R)[8]) {
  constexpr int n = N + 1, NN = Shape<3, N>::NN, st = Stride<D, n>::value;
  const int id = (node / st) % n;
  if (id != 0 && id != N) return;
  const bool plus = (id == N);
  const int oth = plus ? node - N * st : node + N * st;
  const int enbp = elem_nb(g, e, ec, D, 1), enbm = elem_nb(g, e, ec, D, -1);
  const unsigned off = (unsigned)(plus ? enbp : enbm) * NN + (unsigned)oth;
  const unsigned ENN = (unsigned)g.E * NN;
  double un[8], uL[8], uR[8], F[8];
#pragma unroll
  for (int v = 0; v < 8; ++v) un[v] = (a.uin + (size_t)v * ENN)[off];
  MhdPrim qn;
  if (!mhd_prim(un, g.gamma, qn)) *g.flag = 1;
  double cf = 1.0;   // F holds the flux divided by cf
  if (a.surf == SURF_EC) {
    const MhdNode nn = mhd_node(qn);
    mhd_ec_flux<D>(plus ? me : nn, plus ? nn : me, g.inv_gm1, F);
  } else {
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      uL[v] = plus ? um[v] : un[v];
      uR[v] = plus ? un[v] : um[v];
    }
    cf = mhd_surface_flux<D>(a.surf, uL, plus ? qm : qn, uR, plus ? qn : qm, F);
  }
  const double c = plus ? sT[TAB_LIFT + 2 * D + 1] : sT[TAB_LIFT + 2 * D];
  const double cF = c * cf, cB = c * (0.5 * (qm.B[D] + qn.B[D]));
#pragma unroll
  for (int v = 0; v < 8; ++v) R[v] += cF * F[v] + cB * phi[v];
}

// Three waves per SIMD: the register budget of 168 costs a few spilled bytes, which the
// extra wave per SIMD more than repays (173 against 198 us per stage at 32^3, N = 3).
template <int N, int EPI>
__global__ __launch_bounds__((Shape<3, N>::THREADS), 3) void k_stage_mhd_ec(StageArgs a, Geom g) {
  using S = Shape<3, N>;
  using LO = MhdEcLdsOf<N>;
  constexpr int NN = S::NN;
  __shared__ typename LO::type s;
  __shared__ double sT[TAB_SIZE];
  for (int i = threadIdx.x; i < TAB_SIZE; i += blockDim.x) sT[i] = g.tab[i];
  const int tile = (int)xcd_tile(blockIdx.x, gridDim.x);
  const int le = elem_slot<NN>();
  const int node = (int)(threadIdx.x % (unsigned)NN);
  const int e = tile * S::NE + le;
  const bool inb = le < S::NE;
  const bool active = inb && (e < g.E);
  const int base = le * NN;
  const int li = base + node;
  const unsigned ENN = (unsigned)g.E * NN;
  const unsigned own_ix = (unsigned)e * NN + node;
  double um[8], phi[8];
  MhdPrim qm;
  int ec[3] = {0, 0, 0};
  if (active) {
#pragma unroll
    for (int v = 0; v < 8; ++v) um[v] = (a.uin + (size_t)e * NN + (size_t)v * ENN)[(unsigned)node];
    if (!mhd_prim(um, g.gamma, qm)) *g.flag = 1;
    elem_xyz(g, e, ec);
  } else {
#pragma unroll
    for (int v = 0; v < 8; ++v) um[v] = 0.0;
    um[0] = 1.0;
    um[4] = 1.0;
    mhd_prim(um, g.gamma, qm);
  }
  const MhdNode me = mhd_node(qm);
  phi[0] = 0.0;
  phi[4] = me.vB;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    phi[1 + k] = me.B[k];
    phi[5 + k] = me.v[k];
  }
  if (active) {
    s.rho[li] = me.rho;
    s.beta[li] = me.beta;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      s.v[k][li] = me.v[k];
      s.B[k][li] = me.B[k];
    }
    s.v2[li] = me.v2;
    s.B2[li] = me.B2;
    s.vB[li] = me.vB;
  }
  double* x = reinterpret_cast<double*>(s.xb + (le < S::NE ? le : 0) * LO::SLOT);
  if (inb) {
#pragma unroll
    for (int v = 0; v < 8; ++v) x[v * NN + node] = 0.0;
  }
  double R[8];
#pragma unroll
  for (int v = 0; v < 8; ++v) R[v] = 0.0;
  __syncthreads();
  if (a.surf != SURF_NONE && active) {
    mhd_ec_face<N, 0>(g, a, sT, e, ec, node, um, qm, me, phi, R);
    mhd_ec_face<N, 1>(g, a, sT, e, ec, node, um, qm, me, phi, R);
    mhd_ec_face<N, 2>(g, a, sT, e, ec, node, um, qm, me, phi, R);
  }
  const double inv_gm1 = g.inv_gm1;
  mhd_ec_dir<N, 0>(s, x, active, base, node, me, phi, sT + TAB_S, inv_gm1, R);
  mhd_ec_dir<N, 1>(s, x, active, base, node, me, phi, sT + TAB_S, inv_gm1, R);
  mhd_ec_dir<N, 2>(s, x, active, base, node, me, phi, sT + TAB_S, inv_gm1, R);
  elem_sync<3, N>();   // every partner share has landed
  if (active) {
#pragma unroll
    for (int v = 0; v < 8; ++v) R[v] += x[v * NN + node];
  }
  stage_epilogue<3, N, 8, EPI, 256>(
      s.xb, a, g, le, node, e, inb, active, ENN, own_ix, um, R,
      [&](const double (&un)[8], double (&ls)[3]) {
        MhdPrim q;
        const bool ok = mhd_prim(un, g.gamma, q);
        ls[0] = sT[TAB_JAC + 0] * (fabs(q.v[0]) + mhd_cf<0>(q));
        ls[1] = sT[TAB_JAC + 1] * (fabs(q.v[1]) + mhd_cf<1>(q));
        ls[2] = sT[TAB_JAC + 2] * (fabs(q.v[2]) + mhd_cf<2>(q));
        return ok;
      });
}

// CFL partial per element: sum_d (2/h_d) max_nodes (|v_d| + c_f,d).
// Small meshes: a stage of a few elements is a chain of single-wave latencies (the 4^3
// Alfven-wave mesh has 64 elements for 1,024 SIMDs).  Three waves share one element of 4^3
// nodes (lane = node in every wave) and wave d takes direction d: its face term, so that the
// three neighbour loads are in flight together, and its volume term (the weak form's staged
// f^d contraction, or the entropy-conservative pair rounds along d with Powell's term).  Each
// wave adds its partner shares and then its own sum into its own LDS slot (one wave's LDS
// operations complete in issue order); wave 0 sums the three slots in a fixed order and runs
// the epilogue.
template <int VOL>
struct MhdSplitLds {
  MhdEcLds<(VOL == VOL_EC ? 64 : 1), 16> nd;    // EC: node data of the pair flux
  MhdLds<(VOL == VOL_EC ? 1 : 64), 16> f[3];   // weak form: each wave's staged fluxes
  double x[3][8][64];                           // per-wave sums
};

constexpr int MHD_SPLIT_MAX_E = 512;   // element count up to which the split kernel runs

template <int VOL, int EPI>
__global__ __launch_bounds__(192) void k_stage_mhd_split(StageArgs a, Geom g) {
  constexpr int N = 3, NN = 64;
  __shared__ MhdSplitLds<VOL> s;
  __shared__ double sT[TAB_SIZE];
  for (int i = threadIdx.x; i < TAB_SIZE; i += blockDim.x) sT[i] = g.tab[i];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave (uniform)
  const int node = (int)(threadIdx.x & 63u);
  const int e = blockIdx.x;
  const unsigned ENN = (unsigned)g.E * NN;
  const unsigned own_ix = (unsigned)e * NN + node;
  double um[8];
#pragma unroll
  for (int v = 0; v < 8; ++v) um[v] = (a.uin + (size_t)e * NN + (size_t)v * ENN)[(unsigned)node];
  // wave 0 runs the epilogue: its RK register and dt are loaded now, their latency hidden
  // behind the stage (a few blocks leave the chip idle, so registers are not scarce here)
  double kp[8], dtp = 0.0;
  if constexpr (EPI == EPI_RK) {
    if (w == 0) {
      dtp = a.dt_from ? stage_dt_from_partials(a) : *a.dt;
      if (a.A != 0.0) {
#pragma unroll
        for (int v = 0; v < 8; ++v) kp[v] = (a.k + (size_t)e * NN + (size_t)v * ENN)[(unsigned)node];
      }
    }
  }
  MhdPrim qm;
  if (!mhd_prim(um, g.gamma, qm)) *g.flag = 1;
  int ec[3];
  elem_xyz(g, e, ec);
  double* x = &s.x[w][0][0];
#pragma unroll
  for (int v = 0; v < 8; ++v) x[v * NN + node] = 0.0;
  double R[8];
#pragma unroll
  for (int v = 0; v < 8; ++v) R[v] = 0.0;
  if constexpr (VOL == VOL_EC) {
    const MhdNode me = mhd_node(qm);
    double phi[8];
    phi[0] = 0.0;
    phi[4] = me.vB;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      phi[1 + k] = me.B[k];
      phi[5 + k] = me.v[k];
    }
    if (w == 0) {
      s.nd.rho[node] = me.rho;
      s.nd.beta[node] = me.beta;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        s.nd.v[k][node] = me.v[k];
        s.nd.B[k][node] = me.B[k];
      }
      s.nd.v2[node] = me.v2;
      s.nd.B2[node] = me.B2;
      s.nd.vB[node] = me.vB;
    }
    __syncthreads();   // tables, node data and zeroed slots visible
    const double* sS = sT + TAB_S;
    if (w == 0) {
      if (a.surf != SURF_NONE) mhd_ec_face<N, 0>(g, a, sT, e, ec, node, um, qm, me, phi, R);
      mhd_ec_dir<N, 0>(s.nd, x, true, 0, node, me, phi, sS, g.inv_gm1, R);
    } else if (w == 1) {
      if (a.surf != SURF_NONE) mhd_ec_face<N, 1>(g, a, sT, e, ec, node, um, qm, me, phi, R);
      mhd_ec_dir<N, 1>(s.nd, x, true, 0, node, me, phi, sS, g.inv_gm1, R);
    } else {
      if (a.surf != SURF_NONE) mhd_ec_face<N, 2>(g, a, sT, e, ec, node, um, qm, me, phi, R);
      mhd_ec_dir<N, 2>(s.nd, x, true, 0, node, me, phi, sS, g.inv_gm1, R);
    }
  } else {
    __syncthreads();   // tables and zeroed slots visible
    if (w == 0) mhd_dir<N, 0>(s.f[0], g, a, sT, true, e, ec, 0, node, um, qm, R);
    else if (w == 1) mhd_dir<N, 1>(s.f[1], g, a, sT, true, e, ec, 0, node, um, qm, R);
    else mhd_dir<N, 2>(s.f[2], g, a, sT, true, e, ec, 0, node, um, qm, R);
  }
#pragma unroll
  for (int v = 0; v < 8; ++v) lds_add(&x[v * NN + node], R[v]);
  __syncthreads();   // every wave's shares and own sums have landed
  if (w != 0) return;
#pragma unroll
  for (int v = 0; v < 8; ++v) R[v] = (s.x[0][v][node] + s.x[1][v][node]) + s.x[2][v][node];
  // wave 0 alone: the epilogue's element-wide reductions are wave reductions
  stage_epilogue<3, N, 8, EPI, 256>(
      nullptr, a, g, 0, node, e, true, true, ENN, own_ix, um, R,
      [&](const double (&un)[8], double (&ls)[3]) {
        MhdPrim q;
        const bool ok = mhd_prim(un, g.gamma, q);
        ls[0] = sT[TAB_JAC + 0] * (fabs(q.v[0]) + mhd_cf<0>(q));
        ls[1] = sT[TAB_JAC + 1] * (fabs(q.v[1]) + mhd_cf<1>(q));
        ls[2] = sT[TAB_JAC + 2] * (fabs(q.v[2]) + mhd_cf<2>(q));
        return ok;
      },
      nullptr, EPI == EPI_RK ? kp : nullptr, dtp);
  if constexpr (EPI == EPI_RK) {
    if (a.t_step && blockIdx.x == 0 && node == 0) stage_time_publish(a, dtp);
  }
}

template <int N>
__global__ __launch_bounds__((Shape<3, N>::THREADS)) void k_maxspeed_mhd(
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
      double um[8];
#pragma unroll
      for (int v = 0; v < 8; ++v) um[v] = u[v * ENN + (unsigned)e * NN + node];
      MhdPrim q;
      if (!mhd_prim(um, g.gamma, q)) *g.flag = 1;
      sm[0][base + node] = fabs(q.v[0]) + mhd_cf<0>(q);
      sm[1][base + node] = fabs(q.v[1]) + mhd_cf<1>(q);
      sm[2][base + node] = fabs(q.v[2]) + mhd_cf<2>(q);
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
  if (active && node == 0) {
    double lam = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) lam += g.tab[TAB_JAC + d] * sm[d][base];
    partial[e] = lam;
  }
}

}  // namespace dgx
