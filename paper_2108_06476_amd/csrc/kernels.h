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
                                                   //            (weak form: (2/h_d) Dhat_im)
constexpr int TAB_LIFT = TAB_S + 3 * TMAX * TMAX;  // [3][2]     +(2/h_d)/w_0, -(2/h_d)/w_N
constexpr int TAB_FV = TAB_LIFT + 6;               // [3][8]     -(2/h_d)/w_i
constexpr int TAB_VINV = TAB_FV + 3 * TMAX;        // [8][8]     orthonormal-Legendre V^-1
constexpr int TAB_W = TAB_VINV + TMAX * TMAX;      // [8]        LGL weights
constexpr int TAB_X = TAB_W + TMAX;                // [8]        LGL nodes
constexpr int TAB_JAC = TAB_X + TMAX;              // [3]        2/h_d
constexpr int TAB_SIZE = TAB_JAC + 3;

enum { VOL_EC = 0, VOL_CENTRAL = 1, VOL_SHOCKCAP = 2, VOL_WEAK = 3, VOL_NONE = 4,
       VOL_WEAK_MFMA = 5 };
enum { EPI_RHS = 0, EPI_RK = 1 };

// Element tiles: NE elements of NN nodes per block of up to BUDGET threads.
template <int DIM, int N, int BUDGET = 256>
struct Shape {
  static constexpr int n = N + 1;
  static constexpr int NN = DIM == 3 ? n * n * n : n * n;  // nodes per element
  static constexpr int NF = DIM == 3 ? n * n : n;          // nodes per face
  static constexpr int NV = DIM + 2;
  static constexpr int NE = NN >= BUDGET ? 1 : BUDGET / NN;  // elements per block
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
  double inv_gm1 = 0.0;          // 1/(gamma - 1), formed once on the host
  // curvilinear elements (nullptr: Cartesian)
  const double* ja = nullptr;    // (J a^i)_n, [3 (i)][3 (n)][E][NN]
  const double* jac = nullptr;   // J, [E][NN]
  const double* xyz = nullptr;   // node positions, [3][E][NN]
  int source = 0;                // 1: the manufactured solution's source term
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

// Element coordinates (32-bit: the library keeps the element count below 2^30) and the
// periodic face neighbour in a runtime direction d: e + (wrapped c_d +- 1 - c_d) * stride_d.
__device__ __forceinline__ void elem_xyz(const Geom& g, int e, int (&c)[3]) {
  const unsigned q = (unsigned)e / (unsigned)g.K[0];
  c[0] = e - (int)q * g.K[0];
  const unsigned r = q / (unsigned)g.K[1];
  c[1] = (int)q - (int)r * g.K[1];
  c[2] = (int)r;
}

__device__ __forceinline__ int elem_nb(const Geom& g, int e, const int (&c)[3], int d, int s) {
  const int Kd = d == 0 ? g.K[0] : (d == 1 ? g.K[1] : g.K[2]);
  const int cd = d == 0 ? c[0] : (d == 1 ? c[1] : c[2]);
  const int sd = d == 0 ? 1 : (d == 1 ? g.K[0] : g.K[0] * g.K[1]);
  int x = cd + s;
  x = x < 0 ? x + Kd : (x >= Kd ? x - Kd : x);
  return e + (x - cd) * sd;
}

// Orders LDS accesses of one wavefront: the wait retires the wave's outstanding LDS
// operations and the memory clobber keeps the compiler from moving any memory access
// across this point (the wave-barrier intrinsic alone does not order memory).
__device__ __forceinline__ void wave_sync() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_wave_barrier();
}

// An element of exactly one wavefront (64 nodes: N = 3 in 3D, N = 7 in 2D) exchanges data
// only within its wave: wave-level ordering replaces block barriers.
template <int DIM, int N>
struct WaveElem {
  static constexpr bool value = Shape<DIM, N>::NN == 64;
};

// One DPP move of a double (two 32-bit halves with the same control): lanes that the row
// mask leaves out keep `old`.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double old, double src) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(src), CTRL,
                                             ROW_MASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(src), CTRL,
                                             ROW_MASK, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Max over the 64 lanes of a wave (all active), valid in lane 63: swaps within quads, the
// half-row and row mirrors (every lane of a row of 16 then holds the row's max), then the
// broadcasts of lane 15 into row 1 and row 3 and of lane 31 into rows 2 and 3.  Register
// moves only, no LDS round trips.
__device__ __forceinline__ double wave_max_lane63(double x) {
  x = fmax(x, dpp_f64<0xB1, 0xF>(x, x));    // quad_perm [1,0,3,2]
  x = fmax(x, dpp_f64<0x4E, 0xF>(x, x));    // quad_perm [2,3,0,1]
  x = fmax(x, dpp_f64<0x141, 0xF>(x, x));   // row_half_mirror
  x = fmax(x, dpp_f64<0x140, 0xF>(x, x));   // row_mirror
  x = fmax(x, dpp_f64<0x142, 0xA>(x, x));   // row_bcast:15 into rows 1 and 3
  x = fmax(x, dpp_f64<0x143, 0xC>(x, x));   // row_bcast:31 into rows 2 and 3
  return x;
}

// The element slot of this thread in its block.  A wavefront never spans two elements whose
// node count is a multiple of 64: the slot is then wave-uniform, and the element's index
// arithmetic (coordinates, neighbours, plane offsets) and its active branch run on the
// scalar unit.
template <int NN>
__device__ __forceinline__ int elem_slot() {
  return NN % 64 == 0 ? __builtin_amdgcn_readfirstlane(threadIdx.x / NN) : (int)(threadIdx.x / NN);
}

// Sum over the 64 lanes of a wave (all active), valid in lane 63: the steps of
// wave_max_lane63 with additions; lanes that a broadcast leaves out add zero.
__device__ __forceinline__ double wave_sum_lane63(double x) {
  x += dpp_f64<0xB1, 0xF>(0.0, x);    // quad_perm [1,0,3,2]
  x += dpp_f64<0x4E, 0xF>(0.0, x);    // quad_perm [2,3,0,1]
  x += dpp_f64<0x141, 0xF>(0.0, x);   // row_half_mirror
  x += dpp_f64<0x140, 0xF>(0.0, x);   // row_mirror
  x += dpp_f64<0x142, 0xA>(0.0, x);   // row_bcast:15 into rows 1 and 3
  x += dpp_f64<0x143, 0xC>(0.0, x);   // row_bcast:31 into rows 2 and 3
  return x;
}

template <int DIM, int N>
__device__ __forceinline__ void elem_sync() {
  if constexpr (WaveElem<DIM, N>::value) wave_sync();
  else __syncthreads();
}

// Blocks are dispatched round-robin over the 8 XCDs of the chip, each with its own L2.
// Give every XCD a contiguous range of element tiles so that face neighbours (x: the next
// element, y: K_x elements away) are mostly read from the same L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nb) {
  const int64_t per = nb / 8, rem = nb % 8;
  const int64_t x = b % 8, i = b / 8;
  return x * per + (x < rem ? x : rem) + i;
}

// The interface flux itself (factor applied): the subcell fluxes are shared through LDS.
template <int DIM, int D>
__device__ __forceinline__ void face_flux(int surf, const double (&uL)[DIM + 2], const Prim<double>& L,
                                          const double (&uR)[DIM + 2], const Prim<double>& R,
                                          double gamma, double (&f)[DIM + 2]) {
  double c = 1.0;
  if (surf == SURF_LLF) c = llf_flux<DIM, D>(uL, L, uR, R, gamma, f);
  else if (surf == SURF_HLL) c = hll_flux<DIM, D>(uL, L, uR, R, gamma, f);
  else ec_flux<DIM, D, double>(L, R, 1.0 / (gamma - 1.0), f);
#pragma unroll
  for (int v = 0; v < DIM + 2; ++v) f[v] *= c;
}

// --------------------------------------------------------------------------------------
// One stage of the right-hand side, one thread per node, Shape::NE elements per block
// (element-tiled, staged in LDS):
//   surface: the thread of every face node evaluates the numerical flux with the neighbour's
//            node across the face (each interface is evaluated by both of its elements, from
//            the same two states in the same order, so the two agree to rounding) and lifts
//            it to its node:
//            +(2/h_d)/w_0 F* at i_d = 0, -(2/h_d)/w_N F* at i_d = N;
//   volume:  -(2/h_d) sum_{m != i_d} S_{i_d m} f#(u, u_m), each pair evaluated once;
//   shock capturing: R_vol = (1 - alpha) R_DG + alpha R_FV (alpha = 0 skips the FV part);
//   epilogue: RHS: du = R;  RK: k = A k + dt R (not stored in a step's last stage),
//            u_out = u_in + B k, optionally the per-element wave speeds of u_out for the
//            next time step and (shock capturing) the raw indicator of u_out.
// u_in is only read and u_out only written (they must differ in RK mode: neighbours read
// u_in); k is read and written by the owning thread.
// --------------------------------------------------------------------------------------
template <typename RT, int DIM, int NE_NN, int XB, bool CONS>
struct StageLds {
  RT rho[NE_NN], v[DIM][NE_NN], p[NE_NN], beta[NE_NN];
  double c[CONS ? NE_NN : 1];         // sound speed (subcell FV fluxes)
  alignas(16) unsigned char xb[XB];   // per element: partner contributions | wave speeds
  double u[CONS ? DIM + 2 : 1][CONS ? NE_NN : 1];
};

// The scratch buffer xb holds one fixed-size slot per element; every view of it (partner
// contributions [NV][NN], wave speeds [DIM][NN]) stays inside the element's own slot, so
// elements never touch each other's scratch (with one element per wave, waves run without
// block barriers).
template <int DIM, int N, typename RT, int BUDGET = 256>
struct StageShape {
  using S = Shape<DIM, N, BUDGET>;
  static constexpr int NENN = S::NE * S::NN;
  static constexpr int SLOT_X = 8 * S::NV * S::NN;   // float64 partner shares
  static constexpr int SLOT_S = 8 * DIM * S::NN;
  static constexpr int SLOT0 = SLOT_X > SLOT_S ? SLOT_X : SLOT_S;
  static constexpr int SLOT = (SLOT0 + 15) / 16 * 16;
  static constexpr int XB = S::NE * SLOT;
};

// LDS accumulation (ds_add_f64): the partner's share of a pair flux.  The shares are
// summed in float64 also for float32 fluxes: on gfx950 an LDS float32 atomic add costs
// about ten times the LDS cycles of the float64 one, and the float64 sum is the more
// accurate of the two.
__device__ __forceinline__ void lds_add(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// The EC and blended volumes stage the nodes' velocities halved (exact), which saves
// multiplications in the pair flux (ec_flux_h); the subcell FV fluxes double them back and
// the central form reads them whole.
template <int VOL>
struct StagedHalfV {
  static constexpr bool value = VOL == VOL_EC || VOL == VOL_SHOCKCAP;
};

// Unique pairs along direction D.  In round r every node i pairs with i + r (mod n) and
// evaluates the symmetric two-point flux once: it keeps S_{i,m} f and adds S_{m,i} f into
// node m's LDS accumulator x (read back once after all directions).  Rounds r = 1..(n-1)/2
// cover every pair once; for even n the extra round r = n/2 (HALF) is computed by the
// nodes i < n/2 only, unless the caller packs it with another direction's.  In a round
// every node receives at most one share, and one wave's LDS
// operations complete in issue order, so the sums are formed in a fixed order; elements
// spread over several waves put a block barrier between rounds for the same reason.
template <int DIM, int N, int D, int VOL, typename RT, bool HALF, typename L>
__device__ __forceinline__ void volume_dir(const L& s, double* __restrict__ x /* element slot */,
                                           bool on, int base,
                                           int node, const Prim<RT>& me, const RT (&hme)[3],
                                           const double (&ume)[DIM + 2], const double* sS,
                                           RT inv_gm1, RT pref, RT (&acc)[DIM + 2]) {
  constexpr int n = N + 1, st = Stride<D, n>::value;
  constexpr int NN = Shape<DIM, N>::NN;
  constexpr int FULL = (n - 1) / 2;
  constexpr int ROUNDS = FULL + (HALF && n % 2 == 0 ? 1 : 0);
  const int id = (node / st) % n;
  const int nb = base + node - id * st;
#pragma unroll
  for (int r = 1; r <= ROUNDS; ++r) {
    const bool half = (r > FULL);
    int m = id + r;
    if (m >= n) m -= n;
    const int pn = nb + m * st;
    if (on && (!half || id < n / 2)) {
      Prim<RT> q;
      q.rho = s.rho[pn];
#pragma unroll
      for (int k = 0; k < DIM; ++k) q.v[k] = s.v[k][pn];
      q.p = s.p[pn];
      q.beta = s.beta[pn];
      RT f[DIM + 2];
      if constexpr (VOL == VOL_CENTRAL) {
        double uq[DIM + 2], fd[DIM + 2];
        Prim<double> qd, med;
#pragma unroll
        for (int v = 0; v < DIM + 2; ++v) uq[v] = s.u[v][pn];
        qd.rho = q.rho;
        med.rho = me.rho;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          qd.v[k] = k < DIM ? (double)q.v[k] : 0.0;
          med.v[k] = k < DIM ? (double)me.v[k] : 0.0;
        }
        qd.p = q.p;
        med.p = me.p;
        central_flux<DIM, D>(ume, med, uq, qd, fd);
#pragma unroll
        for (int v = 0; v < DIM + 2; ++v) f[v] = (RT)fd[v];
      } else if constexpr (sizeof(RT) == 4) {
        ec_flux_pp<DIM, D>(me, hme, q, inv_gm1, pref, f);
      } else if constexpr (StagedHalfV<VOL>::value) {
        ec_flux_h<DIM, D, RT>(me, hme, q, inv_gm1, f);
      } else {
        ec_flux<DIM, D, RT>(me, q, inv_gm1, f);
      }
      const RT cme = (RT)sS[(D * TMAX + id) * TMAX + m];
      const RT cpa = (RT)sS[(D * TMAX + m) * TMAX + id];
#pragma unroll
      for (int v = 0; v < DIM + 2; ++v) {
        acc[v] += cme * f[v];
        lds_add(&x[v * NN + pn - base], (double)(cpa * f[v]));
      }
    }
    if constexpr (!WaveElem<DIM, N>::value) __syncthreads();
  }
}

// The half rounds of x and y in one full round (even n, EC volume flux).  Every node lies
// in one x pair (i, i + n/2) and one y pair; on each 4-cycle
// (a,b) -> (a+h,b) -> (a+h,b+h) -> (a,b+h) of these pairs (h = n/2, a, b < h) every node
// takes the next edge, so a node whose x and y indices are on the same side of h evaluates
// its x pair and the others their y pair: 64 of 64 lanes busy where the two half rounds
// kept 32.  The y flux is the x flux of the states with v_x and v_y exchanged, its momentum
// components exchanged back.
template <int DIM, int N, int VOL, typename RT, typename L>
__device__ __forceinline__ void volume_xy_half(const L& s, double* __restrict__ x, bool on,
                                               int base, int node, const Prim<RT>& me,
                                               const RT (&hme)[3], const double* sS,
                                               RT inv_gm1, RT pref, RT (&acc)[DIM + 2]) {
  constexpr int n = N + 1, h = n / 2;
  constexpr int NN = Shape<DIM, N>::NN;
  static_assert(n % 2 == 0, "packed half rounds need an even number of nodes per line");
  const int ix = node % n, iy = (node / n) % n;
  const bool dy = (ix < h) != (iy < h);
  const int id = dy ? iy : ix;
  const int m = id < h ? id + h : id - h;
  const int pn = base + node + (m - id) * (dy ? n : 1);
  if (on) {
    Prim<RT> a = me, q;
    q.rho = s.rho[pn];
#pragma unroll
    for (int k = 0; k < DIM; ++k) q.v[k] = s.v[k][pn];
    q.p = s.p[pn];
    q.beta = s.beta[pn];
    const RT q0 = q.v[0], q1 = q.v[1];
    a.v[0] = dy ? me.v[1] : me.v[0];
    a.v[1] = dy ? me.v[0] : me.v[1];
    q.v[0] = dy ? q1 : q0;
    q.v[1] = dy ? q0 : q1;
    const RT ha[3] = {dy ? hme[1] : hme[0], dy ? hme[0] : hme[1], hme[2]};
    RT f[DIM + 2];
    if constexpr (sizeof(RT) == 4) ec_flux_pp<DIM, 0>(a, ha, q, inv_gm1, pref, f);
    else if constexpr (StagedHalfV<VOL>::value) ec_flux_h<DIM, 0, RT>(a, ha, q, inv_gm1, f);
    else ec_flux<DIM, 0, RT>(a, q, inv_gm1, f);
    const RT f1 = f[1], f2 = f[2];
    f[1] = dy ? f2 : f1;
    f[2] = dy ? f1 : f2;
    const int D = dy ? 1 : 0;
    const RT cme = (RT)sS[(D * TMAX + id) * TMAX + m];
    const RT cpa = (RT)sS[(D * TMAX + m) * TMAX + id];
#pragma unroll
    for (int v = 0; v < DIM + 2; ++v) {
      acc[v] += cme * f[v];
      lds_add(&x[v * NN + pn - base], (double)(cpa * f[v]));
    }
  }
  if constexpr (!WaveElem<DIM, N>::value) __syncthreads();
}

// First-order FV on the LGL subcells in direction D with the fv flux (LLF or HLL):
// acc += -(2/h_d)/w_i (F_{i+1/2} - F_{i-1/2}), element-boundary subcell fluxes zero.  Every
// subcell face is evaluated once, by its left node (left state: itself), and shared through
// the element's LDS slot f [NV][NN]: the right node reads it as its F_{i-1/2} (the same
// arguments in the same order as its own evaluation would take).  Called by every thread of
// the block (on: this node's element takes part).
template <int DIM, int N, int D, typename L>
__device__ __forceinline__ void fv_dir(const L& s, double* __restrict__ f, int fvf, bool on,
                                       int base, int node, const Prim<double>& me,
                                       const double (&ume)[DIM + 2], const double* sFV,
                                       double gamma, double (&acc)[DIM + 2]) {
  constexpr int n = N + 1, st = Stride<D, n>::value;
  constexpr int NN = Shape<DIM, N>::NN;
  const int id = (node / st) % n;
  double Fp[DIM + 2];
#pragma unroll
  for (int v = 0; v < DIM + 2; ++v) Fp[v] = 0.0;
  auto load = [&](int pn, double (&uq)[DIM + 2], Prim<double>& q) {
#pragma unroll
    for (int v = 0; v < DIM + 2; ++v) uq[v] = s.u[v][pn];
    q.rho = s.rho[pn];
    q.v[0] = q.v[1] = q.v[2] = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) q.v[k] = 2.0 * s.v[k][pn];   // staged halved (blended volume)
    q.p = s.p[pn];
    q.beta = s.beta[pn];
    q.c = s.c[pn];
  };
  if (on && id < N) {
    double uq[DIM + 2];
    Prim<double> q;
    load(base + node + st, uq, q);
    face_flux<DIM, D>(fvf, ume, me, uq, q, gamma, Fp);
#pragma unroll
    for (int v = 0; v < DIM + 2; ++v) f[v * NN + node] = Fp[v];
  }
  elem_sync<DIM, N>();
  if (on) {
    const double c = sFV[D * TMAX + id];
#pragma unroll
    for (int v = 0; v < DIM + 2; ++v)
      acc[v] += c * (Fp[v] - (id > 0 ? f[v * NN + node - st] : 0.0));
  }
  elem_sync<DIM, N>();   // read before the next direction writes
}

// Surface term of one node in direction D: a node with index_D = 0 (N) lies on the
// element's minus (plus) face; it evaluates the numerical flux with the neighbour's node
// across that face and lifts it, +(2/h_D)/w_0 F* (minus) or -(2/h_D)/w_N F* (plus).  Both
// elements of an interface evaluate the same expression of the (left, right) states; the
// primitives of the two states come from different code (the own node's from the staging,
// the neighbour's here), so the two values agree to rounding, not always bit for bit.
// Issue the loads of the neighbour's node across the face in direction D (if any).
template <int DIM, int N, int D>
__device__ __forceinline__ void face_load(const double* __restrict__ u, const Geom& g, int e,
                                          const int (&ec)[3], int node, double (&un)[DIM + 2]) {
  using S = Shape<DIM, N>;
  constexpr int n = S::n, NN = S::NN, NV = S::NV, st = Stride<D, n>::value;
  const int id = (node / st) % n;
  if (id != 0 && id != N) return;
  const bool plus = (id == N);
  const int oth = plus ? node - N * st : node + N * st;
  // both neighbours' nodes first (uniform when e is), then one per-lane choice
  const double* pp = u + (size_t)elem_nb(g, e, ec, D, 1) * NN;
  const double* pm = u + (size_t)elem_nb(g, e, ec, D, -1) * NN;
  const double* ub = plus ? pp : pm;
  const size_t ENN = (size_t)g.E * NN;
#pragma unroll
  for (int v = 0; v < NV; ++v) un[v] = (ub + (size_t)v * ENN)[(unsigned)oth];
}

template <int DIM, int N, int D, bool PREF>
__device__ __forceinline__ void surface_dir(const Geom& g, int surf, int node,
                                            const double (&um)[DIM + 2], const Prim<double>& qm,
                                            const double (&un)[DIM + 2], const double* sL,
                                            double pref, double (&R)[DIM + 2]) {
  using S = Shape<DIM, N>;
  constexpr int n = S::n, NV = S::NV, st = Stride<D, n>::value;
  const int id = (node / st) % n;
  if (id != 0 && id != N) return;
  const bool plus = (id == N);
  Prim<double> qn;
  const bool ok = surf == SURF_EC ? cons_to_prim<DIM, true>(un, g.gamma, qn)
                                  : cons_to_prim<DIM, false>(un, g.gamma, qn);
  if (!ok) *g.flag = 1;
  double F[NV];
  double half = 1.0;   // F holds the flux divided by half (LLF: 1/2, HLL: 1/(s_R - s_L))
  if (surf == SURF_LLF) {
    // 2 F = (f_L + f_R) - lambda (u_R - u_L) from (own, neighbour): with the sign of the
    // jump term both elements evaluate the same expression of (left, right)
    double fo[NV], fn[NV];
    phys_flux<DIM, D>(um, qm, fo);
    phys_flux<DIM, D>(un, qn, fn);
    const double lam = fmax(fabs(qm.v[D]) + qm.c, fabs(qn.v[D]) + qn.c);
    const double sl = plus ? lam : -lam;
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v] = (fo[v] + fn[v]) - sl * (un[v] - um[v]);
    half = 0.5;
  } else if (surf == SURF_EC) {
    ec_flux_sym<DIM, D>(qm, qn, g.inv_gm1, F);
  } else {
    double uL[NV], uR[NV];
    Prim<double> qL, qR;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
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
    qL.c = plus ? qm.c : qn.c;
    qR.c = plus ? qn.c : qm.c;
    half = hll_flux<DIM, D>(uL, qL, uR, qR, g.gamma, F);
  }
  const double c0 = plus ? sL[2 * D + 1] : sL[2 * D];
  const double c = half * c0;
#pragma unroll
  for (int v = 0; v < NV; ++v) R[v] += c * F[v];
  // PREF: the constant pressure pref left out of a float32 volume sum, removed from the
  // lifted normal momentum flux with it
  if constexpr (PREF) R[1 + D] -= c0 * pref;
}

struct StageArgs {
  const double* uin;     // stage input (and the neighbours' face states)
  double* uout;          // RK: stage output state
  double* du;            // RHS: right-hand side
  double* k;             // RK register
  const double* alpha;   // blending factors (shock capturing)
  const double* dt;      // device dt (RK)
  double* speed;         // RK: per-block max wave speed of uout (nullptr: skip)
  double A, B;           // RK stage coefficients
  int surf;              // SURF_* (SURF_NONE: no surface term)
  int fvf;               // subcell FV flux (SURF_LLF or SURF_HLL)
  // time of the stage (source terms): *t0 + cs * (*dt) when t0 is set, else t
  const double* t0 = nullptr;
  double cs = 0.0;
  double t = 0.0;
  // RK: write k (0 in a step's last stage: k is dead until the next step's first stage,
  // which does not read it)
  int kw = 1;
  // shock capturing, RK: the raw indicator of the stage's output state (nullptr: skip) and
  // its constants (threshold, sharpness, alpha_min, alpha_max)
  double* alpha_next = nullptr;
  double ind_thr = 0.0, ind_sharp = 0.0, ind_amin = 0.0, ind_amax = 0.0, ind_xcut = 0.0;
  // shock capturing: the raw indicator of the stage's input (nullptr: alpha holds the
  // smoothed factors); each element then smooths its own from it and its face neighbours'
  const double* alpha_raw_in = nullptr;
  int alpha_smooth = 0;
  // small meshes (several waves per element): the first stage of an adaptive step derives dt
  // itself from the per-element wave-speed partials dt_from[0, dt_np) (every block alike,
  // dt = dt_cfl 2 / (dt_n1 max)); block 0 publishes it to dt_pub and the step's start time
  // *t_cur to t0_pub (if set).  t_step = 2 marks the second stage, whose block 0 advances
  // *t_cur by the step's dt (nothing reads t_cur while a step runs).
  const double* dt_from = nullptr;
  int64_t dt_np = 0;
  int64_t dt_stride = 1;   // dt_from holds its values dt_stride doubles apart
  // Mid-size Cartesian meshes (api.hip's stage_slots): the last stage folds each element's
  // wave speed into the DT_SLOTS slots of speed_slots (an atomic max on the bits of a
  // positive double, slot e % DT_SLOTS), the next step's first stage reduces them (dt_from,
  // dt_np = DT_SLOTS, dt_stride = DT_SLOT_STRIDE), and block 0 of its second stage clears
  // them (slots_clear).
  double* speed_slots = nullptr;
  double* slots_clear = nullptr;
  double dt_cfl = 0.0, dt_n1 = 0.0;
  double* dt_pub = nullptr;
  double* t_cur = nullptr;
  double* t0_pub = nullptr;
  int t_step = 0;
};

// The wave-speed slots of StageArgs::speed_slots: DT_SLOTS maxima, DT_SLOT_STRIDE doubles
// (512 B) apart so that the atomics of different slots spread over the memory channels.
constexpr int DT_SLOTS = 64;
constexpr int DT_SLOT_STRIDE = 64;

// One element's wave speed into its slot.  Non-negative doubles order as their bit patterns
// do, so an unsigned 64-bit atomic max keeps the exact maximum whatever the order; zero and
// NaN are skipped, as the fmax reductions of the partials skip NaN.
__device__ __forceinline__ void slot_max(double* slots, int e, double lam) {
  if (lam > 0.0)
    __hip_atomic_fetch_max(
        reinterpret_cast<unsigned long long*>(slots + (size_t)(e & (DT_SLOTS - 1)) * DT_SLOT_STRIDE),
        (unsigned long long)__double_as_longlong(lam), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The first-stage dt of StageArgs::dt_from, reduced by one wave (all 64 lanes active): the
// same value as k_dt_final's (max is exact), in every lane.
__device__ __forceinline__ double stage_dt_from_partials(const StageArgs& a) {
  double m[4] = {0.0, 0.0, 0.0, 0.0};
  int64_t i = threadIdx.x & 63u;
  const int64_t sd = a.dt_stride;
  for (; i + 3 * 64 < a.dt_np; i += 4 * 64) {
#pragma unroll
    for (int k = 0; k < 4; ++k) m[k] = fmax(m[k], a.dt_from[(i + k * 64) * sd]);
  }
  for (; i < a.dt_np; i += 64) m[0] = fmax(m[0], a.dt_from[i * sd]);
  const double r = wave_max_lane63(fmax(fmax(m[0], m[1]), fmax(m[2], m[3])));
  const double mx = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(r), 63),
                                     __builtin_amdgcn_readlane(__double2loint(r), 63));
  return a.dt_cfl * 2.0 / (a.dt_n1 * mx);
}

// Block 0's part of StageArgs::t_step (called by one thread after the stage's own reads of
// dt and t): stage 1 publishes dt and the step's start time, stage 2 advances t.
__device__ __forceinline__ void stage_time_publish(const StageArgs& a, double dt_stage1) {
  if (a.t_step == 1) {
    *a.dt_pub = dt_stage1;
    if (a.t0_pub && a.t_cur) *a.t0_pub = *a.t_cur;
  } else if (a.t_step == 2 && a.t_cur) {
    *a.t_cur += *a.dt;
  }
}

// Weak form: the physical fluxes f^d_v of every node, contracted along the lines.
template <int DIM, int NE_NN, int XB>
struct WeakLds {
  double f[DIM][DIM + 2][NE_NN];
  alignas(16) unsigned char xb[XB];   // per element: wave speeds (elements of several waves)
};

template <int DIM, int N, int VOL, typename RT, int BUDGET = 256>
struct StageLdsOf {
  using SS = StageShape<DIM, N, RT, BUDGET>;
  using type = StageLds<RT, DIM, SS::NENN, SS::XB, (VOL == VOL_CENTRAL || VOL == VOL_SHOCKCAP)>;
};

template <int DIM, int N, typename RT, int BUDGET>
struct StageLdsOf<DIM, N, VOL_WEAK, RT, BUDGET> {
  using SS = StageShape<DIM, N, RT, BUDGET>;
  // one-wave elements reduce their wave speeds with DPP moves: no scratch slot
  using type = WeakLds<DIM, SS::NENN, WaveElem<DIM, N>::value ? 16 : SS::XB>;
};

template <int DIM, int N, typename RT, int BUDGET>
struct StageLdsOf<DIM, N, VOL_WEAK_MFMA, RT, BUDGET> {
  using type = typename StageLdsOf<DIM, N, VOL_WEAK, RT, BUDGET>::type;
};

// A double from lane `src` of the wave (ds_bpermute on both halves).
__device__ __forceinline__ double lane_read_f64(double x, int src) {
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, __double2loint(x));
  const int hi = __builtin_amdgcn_ds_bpermute(src << 2, __double2hiint(x));
  return __hiloint2double(hi, lo);
}

// Weak-form volume term of a 3D N = 3 element (one wave, lane = node = ix + 4 iy + 16 iz) on
// the matrix cores: v_mfma_f64_4x4x4f64 multiplies four 4x4 blocks per instruction; with
// (bits 0-1, 2-3, 4-5) of the lane holding (row, block, k) of A, (column, block, k) of B and
// (column, block, row) of the result, one instruction contracts all 16 lines of one variable
// in one direction:
//   z: A = Dhat_z[a][c], B = the lane's own flux: result on the owner lane;
//   x: A = flux of node (c, b, a) (gathered from LDS), B = Dhat_x[a][c] (the transposed
//      product): result on the owner lane;
//   y: A = Dhat_y[a][c], B = flux of node (a, c, b): the result for node (a, c, b) sits on
//      lane (a, b, c); the swap of the two upper bit pairs is its own inverse, so each lane
//      reads its value from lane (a, c, b).
// (a, b, c) = (l & 3, (l >> 2) & 3, l >> 4).  The running sum R is the accumulator input.
template <typename L>
__device__ __forceinline__ void weak_mfma_n3(const L& s, int base, int l, const double* sD,
                                             double (&R)[5]) {
  const int a = l & 3, b = (l >> 2) & 3, c = l >> 4;
  const double dx = sD[(0 * TMAX + a) * TMAX + c];
  const double dy = sD[(1 * TMAX + a) * TMAX + c];
  const double dz = sD[(2 * TMAX + a) * TMAX + c];
  const int nx = c + 4 * b + 16 * a;
  const int ny = a + 4 * c + 16 * b;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    double r = __builtin_amdgcn_mfma_f64_4x4x4f64(dz, s.f[2][v][base + l], R[v], 0, 0, 0);
    r = __builtin_amdgcn_mfma_f64_4x4x4f64(s.f[0][v][base + nx], dx, r, 0, 0, 0);
    const double oy = __builtin_amdgcn_mfma_f64_4x4x4f64(dy, s.f[1][v][base + ny], 0.0, 0, 0, 0);
    R[v] = r + lane_read_f64(oy, ny);
  }
}

// Weak-form volume term along direction D: R_v += sum_m (2/h_D) Dhat_{i m} f^D_v(u_m) over
// the line of the node (i = its index along D), fluxes read from LDS.
template <int DIM, int N, int D, typename L>
__device__ __forceinline__ void weak_dir(const L& s, int base, int node, const double* sD,
                                         double (&R)[DIM + 2]) {
  constexpr int n = N + 1, st = Stride<D, n>::value;
  const int id = (node / st) % n;
  const int nb = base + node - id * st;
#pragma unroll
  for (int m = 0; m < n; ++m) {
    const double c = sD[(D * TMAX + id) * TMAX + m];
#pragma unroll
    for (int v = 0; v < DIM + 2; ++v) R[v] = fma(c, s.f[D][v][nb + m * st], R[v]);
  }
}

// Epilogue of a stage for one node: RHS: du = R; RK: k <- A k + dt R, u_out = u + B k and,
// in the last stage, each element's partial of the next CFL step,
// sum_d max_nodes lam_d of the new state: speeds(u_new, lam) gives the directions' scaled
// wave speeds and returns false for a non-physical state.
// xb: the block's per-element LDS slots (elements of several waves reduce through them).
// DTF: the caller may ask for the first stage's dt to be derived here (a.dt_from) and for
// the last stage's wave speeds to be folded into slots (a.speed_slots).
template <int DIM, int N, int NV, int EPI, int BUDGET, typename SpeedFn, bool DTF = false>
__device__ __forceinline__ double stage_epilogue(unsigned char* xb, const StageArgs& a,
                                               const Geom& g, int le, int node, int e, bool inb,
                                               bool active, size_t ENN, size_t own_ix,
                                               const double (&um)[NV], const double (&R)[NV],
                                               SpeedFn speeds, double* un_out = nullptr,
                                               const double* kpre = nullptr,
                                               double dtpre = 0.0) {
  using S = Shape<DIM, N, BUDGET>;
  using SS = StageShape<DIM, N, double, BUDGET>;
  constexpr int NN = S::NN;
  double dt_used = 0.0;
  if constexpr (EPI == EPI_RHS) {
    if (active) {
#pragma unroll
      for (int v = 0; v < NV; ++v) (a.du + (size_t)(own_ix - node) + (size_t)v * ENN)[(unsigned)node] = R[v];
    }
  } else {
    double un[NV];
    // dtpre (> 0): dt loaded or derived by the caller; a first stage that derives dt itself
    // (a.dt_from) reduces the partials here, where few registers are live (every lane of
    // the wave reaches this point)
    if (dtpre > 0.0) dt_used = dtpre;
    else if constexpr (DTF) {
      if (a.dt_from) dt_used = stage_dt_from_partials(a);
    }
    if (active) {
      // kpre: the RK register loaded by the caller already
      const double dt = dt_used > 0.0 ? dt_used : *a.dt;
      double kv[NV];
      if (a.A == 0.0) {   // first stage: k is not read (uniform branch)
#pragma unroll
        for (int v = 0; v < NV; ++v) kv[v] = dt * R[v];
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v)
          kv[v] = a.A * (kpre ? kpre[v] : (a.k + (size_t)(own_ix - node) + (size_t)v * ENN)[(unsigned)node]) + dt * R[v];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const size_t pb = (size_t)(own_ix - node) + (size_t)v * ENN;   // uniform plane base
        if (a.kw) a.k[pb + (unsigned)node] = kv[v];
        un[v] = um[v] + a.B * kv[v];
        a.uout[pb + (unsigned)node] = un[v];
        if (un_out) un_out[v] = un[v];
      }
    }
    double* const slots = DTF ? a.speed_slots : nullptr;
    if (a.speed != nullptr || slots != nullptr) {
      if constexpr (WaveElem<DIM, N>::value) {
        if (active) {   // uniform per wave: the element is the wave
          double ls[DIM];
          if (!speeds(un, ls)) *g.flag = 1;
          double lam = 0.0;
#pragma unroll
          for (int d = 0; d < DIM; ++d) lam += wave_max_lane63(ls[d]);
          if (node == NN - 1) {
            if (DTF && slots) slot_max(slots, e, lam);
            else a.speed[e] = lam;
          }
        }
      } else {
        constexpr int P2 = NN <= 4 ? 4 : NN <= 16 ? 16 : NN <= 64 ? 64 : NN <= 128 ? 128 : NN <= 256 ? 256 : 512;
        double* sp = reinterpret_cast<double*>(xb + (le < S::NE ? le : 0) * SS::SLOT);   // [DIM][NN]
        __syncthreads();
        if (inb) {
          if (active) {
            double ls[DIM];
            if (!speeds(un, ls)) *g.flag = 1;
#pragma unroll
            for (int d = 0; d < DIM; ++d) sp[d * NN + node] = ls[d];
          } else {
#pragma unroll
            for (int d = 0; d < DIM; ++d) sp[d * NN + node] = 0.0;
          }
        }
        __syncthreads();
        for (int h = P2 / 2; h > 0; h >>= 1) {
          if (inb && node < h && node + h < NN) {
#pragma unroll
            for (int d = 0; d < DIM; ++d)
              sp[d * NN + node] = fmax(sp[d * NN + node], sp[d * NN + node + h]);
          }
          __syncthreads();
        }
        if (active && node == 0) {
          double lam = 0.0;
#pragma unroll
          for (int d = 0; d < DIM; ++d) lam += sp[d * NN];
          if (DTF && slots) slot_max(slots, e, lam);
          else a.speed[e] = lam;
        }
      }
    }
  }
  return dt_used;
}

// The indicator of one element from q = rho p at its nodes: w0, w1, w2 are NN-double LDS
// scratch arrays of the element (w0 holds q on entry), sV the LDS V^-1 table.  Called by
// every thread of the block (inb: the thread has an element slot; active: its element
// exists); a one-wave element uses wave-level ordering, other shapes block barriers.
template <int DIM, int N>
__device__ __forceinline__ void indicator_elem(double* w0, double* w1, double* w2,
                                               const double* sV, int node, bool inb, bool active,
                                               double thr, double sharp, double alpha_min,
                                               double alpha_max, double xcut,
                                               double* __restrict__ alpha_raw,
                                               double* __restrict__ energy, int64_t e) {
  constexpr int NN = Shape<DIM, N>::NN, n = N + 1;
  constexpr bool WAVE = WaveElem<DIM, N>::value;
  elem_sync<DIM, N>();   // q visible
  double* in = w0;
  double* out = w1;
#pragma unroll
  for (int D = 0; D < DIM; ++D) {
    const int st = D == 0 ? 1 : (D == 1 ? n : n * n);
    if (active) {
      const int id = (node / st) % n;
      const int nb = node - id * st;
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < n; ++m) acc += sV[id * TMAX + m] * in[nb + m * st];
      out[node] = acc;
    }
    elem_sync<DIM, N>();
    double* t = in;
    in = out;
    out = t;
  }
  // in[] holds the modal coefficients; the energy of all modes and of the index cubes
  // [0, N-1]^d and [0, N-2]^d, summed over the element's nodes
  double t0 = 0.0, t1 = 0.0, t2 = 0.0;
  if (active) {
    const int i = node % n, j = (node / n) % n, k = DIM == 3 ? node / (n * n) : 0;
    const int mx = max(i, max(j, k));
    const double c = in[node] * in[node];
    t0 = c;
    t1 = mx <= N - 1 ? c : 0.0;
    t2 = mx <= N - 2 ? c : 0.0;
  }
  int last = 0;   // the node that holds the sums
  if constexpr (WAVE) {
    if (active) {   // uniform per wave: the element is the wave
      t0 = wave_sum_lane63(t0);
      t1 = wave_sum_lane63(t1);
      t2 = wave_sum_lane63(t2);
    }
    last = NN - 1;
  } else {
    constexpr int P2 = NN <= 4 ? 4 : NN <= 16 ? 16 : NN <= 64 ? 64 : NN <= 128 ? 128 : NN <= 256 ? 256 : 512;
    double* a0 = out;   // free: the transform's scratch
    elem_sync<DIM, N>();
    if (inb) {
      a0[node] = t0;
      in[node] = t1;
      w2[node] = t2;
    }
    __syncthreads();
    for (int hh = P2 / 2; hh > 0; hh >>= 1) {
      if (inb && node < hh && node + hh < NN) {
        a0[node] += a0[node + hh];
        in[node] += in[node + hh];
        w2[node] += w2[node + hh];
      }
      __syncthreads();
    }
    t0 = a0[0];
    t1 = in[0];
    t2 = w2[0];
  }
  if (active && node == last) {
    // the ratios and the logistic with refined hardware reciprocals (full float64 accuracy)
    const double r1 = t0 != 0.0 ? (t0 - t1) * rcp_nr(t0) : 0.0;
    const double r2 = t1 != 0.0 ? (t1 - t2) * rcp_nr(t1) : 0.0;
    const double en = fmax(r1, r2);
    // the logistic 1/(1 + exp(-x)) lies below alpha_min for x < -xcut and above
    // 1 - alpha_min for x > xcut (xcut = ln(1/alpha_min - 1)); beyond those by a margin the
    // clipped value is known without the exponential
    const double x = sharp * (en - thr);
    double al;
    if (x < -xcut - 1e-3) {
      al = 0.0;
    } else if (x > xcut + 1e-3) {
      al = 1.0;
    } else {
      al = rcp_nr(1.0 + exp(-x));
      if (al < alpha_min) al = 0.0;
      else if (al > 1.0 - alpha_min) al = 1.0;
    }
    al = fmin(al, alpha_max);
    alpha_raw[e] = al;
    if (energy) energy[e] = en;
  }
}

// One tile of elements (the body of the stage kernels).  sT holds the run's operator
// tables in LDS; they are loaded by the caller and become visible at the first barrier.
template <int DIM, int N, int VOL, int EPI, typename RT, int BUDGET>
__device__ __forceinline__ void stage_tile(typename StageLdsOf<DIM, N, VOL, RT, BUDGET>::type& s,
                                           const double* sT, const StageArgs& a, const Geom& g,
                                           int tile) {
  using S = Shape<DIM, N, BUDGET>;
  using SS = StageShape<DIM, N, RT, BUDGET>;
  constexpr int NV = S::NV, NN = S::NN;
  constexpr bool CONS = (VOL == VOL_CENTRAL || VOL == VOL_SHOCKCAP);
  const int le = elem_slot<NN>();
  const int node = (int)(threadIdx.x % (unsigned)NN);
  const int e = tile * S::NE + le;
  const bool inb = le < S::NE;
  const bool active = inb && (e < g.E);
  const int base = le * NN;
  const size_t ENN = (size_t)g.E * NN;
  const size_t own_ix = (size_t)e * NN + node;

  static_assert(sizeof(RT) == 8 || VOL == VOL_EC, "float32 volume fluxes: EC flux differencing only");
  double um[NV];
  double unb[DIM][NV];   // neighbours' face-node states, loaded up front
  Prim<double> qd;
  // float32 volume sums take the pressure relative to one reference per element (node 0's),
  // so they carry no large constant part; the constant's volume sum, p_ref times the row sum
  // of -(2/h_d) S (minus the lift factor at a face node, zero inside), cancels exactly
  // against p_ref in the lifted surface flux, which is removed there in float64 instead.
  double pref = 0.0;
  double al_e = 0.0;   // shock capturing: the element's blending factor
  if (active) {
#pragma unroll
    for (int v = 0; v < NV; ++v) um[v] = (a.uin + (size_t)e * NN + (size_t)v * ENN)[(unsigned)node];
    if constexpr (VOL == VOL_SHOCKCAP) {
      if (a.alpha_raw_in) {   // alpha_e = max(raw_e, raw of the face neighbours / 2)
        const double* ar = a.alpha_raw_in;
        double v = ar[e];
        if (a.alpha_smooth) {
          int ec[3];
          elem_xyz(g, e, ec);
#pragma unroll
          for (int d = 0; d < DIM; ++d) {
            v = fmax(v, 0.5 * ar[elem_nb(g, e, ec, d, -1)]);
            v = fmax(v, 0.5 * ar[elem_nb(g, e, ec, d, 1)]);
          }
        }
        al_e = v;
      } else {
        al_e = a.alpha[e];
      }
    }
    if constexpr (sizeof(RT) == 4 && !WaveElem<DIM, N>::value) {
      double u0[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) u0[v] = a.uin[(size_t)e * NN + (size_t)v * ENN];
      pref = pressure<DIM>(u0, g.gamma);
    }
    if (a.surf != SURF_NONE) {
      int ec[3];
      elem_xyz(g, e, ec);
      face_load<DIM, N, 0>(a.uin, g, e, ec, node, unb[0]);
      face_load<DIM, N, 1>(a.uin, g, e, ec, node, unb[1]);
      if constexpr (DIM == 3) face_load<DIM, N, 2>(a.uin, g, e, ec, node, unb[2]);
    }
    if (!cons_to_prim<DIM>(um, g.gamma, qd)) *g.flag = 1;
    if constexpr (sizeof(RT) == 4 && WaveElem<DIM, N>::value) {   // the wave is the element
      pref = __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(qd.p)),
                              __builtin_amdgcn_readfirstlane(__double2loint(qd.p)));
    }
    const int li = base + node;
    if constexpr (VOL == VOL_WEAK || VOL == VOL_WEAK_MFMA) {   // physical fluxes of this node
      double f[NV];
      phys_flux<DIM, 0>(um, qd, f);
#pragma unroll
      for (int v = 0; v < NV; ++v) s.f[0][v][li] = f[v];
      phys_flux<DIM, 1>(um, qd, f);
#pragma unroll
      for (int v = 0; v < NV; ++v) s.f[1][v][li] = f[v];
      if constexpr (DIM == 3) {
        phys_flux<DIM, 2>(um, qd, f);
#pragma unroll
        for (int v = 0; v < NV; ++v) s.f[2][v][li] = f[v];
      }
    } else {
      if constexpr (CONS) s.c[li] = qd.c;
      s.rho[li] = (RT)qd.rho;
#pragma unroll
      for (int k = 0; k < DIM; ++k) s.v[k][li] = (RT)(StagedHalfV<VOL>::value ? 0.5 * qd.v[k] : qd.v[k]);
      s.p[li] = (RT)(qd.p - pref);
      s.beta[li] = (RT)qd.beta;
      if constexpr (CONS) {
#pragma unroll
        for (int v = 0; v < NV; ++v) s.u[v][li] = um[v];
      }
    }
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) um[v] = 1.0;
    qd.rho = qd.p = qd.beta = qd.c = 1.0;
    qd.v[0] = qd.v[1] = qd.v[2] = 0.0;
  }

  if (VOL != VOL_WEAK && VOL != VOL_WEAK_MFMA && inb) {   // zero the partner-share accumulator
    double* x = reinterpret_cast<double*>(s.xb + le * SS::SLOT);
#pragma unroll
    for (int v = 0; v < NV; ++v) x[v * NN + node] = 0.0;
  }
  double R[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) R[v] = 0.0;
  __syncthreads();   // tables, staged nodes and zeroed accumulators visible

  // ---- surface: each boundary node's face flux, lifted onto the node
  if (a.surf != SURF_NONE && active) {
    constexpr bool PREF = sizeof(RT) == 4;
    surface_dir<DIM, N, 0, PREF>(g, a.surf, node, um, qd, unb[0], sT + TAB_LIFT, pref, R);
    surface_dir<DIM, N, 1, PREF>(g, a.surf, node, um, qd, unb[1], sT + TAB_LIFT, pref, R);
    if constexpr (DIM == 3) surface_dir<DIM, N, 2, PREF>(g, a.surf, node, um, qd, unb[2], sT + TAB_LIFT, pref, R);
  }

  // ---- volume
  if constexpr (VOL == VOL_WEAK_MFMA) {
    static_assert(DIM == 3 && N == 3, "the matrix-core weak form is built for 3D, N = 3");
    if (active) weak_mfma_n3(s, base, node, sT + TAB_S, R);   // uniform: one element per wave
  } else if constexpr (VOL == VOL_WEAK) {
    if (active) {
      weak_dir<DIM, N, 0>(s, base, node, sT + TAB_S, R);
      weak_dir<DIM, N, 1>(s, base, node, sT + TAB_S, R);
      if constexpr (DIM == 3) weak_dir<DIM, N, 2>(s, base, node, sT + TAB_S, R);
    }
  } else if constexpr (VOL != VOL_NONE) {
    double* x = reinterpret_cast<double*>(s.xb + (le < S::NE ? le : 0) * SS::SLOT);
    Prim<RT> me;
    me.rho = (RT)qd.rho;
#pragma unroll
    for (int k = 0; k < 3; ++k) me.v[k] = (RT)qd.v[k];
    RT hme[3];   // this node's velocity halved (the staged form of the EC volume)
#pragma unroll
    for (int k = 0; k < 3; ++k) hme[k] = (RT)(0.5 * qd.v[k]);
    me.p = (RT)(qd.p - pref);
    me.beta = (RT)qd.beta;
    const RT inv_gm1 = (RT)g.inv_gm1;
    // float64 without blending: the surface terms seed the volume accumulator (fewer live
    // registers through the pair rounds)
    constexpr bool SEED = (VOL != VOL_SHOCKCAP) && sizeof(RT) == 8;
    RT acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = SEED ? (RT)R[v] : RT(0);
    // even n with the EC flux: the x and y half rounds run as one packed round
    constexpr bool PACK = (N % 2 == 1) && (VOL == VOL_EC || VOL == VOL_SHOCKCAP);
    volume_dir<DIM, N, 0, VOL, RT, !PACK>(s, x, active, base, node, me, hme, um, sT + TAB_S, inv_gm1, (RT)pref, acc);
    volume_dir<DIM, N, 1, VOL, RT, !PACK>(s, x, active, base, node, me, hme, um, sT + TAB_S, inv_gm1, (RT)pref, acc);
    if constexpr (PACK)
      volume_xy_half<DIM, N, VOL, RT>(s, x, active, base, node, me, hme, sT + TAB_S, inv_gm1, (RT)pref, acc);
    if constexpr (DIM == 3)
      volume_dir<DIM, N, 2, VOL, RT, true>(s, x, active, base, node, me, hme, um, sT + TAB_S, inv_gm1, (RT)pref, acc);
    elem_sync<DIM, N>();   // every partner share has landed
    if (active) {
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] += (RT)x[v * NN + node];
    }
    if constexpr (VOL == VOL_SHOCKCAP) {
      // blended subcell FV part: the partner-share slot x is free once every node has read
      // its shares and holds the shared subcell fluxes; a one-wave element skips it when its
      // alpha is zero, a block of other shapes when every alpha in it is zero
      const double al = al_e;
      double fv[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) fv[v] = 0.0;
      const bool any = WaveElem<DIM, N>::value ? (al != 0.0) : (__syncthreads_or(al != 0.0) != 0);
      if (any) {
        const bool on = active && al != 0.0;
        elem_sync<DIM, N>();
        fv_dir<DIM, N, 0>(s, x, a.fvf, on, base, node, qd, um, sT + TAB_FV, g.gamma, fv);
        fv_dir<DIM, N, 1>(s, x, a.fvf, on, base, node, qd, um, sT + TAB_FV, g.gamma, fv);
        if constexpr (DIM == 3)
          fv_dir<DIM, N, 2>(s, x, a.fvf, on, base, node, qd, um, sT + TAB_FV, g.gamma, fv);
      }
      if (active) {
#pragma unroll
        for (int v = 0; v < NV; ++v)
          R[v] += al != 0.0 ? (1.0 - al) * (double)acc[v] + al * fv[v] : (double)acc[v];
      }
    } else if (active) {
      if constexpr (SEED) {
#pragma unroll
        for (int v = 0; v < NV; ++v) R[v] = (double)acc[v];
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) R[v] += (double)acc[v];
      }
    }
  }

  // ---- epilogue
  constexpr bool IND = VOL == VOL_SHOCKCAP && EPI == EPI_RK;   // indicator of the output
  double un[NV];
  auto speeds = [&](const double (&un)[NV], double (&ls)[DIM]) {
        Prim<double> q;
        const bool ok = cons_to_prim<DIM, false>(un, g.gamma, q);
#pragma unroll
        for (int d = 0; d < DIM; ++d) ls[d] = sT[TAB_JAC + d] * (fabs(q.v[d]) + q.c);
        return ok;
      };
  const double dt_used = stage_epilogue<DIM, N, NV, EPI, BUDGET, decltype(speeds), true>(
      s.xb, a, g, le, node, e, inb, active, ENN, own_ix, um, R, speeds, IND ? un : nullptr);
  // shock capturing: the raw indicator of the state just written, for the next stage (the
  // computation of k_indicator on the same values, in the element's LDS slot)
  if constexpr (IND) {
    if (a.alpha_next) {   // uniform
      double* w = reinterpret_cast<double*>(s.xb + (le < S::NE ? le : 0) * SS::SLOT);
      elem_sync<DIM, N>();   // the epilogue is done with the slot
      if (active) {
        double q;
        if (!rho_p<DIM>(un, g.gamma, q)) *g.flag = 1;
        w[node] = q;
      }
      indicator_elem<DIM, N>(w, w + NN, w + 2 * NN, sT + TAB_VINV, node, inb, active, a.ind_thr,
                             a.ind_sharp, a.ind_amin, a.ind_amax, a.ind_xcut, a.alpha_next,
                             nullptr, e);
    }
  }
  if constexpr (EPI == EPI_RK) {
    if (a.t_step && blockIdx.x == 0 && threadIdx.x == 0) stage_time_publish(a, dt_used);
    if (a.slots_clear && blockIdx.x == 0 && threadIdx.x < (unsigned)DT_SLOTS)
      a.slots_clear[threadIdx.x * DT_SLOT_STRIDE] = 0.0;
  }
}

// The matrix-core variant asks for 4 waves per SIMD (its accumulators would otherwise push
// the register count past 128).
template <int DIM, int N, int VOL, int EPI, typename RT>
__global__ __launch_bounds__((Shape<DIM, N>::THREADS), (VOL == VOL_WEAK_MFMA ? 4 : 1))
void k_stage(StageArgs a, Geom g) {
  __shared__ typename StageLdsOf<DIM, N, VOL, RT>::type s;
  __shared__ double sT[TAB_SIZE];
  for (int i = threadIdx.x; i < TAB_SIZE; i += blockDim.x) sT[i] = g.tab[i];
  stage_tile<DIM, N, VOL, EPI, RT, 256>(s, sT, a, g, (int)xcd_tile(blockIdx.x, gridDim.x));
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
    Geom g, double alpha_min, double alpha_max, double thr, double sharp, double xcut) {
  using S = Shape<DIM, N>;
  constexpr int NN = S::NN;
  __shared__ double sa[S::NE * NN], sb[S::NE * NN], sc[S::NE * NN];
  __shared__ double sV[TMAX * TMAX];
  for (int i = threadIdx.x; i < TMAX * TMAX; i += blockDim.x) sV[i] = g.tab[TAB_VINV + i];
  const int le = elem_slot<NN>();
  const int node = (int)(threadIdx.x % (unsigned)NN);
  const int64_t e = (int64_t)blockIdx.x * S::NE + le;
  const bool active = (le < S::NE) && (e < g.E);
  const int base = (le < S::NE ? le : 0) * NN;
  const int64_t ENN = g.E * NN;
  if (active) {
    double um[S::NV];
#pragma unroll
    for (int v = 0; v < S::NV; ++v) um[v] = u[v * ENN + e * NN + node];
    double q;
    if (!rho_p<DIM>(um, g.gamma, q)) *g.flag = 1;
    sa[base + node] = q;
  }
  __syncthreads();   // V^-1
  indicator_elem<DIM, N>(sa + base, sb + base, sc + base, sV, node, le < S::NE, active, thr,
                         sharp, alpha_min, alpha_max, xcut, alpha_raw, energy, e);
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
// Max of p[0, n) over one block of T threads (T a multiple of 64), valid in thread 0.
// Eight independent loads per thread are kept in flight: the pass reads a few hundred KB
// from a single CU, so it is bound by load latency, not bandwidth.  max is exact, so the
// result does not depend on the order.  s: LDS scratch of T / 64 doubles.
// --------------------------------------------------------------------------------------
template <int T>
__device__ double block_max(const double* __restrict__ p, int64_t n, double* s) {
  static_assert(T % 64 == 0 && T <= 4096, "block of whole waves");
  double m[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int64_t i = threadIdx.x;
  for (; i + 7 * T < n; i += 8 * T) {
#pragma unroll
    for (int k = 0; k < 8; ++k) m[k] = fmax(m[k], p[i + k * T]);
  }
  for (; i < n; i += T) m[0] = fmax(m[0], p[i]);
  double r = fmax(fmax(fmax(m[0], m[1]), fmax(m[2], m[3])), fmax(fmax(m[4], m[5]), fmax(m[6], m[7])));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) r = fmax(r, __shfl_xor(r, o));
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = r;
  __syncthreads();
  if (threadIdx.x < 64) {
    r = (int)threadIdx.x < T / 64 ? s[threadIdx.x] : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) r = fmax(r, __shfl_xor(r, o));
  }
  return r;
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
  constexpr int P2 = NN <= 4 ? 4 : NN <= 16 ? 16 : NN <= 64 ? 64 : NN <= 128 ? 128 : NN <= 256 ? 256 : 512;
  __shared__ double sm[DIM][S::NE * NN];
  const int le = threadIdx.x / NN;
  const int node = threadIdx.x - le * NN;
  const int64_t e = (int64_t)blockIdx.x * S::NE + le;
  const bool inb = le < S::NE;
  const bool active = inb && (e < g.E);
  const int base = le * NN;
  const int64_t ENN = g.E * NN;
  if (inb) {
    if (active) {
      double um[S::NV];
#pragma unroll
      for (int v = 0; v < S::NV; ++v) um[v] = u[v * ENN + e * NN + node];
      Prim<double> q;
      if (!cons_to_prim<DIM>(um, g.gamma, q)) *g.flag = 1;
#pragma unroll
      for (int d = 0; d < DIM; ++d) sm[d][base + node] = fabs(q.v[d]) + q.c;
    } else {
#pragma unroll
      for (int d = 0; d < DIM; ++d) sm[d][base + node] = 0.0;
    }
  }
  __syncthreads();
  for (int half = P2 / 2; half > 0; half >>= 1) {
    if (inb && node < half && node + half < NN) {
#pragma unroll
      for (int d = 0; d < DIM; ++d)
        sm[d][base + node] = fmax(sm[d][base + node], sm[d][base + node + half]);
    }
    __syncthreads();
  }
  if (active && node == 0) {
    double lam = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) lam += g.tab[TAB_JAC + d] * sm[d][base];
    partial[e] = lam;
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
