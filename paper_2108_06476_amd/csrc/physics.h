// physics.h -- pointwise ideal-gas Euler physics for the gfx950 kernels.
//
// Conservation law of Eq. (1) (Section 2) for the Euler equations of an ideal gas,
// no source term.  Two-point and interface fluxes named in Sections 2.3.1 and 3.1:
// the entropy-conservative, kinetic-energy-preserving volume flux, the central flux,
// local Lax-Friedrichs and HLL.  Direction is a compile-time parameter so velocity
// components stay in registers.
#pragma once
#include <hip/hip_runtime.h>

namespace dgx {

// Primitive state kept per node: rho, v, p, beta = rho/p (the argument of the second
// logarithmic mean, computed once per node instead of once per pair) and the sound speed c.
template <typename T>
struct Prim {
  T rho, v[3], p, beta, c;
};

// 1/x from the hardware reciprocal refined by two Newton steps (x > 0, normal).
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// 1/x with one Newton step (relative error 2.2e-15 on gfx950, against 4.6e-8 for the bare
// hardware reciprocal): enough where the reciprocal only forms z = (b - a)/(b + a), whose
// square enters a series with weight <= 1/3 below z^2 = 1e-4, and for float32 results.
__device__ __forceinline__ double rcp_nr1(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

// sqrt(x) for normal x > 0: the hardware reciprocal square root, one Newton step on
// (g, h) = (sqrt x, 1/(2 sqrt x)) and two residual corrections g += (x - g^2) h.
__device__ __forceinline__ double sqrt_pos(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  double d = fma(-g, g, x);
  g = fma(d, h, g);
  d = fma(-g, g, x);
  return fma(d, h, g);
}

// sqrt_pos with one residual correction (within about an ulp): the sound speed of the
// primitive conversion, whose relative error of order 1e-16 stays far below the right-hand
// side's float64 parity bar.
__device__ __forceinline__ double sqrt_pos1(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  return fma(fma(-g, g, x), h, g);
}

// The log means' middle branch (1e-4 <= z^2 < 0.1) as polynomials of degree 10 in x = z^2:
// P(x) = z/(2 artanh z) and 2Q(x) = 2 artanh(z)/z, the interpolants at Chebyshev nodes of
// [0, 0.1] formed at 60 digits (logmean_fit.py beside this file).  Both are analytic for
// |x| < 1, so ten degrees leave about 1e-18 relative error with these float64 coefficients,
// and neither needs a reciprocal or a logarithm.
__device__ __forceinline__ double ln_mean_mid(double x) {
  constexpr double kP[11] = {
      0.5, -0.1666666666666666, -0.04444444444447207, -0.023280423276128673,
      -0.015097002105376345, -0.010898386189257736, -0.008394230906424155,
      -0.00674302519561495, -0.005699575913500763, -0.004061649743847389,
      -0.006793753103187953};
  double p = kP[10];
#pragma unroll
  for (int k = 9; k >= 0; --k) p = fma(p, x, kP[k]);
  return p;
}

__device__ __forceinline__ double inv_ln_mean_mid(double x) {
  constexpr double kQ[11] = {   // Q(x) = artanh(z)/z; the factor 2 is applied exactly below
      1.0, 0.3333333333333325, 0.20000000000033863, 0.14285714280450776,
      0.11111111529834054, 0.09090889710268459, 0.07692864848122398,
      0.06656438300891282, 0.060018248406360414, 0.04412879698538037,
      0.0802184520988054};
  double p = 2.0 * kQ[10];
#pragma unroll
  for (int k = 9; k >= 0; --k) p = fma(p, x, 2.0 * kQ[k]);
  return p;
}

// Logarithmic mean {{a}}_ln = (b - a)/(ln b - ln a) and its reciprocal.  With
// z = (b - a)/(b + a), ln(b/a) = 2 artanh z, so {{a}}_ln = (a + b)/2 * z/artanh(z) and
// 1/{{a}}_ln = 2/(a + b) * artanh(z)/z.  Below z^2 = 1e-4 (the threshold of the efficiency
// reference the paper cites, Section 3.2) both use their Taylor series in z^2 to z^6
// (truncation below 1.2e-17), so one reciprocal of a + b serves the whole evaluation; up to
// z^2 = 0.1 (states within a factor 1.9) the degree-10 polynomials above replace the
// logarithm and its two divisions (MID; a kernel that never meets such jumps and is short of
// registers leaves it out); beyond it the logarithm.
template <bool MID = true>
__device__ __forceinline__ double ln_mean(double a, double b) {
  const double s = a + b, d = b - a;
  const double r = rcp_nr1(s);   // only z is formed from it
  const double z = d * r, z2 = z * z;
  if (z2 < 1.0e-4)   // (s/2)(1 - z^2/3 - 4 z^4/45 - 44 z^6/945), the 1/2 in the coefficients
    return s * (0.5 + z2 * (-1.0 / 6.0 + z2 * (-2.0 / 45.0 + z2 * (-22.0 / 945.0))));
  if (MID && z2 < 0.1) return s * ln_mean_mid(z2);
  const double hi = fmax(a, b), lo = fmin(a, b);   // symmetric in (a, b), bit for bit
  return (hi - lo) / log(hi / lo);
}

// The reciprocal 1/(a + b) takes one Newton step: its relative error (2.2e-15) enters the
// result linearly, two orders below what the right-hand side's float64 parity bar allows.
template <bool MID = true>
__device__ __forceinline__ double inv_ln_mean(double a, double b) {
  const double s = a + b, d = b - a;
  const double r = rcp_nr1(s);
  const double z = d * r, z2 = z * z;
  if (z2 < 1.0e-4)   // (2/s)(1 + z^2/3 + z^4/5 + z^6/7), the 2 in the coefficients
    return r * (2.0 + z2 * (2.0 / 3.0 + z2 * (2.0 / 5.0 + z2 * (2.0 / 7.0))));
  if (MID && z2 < 0.1) return r * inv_ln_mean_mid(z2);
  const double hi = fmax(a, b), lo = fmin(a, b);
  return log(hi / lo) / (hi - lo);
}

// Mixed precision: the near-equal branch is evaluated in float64, the log branch in
// float32.  For a float32 result the series serves up to z^2 = 1e-2: its truncation there
// (the first omitted terms, 428/14175 z^8 and z^8/9) is 3e-10 and 1.1e-9 relative, below
// float32 rounding, while ln(b/a) in float32 loses relative accuracy as b/a -> 1.
__device__ __forceinline__ float ln_mean(float a, float b) {
  const double s = (double)a + (double)b, d = (double)b - (double)a;
  const double r = rcp_nr1(s);
  const double z = d * r, z2 = z * z;
  if (z2 < 1.0e-2)
    return (float)(0.5 * s * (1.0 + z2 * (-1.0 / 3.0 + z2 * (-4.0 / 45.0 + z2 * (-44.0 / 945.0)))));
  return (b - a) / __logf(b / a);
}

__device__ __forceinline__ float inv_ln_mean(float a, float b) {
  const double s = (double)a + (double)b, d = (double)b - (double)a;
  const double r = rcp_nr1(s);   // float32 result
  const double z = d * r, z2 = z * z;
  if (z2 < 1.0e-2)
    return (float)(2.0 * r * (1.0 + z2 * (1.0 / 3.0 + z2 * (1.0 / 5.0 + z2 * (1.0 / 7.0)))));
  return __logf(b / a) / (b - a);
}

// Conserved -> primitive (beta = rho/p only when BETA).  Returns false for a non-physical
// state.  The reciprocals of rho and p take one Newton step (relative error 2.2e-15) and the
// sound speed one residual correction: the errors enter the fluxes linearly, three orders
// below the float64 parity bar, and each conversion runs for every node and again for the
// neighbours' face nodes.
template <int DIM, bool BETA = true>
__device__ __forceinline__ bool cons_to_prim(const double (&u)[DIM + 2], double gamma,
                                             Prim<double>& q) {
  q.rho = u[0];
  const double inv = rcp_nr1(u[0]);
  double v2 = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) q.v[k] = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    q.v[k] = u[1 + k] * inv;
    v2 += q.v[k] * q.v[k];
  }
  q.p = (gamma - 1.0) * (u[DIM + 1] - 0.5 * u[0] * v2);
  q.beta = BETA ? q.rho * rcp_nr1(q.p) : 0.0;
  q.c = sqrt_pos1(gamma * q.p * inv);
  return (q.rho > 0.0) && (q.p > 0.0) && (q.p < 1.0e300) && (q.rho < 1.0e300);
}

// The shock indicator's variable q = rho p of a conserved state, formed without a division:
// rho p = (gamma - 1) (rho (rho E) - |rho v|^2 / 2).  Returns false for a non-physical state
// (rho <= 0, p <= 0, or not finite).
template <int DIM>
__device__ __forceinline__ bool rho_p(const double (&u)[DIM + 2], double gamma, double& q) {
  double m2 = u[1] * u[1];
#pragma unroll
  for (int k = 2; k <= DIM; ++k) m2 = fma(u[k], u[k], m2);
  q = (gamma - 1.0) * fma(u[0], u[DIM + 1], -0.5 * m2);
  return (u[0] > 0.0) && (q > 0.0) && (q < 1.0e300) && (u[0] < 1.0e300);
}

// Entropy-conservative, kinetic-energy-preserving two-point flux in direction D:
//   f_rho  = {{rho}}_ln {{v_D}},  f_rhov = f_rho {{v}} + {{p}} e_D,
//   f_rhoE = f_rho (1/((gamma-1) {{rho/p}}_ln) + v_L.v_R/2) + (p_L v_DR + p_R v_DL)/2.
template <int DIM, int D, typename T>
__device__ __forceinline__ void ec_flux(const Prim<T>& L, const Prim<T>& R, T inv_gm1,
                                        T (&f)[DIM + 2]) {
  const T rho_ln = ln_mean(L.rho, R.rho);
  const T ibeta = inv_ln_mean(L.beta, R.beta);
  const T half = T(0.5);
  T vLvR = L.v[0] * R.v[0];
#pragma unroll
  for (int k = 1; k < DIM; ++k) vLvR += L.v[k] * R.v[k];
  const T frho = rho_ln * (half * (L.v[D] + R.v[D]));
  const T pavg = half * (L.p + R.p);
  f[0] = frho;
#pragma unroll
  for (int k = 0; k < DIM; ++k) f[1 + k] = frho * (half * (L.v[k] + R.v[k])) + (k == D ? pavg : T(0));
  f[DIM + 1] = frho * (ibeta * inv_gm1 + half * vLvR) + half * (L.p * R.v[D] + R.p * L.v[D]);
}

// The EC flux with the partner's velocities stored halved (R.v = v_R/2) and the node's own
// halves hL = v_L/2 beside its full L.v: {{v}} = hL + R.v, v_L.v_R/2 = L.v . R.v and
// (p_L v_DR + p_R v_DL)/2 = p_L R.v_D + p_R hL_D.  Halving is exact, so the values are those
// of ec_flux with five multiplications fewer per pair.
template <int DIM, int D, typename T>
__device__ __forceinline__ void ec_flux_h(const Prim<T>& L, const T (&hL)[3], const Prim<T>& R,
                                          T inv_gm1, T (&f)[DIM + 2]) {
  const T rho_ln = ln_mean(L.rho, R.rho);
  const T ibeta = inv_ln_mean(L.beta, R.beta);
  T vv = L.v[0] * R.v[0];   // v_L . v_R / 2
#pragma unroll
  for (int k = 1; k < DIM; ++k) vv += L.v[k] * R.v[k];
  const T frho = rho_ln * (hL[D] + R.v[D]);
  const T pavg = T(0.5) * (L.p + R.p);
  f[0] = frho;
#pragma unroll
  for (int k = 0; k < DIM; ++k) f[1 + k] = frho * (hL[k] + R.v[k]) + (k == D ? pavg : T(0));
  f[DIM + 1] = frho * (ibeta * inv_gm1 + vv) + (L.p * R.v[D] + R.p * hL[D]);
}

// The EC flux of float32 states whose pressures are perturbations p - p_ref about one
// reference per element: the momentum flux carries {{p - p_ref}} (the constant part's volume
// sum is p_ref times a row sum of the volume operator, which the caller accounts for with
// the lifted surface flux), the energy flux the full (p_L v_DR + p_R v_DL)/2, split as the
// perturbations' products plus p_ref {{v_D}}.  Velocities as in ec_flux_h: the partner's
// halved, the node's own full in L.v and halved in hL.
template <int DIM, int D>
__device__ __forceinline__ void ec_flux_pp(const Prim<float>& L, const float (&hL)[3],
                                           const Prim<float>& R, float inv_gm1, float pref,
                                           float (&f)[DIM + 2]) {
  const float rho_ln = ln_mean(L.rho, R.rho);
  const float ibeta = inv_ln_mean(L.beta, R.beta);
  float vv = L.v[0] * R.v[0];   // v_L . v_R / 2
#pragma unroll
  for (int k = 1; k < DIM; ++k) vv += L.v[k] * R.v[k];
  const float vd = hL[D] + R.v[D];
  const float frho = rho_ln * vd;
  f[0] = frho;
#pragma unroll
  for (int k = 0; k < DIM; ++k)
    f[1 + k] = frho * (hL[k] + R.v[k]) + (k == D ? 0.5f * (L.p + R.p) : 0.0f);
  f[DIM + 1] = frho * (ibeta * inv_gm1 + vv) + (L.p * R.v[D] + R.p * hL[D]) + pref * vd;
}

// Pressure of a conserved state (the reference of the float32 volume path).
template <int DIM>
__device__ __forceinline__ double pressure(const double (&u)[DIM + 2], double gamma) {
  double m2 = u[1] * u[1];
#pragma unroll
  for (int k = 2; k <= DIM; ++k) m2 += u[k] * u[k];
  return (gamma - 1.0) * (u[DIM + 1] - 0.5 * m2 / u[0]);
}

// The EC flux with its state-pair products kept apart, so that f#(L, R) and f#(R, L) agree
// bit for bit (both elements of an interface evaluate it).
template <int DIM, int D>
__device__ __forceinline__ void ec_flux_sym(const Prim<double>& L, const Prim<double>& R,
                                            double inv_gm1, double (&f)[DIM + 2]) {
  const double rho_ln = ln_mean(L.rho, R.rho);
  const double ibeta = inv_ln_mean(L.beta, R.beta);
  double vLvR = L.v[0] * R.v[0];
#pragma unroll
  for (int k = 1; k < DIM; ++k) vLvR += L.v[k] * R.v[k];
  const double frho = rho_ln * (0.5 * (L.v[D] + R.v[D]));
  const double pavg = 0.5 * (L.p + R.p);
  f[0] = frho;
#pragma unroll
  for (int k = 0; k < DIM; ++k) f[1 + k] = frho * (0.5 * (L.v[k] + R.v[k])) + (k == D ? pavg : 0.0);
  const double pv = __dadd_rn(__dmul_rn(L.p, R.v[D]), __dmul_rn(R.p, L.v[D]));
  f[DIM + 1] = frho * (ibeta * inv_gm1 + 0.5 * vLvR) + 0.5 * pv;
}

// Physical flux f^D(u) = (rho v_D, rho v_D v + p e_D, v_D (rho E + p)).
template <int DIM, int D>
__device__ __forceinline__ void phys_flux(const double (&u)[DIM + 2], const Prim<double>& q,
                                          double (&f)[DIM + 2]) {
  f[0] = u[1 + D];
#pragma unroll
  for (int k = 0; k < DIM; ++k) f[1 + k] = u[1 + D] * q.v[k] + (k == D ? q.p : 0.0);
  f[DIM + 1] = q.v[D] * (u[DIM + 1] + q.p);
}

// Central flux (f(u_L) + f(u_R))/2 (flux differencing with it is the weak form).
template <int DIM, int D>
__device__ __forceinline__ void central_flux(const double (&uL)[DIM + 2], const Prim<double>& L,
                                             const double (&uR)[DIM + 2], const Prim<double>& R,
                                             double (&f)[DIM + 2]) {
  double fL[DIM + 2], fR[DIM + 2];
  phys_flux<DIM, D>(uL, L, fL);
  phys_flux<DIM, D>(uR, R, fR);
#pragma unroll
  for (int v = 0; v < DIM + 2; ++v) f[v] = 0.5 * (fL[v] + fR[v]);
}

// The interface fluxes below return f up to a scalar factor, which they return: the flux is
// factor * f.  A caller that scales the result anyway (the lift) folds the factor into its
// coefficient and saves one multiplication per variable.

// Local Lax-Friedrichs: (f_L + f_R)/2 - lambda (u_R - u_L)/2,
// lambda = max(|v_DL| + c_L, |v_DR| + c_R); f holds twice the flux (factor 1/2).
template <int DIM, int D>
__device__ __forceinline__ double llf_flux(const double (&uL)[DIM + 2], const Prim<double>& L,
                                           const double (&uR)[DIM + 2], const Prim<double>& R,
                                           double /*gamma: in the primitives*/, double (&f)[DIM + 2]) {
  double fL[DIM + 2], fR[DIM + 2];
  phys_flux<DIM, D>(uL, L, fL);
  phys_flux<DIM, D>(uR, R, fR);
  const double lam = fmax(fabs(L.v[D]) + L.c, fabs(R.v[D]) + R.c);
#pragma unroll
  for (int v = 0; v < DIM + 2; ++v) f[v] = (fL[v] + fR[v]) - lam * (uR[v] - uL[v]);
  return 0.5;
}

// HLL with s_L = min(v_DL - c_L, v_DR - c_R), s_R = max(v_DL + c_L, v_DR + c_R): f_L for
// s_L >= 0, f_R for s_R <= 0, else (s_R f_L - s_L f_R + s_L s_R (u_R - u_L)) / (s_R - s_L),
// returned without the division (factor 1/(s_R - s_L)).
template <int DIM, int D>
__device__ __forceinline__ double hll_flux(const double (&uL)[DIM + 2], const Prim<double>& L,
                                           const double (&uR)[DIM + 2], const Prim<double>& R,
                                           double /*gamma: in the primitives*/, double (&f)[DIM + 2]) {
  double fL[DIM + 2], fR[DIM + 2];
  phys_flux<DIM, D>(uL, L, fL);
  phys_flux<DIM, D>(uR, R, fR);
  const double sL = fmin(L.v[D] - L.c, R.v[D] - R.c);
  const double sR = fmax(L.v[D] + L.c, R.v[D] + R.c);
  if (sL >= 0.0) {
#pragma unroll
    for (int v = 0; v < DIM + 2; ++v) f[v] = fL[v];
    return 1.0;
  }
  if (sR <= 0.0) {
#pragma unroll
    for (int v = 0; v < DIM + 2; ++v) f[v] = fR[v];
    return 1.0;
  }
#pragma unroll
  for (int v = 0; v < DIM + 2; ++v) f[v] = sR * fL[v] - sL * fR[v] + sL * sR * (uR[v] - uL[v]);
  return rcp_nr(sR - sL);
}

enum { SURF_LLF = 0, SURF_HLL = 1, SURF_EC = 2, SURF_NONE = 3 };

}  // namespace dgx

namespace dgx {

// ---- curvilinear elements (3D): fluxes along a (not necessarily unit) vector a -----------

// sum_n a_n f^n(u) = (rho v.a, rho v (v.a) + p a, (v.a)(rho E + p)).
__device__ __forceinline__ void flux_vec(const double (&u)[5], const Prim<double>& q,
                                         const double (&a)[3], double (&f)[5]) {
  const double va = q.v[0] * a[0] + q.v[1] * a[1] + q.v[2] * a[2];
  f[0] = u[0] * va;
#pragma unroll
  for (int k = 0; k < 3; ++k) f[1 + k] = u[1 + k] * va + q.p * a[k];
  f[4] = va * (u[4] + q.p);
}

// The EC two-point flux contracted with a, sum_n a_n f#_n(L, R): the volume flux of a
// curvilinear element with a the average of the two nodes' metric vectors (J a^i).
__device__ __forceinline__ void ec_flux_vec(const Prim<double>& L, const Prim<double>& R,
                                            const double (&a)[3], double inv_gm1,
                                            double (&f)[5]) {
  const double rho_ln = ln_mean(L.rho, R.rho);
  const double ibeta = inv_ln_mean(L.beta, R.beta);
  double vs[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) vs[k] = 0.5 * (L.v[k] + R.v[k]);
  const double vLvR = L.v[0] * R.v[0] + L.v[1] * R.v[1] + L.v[2] * R.v[2];
  const double frho = rho_ln * (vs[0] * a[0] + vs[1] * a[1] + vs[2] * a[2]);
  const double pavg = 0.5 * (L.p + R.p);
  f[0] = frho;
#pragma unroll
  for (int k = 0; k < 3; ++k) f[1 + k] = frho * vs[k] + pavg * a[k];
  const double vRa = R.v[0] * a[0] + R.v[1] * a[1] + R.v[2] * a[2];
  const double vLa = L.v[0] * a[0] + L.v[1] * a[1] + L.v[2] * a[2];
  f[4] = frho * (ibeta * inv_gm1 + 0.5 * vLvR) + 0.5 * (L.p * vRa + R.p * vLa);
}

// ec_flux_vec with the partner's velocities stored halved (R.v = v_R/2), the node's own
// halves hL beside its full L.v (as ec_flux_h), returning the flux contracted with a.
__device__ __forceinline__ void ec_flux_vec_h(const Prim<double>& L, const double (&hL)[3],
                                              const Prim<double>& R, const double (&a)[3],
                                              double inv_gm1, double (&f)[5]) {
  const double rho_ln = ln_mean(L.rho, R.rho);
  const double ibeta = inv_ln_mean(L.beta, R.beta);
  double vs[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) vs[k] = hL[k] + R.v[k];
  const double vv = L.v[0] * R.v[0] + L.v[1] * R.v[1] + L.v[2] * R.v[2];   // v_L.v_R/2
  const double frho = rho_ln * (vs[0] * a[0] + vs[1] * a[1] + vs[2] * a[2]);
  const double pavg = 0.5 * (L.p + R.p);
  f[0] = frho;
#pragma unroll
  for (int k = 0; k < 3; ++k) f[1 + k] = frho * vs[k] + pavg * a[k];
  const double hRa = R.v[0] * a[0] + R.v[1] * a[1] + R.v[2] * a[2];
  const double hLa = hL[0] * a[0] + hL[1] * a[1] + hL[2] * a[2];
  f[4] = frho * (ibeta * inv_gm1 + vv) + (L.p * hRa + R.p * hLa);
}

// Central two-point flux contracted with a: (f_a(u_L) + f_a(u_R))/2.
__device__ __forceinline__ void central_flux_vec(const double (&uL)[5], const Prim<double>& L,
                                                 const double (&uR)[5], const Prim<double>& R,
                                                 const double (&a)[3], double (&f)[5]) {
  double fL[5], fR[5];
  flux_vec(uL, L, a, fL);
  flux_vec(uR, R, a, fR);
#pragma unroll
  for (int v = 0; v < 5; ++v) f[v] = 0.5 * (fL[v] + fR[v]);
}

// Interface flux through a face with contravariant vector a (from L to R): LLF and HLL
// with the wave speeds scaled by |a| (|a| f*(u_L, u_R; a/|a|)), EC as ec_flux_vec.  Returns
// the factor that turns f into the flux (as llf_flux and hll_flux; the caller folds it into
// its lift coefficient): 0.5 for LLF, 1/(s_R - s_L) for HLL between its wave speeds, else 1.
__device__ __forceinline__ double surface_flux_vec(int surf, const double (&uL)[5],
                                                   const Prim<double>& L, const double (&uR)[5],
                                                   const Prim<double>& R, const double (&a)[3],
                                                   double inv_gm1, double (&f)[5]) {
  if (surf == SURF_EC) {
    ec_flux_vec(L, R, a, inv_gm1, f);
    return 1.0;
  }
  double fL[5], fR[5];
  flux_vec(uL, L, a, fL);
  flux_vec(uR, R, a, fR);
  const double al = sqrt_pos(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
  const double vL = L.v[0] * a[0] + L.v[1] * a[1] + L.v[2] * a[2];
  const double vR = R.v[0] * a[0] + R.v[1] * a[1] + R.v[2] * a[2];
  if (surf == SURF_LLF) {
    const double lam = fmax(fabs(vL) + L.c * al, fabs(vR) + R.c * al);
#pragma unroll
    for (int v = 0; v < 5; ++v) f[v] = (fL[v] + fR[v]) - lam * (uR[v] - uL[v]);
    return 0.5;
  }
  const double sL = fmin(vL - L.c * al, vR - R.c * al);
  const double sR = fmax(vL + L.c * al, vR + R.c * al);
  if (sL >= 0.0) {
#pragma unroll
    for (int v = 0; v < 5; ++v) f[v] = fL[v];
    return 1.0;
  }
  if (sR <= 0.0) {
#pragma unroll
    for (int v = 0; v < 5; ++v) f[v] = fR[v];
    return 1.0;
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) f[v] = sR * fL[v] - sL * fR[v] + sL * sR * (uR[v] - uL[v]);
  return rcp_nr(sR - sL);
}

// Source term of the manufactured solution rho = 2 + A sin(theta), theta = k (x+y+z) - om t,
// v = (1,1,1), rho E = rho^2 (A = 0.1, k = pi, om = 2 pi): s = du/dt + div f(u), with
// h = A cos(theta): s_rho = (3k - om) h, s_rhov = s_rho + (gamma-1)(2 rho - 1.5) k h,
// s_rhoE = -2 rho om h + 3 k (2 rho + (gamma-1)(2 rho - 1.5)) h.
__device__ __forceinline__ void mms_source(double gamma, double x, double y, double z, double t,
                                           double (&s)[5]) {
  constexpr double pi = 3.14159265358979323846;
  constexpr double A = 0.1, k = pi, om = 2.0 * pi;
  double sn, cs;
  sincos(k * (x + y + z) - om * t, &sn, &cs);
  const double rho = 2.0 + A * sn, h = A * cs;
  const double dp = (gamma - 1.0) * (2.0 * rho - 1.5) * k * h;
  s[0] = (3.0 * k - om) * h;
  s[1] = s[0] + dp;
  s[2] = s[0] + dp;
  s[3] = s[0] + dp;
  s[4] = -2.0 * rho * om * h + 3.0 * k * (2.0 * rho + (gamma - 1.0) * (2.0 * rho - 1.5)) * h;
}

}  // namespace dgx
