// registry.h -- host launchers of the templated kernels, one table per (dim, polydeg).
#pragma once
#include <cmath>
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "curv.h"
#include "mhd.h"
#include <limits>

namespace dgx {

enum { PREC_FP64 = 0, PREC_MIXED = 1 };

// Hennemann-Gassner constants of polydeg N: threshold T = 0.5 10^(-1.8 (N+1)^(1/4)) and
// sharpness ln((1 - 1e-4)/1e-4) / T.
inline void indicator_constants(int N, double& thr, double& sharp) {
  thr = 0.5 * std::pow(10.0, -1.8 * std::pow((double)(N + 1), 0.25));
  sharp = std::log((1.0 - 0.0001) / 0.0001) / thr;
}

// x beyond which the clipped logistic is known: 1/(1 + exp(-x)) < alpha_min for
// x < -ln(1/alpha_min - 1) and > 1 - alpha_min for x > ln(1/alpha_min - 1); infinite (never
// skip the exponential) unless 0 < alpha_min < 1/2.
inline double indicator_xcut(double alpha_min) {
  return (alpha_min > 0.0 && alpha_min < 0.5) ? std::log(1.0 / alpha_min - 1.0)
                                              : std::numeric_limits<double>::infinity();
}

struct Launchers {
  int threads = 0;   // block size of the element-tiled kernels
  int ne = 0;        // elements per block
  // returns hipErrorInvalidValue for an unsupported combination
  hipError_t (*stage)(hipStream_t, const StageArgs&, const Geom&, int vol, int epi, int prec) = nullptr;
  hipError_t (*indicator)(hipStream_t, const double* u, double* ar, double* en, const Geom&,
                          double amin, double amax) = nullptr;
  hipError_t (*smooth)(hipStream_t, const double* ar, double* a, const Geom&, int smooth) = nullptr;
  hipError_t (*maxspeed)(hipStream_t, const double* u, double* partial, const Geom&) = nullptr;
  hipError_t (*integrals)(hipStream_t, const double* u, const double* du, double* partial,
                          const Geom&) = nullptr;
  hipError_t (*coords)(hipStream_t, double* xyz, const Geom&, const double* xmin) = nullptr;
  // curvilinear elements (3D only; nullptr in 2D)
  hipError_t (*stage_curv)(hipStream_t, const StageArgs&, const Geom&, int vol, int epi) = nullptr;
  hipError_t (*maxspeed_curv)(hipStream_t, const double* u, double* partial, const Geom&) = nullptr;
  hipError_t (*geometry)(hipStream_t, const Geom&, const double* Dm, double warp, double* xyz,
                         double* ja, double* jac) = nullptr;
  // ideal MHD, weak form (3D only)
  hipError_t (*stage_mhd)(hipStream_t, const StageArgs&, const Geom&, int vol, int epi) = nullptr;
  hipError_t (*maxspeed_mhd)(hipStream_t, const double* u, double* partial, const Geom&) = nullptr;
  const char* volume_name = "";
};

// Filled by the per-dimension translation units; nullptr if (dim, N) is not compiled.
const Launchers* launchers_2d(int N);
const Launchers* launchers_3d(int N);

inline const Launchers* launchers(int dim, int N) {
  return dim == 2 ? launchers_2d(N) : (dim == 3 ? launchers_3d(N) : nullptr);
}

// Host launch helpers shared by the instantiation units.
template <int DIM, int N>
struct Launch {
  using S = Shape<DIM, N>;
  static unsigned blocks(int64_t E) { return (unsigned)((E + S::NE - 1) / S::NE); }

  template <int VOL, int EPI, typename RT>
  static hipError_t stage1(hipStream_t st, const StageArgs& a, const Geom& g) {
    hipLaunchKernelGGL((k_stage<DIM, N, VOL, EPI, RT>), dim3(blocks(g.E)), dim3(S::THREADS), 0, st,
                       a, g);
    return hipGetLastError();
  }

  template <int EPI>
  static hipError_t stage_epi(hipStream_t st, const StageArgs& a, const Geom& g, int vol, int prec) {
    if (vol == VOL_EC) {
      if (prec == PREC_MIXED) return stage1<VOL_EC, EPI, float>(st, a, g);
      return stage1<VOL_EC, EPI, double>(st, a, g);
    }
    if (prec != PREC_FP64) return hipErrorInvalidValue;
    if (vol == VOL_CENTRAL) return stage1<VOL_CENTRAL, EPI, double>(st, a, g);
    if (vol == VOL_NONE) return stage1<VOL_NONE, EPI, double>(st, a, g);
    if (vol == VOL_SHOCKCAP) return stage1<VOL_SHOCKCAP, EPI, double>(st, a, g);
    if (vol == VOL_WEAK) return stage1<VOL_WEAK, EPI, double>(st, a, g);
    if (vol == VOL_WEAK_MFMA) {
      if constexpr (DIM == 3 && N == 3) return stage1<VOL_WEAK_MFMA, EPI, double>(st, a, g);
      return hipErrorInvalidValue;
    }
    return hipErrorInvalidValue;
  }

  static hipError_t stage(hipStream_t st, const StageArgs& a, const Geom& g, int vol, int epi,
                          int prec) {
    if (epi == EPI_RK) return stage_epi<EPI_RK>(st, a, g, vol, prec);
    return stage_epi<EPI_RHS>(st, a, g, vol, prec);
  }

  static hipError_t indicator(hipStream_t st, const double* u, double* ar, double* en,
                              const Geom& g, double amin, double amax) {
    double thr, sharp;
    indicator_constants(N, thr, sharp);
    hipLaunchKernelGGL((k_indicator<DIM, N>), dim3(blocks(g.E)), dim3(S::THREADS), 0, st, u, ar,
                       en, g, amin, amax, thr, sharp, indicator_xcut(amin));
    return hipGetLastError();
  }

  static hipError_t smooth(hipStream_t st, const double* ar, double* a, const Geom& g, int sm) {
    hipLaunchKernelGGL((k_smooth<DIM>), dim3((unsigned)((g.E + 255) / 256)), dim3(256), 0, st, ar,
                       a, g, sm);
    return hipGetLastError();
  }

  static hipError_t maxspeed(hipStream_t st, const double* u, double* partial, const Geom& g) {
    hipLaunchKernelGGL((k_maxspeed<DIM, N>), dim3(blocks(g.E)), dim3(S::THREADS), 0, st, u,
                       partial, g);
    return hipGetLastError();
  }

  static hipError_t integrals(hipStream_t st, const double* u, const double* du, double* partial,
                              const Geom& g) {
    hipLaunchKernelGGL((k_integrals<DIM, N>), dim3(blocks(g.E)), dim3(S::THREADS), 0, st, u, du,
                       partial, g);
    return hipGetLastError();
  }

  static hipError_t coords(hipStream_t st, double* xyz, const Geom& g, const double* xmin) {
    const int64_t tot = g.E * S::NN;
    hipLaunchKernelGGL((k_coords<DIM, N>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                       xyz, g, xmin[0], xmin[1], xmin[2]);
    return hipGetLastError();
  }

  template <int VOL, int EPI>
  static hipError_t stage_curv1(hipStream_t st, const StageArgs& a, const Geom& g) {
    if constexpr (N == 3) {
      if (g.E <= CURV_SPLIT_MAX_E) {   // small meshes: four waves per element
        hipLaunchKernelGGL((k_stage_curv_split<VOL, EPI>), dim3((unsigned)g.E), dim3(256), 0, st, a, g);
        return hipGetLastError();
      }
    }
    hipLaunchKernelGGL((k_stage_curv<N, VOL, EPI>), dim3(blocks(g.E)), dim3(S::THREADS), 0, st, a, g);
    return hipGetLastError();
  }

  static hipError_t stage_curv(hipStream_t st, const StageArgs& a, const Geom& g, int vol, int epi) {
    if constexpr (DIM == 3) {
      if (epi == EPI_RK) {
        if (vol == VOL_EC) return stage_curv1<VOL_EC, EPI_RK>(st, a, g);
        if (vol == VOL_CENTRAL) return stage_curv1<VOL_CENTRAL, EPI_RK>(st, a, g);
        if (vol == VOL_NONE) return stage_curv1<VOL_NONE, EPI_RK>(st, a, g);
      } else {
        if (vol == VOL_EC) return stage_curv1<VOL_EC, EPI_RHS>(st, a, g);
        if (vol == VOL_CENTRAL) return stage_curv1<VOL_CENTRAL, EPI_RHS>(st, a, g);
        if (vol == VOL_NONE) return stage_curv1<VOL_NONE, EPI_RHS>(st, a, g);
      }
    }
    return hipErrorInvalidValue;
  }

  static hipError_t maxspeed_curv(hipStream_t st, const double* u, double* partial, const Geom& g) {
    if constexpr (DIM == 3) {
      hipLaunchKernelGGL((k_maxspeed_curv<N>), dim3(blocks(g.E)), dim3(S::THREADS), 0, st, u,
                         partial, g);
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }

  static hipError_t geometry(hipStream_t st, const Geom& g, const double* Dm, double warp,
                             double* xyz, double* ja, double* jac) {
    if constexpr (DIM == 3) {
      hipLaunchKernelGGL((k_curv_geometry<N>), dim3((unsigned)g.E), dim3(S::NN), 0, st, g, Dm,
                         warp, xyz, ja, jac);
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }

  static hipError_t stage_mhd(hipStream_t st, const StageArgs& a, const Geom& g, int vol, int epi) {
    if constexpr (DIM == 3) {
      if constexpr (N == 3) {
        if (g.E <= MHD_SPLIT_MAX_E) {   // small meshes: three waves per element
          const dim3 eg((unsigned)g.E), eb(192);
          if (vol == VOL_EC) {
            if (epi == EPI_RK) hipLaunchKernelGGL((k_stage_mhd_split<VOL_EC, EPI_RK>), eg, eb, 0, st, a, g);
            else hipLaunchKernelGGL((k_stage_mhd_split<VOL_EC, EPI_RHS>), eg, eb, 0, st, a, g);
          } else {
            if (epi == EPI_RK) hipLaunchKernelGGL((k_stage_mhd_split<VOL_WEAK, EPI_RK>), eg, eb, 0, st, a, g);
            else hipLaunchKernelGGL((k_stage_mhd_split<VOL_WEAK, EPI_RHS>), eg, eb, 0, st, a, g);
          }
          return hipGetLastError();
        }
      }
      const dim3 grid(blocks(g.E)), block(S::THREADS);
      if (vol == VOL_EC) {
        if (epi == EPI_RK) hipLaunchKernelGGL((k_stage_mhd_ec<N, EPI_RK>), grid, block, 0, st, a, g);
        else hipLaunchKernelGGL((k_stage_mhd_ec<N, EPI_RHS>), grid, block, 0, st, a, g);
      } else {
        if (epi == EPI_RK) hipLaunchKernelGGL((k_stage_mhd<N, EPI_RK>), grid, block, 0, st, a, g);
        else hipLaunchKernelGGL((k_stage_mhd<N, EPI_RHS>), grid, block, 0, st, a, g);
      }
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }

  static hipError_t maxspeed_mhd(hipStream_t st, const double* u, double* partial, const Geom& g) {
    if constexpr (DIM == 3) {
      hipLaunchKernelGGL((k_maxspeed_mhd<N>), dim3(blocks(g.E)), dim3(S::THREADS), 0, st, u,
                         partial, g);
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }

  static Launchers make() {
    Launchers L;
    L.threads = S::THREADS;
    L.ne = S::NE;
    L.stage = &stage;
    L.indicator = &indicator;
    L.smooth = &smooth;
    L.maxspeed = &maxspeed;
    L.integrals = &integrals;
    L.coords = &coords;
    if constexpr (DIM == 3) {
      L.stage_curv = &stage_curv;
      L.maxspeed_curv = &maxspeed_curv;
      L.geometry = &geometry;
      L.stage_mhd = &stage_mhd;
      L.maxspeed_mhd = &maxspeed_mhd;
    }
    L.volume_name = "k_stage";
    return L;
  }
};

}  // namespace dgx
