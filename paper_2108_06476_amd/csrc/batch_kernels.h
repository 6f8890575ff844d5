// batch_kernels.h -- ensembles of independent 3D runs (uneven grids, polydeg 3..5)
// advanced by one launch per RK stage over the element tiles of all runs.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace dgx {

constexpr int BATCH_NMIN = 3, BATCH_NMAX = 5;

// Everything a block needs to process a tile of run r (device-resident array).
struct RunDesc {
  double* u;            // the caller's state (stage parity 0 reads it)
  double* u2;           // the library's second state buffer
  double* k;            // RK register
  double* du;           // right-hand side output (dgx_batch_rhs)
  double* dt;           // this run's time step
  double* t;            // this run's time (caller's), or nullptr
  double* speed;        // per-element wave-speed partials [E]
  const double* tab;    // operator tables
  int* flag;            // non-physical-state flag (shared by the batch)
  double gamma, inv_gm1;   // inv_gm1 = 1/(gamma - 1)
  int E, K[3], N, surf;
};

struct BatchLaunch {
  const RunDesc* runs;
  const int* order;     // runs sorted by polydeg (heaviest first)
  const int* prefix;    // prefix[i] = tiles of order[0..i-1]; prefix[nruns] = all tiles
  int nruns;
  int total;            // work items = tiles of all runs
};

// Host launchers (batch_kernels.hip).  budget: threads per block (256 or 512); grid: number
// of blocks (a multiple of 8; below the number of work items the blocks persist and loop
// over them); kw: the RK stage writes k (0 in a step's last stage).
hipError_t batch_stage(hipStream_t st, const BatchLaunch& b, int budget, int grid, int prec,
                       int epi, int cur, double A, double B, int emit_speed, int kw);
hipError_t batch_maxspeed(hipStream_t st, const BatchLaunch& b, int budget, int grid);
hipError_t batch_dt(hipStream_t st, const RunDesc* runs, int nruns, double cfl);
hipError_t batch_copy(hipStream_t st, const RunDesc* runs, int nruns, int64_t max_len);
// elements per tile of polydeg N for a block budget
int batch_tile_elems(int N, int budget);

}  // namespace dgx
