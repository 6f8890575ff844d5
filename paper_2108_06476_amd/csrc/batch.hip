// batch.hip -- ensembles of independent solvers (dgx_batch_*): runs of different grid
// sizes and polynomial degrees advanced together on one stream.  Each run owns a solver
// handle; no state is shared between runs (there is no global state, Section 2.3.3).
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/dgx.h"

struct dgx_batch_s {
  std::vector<dgx_handle> runs;
  hipStream_t stream = nullptr;
  std::string err;
};

extern "C" {

dgx_status dgx_batch_create(const dgx_config* cfgs, int32_t nruns, void* hip_stream,
                            dgx_batch* out) {
  if (!cfgs || !out || nruns < 1) return DGX_EINVAL;
  *out = nullptr;
  for (int r = 0; r < nruns; ++r) {
    const dgx_config& c = cfgs[r];
    if (c.dim != 3 || (c.volume != DGX_VOL_EC) ||
        (c.surface != DGX_SURF_LLF && c.surface != DGX_SURF_HLL) ||
        c.precision != cfgs[0].precision)
      return DGX_EINVAL;
  }
  dgx_batch b = new dgx_batch_s();
  b->stream = (hipStream_t)hip_stream;
  for (int r = 0; r < nruns; ++r) {
    dgx_handle h = nullptr;
    dgx_status st = dgx_create(&cfgs[r], hip_stream, &h);
    if (st != DGX_OK) {
      dgx_batch_destroy(b);
      return st;
    }
    b->runs.push_back(h);
  }
  *out = b;
  return DGX_OK;
}

dgx_status dgx_batch_destroy(dgx_batch b) {
  if (!b) return DGX_EINVAL;
  for (dgx_handle h : b->runs) dgx_destroy(h);
  delete b;
  return DGX_OK;
}

int64_t dgx_batch_num_nodes(dgx_batch b, int32_t r) {
  if (!b || r < 0 || r >= (int32_t)b->runs.size()) return -1;
  return dgx_num_nodes(b->runs[r]);
}

dgx_status dgx_batch_step(dgx_batch b, double* const* u, int32_t nsteps, double cfl, double* t) {
  if (!b || !u) return DGX_EINVAL;
  if (!(cfl > 0.0)) {
    b->err = "cfl must be > 0";
    return DGX_EINVAL;
  }
  for (size_t r = 0; r < b->runs.size(); ++r) {
    dgx_status st = dgx_step(b->runs[r], u[r], nsteps, cfl, 0.0, t ? t + r : nullptr);
    if (st != DGX_OK) {
      b->err = "run " + std::to_string(r) + ": " + dgx_last_error(b->runs[r]);
      return st;
    }
  }
  return DGX_OK;
}

dgx_status dgx_batch_rhs(dgx_batch b, const double* const* u, double* const* du) {
  if (!b || !u || !du) return DGX_EINVAL;
  for (size_t r = 0; r < b->runs.size(); ++r) {
    dgx_status st = dgx_rhs(b->runs[r], u[r], du[r], 0.0);
    if (st != DGX_OK) {
      b->err = "run " + std::to_string(r) + ": " + dgx_last_error(b->runs[r]);
      return st;
    }
  }
  return DGX_OK;
}

dgx_status dgx_batch_tune(dgx_batch b, double* const* u, int32_t budget_ms) {
  (void)u;
  (void)budget_ms;
  if (!b) return DGX_EINVAL;
  return DGX_OK;
}

const char* dgx_batch_last_error(dgx_batch b) { return b ? b->err.c_str() : "invalid batch"; }

}  // extern "C"
