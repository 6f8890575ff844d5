// batch.hip -- ensembles of independent solvers (dgx_batch_*): runs of different grid
// sizes and polynomial degrees advanced together.  Each RK stage of all runs is one launch
// over (run, element tile) work items: one block per item, or a persistent grid whose
// blocks loop over the items; a step (per-run time step + 5 stages) is replayed from a
// captured hipGraph.  The tile shape (block size) and the grid are chosen by timing the
// candidates on the batch (dgx_batch_tune) or set by hand (dgx_batch_set_shape).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/dgx.h"
#include "batch_kernels.h"
#include "tables.h"

using namespace dgx;

namespace {

const double CK_A[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                        -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
const double CK_B[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                        1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                        2277821191437.0 / 14882151754819.0};

}  // namespace

struct dgx_batch_s {
  int nruns = 0;
  int prec = 0;
  hipStream_t stream = nullptr;
  std::vector<dgx_config> cfgs;
  std::vector<int64_t> nodes;     // per run, per variable
  std::vector<void*> allocs;
  std::vector<RunDesc> desc;      // host copy
  RunDesc* desc_d = nullptr;
  int* order_d = nullptr;
  int* prefix_d = nullptr;
  int* flag_d = nullptr;
  std::vector<int> order;
  int budget = 256;
  int grid = 0;
  int cus = 0;
  BatchLaunch bl{};
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  double graph_cfl = -1.0;
  std::string err;
};

namespace {

dgx_status bfail(dgx_batch b, dgx_status st, const std::string& m) {
  if (b) b->err = m;
  return st;
}

#define BHIP(b, expr)                                                                 \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return bfail(b, DGX_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));   \
  } while (0)

bool dev_alloc(dgx_batch b, void** p, size_t bytes) {
  if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  b->allocs.push_back(*p);
  return true;
}

// array argument: inside one device allocation of at least `bytes`
bool dev_ok(const void* p, size_t bytes) {
  if (!p) return false;
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged) return false;
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return (const char*)p + bytes <= (const char*)base + size;
}

void drop_graph(dgx_batch b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
  b->graph_cfl = -1.0;
}

// work items of the current block size: runs heaviest (highest polydeg) first
dgx_status set_shape(dgx_batch b, int budget, int grid) {
  std::vector<int> prefix(b->nruns + 1, 0);
  for (int i = 0; i < b->nruns; ++i) {
    const int r = b->order[i];
    const int ne = batch_tile_elems(b->desc[r].N, budget);
    prefix[i + 1] = prefix[i] + (b->desc[r].E + ne - 1) / ne;
  }
  BHIP(b, hipStreamSynchronize(b->stream));
  BHIP(b, hipMemcpy(b->prefix_d, prefix.data(), sizeof(int) * (b->nruns + 1), hipMemcpyHostToDevice));
  b->budget = budget;
  b->bl.total = prefix[b->nruns];
  // grid 0 or >= the items: one block per item (rounded to the 8 XCDs)
  b->grid = (grid <= 0 || grid >= b->bl.total) ? ((b->bl.total + 7) / 8) * 8 : grid;
  drop_graph(b);
  return DGX_OK;
}

dgx_status upload_desc(dgx_batch b) {
  // work already enqueued may still read the descriptors
  BHIP(b, hipStreamSynchronize(b->stream));
  BHIP(b, hipMemcpy(b->desc_d, b->desc.data(), sizeof(RunDesc) * b->nruns, hipMemcpyHostToDevice));
  return DGX_OK;
}

// Point the descriptors at the caller's arrays; re-upload only when something changed.
dgx_status bind(dgx_batch b, double* const* u, double* const* du, double* t) {
  bool changed = false;
  for (int r = 0; r < b->nruns; ++r) {
    const size_t bytes = sizeof(double) * 5 * (size_t)b->nodes[r];
    if (u && !dev_ok(u[r], bytes))
      return bfail(b, DGX_EINVAL, "u[" + std::to_string(r) + "]: not a device array of the run's size");
    if (du && !dev_ok(du[r], bytes))
      return bfail(b, DGX_EINVAL, "du[" + std::to_string(r) + "]: not a device array of the run's size");
    RunDesc& d = b->desc[r];
    double* nu = u ? u[r] : d.u;
    double* ndu = du ? du[r] : d.du;
    double* nt = t ? t + r : nullptr;
    changed |= (nu != d.u) || (ndu != d.du) || (nt != d.t);
    d.u = nu;
    d.du = ndu;
    d.t = nt;
  }
  if (t && !dev_ok(t, sizeof(double) * b->nruns)) return bfail(b, DGX_EINVAL, "t: not a device array of nruns");
  if (changed) return upload_desc(b);
  return DGX_OK;
}

dgx_status enqueue_step(dgx_batch b, hipStream_t st, double cfl, bool emit) {
  BHIP(b, batch_dt(st, b->desc_d, b->nruns, cfl));
  int cur = 0;
  for (int s = 0; s < 5; ++s) {
    BHIP(b, batch_stage(st, b->bl, b->budget, b->grid, b->prec, EPI_RK, cur, CK_A[s], CK_B[s],
                        (emit && s == 4) ? 1 : 0, s < 4));
    cur = 1 - cur;
  }
  return DGX_OK;
}

// Two steps: the state returns to the caller's buffer (10 stages).  The second step's
// last stage emits the wave speeds of the next step, so the graph can be replayed.
dgx_status enqueue_two_steps(dgx_batch b, hipStream_t st, double cfl) {
  BHIP(b, batch_dt(st, b->desc_d, b->nruns, cfl));
  int cur = 0;
  for (int s = 0; s < 10; ++s) {
    if (s == 5) BHIP(b, batch_dt(st, b->desc_d, b->nruns, cfl));
    BHIP(b, batch_stage(st, b->bl, b->budget, b->grid, b->prec, EPI_RK, cur, CK_A[s % 5],
                        CK_B[s % 5], (s == 4 || s == 9) ? 1 : 0, s % 5 < 4));
    cur = 1 - cur;
  }
  return DGX_OK;
}

dgx_status ensure_graph(dgx_batch b, double cfl) {
  if (b->gexec && b->graph_cfl == cfl) return DGX_OK;
  drop_graph(b);
  if (!b->cap) BHIP(b, hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  BHIP(b, hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  dgx_status st = enqueue_two_steps(b, b->cap, cfl);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->cap, &g);
  if (st != DGX_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return bfail(b, DGX_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  b->graph = g;
  BHIP(b, hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0));
  b->graph_cfl = cfl;
  return DGX_OK;
}

}  // namespace

extern "C" {

dgx_status dgx_batch_create(const dgx_config* cfgs, int32_t nruns, void* hip_stream,
                            dgx_batch* out) {
  if (!cfgs || !out || nruns < 1) return DGX_EINVAL;
  *out = nullptr;
  for (int r = 0; r < nruns; ++r) {
    const dgx_config& c = cfgs[r];
    if (c.dim != 3 || c.volume != DGX_VOL_EC ||
        (c.surface != DGX_SURF_LLF && c.surface != DGX_SURF_HLL) || !(c.gamma > 1.0) ||
        (c.precision != DGX_FP64 && c.precision != DGX_MIXED) || c.precision != cfgs[0].precision)
      return DGX_EINVAL;
    for (int d = 0; d < 3; ++d)
      if (c.cells[d] < 1 || !(c.xmax[d] > c.xmin[d])) return DGX_EINVAL;
    if (c.polydeg < BATCH_NMIN || c.polydeg > BATCH_NMAX) return DGX_EUNSUPPORTED;
    const int n = c.polydeg + 1;
    if ((int64_t)5 * c.cells[0] * c.cells[1] * c.cells[2] * n * n * n >= ((int64_t)1 << 31))
      return DGX_EUNSUPPORTED;
  }
  dgx_batch b = new dgx_batch_s();
  b->nruns = nruns;
  b->prec = cfgs[0].precision;
  b->stream = (hipStream_t)hip_stream;
  b->cfgs.assign(cfgs, cfgs + nruns);
  b->desc.resize(nruns);
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      b->cus < 1)
    b->cus = 256;
  bool ok = dev_alloc(b, (void**)&b->desc_d, sizeof(RunDesc) * nruns) &&
            dev_alloc(b, (void**)&b->order_d, sizeof(int) * nruns) &&
            dev_alloc(b, (void**)&b->prefix_d, sizeof(int) * (nruns + 1)) &&
            dev_alloc(b, (void**)&b->flag_d, sizeof(int) * 2);
  for (int r = 0; ok && r < nruns; ++r) {
    const dgx_config& c = cfgs[r];
    const int n = c.polydeg + 1;
    RunDesc& d = b->desc[r];
    d.E = c.cells[0] * c.cells[1] * c.cells[2];
    d.K[0] = c.cells[0];
    d.K[1] = c.cells[1];
    d.K[2] = c.cells[2];
    d.N = c.polydeg;
    d.surf = c.surface;
    d.gamma = c.gamma;
    d.inv_gm1 = 1.0 / (c.gamma - 1.0);
    d.flag = b->flag_d;
    d.u = d.du = d.t = nullptr;
    b->nodes.push_back((int64_t)d.E * n * n * n);
    const size_t sb = sizeof(double) * 5 * (size_t)b->nodes[r];
    double h[3];
    for (int k = 0; k < 3; ++k) h[k] = (c.xmax[k] - c.xmin[k]) / c.cells[k];
    std::vector<double> T(TAB_SIZE, 0.0);
    ok = stage_tables(c.polydeg, h, T.data()) && dev_alloc(b, (void**)&d.u2, sb) &&
         dev_alloc(b, (void**)&d.k, sb) && dev_alloc(b, (void**)&d.speed, sizeof(double) * d.E) &&
         dev_alloc(b, (void**)&d.dt, sizeof(double)) &&
         dev_alloc(b, (void**)&d.tab, sizeof(double) * TAB_SIZE) &&
         hipMemcpy((void*)d.tab, T.data(), sizeof(double) * TAB_SIZE, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemset(d.k, 0, sb) == hipSuccess;
  }
  if (!ok || hipMemset(b->flag_d, 0, sizeof(int) * 2) != hipSuccess) {
    dgx_batch_destroy(b);
    return DGX_ENOMEM;
  }
  b->order.resize(nruns);
  for (int r = 0; r < nruns; ++r) b->order[r] = r;
  std::stable_sort(b->order.begin(), b->order.end(),
                   [&](int x, int y) { return b->desc[x].N > b->desc[y].N; });
  b->bl.runs = b->desc_d;
  b->bl.order = b->order_d;
  b->bl.prefix = b->prefix_d;
  b->bl.nruns = nruns;
  if (hipMemcpy(b->order_d, b->order.data(), sizeof(int) * nruns, hipMemcpyHostToDevice) != hipSuccess ||
      upload_desc(b) != DGX_OK || set_shape(b, 256, 0) != DGX_OK) {
    dgx_batch_destroy(b);
    return DGX_EHIP;
  }
  *out = b;
  return DGX_OK;
}

dgx_status dgx_batch_destroy(dgx_batch b) {
  if (!b) return DGX_EINVAL;
  (void)hipDeviceSynchronize();
  drop_graph(b);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  for (void* p : b->allocs) (void)hipFree(p);
  delete b;
  return DGX_OK;
}

int64_t dgx_batch_num_nodes(dgx_batch b, int32_t r) {
  if (!b || r < 0 || r >= b->nruns) return -1;
  return b->nodes[r];
}

dgx_status dgx_batch_step(dgx_batch b, double* const* u, int32_t nsteps, double cfl, double* t) {
  if (!b || !u) return DGX_EINVAL;
  if (!(cfl > 0.0)) return bfail(b, DGX_EINVAL, "cfl must be > 0");
  if (nsteps < 0) return bfail(b, DGX_EINVAL, "nsteps < 0");
  dgx_status st = bind(b, u, nullptr, t);
  if (st != DGX_OK) return st;
  if (nsteps == 0) return DGX_OK;
  BHIP(b, batch_maxspeed(b->stream, b->bl, b->budget, b->grid));
  int pairs = nsteps / 2;
  if (pairs > 0) {
    st = ensure_graph(b, cfl);
    if (st != DGX_OK) return st;
    for (int p = 0; p < pairs; ++p) BHIP(b, hipGraphLaunch(b->gexec, b->stream));
  }
  if (nsteps % 2) {
    st = enqueue_step(b, b->stream, cfl, false);
    if (st != DGX_OK) return st;
    int64_t mx = 0;
    for (int64_t v : b->nodes) mx = std::max(mx, 5 * v);
    BHIP(b, batch_copy(b->stream, b->desc_d, b->nruns, mx));
  }
  return DGX_OK;
}

dgx_status dgx_batch_rhs(dgx_batch b, const double* const* u, double* const* du) {
  if (!b || !u || !du) return DGX_EINVAL;
  for (int r = 0; r < b->nruns; ++r) {
    const size_t bytes = sizeof(double) * 5 * (size_t)b->nodes[r];
    const char *pu = (const char*)u[r], *pd = (const char*)du[r];
    if (pu < pd + bytes && pd < pu + bytes)
      return bfail(b, DGX_EINVAL, "u[" + std::to_string(r) + "] and du[" + std::to_string(r) + "] overlap");
  }
  dgx_status st = bind(b, const_cast<double* const*>(u), du, nullptr);
  if (st != DGX_OK) return st;
  BHIP(b, batch_stage(b->stream, b->bl, b->budget, b->grid, b->prec, EPI_RHS, 0, 0.0, 0.0, 0, 0));
  return DGX_OK;
}

dgx_status dgx_batch_tune(dgx_batch b, double* const* u, int32_t budget_ms) {
  if (!b || !u) return DGX_EINVAL;
  // times one right-hand side of every run (written into the RK registers, which hold no
  // state between steps) for each candidate tile shape and persistent grid
  std::vector<double*> kbuf(b->nruns);
  for (int r = 0; r < b->nruns; ++r) kbuf[r] = b->desc[r].k;
  dgx_status st = bind(b, u, kbuf.data(), nullptr);
  if (st != DGX_OK) return st;
  hipEvent_t e0, e1;
  BHIP(b, hipEventCreate(&e0));
  BHIP(b, hipEventCreate(&e1));
  const int budgets[2] = {256, 512};
  const int mult[4] = {0, 2, 4, 8};   // 0: one block per work item; else persistent blocks per CU
  double best = 1e300, used = 0.0;
  int bb = b->budget, bg = b->grid;
  for (int budget : budgets) {
    for (int m : mult) {   // (persistent candidates beyond the item count are skipped)
      if (used > budget_ms) break;
      st = set_shape(b, budget, m ? ((b->cus * m + 7) / 8) * 8 : 0);
      if (st != DGX_OK) break;
      const int grid = b->grid;
      float ms = 0.f, total = 0.f;
      bool fail = false;
      for (int rep = 0; rep < 4 && !fail; ++rep) {
        fail |= hipEventRecord(e0, b->stream) != hipSuccess;
        fail |= batch_stage(b->stream, b->bl, budget, grid, b->prec, EPI_RHS, 0, 0.0, 0.0, 0, 0) != hipSuccess;
        fail |= hipEventRecord(e1, b->stream) != hipSuccess;
        fail |= hipEventSynchronize(e1) != hipSuccess;
        fail |= hipEventElapsedTime(&ms, e0, e1) != hipSuccess;
        if (rep > 0) total += ms;   // the first launch warms up
        used += ms;
      }
      if (fail) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return bfail(b, DGX_EHIP, "tuning launch failed");
      }
      if (total / 3 < best) {
        best = total / 3;
        bb = budget;
        bg = grid;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (int r = 0; r < b->nruns; ++r) b->desc[r].du = nullptr;
  st = upload_desc(b);
  if (st != DGX_OK) return st;
  return set_shape(b, bb, bg);
}

dgx_status dgx_batch_check(dgx_batch b, int32_t* flag) {
  if (!b || !flag) return DGX_EINVAL;
  BHIP(b, hipStreamSynchronize(b->stream));
  int f = 0;
  BHIP(b, hipMemcpy(&f, b->flag_d, sizeof(int), hipMemcpyDeviceToHost));
  BHIP(b, hipMemset(b->flag_d, 0, sizeof(int)));
  *flag = f;
  return f ? DGX_ENONPHYS : DGX_OK;
}

dgx_status dgx_batch_set_shape(dgx_batch b, int32_t block, int32_t grid) {
  if (!b) return DGX_EINVAL;
  if (block != 256 && block != 512) return bfail(b, DGX_EINVAL, "block must be 256 or 512");
  if (grid < 0 || grid % 8 != 0) return bfail(b, DGX_EINVAL, "grid must be 0 or a positive multiple of 8");
  return set_shape(b, block, grid);
}

dgx_status dgx_batch_shape(dgx_batch b, int32_t* block, int32_t* grid) {
  if (!b) return DGX_EINVAL;
  if (block) *block = b->budget;
  if (grid) *grid = b->grid;
  return DGX_OK;
}

const char* dgx_batch_last_error(dgx_batch b) { return b ? b->err.c_str() : "invalid batch"; }

}  // extern "C"
