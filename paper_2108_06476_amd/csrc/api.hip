// api.hip -- the dgx C ABI (include/dgx.h): handle management, argument checks and the
// launch sequences of the right-hand side, the indicator, the CFL time step, the
// low-storage Runge-Kutta step and the integrals.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dgx.h"
#include "registry.h"
#include "tables.h"

namespace dgx {
const Launchers* launchers_d2_n1();
const Launchers* launchers_d2_n2();
const Launchers* launchers_d2_n3();
const Launchers* launchers_d2_n4();
const Launchers* launchers_d2_n5();
const Launchers* launchers_d2_n6();
const Launchers* launchers_d2_n7();
const Launchers* launchers_d3_n1();
const Launchers* launchers_d3_n2();
const Launchers* launchers_d3_n3();
const Launchers* launchers_d3_n4();
const Launchers* launchers_d3_n5();
const Launchers* launchers_d3_n6();
const Launchers* launchers_d3_n7();

const Launchers* launchers_2d(int N) {
  switch (N) {
    case 1: return launchers_d2_n1();
    case 2: return launchers_d2_n2();
    case 3: return launchers_d2_n3();
    case 4: return launchers_d2_n4();
    case 5: return launchers_d2_n5();
    case 6: return launchers_d2_n6();
    case 7: return launchers_d2_n7();
    default: return nullptr;
  }
}

const Launchers* launchers_3d(int N) {
  switch (N) {
    case 1: return launchers_d3_n1();
    case 2: return launchers_d3_n2();
    case 3: return launchers_d3_n3();
    case 4: return launchers_d3_n4();
    case 5: return launchers_d3_n5();
    case 6: return launchers_d3_n6();
    case 7: return launchers_d3_n7();
    default: return nullptr;
  }
}

// Carpenter-Kennedy (1994) five-stage fourth-order 2N-storage coefficients (the time
// integrator of Section 3.1): k <- A_s k + dt R, u <- u + B_s k.
static const double CK_A[5] = {0.0, -567301805773.0 / 1357537059087.0,
                               -2404267990393.0 / 2016746695238.0,
                               -3550918686646.0 / 2091501179385.0,
                               -1275806237668.0 / 842570457699.0};
static const double CK_B[5] = {1432997174477.0 / 9575080441755.0,
                               5161836677717.0 / 13612068292357.0,
                               1720146321549.0 / 2090206949498.0,
                               3134564353537.0 / 4481467310338.0,
                               2277821191437.0 / 14882151754819.0};

// Stage times c_s of the same scheme (for time-dependent source terms: t + c_s dt).
static const double CK_C[5] = {0.0, 1432997174477.0 / 9575080441755.0,
                               2526269341429.0 / 6820363183890.0,
                               2006345519317.0 / 3224310063776.0,
                               2802321613138.0 / 2924317926251.0};

// dt = cfl * 2 / ((N+1) * max partial); t0 = t (the step's start time, when asked); t += dt.
// T = 1024 threads, or one wave (T = 64) for up to DT_WAVE_MAX partials: a small mesh's step
// is a chain of short launches, and one wave reduces with DPP moves and no barrier.  max is
// exact, so both give the same dt.
constexpr int64_t DT_WAVE_MAX = 4096;

template <int T>
__global__ __launch_bounds__(T) void k_dt_final(const double* __restrict__ partial, int64_t np,
                                                double cfl, double n1, double* __restrict__ dt,
                                                double* __restrict__ t, double* __restrict__ t0) {
  double m;
  int owner;
  if constexpr (T == 64) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};   // four loads in flight per lane
    int64_t i = threadIdx.x;
    for (; i + 3 * 64 < np; i += 4 * 64) {
#pragma unroll
      for (int k = 0; k < 4; ++k) a[k] = fmax(a[k], partial[i + k * 64]);
    }
    for (; i < np; i += 64) a[0] = fmax(a[0], partial[i]);
    m = wave_max_lane63(fmax(fmax(a[0], a[1]), fmax(a[2], a[3])));
    owner = 63;
  } else {
    __shared__ double s[T / 64];
    m = block_max<T>(partial, np, s);
    owner = 0;
  }
  if ((int)threadIdx.x == owner) {
    const double d = cfl * 2.0 / (n1 * m);
    *dt = d;
    if (t) {
      if (t0) *t0 = *t;
      *t += d;
    }
  }
}

static void launch_dt_final(hipStream_t st, const double* partial, int64_t np, double cfl,
                            double n1, double* dt, double* t, double* t0) {
  if (np <= DT_WAVE_MAX)
    hipLaunchKernelGGL(k_dt_final<64>, dim3(1), dim3(64), 0, st, partial, np, cfl, n1, dt, t, t0);
  else
    hipLaunchKernelGGL(k_dt_final<1024>, dim3(1), dim3(1024), 0, st, partial, np, cfl, n1, dt, t, t0);
}

// The start of a dgx_step call on a mesh whose stages keep the wave speeds in slots: the
// max of k_maxspeed's per-element partials into slot 0, the other slots cleared; the first
// stage then takes dt from the slots as in every later step.
__global__ __launch_bounds__(1024) void k_dt_seed(const double* __restrict__ partial, int64_t np,
                                                  double* __restrict__ slots) {
  __shared__ double s[16];
  const double m = block_max<1024>(partial, np, s);
  if (threadIdx.x == 0) slots[0] = m;
  else if (threadIdx.x < (unsigned)DT_SLOTS) slots[threadIdx.x * DT_SLOT_STRIDE] = 0.0;
}

__global__ void k_set_dt(double v, double* __restrict__ dt, double* __restrict__ t,
                         double* __restrict__ t0) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *dt = v;
    if (t) {
      if (t0) *t0 = *t;
      *t += v;
    }
  }
}

// out[c] = sum over blocks of partial[b*7 + c], fixed order
__global__ __launch_bounds__(256) void k_sum_final(const double* __restrict__ partial, int64_t np,
                                                   double* __restrict__ out) {
  __shared__ double s[7][256];
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int64_t i = threadIdx.x; i < np; i += 256)
    for (int c = 0; c < 7; ++c) acc[c] += partial[i * 7 + c];
  for (int c = 0; c < 7; ++c) s[c][threadIdx.x] = acc[c];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int c = 0; c < 7; ++c) s[c][threadIdx.x] += s[c][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < 7) out[threadIdx.x] = s[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_copy(const double* __restrict__ src,
                                              double* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    dst[i] = src[i];
}

__global__ void k_zero_int(int* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

// Scratch of dgx_max_dt_noalloc: the per-element wave-speed partials, in a file-scope
// device array (each device holds its own copy for the life of the process).  Host code
// never uses the name as an address: the device address comes from hipGetSymbolAddress,
// taken once per device when a handle is created on it.
constexpr int64_t NOALLOC_MAX_ELEMS = (int64_t)1 << 20;   // 8 MiB of float64
static __device__ __align__(256) double scratch[NOALLOC_MAX_ELEMS];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mutex;
double* scratch_ptr[MAX_DEVICES] = {};

// The device address of `scratch` on device `dev` (the current device), looked up on the
// first call for that device.
hipError_t scratch_address(int dev, double** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mutex);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace dgx

using namespace dgx;

struct dgx_solver {
  dgx_config cfg{};
  int dim = 0, N = 0, n = 0, NN = 0, NF = 0, NV = 0;
  int64_t E = 0;
  double h[3] = {1, 1, 1};
  hipStream_t stream = nullptr;
  const Launchers* L = nullptr;
  Geom g{};
  double* tab = nullptr;
  double* u2 = nullptr;   // second state buffer of the double-buffered RK stages
  double* k = nullptr;
  double* alpha = nullptr;
  double* alpha_raw = nullptr;
  double* energy = nullptr;
  double* partial = nullptr;
  int64_t npart = 0;   // wave-speed partials (one per element)
  double* slots = nullptr;   // DT_SLOTS wave-speed maxima, DT_SLOT_STRIDE doubles apart
  int64_t nblk = 0;    // blocks of the element-tiled kernels (integral partials)
  double* dt = nullptr;
  int* flag = nullptr;
  // curvilinear mesh (dgx_create_curved)
  bool curved = false;
  double* ja = nullptr;     // (J a^i)_n [3][3][E][NN]
  double* jac = nullptr;    // J [E][NN]
  double* xyz = nullptr;    // node positions [3][E][NN]
  double* dmat = nullptr;   // LGL differentiation matrix [n][n]
  double* t0 = nullptr;     // start time of the current step
  bool mhd = false;         // ideal MHD (dgx_create_mhd): 8 variables
  // two RK steps captured in a hipGraph (replayed by dgx_step), valid for one key
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;     // a step pair starting a call (shock capturing: fresh)
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph2 = nullptr;    // shock capturing: a step pair continuing one
  hipGraphExec_t gexec2 = nullptr;
  const double* g_u = nullptr;
  const double* g_t = nullptr;
  double g_cfl = 0.0, g_dtf = 0.0;
  std::string err;
  bool prof = false;
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
  std::vector<int> ev_count;   // stage launches inside each event pair
  int64_t launches = 0;
  double prof_ms = 0.0;
  int device = 0;                    // the device the handle was created on
  double* noalloc_partial = nullptr; // that device's static scratch (dgx_max_dt_noalloc)
};

namespace {

dgx_status fail(dgx_handle h, dgx_status st, const std::string& msg) {
  if (h) h->err = msg;
  return st;
}

#define HIPCHK(h, expr)                                                                \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(h, DGX_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

// A device array argument must lie inside one device allocation of at least `bytes`.
dgx_status check_dev(dgx_handle h, const void* p, size_t bytes, const char* name) {
  if (!p) return fail(h, DGX_EINVAL, std::string(name) + ": NULL pointer");
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return fail(h, DGX_EINVAL, std::string(name) + ": not a device pointer");
  }
  if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)
    return fail(h, DGX_EINVAL, std::string(name) + ": not device memory");
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p) != hipSuccess) {
    (void)hipGetLastError();
    return fail(h, DGX_EINVAL, std::string(name) + ": no allocation range");
  }
  const char* b = (const char*)base;
  const char* q = (const char*)p;
  if (q + bytes > b + size)
    return fail(h, DGX_EINVAL, std::string(name) + ": allocation too small (" +
                                   std::to_string(size - (size_t)(q - b)) + " < " +
                                   std::to_string(bytes) + " bytes)");
  return DGX_OK;
}

#define CHKDEV(h, p, bytes, name)                             \
  do {                                                        \
    dgx_status s_ = check_dev(h, p, bytes, name);             \
    if (s_ != DGX_OK) return s_;                              \
  } while (0)

size_t state_bytes(dgx_handle h) { return sizeof(double) * (size_t)h->NV * h->E * h->NN; }

// Two byte ranges [a, a + n) and [b, b + n) share an address.
bool overlap(const void* a, const void* b, size_t n) {
  const char *p = (const char*)a, *q = (const char*)b;
  return p < q + n && q < p + n;
}

// Timing of the dominant kernel: one event pair brackets a run of consecutive stage
// launches (an event recorded between two kernels leaves the stream idle for microseconds),
// and the pair's time is shared by the launches inside it.
hipError_t launch_stage(dgx_handle h, const StageArgs& a, int epi, bool last) {
  const size_t pair = h->ev_used / 2;
  if (h->prof && h->ev_count.size() <= pair) {   // open a bracket
    if (h->ev_used + 2 > h->ev.size()) {
      for (int i = 0; i < 2; ++i) {
        hipEvent_t ev;
        hipError_t r = hipEventCreate(&ev);
        if (r != hipSuccess) return r;
        h->ev.push_back(ev);
      }
    }
    h->ev_count.push_back(0);
    hipError_t r = hipEventRecord(h->ev[h->ev_used], h->stream);
    if (r != hipSuccess) return r;
  }
  hipError_t r = h->mhd      ? h->L->stage_mhd(h->stream, a, h->g, h->cfg.volume, epi)
                 : h->curved ? h->L->stage_curv(h->stream, a, h->g, h->cfg.volume, epi)
                             : h->L->stage(h->stream, a, h->g, h->cfg.volume, epi, h->cfg.precision);
  if (r != hipSuccess || !h->prof) return r;
  h->ev_count[pair] += 1;
  if (last) {   // close it
    r = hipEventRecord(h->ev[h->ev_used + 1], h->stream);
    h->ev_used += 2;
  }
  return r;
}

dgx_status enqueue_indicator(dgx_handle h, const double* u, double* alpha, double* ar,
                             double* en) {
  HIPCHK(h, h->L->indicator(h->stream, u, ar, en, h->g, h->cfg.alpha_min, h->cfg.alpha_max));
  HIPCHK(h, h->L->smooth(h->stream, ar, alpha, h->g, h->cfg.alpha_smooth));
  return DGX_OK;
}

StageArgs stage_args(dgx_handle h, const double* uin, const double* alpha) {
  StageArgs a;
  a.uin = uin;
  a.uout = nullptr;
  a.du = nullptr;
  a.k = h->k;
  a.alpha = alpha;
  a.dt = h->dt;
  a.speed = nullptr;
  a.A = 0.0;
  a.B = 0.0;
  a.surf = h->cfg.surface;
  a.fvf = h->cfg.fv_flux;
  return a;
}

// du = R(u); alpha_in (shock capturing) may be NULL: then the indicator runs first.
dgx_status enqueue_rhs(dgx_handle h, const double* u, double* du, const double* alpha_in,
                       double t = 0.0) {
  const double* alpha = alpha_in;
  if (h->cfg.volume == DGX_VOL_SHOCKCAP_HG && !alpha) {
    dgx_status st = enqueue_indicator(h, u, h->alpha, h->alpha_raw, nullptr);
    if (st != DGX_OK) return st;
    alpha = h->alpha;
  }
  StageArgs a = stage_args(h, u, alpha);
  a.du = du;
  a.t = t;
  HIPCHK(h, launch_stage(h, a, EPI_RHS, true));
  return DGX_OK;
}


// One RK step on h->stream: dt (adaptive: from the partials in h->partial, or, see
// stage_slots, from the slots in h->slots), then the five stages; emit: the last stage writes
// the next step's partials (or folds them into the slots).  cur: which of buf holds
// the state (toggled by every stage).  Shock capturing: every stage writes the raw
// indicator of its output state and smooths its input's itself; the first stage of a step
// with fresh set (the first of a call) has it computed first.  j0: the parity of the
// number of stages since then, which picks the buffer each stage reads.
bool shock_steps(dgx_handle h) {
  return h->cfg.volume == DGX_VOL_SHOCKCAP_HG && !h->curved && !h->mhd;
}

// Small meshes (at most STAGE_DT_MAX_E elements; for curvilinear and MHD handles those whose
// N = 3 stages run several waves per element): the first stage of an adaptive step derives
// dt itself, every wave reducing the partials (one launch fewer per step on a latency-bound
// mesh), with the same value and time updates as k_dt_final.
constexpr int64_t STAGE_DT_MAX_E = 512;

static bool stage_derives_dt(dgx_handle h) {
  if (h->E > STAGE_DT_MAX_E) return false;
  if (h->curved) return h->N == 3 && h->E <= CURV_SPLIT_MAX_E;
  if (h->mhd) return h->N == 3 && h->E <= MHD_SPLIT_MAX_E;
  return true;
}

// Mid-size Cartesian meshes: the last stage of a step folds the element wave speeds into
// DT_SLOTS slots by atomic max, and the next step's first stage derives dt from those
// (every wave reducing 64 values): no dt kernel between the steps.  From STAGE_SLOTS_MAX_E
// elements on, the 6 us that k_dt_final takes are a small part of a step and the atomics
// and slot reads cost about as much, so those meshes keep k_dt_final.
constexpr int64_t STAGE_SLOTS_MAX_E = 16384;

static bool stage_slots(dgx_handle h) {
  return !h->curved && !h->mhd && h->E > STAGE_DT_MAX_E && h->E < STAGE_SLOTS_MAX_E;
}

dgx_status enqueue_step(dgx_handle h, double* const (&buf)[2], int& cur, double cfl,
                        double dt_fixed, double* t, bool emit, bool fresh, int j0) {
  const bool adaptive = cfl > 0.0;
  double* t0 = h->g.source ? h->t0 : nullptr;   // step start time for the stage times
  const bool slots = adaptive && stage_slots(h);
  const bool in_stage = adaptive && (stage_derives_dt(h) || slots);
  if (in_stage) {
    // dt from the partials in the first stage, the time advanced by the second
  } else if (adaptive) {
    launch_dt_final(h->stream, h->partial, h->npart, cfl, (double)(h->N + 1), h->dt, t, t0);
  } else {
    hipLaunchKernelGGL(k_set_dt, dim3(1), dim3(64), 0, h->stream, dt_fixed, h->dt, t, t0);
  }
  HIPCHK(h, hipGetLastError());
  // shock capturing: the raw indicator alternates between two buffers, each stage smoothing
  // its input's and emitting its output's; a fresh step starts from k_indicator's
  const bool shock = shock_steps(h);
  double* const araw[2] = {h->alpha_raw, h->alpha};
  for (int st = 0; st < 5; ++st) {
    const double* uin = buf[cur];
    const int j = j0 + st;   // parity of the stages since the indicator ran on a state
    if (shock && st == 0 && fresh) {
      HIPCHK(h, h->L->indicator(h->stream, uin, araw[0], nullptr, h->g, h->cfg.alpha_min,
                                h->cfg.alpha_max));
    }
    StageArgs a = stage_args(h, uin, nullptr);
    if (shock) {
      a.alpha_raw_in = araw[j % 2];
      a.alpha_smooth = h->cfg.alpha_smooth;
      a.alpha_next = araw[(j + 1) % 2];
      indicator_constants(h->N, a.ind_thr, a.ind_sharp);
      a.ind_xcut = indicator_xcut(h->cfg.alpha_min);
      a.ind_amin = h->cfg.alpha_min;
      a.ind_amax = h->cfg.alpha_max;
    }
    a.uout = buf[1 - cur];
    a.A = CK_A[st];
    a.B = CK_B[st];
    a.speed = (adaptive && st == 4 && emit && !slots) ? h->partial : nullptr;
    a.speed_slots = (st == 4 && emit && slots) ? h->slots : nullptr;
    a.t0 = t0;
    a.cs = CK_C[st];
    if (in_stage && st == 0) {   // c_1 = 0: the source time is the step's start, t itself
      a.dt_from = slots ? h->slots : h->partial;
      a.dt_np = slots ? DT_SLOTS : h->npart;
      a.dt_stride = slots ? DT_SLOT_STRIDE : 1;
      a.dt_cfl = cfl;
      a.dt_n1 = (double)(h->N + 1);
      a.dt_pub = h->dt;
      a.t_cur = t;
      a.t0_pub = t0;
      a.t0 = t0 ? t : nullptr;
      a.t_step = 1;
    } else if (in_stage && st == 1) {
      a.t_cur = t;
      a.t_step = 2;
      if (slots) a.slots_clear = h->slots;   // read by stage 0, written again by stage 4
    }
    a.kw = st < 4;
    // the stages of one step run back to back (an indicator kernel only precedes stage 0)
    HIPCHK(h, launch_stage(h, a, EPI_RK, st == 4));
    cur = 1 - cur;
  }
  return DGX_OK;
}

void drop_step_graph(dgx_handle h) {
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  if (h->gexec2) (void)hipGraphExecDestroy(h->gexec2);
  if (h->graph2) (void)hipGraphDestroy(h->graph2);
  h->gexec = nullptr;
  h->graph = nullptr;
  h->gexec2 = nullptr;
  h->graph2 = nullptr;
  h->g_u = nullptr;
}

// One pair of RK steps (both emitting the next partials) captured on a private stream;
// fresh: its first step starts a call.
dgx_status capture_step_pair(dgx_handle h, double* u, double cfl, double dt_fixed, double* t,
                             bool fresh, hipGraph_t& graph, hipGraphExec_t& exec) {
  if (!h->cap) HIPCHK(h, hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
  HIPCHK(h, hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
  hipStream_t user = h->stream;
  h->stream = h->cap;
  double* buf[2] = {u, h->u2};
  int cur = 0;
  dgx_status st = enqueue_step(h, buf, cur, cfl, dt_fixed, t, true, fresh, 0);
  if (st == DGX_OK) st = enqueue_step(h, buf, cur, cfl, dt_fixed, t, true, false, 1);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(h->cap, &g);
  h->stream = user;
  if (st != DGX_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return st != DGX_OK ? st : fail(h, DGX_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  }
  graph = g;
  HIPCHK(h, hipGraphInstantiate(&exec, g, nullptr, nullptr, 0));
  return DGX_OK;
}

// The captured step pairs, reused while the state pointer, t and the step rule stay the
// same: one that starts a call and, with shock capturing (whose first stage of a call runs
// the indicator), one that continues it.
dgx_status ensure_step_graph(dgx_handle h, double* u, double cfl, double dt_fixed, double* t) {
  if (h->gexec && h->g_u == u && h->g_t == t && h->g_cfl == cfl && h->g_dtf == dt_fixed)
    return DGX_OK;
  drop_step_graph(h);
  dgx_status st = capture_step_pair(h, u, cfl, dt_fixed, t, true, h->graph, h->gexec);
  if (st != DGX_OK) return st;
  if (shock_steps(h)) {
    st = capture_step_pair(h, u, cfl, dt_fixed, t, false, h->graph2, h->gexec2);
    if (st != DGX_OK) return st;
  }
  h->g_u = u;
  h->g_t = t;
  h->g_cfl = cfl;
  h->g_dtf = dt_fixed;
  return DGX_OK;
}

// Per-element CFL partials of u into h->partial.
hipError_t enqueue_maxspeed(dgx_handle h, const double* u) {
  return h->mhd      ? h->L->maxspeed_mhd(h->stream, u, h->partial, h->g)
         : h->curved ? h->L->maxspeed_curv(h->stream, u, h->partial, h->g)
                     : h->L->maxspeed(h->stream, u, h->partial, h->g);
}

// The solver behind dgx_create (cv == nullptr) and dgx_create_curved.
dgx_status create_impl(const dgx_config& c, const dgx_curv_config* cv, void* hip_stream,
                       dgx_handle* out, bool mhd = false) {
  *out = nullptr;
  if (c.dim != 2 && c.dim != 3) return DGX_EINVAL;
  if (c.polydeg < 1) return DGX_EINVAL;
  if (!(c.gamma > 1.0)) return DGX_EINVAL;
  for (int d = 0; d < c.dim; ++d)
    if (c.cells[d] < 1 || !(c.xmax[d] > c.xmin[d])) return DGX_EINVAL;
  if (c.dim == 2 && c.cells[2] != 1) return DGX_EINVAL;
  if (c.volume != DGX_VOL_EC && c.volume != DGX_VOL_CENTRAL && c.volume != DGX_VOL_SHOCKCAP_HG &&
      c.volume != DGX_VOL_WEAK && c.volume != DGX_VOL_NONE && c.volume != DGX_VOL_WEAK_MFMA)
    return DGX_EINVAL;
  if (c.volume == DGX_VOL_WEAK_MFMA && (c.dim != 3 || c.polydeg != 3)) return DGX_EUNSUPPORTED;
  if (c.surface < DGX_SURF_LLF || c.surface > DGX_SURF_NONE) return DGX_EINVAL;
  if (c.volume == DGX_VOL_SHOCKCAP_HG) {
    if (c.fv_flux != DGX_SURF_LLF && c.fv_flux != DGX_SURF_HLL) return DGX_EINVAL;
    if (!(c.alpha_max >= 0.0 && c.alpha_max <= 1.0) || !(c.alpha_min >= 0.0 && c.alpha_min < 0.5))
      return DGX_EINVAL;
  }
  if (c.precision != DGX_FP64 && c.precision != DGX_MIXED) return DGX_EINVAL;
  if (c.precision == DGX_MIXED && c.volume != DGX_VOL_EC) return DGX_EUNSUPPORTED;
  const Launchers* L = launchers(c.dim, c.polydeg);
  if (!L) return DGX_EUNSUPPORTED;

  dgx_handle h = new dgx_solver();
  h->cfg = c;
  h->dim = c.dim;
  h->N = c.polydeg;
  h->n = c.polydeg + 1;
  h->NN = c.dim == 3 ? h->n * h->n * h->n : h->n * h->n;
  h->NF = c.dim == 3 ? h->n * h->n : h->n;
  h->NV = mhd ? 8 : c.dim + 2;
  h->mhd = mhd;
  h->E = 1;
  for (int d = 0; d < 3; ++d) {
    const int K = d < c.dim ? c.cells[d] : 1;
    h->E *= K;
    h->h[d] = d < c.dim ? (c.xmax[d] - c.xmin[d]) / K : 1.0;
  }
  h->stream = (hipStream_t)hip_stream;
  h->L = L;
  const int64_t nodes = h->E * h->NN;
  // The curvilinear and MHD kernels index a whole state (or metric) array in 32 bits; the
  // Cartesian Euler kernels use 64-bit offsets and only keep the element index in an int.
  const bool fits = (cv || mhd) ? (int64_t)(cv ? 9 : h->NV) * nodes < ((int64_t)1 << 31)
                                : h->E < ((int64_t)1 << 30);
  if (!fits) {
    delete h;
    return DGX_EUNSUPPORTED;
  }
  // set-up of dgx_max_dt_noalloc: the device address of this device's static scratch
  if (hipGetDevice(&h->device) != hipSuccess ||
      scratch_address(h->device, &h->noalloc_partial) != hipSuccess) {
    (void)hipGetLastError();
    delete h;
    return DGX_EHIP;
  }
  // curvilinear: the reference element's tables (2/h = 1); the metric terms carry the scale
  const double href[3] = {2.0, 2.0, 2.0};

  // operator tables
  std::vector<double> T(TAB_SIZE, 0.0);
  if (!stage_tables(h->N, cv ? href : h->h, T.data(),
                    c.volume == DGX_VOL_WEAK || c.volume == DGX_VOL_WEAK_MFMA)) {
    delete h;
    return DGX_EINVAL;
  }
  // curvilinear volume rounds contract with the sum of the pair's metric vectors: -S/2
  if (cv)
    for (int i = TAB_S; i < TAB_S + 3 * TMAX * TMAX; ++i) T[i] *= 0.5;

  const int64_t nblk = (h->E + L->ne - 1) / L->ne;
  h->npart = h->E;   // wave-speed partials: one per element
  h->nblk = nblk;
  auto alloc = [&](void** p, size_t bytes) -> bool {
    if (hipMalloc(p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    return true;
  };
  bool ok = alloc((void**)&h->tab, sizeof(double) * TAB_SIZE) &&
            alloc((void**)&h->u2, state_bytes(h)) &&
            alloc((void**)&h->k, state_bytes(h)) &&
            alloc((void**)&h->alpha, sizeof(double) * h->E) &&
            alloc((void**)&h->alpha_raw, sizeof(double) * h->E) &&
            alloc((void**)&h->energy, sizeof(double) * h->E) &&
            alloc((void**)&h->partial, sizeof(double) * std::max<size_t>(7 * (size_t)nblk, (size_t)h->E)) &&
            alloc((void**)&h->dt, sizeof(double) * 2) && alloc((void**)&h->flag, sizeof(int) * 2) &&
            alloc((void**)&h->slots, sizeof(double) * DT_SLOTS * DT_SLOT_STRIDE);
  if (!ok) {
    dgx_destroy(h);
    return DGX_ENOMEM;
  }
  if (hipMemcpy(h->tab, T.data(), sizeof(double) * TAB_SIZE, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(h->slots, 0, sizeof(double) * DT_SLOTS * DT_SLOT_STRIDE) != hipSuccess ||
      hipMemset(h->k, 0, state_bytes(h)) != hipSuccess ||
      hipMemset(h->alpha, 0, sizeof(double) * h->E) != hipSuccess ||
      hipMemset(h->flag, 0, sizeof(int) * 2) != hipSuccess ||
      hipMemset(h->dt, 0, sizeof(double) * 2) != hipSuccess) {
    dgx_destroy(h);
    return DGX_EHIP;
  }
  h->g.E = h->E;
  for (int d = 0; d < 3; ++d) h->g.K[d] = d < c.dim ? c.cells[d] : 1;
  h->g.gamma = c.gamma;
  h->g.inv_gm1 = 1.0 / (c.gamma - 1.0);
  h->g.tab = h->tab;
  h->g.flag = h->flag;
  if (cv) {
    h->curved = true;
    const int n = h->n;
    double x[16], w[16], D[256], Vinv[256];
    if (!lgl_tables(h->N, x, w, D, Vinv)) {
      dgx_destroy(h);
      return DGX_EINVAL;
    }
    if (!alloc((void**)&h->ja, sizeof(double) * 9 * nodes) ||
        !alloc((void**)&h->jac, sizeof(double) * nodes) ||
        !alloc((void**)&h->xyz, sizeof(double) * 3 * nodes) ||
        !alloc((void**)&h->dmat, sizeof(double) * n * n) || !alloc((void**)&h->t0, sizeof(double))) {
      dgx_destroy(h);
      return DGX_ENOMEM;
    }
    if (hipMemcpy(h->dmat, D, sizeof(double) * n * n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(h->t0, 0, sizeof(double)) != hipSuccess ||
        h->L->geometry(h->stream, h->g, h->dmat, cv->warp, h->xyz, h->ja, h->jac) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess) {
      dgx_destroy(h);
      return DGX_EHIP;
    }
    h->g.ja = h->ja;
    h->g.jac = h->jac;
    h->g.xyz = h->xyz;
    h->g.source = cv->source == DGX_SOURCE_MMS ? 1 : 0;
  }
  *out = h;
  return DGX_OK;
}

}  // namespace

extern "C" {

dgx_status dgx_create(const dgx_config* cfg, void* hip_stream, dgx_handle* out) {
  if (!cfg || !out) return DGX_EINVAL;
  return create_impl(*cfg, nullptr, hip_stream, out);
}

dgx_status dgx_create_curved(const dgx_curv_config* cv, void* hip_stream, dgx_handle* out) {
  if (!cv || !out) return DGX_EINVAL;
  *out = nullptr;
  if (cv->polydeg < 1 || cv->cells < 1 || !(cv->gamma > 1.0) || !(cv->warp >= 0.0 && cv->warp < 0.5))
    return DGX_EINVAL;
  if (cv->volume != DGX_VOL_EC && cv->volume != DGX_VOL_CENTRAL && cv->volume != DGX_VOL_NONE)
    return DGX_EUNSUPPORTED;
  if (cv->surface < DGX_SURF_LLF || cv->surface > DGX_SURF_NONE) return DGX_EINVAL;
  if (cv->source != DGX_SOURCE_NONE && cv->source != DGX_SOURCE_MMS) return DGX_EINVAL;
  dgx_config c{};
  c.dim = 3;
  c.polydeg = cv->polydeg;
  for (int d = 0; d < 3; ++d) {
    c.cells[d] = cv->cells;
    c.xmin[d] = -1.0;
    c.xmax[d] = 1.0;
  }
  c.gamma = cv->gamma;
  c.volume = cv->volume;
  c.surface = cv->surface;
  c.fv_flux = DGX_SURF_LLF;
  c.precision = DGX_FP64;
  return create_impl(c, cv, hip_stream, out);
}

dgx_status dgx_create_mhd(const dgx_mhd_config* mc, void* hip_stream, dgx_handle* out) {
  if (!mc || !out) return DGX_EINVAL;
  *out = nullptr;
  if (mc->polydeg < 1 || mc->cells < 1 || !(mc->gamma > 1.0)) return DGX_EINVAL;
  if (mc->volume != DGX_VOL_WEAK && mc->volume != DGX_VOL_EC) return DGX_EINVAL;
  if (mc->surface != DGX_SURF_HLL && mc->surface != DGX_SURF_LLF &&
      !(mc->surface == DGX_SURF_EC && mc->volume == DGX_VOL_EC))
    return DGX_EINVAL;
  dgx_config c{};
  c.dim = 3;
  c.polydeg = mc->polydeg;
  for (int d = 0; d < 3; ++d) {
    c.cells[d] = mc->cells;
    c.xmin[d] = -1.0;
    c.xmax[d] = 1.0;
  }
  c.gamma = mc->gamma;
  c.volume = mc->volume;   // the weak form's tables (Dhat) or flux differencing's (S)
  c.surface = mc->surface;
  c.fv_flux = DGX_SURF_LLF;
  c.precision = DGX_FP64;
  return create_impl(c, nullptr, hip_stream, out, true);
}

dgx_status dgx_geometry(dgx_handle h, double* ja, double* jac) {
  if (!h) return DGX_EINVAL;
  if (!h->curved) return fail(h, DGX_EINVAL, "dgx_geometry needs a curvilinear handle");
  const size_t nodes = (size_t)h->E * h->NN;
  if (ja) {
    CHKDEV(h, ja, sizeof(double) * 9 * nodes, "ja");
    HIPCHK(h, hipMemcpyAsync(ja, h->ja, sizeof(double) * 9 * nodes, hipMemcpyDeviceToDevice, h->stream));
  }
  if (jac) {
    CHKDEV(h, jac, sizeof(double) * nodes, "jac");
    HIPCHK(h, hipMemcpyAsync(jac, h->jac, sizeof(double) * nodes, hipMemcpyDeviceToDevice, h->stream));
  }
  return DGX_OK;
}

dgx_status dgx_destroy(dgx_handle h) {
  if (!h) return DGX_EINVAL;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  else (void)hipDeviceSynchronize();
  for (void* p : {(void*)h->tab, (void*)h->u2, (void*)h->k, (void*)h->alpha, (void*)h->alpha_raw,
                  (void*)h->energy, (void*)h->partial, (void*)h->dt, (void*)h->flag, (void*)h->ja,
                  (void*)h->jac, (void*)h->xyz, (void*)h->dmat, (void*)h->t0, (void*)h->slots})
    if (p) (void)hipFree(p);
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  drop_step_graph(h);
  if (h->cap) (void)hipStreamDestroy(h->cap);
  delete h;
  return DGX_OK;
}

dgx_status dgx_set_stream(dgx_handle h, void* hip_stream) {
  if (!h) return DGX_EINVAL;
  h->stream = (hipStream_t)hip_stream;
  return DGX_OK;
}

int64_t dgx_num_nodes(dgx_handle h) { return h ? h->E * h->NN : -1; }
int64_t dgx_num_elements(dgx_handle h) { return h ? h->E : -1; }

dgx_status dgx_node_coords(dgx_handle h, double* xyz) {
  if (!h) return DGX_EINVAL;
  CHKDEV(h, xyz, sizeof(double) * (size_t)h->dim * h->E * h->NN, "xyz");
  if (h->curved) {
    HIPCHK(h, hipMemcpyAsync(xyz, h->xyz, sizeof(double) * 3 * (size_t)h->E * h->NN,
                             hipMemcpyDeviceToDevice, h->stream));
    return DGX_OK;
  }
  HIPCHK(h, h->L->coords(h->stream, xyz, h->g, h->cfg.xmin));
  return DGX_OK;
}

dgx_status dgx_rhs(dgx_handle h, const double* u, double* du, double t) {
  if (!h) return DGX_EINVAL;
  CHKDEV(h, u, state_bytes(h), "u");
  CHKDEV(h, du, state_bytes(h), "du");
  if (overlap(u, du, state_bytes(h))) return fail(h, DGX_EINVAL, "u and du overlap");
  return enqueue_rhs(h, u, du, nullptr, t);
}

dgx_status dgx_rhs_alpha(dgx_handle h, const double* u, const double* alpha, double* du) {
  if (!h) return DGX_EINVAL;
  if (h->cfg.volume != DGX_VOL_SHOCKCAP_HG || h->curved)
    return fail(h, DGX_EINVAL, "dgx_rhs_alpha needs DGX_VOL_SHOCKCAP_HG");
  CHKDEV(h, u, state_bytes(h), "u");
  CHKDEV(h, du, state_bytes(h), "du");
  CHKDEV(h, alpha, sizeof(double) * h->E, "alpha");
  if (overlap(u, du, state_bytes(h))) return fail(h, DGX_EINVAL, "u and du overlap");
  return enqueue_rhs(h, u, du, alpha);
}

dgx_status dgx_indicator(dgx_handle h, const double* u, double* alpha, double* alpha_raw,
                         double* energy) {
  if (!h) return DGX_EINVAL;
  if (h->curved || h->mhd) return fail(h, DGX_EUNSUPPORTED, "no indicator on this handle");
  CHKDEV(h, u, state_bytes(h), "u");
  CHKDEV(h, alpha, sizeof(double) * h->E, "alpha");
  if (alpha_raw) CHKDEV(h, alpha_raw, sizeof(double) * h->E, "alpha_raw");
  if (energy) CHKDEV(h, energy, sizeof(double) * h->E, "energy");
  if (alpha_raw == alpha) return fail(h, DGX_EINVAL, "alpha and alpha_raw must differ");
  return enqueue_indicator(h, u, alpha, alpha_raw ? alpha_raw : h->alpha_raw, energy);
}

dgx_status dgx_max_dt(dgx_handle h, const double* u, double cfl, double* dt) {
  if (!h) return DGX_EINVAL;
  if (!(cfl > 0.0)) return fail(h, DGX_EINVAL, "cfl must be > 0");
  CHKDEV(h, u, state_bytes(h), "u");
  CHKDEV(h, dt, sizeof(double), "dt");
  HIPCHK(h, enqueue_maxspeed(h, u));
  launch_dt_final(h->stream, h->partial, h->npart, cfl, (double)(h->N + 1), dt, nullptr, nullptr);
  HIPCHK(h, hipGetLastError());
  return DGX_OK;
}

dgx_status dgx_max_dt_noalloc(dgx_handle h, const double* u, double cfl, double* dt) {
  if (!h) return DGX_EINVAL;
  if (!(cfl > 0.0)) return fail(h, DGX_EINVAL, "cfl must be > 0");
  if (h->E > NOALLOC_MAX_ELEMS)
    return fail(h, DGX_EINVAL, "dgx_max_dt_noalloc: " + std::to_string(h->E) +
                                   " elements exceed its static scratch of " +
                                   std::to_string(NOALLOC_MAX_ELEMS));
  int dev = -1;
  HIPCHK(h, hipGetDevice(&dev));
  if (dev != h->device)
    return fail(h, DGX_EINVAL, "dgx_max_dt_noalloc: the current device is not the handle's");
  CHKDEV(h, u, state_bytes(h), "u");
  CHKDEV(h, dt, sizeof(double), "dt");
  // every partial in [0, E) is written by the first kernel before the second reads it, so
  // nothing needs clearing
  double* part = h->noalloc_partial;
  HIPCHK(h, h->mhd      ? h->L->maxspeed_mhd(h->stream, u, part, h->g)
            : h->curved ? h->L->maxspeed_curv(h->stream, u, part, h->g)
                        : h->L->maxspeed(h->stream, u, part, h->g));
  launch_dt_final(h->stream, part, h->E, cfl, (double)(h->N + 1), dt, nullptr, nullptr);
  HIPCHK(h, hipGetLastError());
  return DGX_OK;
}

dgx_status dgx_step(dgx_handle h, double* u, int32_t nsteps, double cfl, double dt_fixed,
                    double* t) {
  if (!h) return DGX_EINVAL;
  if (nsteps < 0) return fail(h, DGX_EINVAL, "nsteps < 0");
  if (!(cfl > 0.0) && !(dt_fixed > 0.0)) return fail(h, DGX_EINVAL, "need cfl > 0 or dt_fixed > 0");
  CHKDEV(h, u, state_bytes(h), "u");
  if (t) CHKDEV(h, t, sizeof(double), "t");
  if (h->g.source && !t) return fail(h, DGX_EINVAL, "the source term needs the device time t");
  if (nsteps == 0) return DGX_OK;
  const bool adaptive = cfl > 0.0;
  // the state alternates between u and the library's u2, stage by stage: a stage reads the
  // neighbours' face states of its input while other blocks write their output
  double* buf[2] = {u, h->u2};
  int cur = 0;
  if (adaptive) {
    HIPCHK(h, enqueue_maxspeed(h, u));
    if (stage_slots(h)) {
      hipLaunchKernelGGL(k_dt_seed, dim3(1), dim3(1024), 0, h->stream, h->partial, h->npart, h->slots);
      HIPCHK(h, hipGetLastError());
    }
  }
  int s = 0;
  if (nsteps >= 2 && !h->prof) {
    // pairs of steps from the captured graph (ten stages: the state is back in u)
    dgx_status st = ensure_step_graph(h, u, cfl, dt_fixed, t);
    if (st != DGX_OK) return st;
    for (; s + 2 <= nsteps; s += 2)
      HIPCHK(h, hipGraphLaunch(s == 0 || !h->gexec2 ? h->gexec : h->gexec2, h->stream));
  }
  for (; s < nsteps; ++s) {
    // the indicator only before the call's first stage: the replayed pairs and these steps
    // run the same kernels on the same numbers
    dgx_status st = enqueue_step(h, buf, cur, cfl, dt_fixed, t, s + 1 < nsteps, s == 0, s % 2);
    if (st != DGX_OK) return st;
  }
  if (cur != 0) {
    const int64_t n = (int64_t)h->NV * h->E * h->NN;
    hipLaunchKernelGGL(k_copy, dim3(2048), dim3(256), 0, h->stream, h->u2, u, n);
    HIPCHK(h, hipGetLastError());
  }
  return DGX_OK;
}

dgx_status dgx_integrals(dgx_handle h, const double* u, const double* du, double* out7) {
  if (!h) return DGX_EINVAL;
  if (h->curved || h->mhd) return fail(h, DGX_EUNSUPPORTED, "no integrals on this handle");
  CHKDEV(h, u, state_bytes(h), "u");
  if (du) CHKDEV(h, du, state_bytes(h), "du");
  CHKDEV(h, out7, sizeof(double) * 7, "out7");
  HIPCHK(h, h->L->integrals(h->stream, u, du, h->partial, h->g));
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, h->stream, h->partial, h->nblk, out7);
  HIPCHK(h, hipGetLastError());
  return DGX_OK;
}

dgx_status dgx_check(dgx_handle h, int32_t* flag) {
  if (!h || !flag) return DGX_EINVAL;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  int f = 0;
  HIPCHK(h, hipMemcpy(&f, h->flag, sizeof(int), hipMemcpyDeviceToHost));
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, h->stream, h->flag);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipStreamSynchronize(h->stream));
  *flag = f;
  return f ? DGX_ENONPHYS : DGX_OK;
}

const char* dgx_last_error(dgx_handle h) { return h ? h->err.c_str() : "invalid handle"; }

dgx_status dgx_profile_enable(dgx_handle h, int32_t on) {
  if (!h) return DGX_EINVAL;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->prof = on != 0;
  h->ev_used = 0;
  h->ev_count.clear();
  h->launches = 0;
  h->prof_ms = 0.0;
  return DGX_OK;
}

dgx_status dgx_profile_read(dgx_handle h, double* avg_ms, int64_t* launches, const char** name) {
  if (!h) return DGX_EINVAL;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  for (size_t i = 0; i + 1 < h->ev_used; i += 2) {
    float ms = 0.f;
    HIPCHK(h, hipEventElapsedTime(&ms, h->ev[i], h->ev[i + 1]));
    h->prof_ms += ms;
    h->launches += h->ev_count[i / 2];
  }
  h->ev_used = 0;
  h->ev_count.clear();
  if (avg_ms) *avg_ms = h->launches ? h->prof_ms / h->launches : 0.0;
  if (launches) *launches = h->launches;
  if (name) *name = h->L->volume_name;
  return DGX_OK;
}

}  // extern "C"
