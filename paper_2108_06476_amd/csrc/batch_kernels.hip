// batch_kernels.hip -- stage kernels of the ensemble API: every launch processes the
// element tiles of all runs (work items), each tile with the same stage body as the
// single-run kernel, specialised per polydeg (3, 4, 5) behind a uniform branch.
#include "batch_kernels.h"

namespace dgx {

template <typename RT, int BUDGET>
struct BatchSmem {
  static constexpr size_t s3 = sizeof(typename StageLdsOf<3, 3, VOL_EC, RT, BUDGET>::type);
  static constexpr size_t s4 = sizeof(typename StageLdsOf<3, 4, VOL_EC, RT, BUDGET>::type);
  static constexpr size_t s5 = sizeof(typename StageLdsOf<3, 5, VOL_EC, RT, BUDGET>::type);
  static constexpr size_t m34 = s3 > s4 ? s3 : s4;
  static constexpr size_t bytes = m34 > s5 ? m34 : s5;
};

// Work items are split into 8 contiguous ranges, one per XCD (blocks are dispatched
// round-robin over the XCDs), so consecutive tiles of a run share an L2.  The grid is a
// multiple of 8.
__device__ __forceinline__ void xcd_range(int total, int& first, int& end, int& stride) {
  const int x = blockIdx.x % 8, i = blockIdx.x / 8;
  const int chunk = (total + 7) / 8;
  first = x * chunk + i;
  end = min(total, (x + 1) * chunk);
  stride = gridDim.x / 8;
}

__device__ __forceinline__ int find_run(const BatchLaunch& b, int item) {
  int lo = 0, hi = b.nruns;   // prefix[lo] <= item < prefix[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (b.prefix[mid] <= item) lo = mid;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ Geom run_geom(const RunDesc& d) {
  Geom g;
  g.E = d.E;
  g.K[0] = d.K[0];
  g.K[1] = d.K[1];
  g.K[2] = d.K[2];
  g.gamma = d.gamma;
  g.inv_gm1 = d.inv_gm1;
  g.tab = d.tab;
  g.flag = d.flag;
  return g;
}

template <int N, typename RT, int BUDGET, int EPI>
__device__ __forceinline__ void batch_tile(unsigned char* smem, const double* sT, const RunDesc& d,
                                           int tile, int cur, double A, double B, int emit,
                                           int kw) {
  using L = typename StageLdsOf<3, N, VOL_EC, RT, BUDGET>::type;
  StageArgs a;
  a.uin = cur ? d.u2 : d.u;
  a.uout = cur ? d.u : d.u2;
  a.du = d.du;
  a.k = d.k;
  a.alpha = nullptr;
  a.dt = d.dt;
  a.speed = emit ? d.speed : nullptr;
  a.A = A;
  a.B = B;
  a.surf = d.surf;
  a.fvf = SURF_LLF;
  a.kw = kw;
  stage_tile<3, N, VOL_EC, EPI, RT, BUDGET>(*reinterpret_cast<L*>(smem), sT, a, run_geom(d), tile);
}

__device__ __forceinline__ void batch_item_tables(const RunDesc& d, double* sT, int budget) {
  for (int i = threadIdx.x; i < TAB_SIZE; i += budget) sT[i] = d.tab[i];
}

// One launch covers every work item of every run.  PERSIST = false: one block per item
// (block b takes item xcd_tile(b)), asked for 4 waves per SIMD (the float32 body would
// otherwise take 130 VGPRs and 3); PERSIST = true: a fixed grid whose blocks loop over
// XCD-contiguous item ranges.  The loop costs registers (the compiler keeps ~200 VGPRs
// live across it against 128 for one item), so the tuner times both.
template <typename RT, int BUDGET, int EPI, bool PERSIST>
__global__ __launch_bounds__(BUDGET, PERSIST ? 1 : 4) void k_batch_stage(BatchLaunch b, int cur, double A, double B,
                                                        int emit, int kw) {
  __shared__ __align__(16) unsigned char smem[BatchSmem<RT, BUDGET>::bytes];
  __shared__ double sT[TAB_SIZE];
  if constexpr (!PERSIST) {
    const int item = (int)xcd_tile(blockIdx.x, gridDim.x);
    if (item >= b.total) return;
    const int ri = find_run(b, item);
    const RunDesc d = b.runs[b.order[ri]];
    const int tile = item - b.prefix[ri];
    batch_item_tables(d, sT, BUDGET);
    if (d.N == 3) batch_tile<3, RT, BUDGET, EPI>(smem, sT, d, tile, cur, A, B, emit, kw);
    else if (d.N == 4) batch_tile<4, RT, BUDGET, EPI>(smem, sT, d, tile, cur, A, B, emit, kw);
    else batch_tile<5, RT, BUDGET, EPI>(smem, sT, d, tile, cur, A, B, emit, kw);
  } else {
    int first, end, stride;
    xcd_range(b.total, first, end, stride);
    for (int item = first; item < end; item += stride) {
      const int ri = find_run(b, item);
      const RunDesc d = b.runs[b.order[ri]];
      const int tile = item - b.prefix[ri];
      __syncthreads();   // the previous tile is done with the LDS
      batch_item_tables(d, sT, BUDGET);
      if (d.N == 3) batch_tile<3, RT, BUDGET, EPI>(smem, sT, d, tile, cur, A, B, emit, kw);
      else if (d.N == 4) batch_tile<4, RT, BUDGET, EPI>(smem, sT, d, tile, cur, A, B, emit, kw);
      else batch_tile<5, RT, BUDGET, EPI>(smem, sT, d, tile, cur, A, B, emit, kw);
    }
  }
}

// Per element of one tile: sum_d (2/h_d) max over the nodes of |v_d| + c -> speed[e].
template <int N, int BUDGET>
__device__ __forceinline__ void speed_tile(double (*sm)[BUDGET], const RunDesc& d, int tile) {
  using S = Shape<3, N, BUDGET>;
  constexpr int NN = S::NN;
  constexpr int P2 = NN <= 64 ? 64 : (NN <= 128 ? 128 : 256);
  const int le = threadIdx.x / NN;
  const int node = threadIdx.x - le * NN;
  const int e = tile * S::NE + le;
  const bool inb = le < S::NE;
  const bool active = inb && e < d.E;
  const int base = le * NN;
  if (inb) {
    if (active) {
      const unsigned ENN = (unsigned)d.E * NN;
      double um[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) um[v] = d.u[v * ENN + (unsigned)e * NN + node];
      Prim<double> q;
      if (!cons_to_prim<3>(um, d.gamma, q)) *d.flag = 1;
#pragma unroll
      for (int k = 0; k < 3; ++k) sm[k][base + node] = fabs(q.v[k]) + q.c;
    } else {
#pragma unroll
      for (int k = 0; k < 3; ++k) sm[k][base + node] = 0.0;
    }
  }
  __syncthreads();
  for (int h = P2 / 2; h > 0; h >>= 1) {
    if (inb && node < h && node + h < NN) {
#pragma unroll
      for (int k = 0; k < 3; ++k) sm[k][base + node] = fmax(sm[k][base + node], sm[k][base + node + h]);
    }
    __syncthreads();
  }
  if (active && node == 0) {
    double lam = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) lam += d.tab[TAB_JAC + k] * sm[k][base];
    d.speed[e] = lam;
  }
}

template <int BUDGET>
__global__ __launch_bounds__(BUDGET) void k_batch_maxspeed(BatchLaunch b) {
  __shared__ double sm[3][BUDGET];
  int first, end, stride;
  xcd_range(b.total, first, end, stride);
  for (int item = first; item < end; item += stride) {
    const int ri = find_run(b, item);
    const RunDesc d = b.runs[b.order[ri]];
    const int tile = item - b.prefix[ri];
    __syncthreads();
    if (d.N == 3) speed_tile<3, BUDGET>(sm, d, tile);
    else if (d.N == 4) speed_tile<4, BUDGET>(sm, d, tile);
    else speed_tile<5, BUDGET>(sm, d, tile);
  }
}

// One block per run: dt = cfl * 2 / ((N+1) * max_e speed[e]); t += dt.
__global__ __launch_bounds__(512) void k_batch_dt(const RunDesc* __restrict__ runs, double cfl) {
  __shared__ double s[8];
  const RunDesc d = runs[blockIdx.x];
  const double m = block_max<512>(d.speed, d.E, s);
  if (threadIdx.x == 0) {
    const double dt = cfl * 2.0 / ((d.N + 1.0) * m);
    *d.dt = dt;
    if (d.t) *d.t += dt;
  }
}

// u <- u2 for every run (the state sits in u2 after an odd number of stages).
__global__ __launch_bounds__(256) void k_batch_copy(const RunDesc* __restrict__ runs) {
  const RunDesc d = runs[blockIdx.y];
  const int n = d.N + 1;
  const int64_t len = (int64_t)5 * d.E * n * n * n;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < len; i += (int64_t)gridDim.x * 256)
    d.u[i] = d.u2[i];
}

int batch_tile_elems(int N, int budget) {
  const int NN = (N + 1) * (N + 1) * (N + 1);
  return NN >= budget ? 1 : budget / NN;
}

template <typename RT, int BUDGET, bool PERSIST>
static hipError_t stage_launch(hipStream_t st, const BatchLaunch& b, int grid, int epi, int cur,
                               double A, double B, int emit, int kw) {
  if (epi == EPI_RK)
    hipLaunchKernelGGL((k_batch_stage<RT, BUDGET, EPI_RK, PERSIST>), dim3(grid), dim3(BUDGET), 0, st,
                       b, cur, A, B, emit, kw);
  else
    hipLaunchKernelGGL((k_batch_stage<RT, BUDGET, EPI_RHS, PERSIST>), dim3(grid), dim3(BUDGET), 0, st,
                       b, cur, A, B, emit, kw);
  return hipGetLastError();
}

template <typename RT>
static hipError_t stage_launch_rt(hipStream_t st, const BatchLaunch& b, int budget, int grid,
                                  int epi, int cur, double A, double B, int emit,
                                  int kw) {
  // grid >= items: one block per item; otherwise persistent blocks
  const bool persist = grid < b.total;
  if (budget == 512) {
    if (persist) return stage_launch<RT, 512, true>(st, b, grid, epi, cur, A, B, emit, kw);
    return stage_launch<RT, 512, false>(st, b, grid, epi, cur, A, B, emit, kw);
  }
  if (persist) return stage_launch<RT, 256, true>(st, b, grid, epi, cur, A, B, emit, kw);
  return stage_launch<RT, 256, false>(st, b, grid, epi, cur, A, B, emit, kw);
}

hipError_t batch_stage(hipStream_t st, const BatchLaunch& b, int budget, int grid, int prec,
                       int epi, int cur, double A, double B, int emit_speed, int kw) {
  if (grid % 8 != 0 || grid <= 0) return hipErrorInvalidValue;
  if (prec == 1) return stage_launch_rt<float>(st, b, budget, grid, epi, cur, A, B, emit_speed, kw);
  return stage_launch_rt<double>(st, b, budget, grid, epi, cur, A, B, emit_speed, kw);
}

hipError_t batch_maxspeed(hipStream_t st, const BatchLaunch& b, int budget, int grid) {
  if (grid % 8 != 0 || grid <= 0) return hipErrorInvalidValue;
  if (budget == 512) hipLaunchKernelGGL((k_batch_maxspeed<512>), dim3(grid), dim3(512), 0, st, b);
  else hipLaunchKernelGGL((k_batch_maxspeed<256>), dim3(grid), dim3(256), 0, st, b);
  return hipGetLastError();
}

hipError_t batch_dt(hipStream_t st, const RunDesc* runs, int nruns, double cfl) {
  hipLaunchKernelGGL(k_batch_dt, dim3(nruns), dim3(512), 0, st, runs, cfl);
  return hipGetLastError();
}

hipError_t batch_copy(hipStream_t st, const RunDesc* runs, int nruns, int64_t max_len) {
  const int64_t bx = (max_len + 255) / 256;
  hipLaunchKernelGGL(k_batch_copy, dim3((unsigned)(bx < 1024 ? bx : 1024), nruns), dim3(256), 0, st,
                     runs);
  return hipGetLastError();
}

}  // namespace dgx
