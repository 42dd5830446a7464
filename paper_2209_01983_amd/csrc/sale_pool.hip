// sale_pool.hip -- the persistent multi-run kernel of libsale (gfx950).
//
// A pool advance is one launch of k_pool. Its blocks pull work items from a
// device queue in a fixed global order:
//
//   for round s = 0 .. rounds-1:
//     for every active run q: the Lagrange tiles of q's step s   (phase 2s)
//     for every active run q: the remap tiles of q's step s      (phase 2s+1)
//
// Item j of a run's phase p may start only when the run's phase counter has
// reached p; the last tile to finish a phase advances the counter (and, after
// a remap phase other than the last round's, starts the run's next time step:
// dt from the signal speed, t and the step count advanced). A block holds one item
// at a time and every item depends only on items earlier in the queue, so the
// earliest unfinished item can always progress: the waits end. They are also
// capped in time; a wait that hits the cap aborts the advance (every later
// wait gives up at once, the runs concerned are flagged) so that every wave
// exits soon. Writes of a finished tile are released at agent scope (an L2
// write-back, no invalidation) before the counter moves and acquired at agent
// scope by the waiting block after it sees the counter, which covers the
// per-XCD L2 caches.
//
// A run's current state buffer follows its own step count, so a run that is
// done (step target or t_end reached, or flagged) simply skips its items.
#include "sale_tiles.h"

// waves per SIMD the persistent kernel is compiled for: with both tile kinds in
// one kernel, 2 (one 512-thread block per CU) keeps every value in registers
#ifndef SALE_WAVES_POOL
#define SALE_WAVES_POOL 2
#endif

namespace sale {

namespace {

constexpr int CH = kPoolRows, CW = kPoolWidth;
// register cap of the lockstep tile kernels (4 waves per SIMD)
constexpr int waves_of_lock() { return 4; }
// the FP32 bulk remap tile of 16 rows fits 80 VGPRs and 40 KB of LDS: three
// blocks per CU
template <typename R>
constexpr int waves_of_lock_remap() { return sizeof(R) == 4 && CH == 16 ? 6 : waves_of_lock(); }
constexpr int NT = tile_threads<CH, CW>();
constexpr int LDS_L = lagrange_lds_doubles<CH, CW, NT>();
template <typename R>
constexpr int LDS_R = remap_lds_doubles<R, CH, CW, NT>();
constexpr int LDS_DOUBLES = LDS_L > LDS_R<double> ? LDS_L : LDS_R<double>;
// Cap of one wait, in ticks of the 100 MHz constant clock. A wait normally
// lasts at most one tile of the same run (milliseconds).
constexpr long long kWaitTicks = 200000000ll;  // 2 s

template <typename R>
__device__ RunArgs<R> args_of(const PoolRun<R> &p) {
  RunArgs<R> a;
  a.m = p.m;
  a.ctl = p.ctl;
  const int cur = (int)((p.ctl->step - 1 - p.step0) & 1);  // the step in flight was counted
  a.cur = p.s[cur];
  a.nxt = p.s[1 - cur];
  a.up = p.up;
  a.vp = p.vp;
  a.wp = p.wp;
  a.geo = p.geo;
  a.ga = p.ga;
  a.gb = p.gb;
  return a;
}

// prepare an advance: queue head, per-run counters and the first step's dt
template <typename R>
__global__ void k_pool_prepare(PoolRun<R> *runs, const int *act, PoolQueue *qh) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q == 0) {
    qh->head = 0ull;
    qh->timeouts = 0u;
    qh->abort = 0u;
  }
  if (q >= qh->nact) return;
  const PoolRun<R> &p = runs[act[q]];
  Ctl *c = p.ctl;
  c->tiles_done = 0u;
  c->phase = 0u;
  c->step_target = p.step_target;
  if (c->clk_first == 0) c->clk_first = wall_clock64();
  begin_step(p.m, c, p.step_target);
}

// index of the last prefix entry <= j (pref is non-decreasing, pref[0] = 0)
__device__ __forceinline__ int find_run(const int *pref, int n, int j) {
  int lo = 0, hi = n;  // invariant: pref[lo] <= j < pref[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pref[mid] <= j)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

template <typename R>
__global__ __launch_bounds__(NT, SALE_WAVES_POOL) void k_pool(const PoolRun<R> *__restrict__ runs, const int *__restrict__ act,
                                             const int *__restrict__ prefA, const int *__restrict__ prefB,
                                             PoolQueue *qh) {
  __shared__ double lds[LDS_DOUBLES];
  __shared__ unsigned long long s_item;
  __shared__ int s_go;
  const int nact = qh->nact, totA = qh->totA, totB = qh->totB;
  const unsigned long long per_round = (unsigned long long)(totA + totB);
  const int rounds = qh->rounds;
  const unsigned long long total = per_round * (unsigned long long)rounds;
  for (;;) {
    __syncthreads();  // the previous item's LDS reads are done
    if (threadIdx.x == 0) s_item = atomicAdd(&qh->head, 1ull);
    __syncthreads();
    const unsigned long long item = s_item;
    if (item >= total) break;
    const int round = (int)(item / per_round);
    int j = (int)(item % per_round);
    const bool remap = j >= totA;
    if (remap) j -= totA;
    const int q = find_run(remap ? prefB : prefA, nact, j);
    const int tile = j - (remap ? prefB[q] : prefA[q]);
    const PoolRun<R> &p = runs[act[q]];
    Ctl *ctl = p.ctl;
    const unsigned int want = 2u * (unsigned)round + (remap ? 1u : 0u);
    // wait for the run's previous phase
    if (threadIdx.x == 0) {
      int go = 1;
      const long long t0 = wall_clock64();
      while (__hip_atomic_load(&ctl->phase, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < want) {
        if (__hip_atomic_load(&qh->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          go = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
        if (wall_clock64() - t0 > kWaitTicks) {
          go = 0;
          atomicAdd(&qh->timeouts, 1u);
          atomicOr(&qh->abort, 1u);
          break;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // see the previous phase's writes
      // a run whose item could not wait is flagged: its state is not trusted
      if (!go) atomicOr(&ctl->status, SALE_FLAG_NUMERIC);
      s_go = go;
    }
    __syncthreads();
    const bool ran = s_go && !__hip_atomic_load(&ctl->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (ran) {
      const RunArgs<R> a = args_of(p);
      if (!remap) {
        const bool t = lagrange_tile<R, CH, CW, NT>(a, tile, ctl->dt, lds);
        if (t) atomicOr(&ctl->status, SALE_FLAG_TANGLE);
      } else {
        double amax;
        bool bad, tangle;
        remap_tile<R, CH, CW, NT>(a, tile, lds, &amax, &bad, &tangle);
        block_max_to_ctl<NT>(ctl, amax, bad);
        if (tangle) atomicOr(&ctl->status, SALE_FLAG_TANGLE);
      }
    }
    // finish the item: release its writes, count it; the last tile of the
    // phase opens the next phase (after a remap phase: the next time step)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
      const unsigned int ntiles = (unsigned)(remap ? p.gb.blocks() : p.ga.blocks());
      const unsigned int old = atomicAdd(&ctl->tiles_done, 1u);
      if (old == ntiles - 1u) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        atomicExch(&ctl->tiles_done, 0u);
        if (remap && ran) ctl->clk_last = wall_clock64();  // the step just completed
        // the next advance's prepare starts the step after the last round
        if (remap && round + 1 < rounds) begin_step(p.m, ctl, p.step_target);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        atomicAdd(&ctl->phase, 1u);
      }
    }
  }
}

// ---- lockstep advance: one launch per phase over the tiles of every active run
// A round is four launches: begin (dt and done of every run), the Lagrange
// tiles of all runs, the remap tiles of all runs, the clock stamp of the
// runs' completed steps. Kernel boundaries order the phases, so nothing waits
// on the device; a run that is done skips its tiles (its state stays in its
// buffer). Each run's grids carry a z split sized to its share of the
// advance's cells. Kernel arguments never change between the rounds of an
// advance (the run descriptors and tables live in device memory), so every
// round after the first can be the replay of one captured graph.
template <typename R>
__global__ void k_lock_begin(const PoolRun<R> *__restrict__ runs, const int *__restrict__ act, int nact,
                             int first) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nact) return;
  const PoolRun<R> &p = runs[act[q]];
  Ctl *c = p.ctl;
  if (first) {
    c->step_target = p.step_target;
    if (c->clk_first == 0) c->clk_first = wall_clock64();
  }
  begin_step(p.m, c, p.step_target);
}

template <typename R>
__global__ __launch_bounds__(NT, waves_of_lock()) void k_lock_lagrange(const PoolRun<R> *__restrict__ runs,
                                                                      const int *__restrict__ act,
                                                                      const int *__restrict__ prefA, int nact) {
  __shared__ double lds[LDS_L];
  const int g = xcd_logical_block(blockIdx.x, gridDim.x);
  const int q = find_run(prefA, nact, g);
  const PoolRun<R> &p = runs[act[q]];
  Ctl *ctl = p.ctl;
  if (ctl->done) return;
  const RunArgs<R> a = args_of(p);
  if (lagrange_tile<R, CH, CW, NT>(a, g - prefA[q], ctl->dt, lds)) atomicOr(&ctl->status, SALE_FLAG_TANGLE);
}

template <typename R>
__global__ __launch_bounds__(NT, waves_of_lock_remap<R>()) void k_lock_remap(const PoolRun<R> *__restrict__ runs,
                                                                            const int *__restrict__ act,
                                                                            const int *__restrict__ prefB, int nact) {
  __shared__ double lds[LDS_R<R>];
  const int g = xcd_logical_block(blockIdx.x, gridDim.x);
  const int q = find_run(prefB, nact, g);
  const PoolRun<R> &p = runs[act[q]];
  Ctl *ctl = p.ctl;
  if (ctl->done) return;
  const RunArgs<R> a = args_of(p);
  double amax;
  bool bad, tangle;
  remap_tile<R, CH, CW, NT>(a, g - prefB[q], lds, &amax, &bad, &tangle);
  block_max_to_ctl<NT>(ctl, amax, bad);
  if (tangle) atomicOr(&ctl->status, SALE_FLAG_TANGLE);
}

// device clock of each run's last completed step
template <typename R>
__global__ void k_lock_stamp(const PoolRun<R> *__restrict__ runs, const int *__restrict__ act, int nact) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nact) return;
  Ctl *c = runs[act[q]].ctl;
  if (!c->done) c->clk_last = wall_clock64();
}

}  // namespace

template <typename R>
hipError_t launch_pool_lockstep(const PoolRun<R> *runs, const int *act, const int *prefA, const int *prefB,
                                int nact, int totA, int totB, int rounds, int first, hipStream_t s) {
  const int nb = (nact + 255) / 256;
  for (int r = 0; r < rounds; r++) {
    hipLaunchKernelGGL(k_lock_begin<R>, dim3(nb), dim3(256), 0, s, runs, act, nact, first && r == 0 ? 1 : 0);
    hipLaunchKernelGGL(k_lock_lagrange<R>, dim3(totA), dim3(NT), 0, s, runs, act, prefA, nact);
    hipLaunchKernelGGL(k_lock_remap<R>, dim3(totB), dim3(NT), 0, s, runs, act, prefB, nact);
    hipLaunchKernelGGL(k_lock_stamp<R>, dim3(nb), dim3(256), 0, s, runs, act, nact);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
template hipError_t launch_pool_lockstep<double>(const PoolRun<double> *, const int *, const int *, const int *,
                                                 int, int, int, int, int, hipStream_t);
template hipError_t launch_pool_lockstep<float>(const PoolRun<float> *, const int *, const int *, const int *, int,
                                                int, int, int, int, hipStream_t);

template <typename R>
hipError_t launch_pool_advance(PoolRun<R> *runs, const int *act, const int *prefA, const int *prefB,
                               PoolQueue *qh, int nact, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_pool_prepare<R>, dim3((nact + 255) / 256), dim3(256), 0, s, runs, act, qh);
  hipLaunchKernelGGL(k_pool<R>, dim3(blocks), dim3(NT), 0, s, runs, act, prefA, prefB, qh);
  return hipGetLastError();
}

template <typename R>
int pool_resident_blocks() {
  int per_cu = 0, cus = 0, dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_pool<R>, NT, 0) != hipSuccess) per_cu = 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
  if (per_cu < 1) per_cu = 1;
  return per_cu * cus;
}

template hipError_t launch_pool_advance<double>(PoolRun<double> *, const int *, const int *, const int *,
                                                PoolQueue *, int, int, hipStream_t);
template hipError_t launch_pool_advance<float>(PoolRun<float> *, const int *, const int *, const int *,
                                               PoolQueue *, int, int, hipStream_t);
template int pool_resident_blocks<double>();
template int pool_resident_blocks<float>();

}  // namespace sale
