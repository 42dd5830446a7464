// sale_pool.hip -- the multi-run kernels of libsale (gfx950).
//
// A persistent pool advance is one launch of k_pool. The active runs are
// split into one group per XCD (balanced by cells on the host), and a block
// serves only the queue of the XCD it runs on, pulling work items in a fixed
// order:
//
//   for round s = 0 .. rounds-1:
//     for every run q of the XCD: the Lagrange tiles of q's step s   (phase 2s)
//     for every run q of the XCD: the remap tiles of q's step s      (phase 2s+1)
//
// Item j of a run's phase p may start only when the run's phase counter has
// reached p; the last tile to finish a phase advances the counter (and, after
// a remap phase other than the last round's, starts the run's next time step:
// dt from the signal speed, t and the step count advanced). A block holds one item
// at a time and every item depends only on items earlier in its XCD's queue,
// so the earliest unfinished item of every served queue can always progress:
// the waits end. They are also capped in time; a wait that hits the cap
// aborts the advance (every later wait gives up at once, the runs concerned
// are flagged) so that every wave exits soon. A queue whose XCD received no
// block of the launch is never served: the last block to leave flags its runs.
//
// Coherence. All tiles of a run execute on one XCD, whose L2 is the point
// where they meet: a finished tile waits until its stores have reached the L2
// (vmcnt 0 in every wave, then the block barrier) before it counts itself, and
// a block that sees a phase counter move takes an agent-scope acquire (its
// CU's L1 lines are dropped) before it reads. No tile writes the L2 back to
// memory, as an agent-scope release after every tile would: where a run's
// tiles met in memory, those write-backs took most of the launch's time. The
// writes reach memory at the end of the kernel. Run-control
// fields are accessed one way only during the launch: the counters, the
// signal-speed maximum and the status flags by device-scope atomics, the step
// fields (dt, t, step, done) by plain loads and stores on the run's XCD.
//
// A run's current state buffer follows its own step count, so a run that is
// done (step target or t_end reached, or flagged) simply skips its items.
#include "sale_pool.h"
#include "sale_tiles.h"

// waves per SIMD the persistent kernel is compiled for: 4 (two 512-thread
// blocks per CU, 128 VGPRs)
#ifndef SALE_WAVES_POOL
#define SALE_WAVES_POOL 4
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

// the tile planes of the persistent kernel (both tile kinds)
__shared__ double pool_lds[LDS_DOUBLES];

// id of the XCD this wave runs on (hardware register XCC_ID, bits 3:0)
__device__ __forceinline__ int xcc_id() {
  unsigned int x;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(x));
  return (int)x;
}

// Release of a finished tile to its XCD: every store of the wave has reached
// the L2 (vmcnt 0; gfx9 counts stores in vmcnt).
__device__ __forceinline__ void stores_reached_l2() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Acquire of a phase: an agent-scope acquire fence, whose invalidation drops
// the CU's vector L1 lines (a workgroup-scope acquire does not, outside
// thread-group split mode); the run's other tiles' writes are in this XCD's
// L2 and are read from there.
__device__ __forceinline__ void acquire_phase() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

template <typename T>
__device__ __forceinline__ T *uniform_ptr(T *p) {
  const unsigned long long v = (unsigned long long)p;
  const unsigned int lo = (unsigned int)__builtin_amdgcn_readfirstlane((int)(unsigned int)v);
  const unsigned int hi = (unsigned int)__builtin_amdgcn_readfirstlane((int)(unsigned int)(v >> 32));
  return (T *)(((unsigned long long)hi << 32) | lo);
}

// A block-uniform copy of *p, every dword read into scalar registers: the
// run descriptor's pointers and sizes then address the tiles' loads from
// scalar registers, as in the lockstep kernels.
template <typename T>
__device__ __forceinline__ T uniform_copy(const T *p) {
  static_assert(sizeof(T) % 4 == 0, "a whole number of dwords");
  int w[sizeof(T) / 4];
  const int *q = reinterpret_cast<const int *>(p);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); i++) w[i] = __builtin_amdgcn_readfirstlane(q[i]);
  T t;
  __builtin_memcpy(&t, w, sizeof(T));
  return t;
}

// step arguments of a pool run: the state buffer follows the run's step count
// (the step in flight was counted). SEL: choose the buffers by selects, for a
// descriptor held in registers (an index would put it in scratch memory).
template <typename R, bool SEL = false>
__device__ __forceinline__ RunArgs<R> args_of(const PoolRun<R> &p, int cur) {
  RunArgs<R> a;
  a.m = p.m;
  a.ctl = p.ctl;
  if (SEL) {
    a.cur = cur ? p.s[1] : p.s[0];
    a.nxt = cur ? p.s[0] : p.s[1];
  } else {
    a.cur = p.s[cur];
    a.nxt = p.s[1 - cur];
  }
  a.up = p.up;
  a.vp = p.vp;
  a.wp = p.wp;
  a.geo = p.geo;
  a.ga = p.ga;
  a.gb = p.gb;
  return a;
}
template <typename R>
__device__ __forceinline__ int cur_of(const PoolRun<R> &p) {
  return (int)((p.ctl->step - 1 - p.step0) & 1);
}

// One work item of the persistent kernel. The run descriptor is read into
// scalar registers (it arrives through a vector pointer), so the tiles
// address their loads from scalar registers as in the lockstep kernels.
template <typename R>
__device__ __forceinline__ void lagrange_item(const PoolRun<R> *pp, int tile) {
  const PoolRun<R> p = uniform_copy(uniform_ptr(pp));
  const RunArgs<R> a = args_of<R, true>(p, __builtin_amdgcn_readfirstlane(cur_of(p)));
  if (lagrange_tile<R, CH, CW, NT>(a, __builtin_amdgcn_readfirstlane(tile), p.ctl->dt, pool_lds))
    atomicOr(&p.ctl->status, SALE_FLAG_TANGLE);
}

template <typename R>
__device__ __forceinline__ void remap_item(const PoolRun<R> *pp, int tile) {
  const PoolRun<R> p = uniform_copy(uniform_ptr(pp));
  const RunArgs<R> a = args_of<R, true>(p, __builtin_amdgcn_readfirstlane(cur_of(p)));
  double amax;
  bool bad, tangle;
  remap_tile<R, CH, CW, NT>(a, __builtin_amdgcn_readfirstlane(tile), pool_lds, &amax, &bad, &tangle);
  block_max_to_ctl<NT>(p.ctl, amax, bad);
  if (tangle) atomicOr(&p.ctl->status, SALE_FLAG_TANGLE);
}

// The same items as calls of their own (not inlined). Both ways fit the
// kernel in 128 VGPRs (two blocks per CU). Inlined, the tile loops run a few
// percent more instructions per plane; called, every item stores and reloads
// the callee-saved registers (about 12 KB per wave). The FP32-bulk kernel is
// bound by instruction issue and takes the calls (256 runs: 1.79e10 against
// 1.70e10 cell-updates/s inlined); the FP64 kernel inlines (32 runs: 8.5e9
// against 7.8e9 with calls; 256 runs: equal).
template <typename R>
__device__ __attribute__((noinline)) void lagrange_item_call(const PoolRun<R> *pp, int tile) {
  lagrange_item<R>(pp, tile);
}
template <typename R>
__device__ __attribute__((noinline)) void remap_item_call(const PoolRun<R> *pp, int tile) {
  remap_item<R>(pp, tile);
}
template <typename R>
constexpr bool pool_calls() { return sizeof(R) == 4; }

// The next time step of a pool run, taken inside the persistent kernel by the
// last tile of its remap phase: begin_step's arithmetic, with the status
// flags and the signal-speed maximum (updated by atomics) read and reset by
// atomics.
__device__ __forceinline__ void pool_begin_step(const Mesh &m, Ctl *ctl, long long step_target) {
  const unsigned int status = __hip_atomic_load(&ctl->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (status != 0u || ctl->t >= ctl->t_end || ctl->step >= step_target) {
    ctl->done = 1u;
    return;
  }
  const unsigned long long bits = __hip_atomic_load(&ctl->amax_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const double amax = __longlong_as_double((long long)bits);
  const double rem = ctl->t_end - ctl->t;
  double dt = amax > 0.0 ? m.cfl * m.h / amax : rem;
  if (dt > rem) dt = rem;
  if (!(dt > 0.0) || !isfinite(dt)) {
    atomicOr(&ctl->status, SALE_FLAG_NUMERIC);
    ctl->done = 1u;
    return;
  }
  ctl->dt = dt;
  ctl->done = 0u;
  ctl->t = ctl->t + dt;
  ctl->step += 1;
  __hip_atomic_store(&ctl->amax_bits, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// prepare an advance: queue heads, per-run counters and the first step's dt
template <typename R>
__global__ void k_pool_prepare(PoolRun<R> *runs, const int *act, PoolQueue *qh) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < kPoolGroups) qh->head[q] = 0ull;
  if (q == 0) {
    qh->timeouts = 0u;
    qh->abort = 0u;
    qh->exited = 0u;
    qh->starved = 0u;
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

// index of the last prefix entry <= j in pref[lo .. hi) (pref is
// non-decreasing, pref[lo] <= j)
__device__ __forceinline__ int find_run(const int *pref, int lo, int hi, int j) {
  // invariant: pref[lo] <= j < pref[hi]
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
__global__ __launch_bounds__(NT, SALE_WAVES_POOL) void k_pool(const PoolRun<R> *__restrict__ runs,
                                                              const int *__restrict__ act,
                                                              const int *__restrict__ prefA,
                                                              const int *__restrict__ prefB, PoolQueue *qh) {
  __shared__ unsigned long long s_item;
  __shared__ int s_go;
  const int g = xcc_id();
  const int a0 = qh->gact[g], a1 = qh->gact[g + 1];
  const int baseA = prefA[a0], baseB = prefB[a0];
  const int nA = prefA[a1] - baseA;
  const unsigned long long per_round = (unsigned long long)(nA + prefB[a1] - baseB);
  const int rounds = qh->rounds;
  const long long wait_ticks = qh->wait_ticks;
  const unsigned long long total = per_round * (unsigned long long)rounds;
  for (;;) {
    __syncthreads();  // the previous item's LDS reads are done
    if (threadIdx.x == 0) s_item = atomicAdd(&qh->head[g], 1ull);
    __syncthreads();
    const unsigned long long item = s_item;
    if (item >= total) break;
    const int round = (int)(item / per_round);
    int j = (int)(item % per_round);
    const bool remap = j >= nA;
    j += remap ? baseB - nA : baseA;  // index into the prefix sums of all active runs
    const int *pref = remap ? prefB : prefA;
    const int q = find_run(pref, a0, a1, j);
    const int tile = j - pref[q];
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
        if (wall_clock64() - t0 > wait_ticks) {
          go = 0;
          atomicAdd(&qh->timeouts, 1u);
          atomicOr(&qh->abort, 1u);
          break;
        }
      }
      acquire_phase();  // see the previous phase's writes
      // a run whose item could not wait is flagged: its state is not trusted
      if (!go) atomicOr(&ctl->status, SALE_FLAG_NUMERIC);
      s_go = go;
    }
    __syncthreads();
    const bool ran = s_go && !ctl->done;
    if (ran) {
      if (pool_calls<R>()) {
        if (!remap)
          lagrange_item_call<R>(&p, tile);
        else
          remap_item_call<R>(&p, tile);
      } else {
        if (!remap)
          lagrange_item<R>(&p, tile);
        else
          remap_item<R>(&p, tile);
      }
    }
    // finish the item: its writes reach the XCD's L2, then it is counted; the
    // last tile of the phase opens the next phase (after a remap phase: the
    // next time step)
    stores_reached_l2();
    __syncthreads();
    if (threadIdx.x == 0) {
      const unsigned int ntiles = (unsigned)(remap ? p.gb.blocks() : p.ga.blocks());
      const unsigned int old = atomicAdd(&ctl->tiles_done, 1u);
      if (old == ntiles - 1u) {
        acquire_phase();  // the step fields as the run's other tiles left them
        atomicExch(&ctl->tiles_done, 0u);
        if (remap && ran) ctl->clk_last = wall_clock64();  // the step just completed
        // the next advance's prepare starts the step after the last round
        if (remap && round + 1 < rounds) pool_begin_step(p.m, ctl, p.step_target);
        stores_reached_l2();
        atomicAdd(&ctl->phase, 1u);
      }
    }
  }
  // the last block to leave flags the runs of every queue that no block
  // served (its XCD received no block of the launch)
  if (threadIdx.x == 0 && atomicAdd(&qh->exited, 1u) == gridDim.x - 1u) {
    for (int h = 0; h < kPoolGroups; h++) {
      const int b0 = qh->gact[h], b1 = qh->gact[h + 1];
      if (b1 == b0) continue;
      const unsigned long long n =
          (unsigned long long)(prefA[b1] - prefA[b0] + prefB[b1] - prefB[b0]) * (unsigned long long)rounds;
      if (__hip_atomic_load(&qh->head[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= n) continue;
      atomicAdd(&qh->starved, 1u);
      for (int r = b0; r < b1; r++) atomicOr(&runs[act[r]].ctl->status, SALE_FLAG_NUMERIC);
    }
  }
}

// one thread per block reports its XCD
__global__ void k_xcc_probe(PoolQueue *qh) {
  if (threadIdx.x == 0) atomicOr(&qh->xcc_mask, 1u << xcc_id());
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
  const int q = find_run(prefA, 0, nact, g);
  const PoolRun<R> &p = runs[act[q]];
  Ctl *ctl = p.ctl;
  if (ctl->done) return;
  const RunArgs<R> a = args_of(p, cur_of(p));
  if (lagrange_tile<R, CH, CW, NT>(a, g - prefA[q], ctl->dt, lds)) atomicOr(&ctl->status, SALE_FLAG_TANGLE);
}

template <typename R>
__global__ __launch_bounds__(NT, waves_of_lock_remap<R>()) void k_lock_remap(const PoolRun<R> *__restrict__ runs,
                                                                            const int *__restrict__ act,
                                                                            const int *__restrict__ prefB, int nact) {
  __shared__ double lds[LDS_R<R>];
  const int g = xcd_logical_block(blockIdx.x, gridDim.x);
  const int q = find_run(prefB, 0, nact, g);
  const PoolRun<R> &p = runs[act[q]];
  Ctl *ctl = p.ctl;
  if (ctl->done) return;
  const RunArgs<R> a = args_of(p, cur_of(p));
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

hipError_t launch_xcc_probe(PoolQueue *qh, hipStream_t s) {
  hipLaunchKernelGGL(k_xcc_probe, dim3(4096), dim3(64), 0, s, qh);
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
