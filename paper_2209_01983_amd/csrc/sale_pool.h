// sale_pool.h -- internal declarations of the pool (many independent runs
// advanced together): run descriptors, queue header, tile shape and the
// launchers of the multi-run kernels. Not part of the ABI.
#pragma once

#include "sale_impl.h"

namespace sale {

// Device-side description of one pool slot.
template <typename R>
struct PoolRun {
  Mesh m;
  Ctl *ctl;
  State<R> s[2];
  R *up, *vp, *wp;
  Geo<R> geo;
  Grid2 ga, gb;
  long long step0;  // step count at admission: state buffer = (step - step0) & 1
  long long step_target;
};

// XCD queues of the persistent advance: every run is served by the blocks
// of one XCD (the ids the hardware reports fit in 4 bits).
constexpr int kPoolGroups = 16;

// Queue header and the active-run tables of one advance.
struct PoolQueue {
  unsigned long long head[kPoolGroups];  // next item of each XCD's queue
  int nact;                              // active runs in this advance
  int rounds;                            // steps per run in this advance
  int totA, totB;                        // Lagrange / remap tiles over all active runs
  int gact[kPoolGroups + 1];             // XCD g serves the runs act[gact[g] .. gact[g+1])
  long long wait_ticks;                  // cap of one wait (100 MHz clock ticks)
  unsigned int timeouts;                 // waits that hit the time cap
  unsigned int abort;                    // set by a timed-out wait: later waits give up at once
  unsigned int exited;                   // blocks that have left the item loop
  unsigned int starved;                  // queues with runs that no block served
  unsigned int xcc_mask;                 // XCD ids seen by the probe
};

// Tile shape of the multi-run kernels: kPoolWidth x kPoolRows columns (their
// meshes are small: narrower tiles than the single-run kernels').
#ifndef SALE_POOL_ROWS
#define SALE_POOL_ROWS 16
#endif
constexpr int kPoolRows = SALE_POOL_ROWS, kPoolWidth = 32;
// Tiles per phase the persistent advance splits the runs' z extents into, in
// proportion to their cells (0: one z segment per tile column); about two per
// resident block. The lockstep advance aims at 3072 blocks per launch.
#ifndef SALE_POOL_PERSISTENT_BLOCKS
#define SALE_POOL_PERSISTENT_BLOCKS 1024
#endif

// Persistent multi-run advance: prepare (queue heads, per-run counters, first
// dt) and the persistent kernel over `blocks` blocks; tables on the device
// (act grouped by XCD as qh->gact says).
template <typename R>
hipError_t launch_pool_advance(PoolRun<R> *runs, const int *act, const int *prefA, const int *prefB,
                               PoolQueue *qh, int nact, int blocks, hipStream_t s);
// Lockstep advance: `rounds` rounds of (begin, Lagrange tiles of all runs,
// remap tiles of all runs, clock stamp), the grids of the run descriptors
// and the prefix sums of their block counts (prefA, prefB, nact + 1 entries)
// describing the launches; `first`: the first of these rounds opens the
// advance (step targets and first clocks are set).
template <typename R>
hipError_t launch_pool_lockstep(const PoolRun<R> *runs, const int *act, const int *prefA, const int *prefB,
                                int nact, int totA, int totB, int rounds, int first, hipStream_t s);
// Blocks of the persistent kernel that fit on the device at once.
template <typename R>
int pool_resident_blocks();
// OR of 1 << (XCD id) over the blocks of a wide launch into qh->xcc_mask
// (which the caller clears first).
hipError_t launch_xcc_probe(PoolQueue *qh, hipStream_t s);

}  // namespace sale
