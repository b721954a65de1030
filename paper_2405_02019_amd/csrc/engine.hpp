// engine.hpp -- device buffers of a simulator handle and the launchers of its
// HIP kernels (kernels.hip), as seen by the runtime (runtime.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "snn_internal.hpp"

namespace snn {

// LDS copies of the thalamic tables (thresholds, and per (instance,
// population) offset and length): used when the batch's tables fit.
constexpr uint32_t kThrLds = 8192;
constexpr uint32_t kMetaLds = 512;

// LDS engine: blocks of one launch (one per CU), thalamic table entries its
// LDS copies hold, and sender classes (the populations of the window's
// instance) a window receives from.
constexpr uint32_t kLdsMaxGrid = 256;
// Banded engine, variants of fewer than 1,024 threads: sender ids per step a
// block keeps in device memory of its own after its LDS history (read back
// through its own XCD's L2; the ids past these come from the shared history
// at device scope).
constexpr uint32_t kBandPrivHist = 192;
constexpr uint32_t kLdsTab = 32;
constexpr uint32_t kWinClasses = 8;
// Flag and list slots of the LDS engine: a block publishes step t only after
// every block it reads from has published step t-2, so four slots are never
// overwritten while a reader still needs them.
constexpr uint32_t kSlots = 4;

// One sender class as seen from one target window: senders [first, first + n)
// (global ids) own `cap` record slots each in the window, the first at `base`.
struct WinClass {
  uint64_t base;
  uint32_t first, n, cap, pad;
};

// Small control block in device memory.
struct Control {
  uint64_t t_base;        // first step of the next launch
  uint64_t raster_n;      // raster entries written since the last drain
  uint32_t spk_cnt[2];    // stepwise: senders of step t live in slot t & 1
  uint32_t overflow;      // raster capacity exceeded
  uint32_t error;         // a bounded wait of the persistent kernel expired
  uint64_t barrier;       // persistent kernel: arrivals at the grid barrier
  uint64_t exit_count;    // persistent kernel: blocks that have finished
  uint32_t lcnt[4];       // persistent: segment-list lengths, 3 rotating slots
  uint32_t epoch;         // LDS engine: barriers completed so far (flag epochs)
  uint32_t pad32;
  uint64_t pad[1];
};

// One storage segment of a sender, as published by the persistent engine for
// the transfer phase of the next iteration.
struct SegEntry {
  uint64_t start;         // first record
  uint32_t len;           // records
  uint32_t tbase;         // global id of the segment's target block
};

struct DeviceNet {
  uint32_t n_inst = 0;
  uint32_t nquads = 0;          // all instances, padded
  uint32_t ntot = 0;            // 4 * nquads = ring row stride
  uint32_t nwin_max = 1;
  uint32_t syn_format = SNN_SYN_PLAIN8;
  const InstDev *inst = nullptr;
  const uint32_t *qinfo = nullptr;  // per quad: instance << 24 | local quad
  const uint32_t *thr = nullptr;    // thalamic thresholds of every (instance, population),
                                    // followed by 8 padding entries
  const uint2 *pmeta = nullptr;     // [n_inst * 8]: (first threshold, count)
  uint32_t nthr = 0;                // thresholds without the padding
  uint32_t thr_lds = 0;             // 1: tables fit the kernels' LDS copies
  float *U = nullptr, *I = nullptr;
  uint32_t *R4 = nullptr;           // 4 refractory counters per quad (bytes)
  int32_t *W = nullptr;             // [64][ntot]
  const uint64_t *seg_ptr = nullptr;
  const uint64_t *rec8 = nullptr;
  const uint32_t *rec4 = nullptr;   // LDS engine, compressed: w16 << 16 | delay << 10 | offset
  const uint16_t *rec2 = nullptr;   // LDS engine, deviation format: doubled << 15 | delay << 9 | offset
  const int8_t *dev8 = nullptr;     // and the weight's deviation (steps of InstDev::dev_sq)
  const uint16_t *tgt16 = nullptr;
  const int16_t *w16 = nullptr;
  const uint8_t *d8 = nullptr;
  uint32_t *spk_list = nullptr;     // [2][ntot]
  uint64_t *raster = nullptr;       // (step << 32) | global id
  uint64_t raster_cap = 0;
  int64_t *wave_ctr = nullptr;      // [nquads / 64][4]: spikes, thalamic, consumed, events
  uint64_t *events = nullptr;       // [n_inst]
  DevConsts *consts = nullptr;
  Control *ctl = nullptr;
  SegEntry *seg_list = nullptr;     // persistent: [3][ntot * nwin_max]
  uint32_t lds_window = 0;          // LDS engine: window capacity of the kernel (320, 512), else 0
  uint32_t n_lwin = 0;              // LDS engine: windows of all instances
  const uint4 *lwin = nullptr;      // LDS engine: per window (first neuron, neurons, instance, 0)
  const WinClass *wcls = nullptr;   // LDS engine: [windows][kWinClasses]
  const uint2 *wrel = nullptr;      // LDS engine: per window, the windows [x, y) of its instance
  int64_t *blk_ctr = nullptr;       // LDS engine: [windows][4] spikes, thalamic, consumed, events
  uint2 *lgroup = nullptr;          // LDS engine: per launch group (flag epoch, blocks finished)
  const uint32_t *outdeg = nullptr; // LDS engine: synapses per sender [ntot]
  uint64_t *lflags = nullptr;       // LDS engine: [kSlots][windows] flag words
  uint32_t *llist = nullptr;        // LDS engine: [kSlots][ntot] senders beyond the inline ones
  uint32_t band_h = 0;              // banded engine: ring rows in LDS (64, 16 or 8), else 0
  uint32_t *ghist = nullptr;        // banded engine: [64][ntot] sender ids of each step beyond
                                    // the block's LDS and private history (same values from
                                    // every block)
  uint32_t *phist = nullptr;        // banded engine below 1,024 threads: [blocks][64][kBandPrivHist]
                                    // the block's own sender ids of each step past its LDS
                                    // history
};

struct LaunchShape {
  uint32_t block = 256;
  uint32_t scatter_blocks = 1024;   // stepwise transfer grid
  uint32_t grid = 0;                // persistent grid (blocks)
  uint32_t qpt = 1;                 // quads per thread (persistent)
};

hipError_t launch_propagators(const DeviceNet &d, hipStream_t s);
// Queue `n` steps of the stepwise engine; step k of the launch is
// ctl->t_base + k.  Advances ctl->t_base by n at the end.
hipError_t launch_stepwise(const DeviceNet &d, const LaunchShape &sh, uint32_t n, hipStream_t s);
hipError_t launch_reset_raster(const DeviceNet &d, hipStream_t s);
// Persistent engine: one cooperative launch of sh.grid blocks runs n steps
// (n grid barriers); the device state is canonical again when it returns.
hipError_t launch_persistent(const DeviceNet &d, const LaunchShape &sh, uint32_t n, hipStream_t s);
// Largest co-resident grid of the persistent kernel for a shape, and the
// quad capacity per thread it was compiled for.
int persistent_max_grid(const DeviceNet &d, uint32_t block, uint32_t qpt);
uint32_t persistent_qmax(uint32_t qpt);
// LDS engine: one cooperative launch of group `group` (windows [win0, win0 +
// nwin), whole instances) runs n steps from ctl->t_base; the last of the
// n_groups launches of a chunk advances ctl->t_base.
hipError_t launch_lds(const DeviceNet &d, uint32_t group, uint32_t n_groups, uint32_t win0,
                      uint32_t nwin, uint32_t n, hipStream_t s);
// Co-resident blocks of the LDS kernel with window capacity wn (320 or 512).
int lds_max_grid(uint32_t wn);

// Banded LDS engine (band.hip): kernel variants, each a block size, a window
// capacity (neurons), the ring rows kept in LDS and the sender ids per step
// its LDS history holds.  Variants are ordered by window capacity.
struct BandVariant {
  uint32_t block, wn, h, hc;
};
constexpr uint32_t kNumBandVariants = 4;
extern const BandVariant kBandVariants[kNumBandVariants];
// One cooperative launch of every window (d.n_lwin blocks) runs n steps from
// ctl->t_base and advances it.
hipError_t launch_band(const DeviceNet &d, uint32_t variant, uint32_t n, hipStream_t s);
// Co-resident blocks of a variant (at most one per CU, at most kLdsMaxGrid).
int band_max_grid(uint32_t variant);

}  // namespace snn
