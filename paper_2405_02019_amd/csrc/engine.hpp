// engine.hpp -- device buffers of a simulator handle and the launchers of its
// HIP kernels (kernels.hip), as seen by the runtime (runtime.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "snn_internal.hpp"

namespace snn {

// Small control block in device memory.
struct Control {
  uint64_t t_base;        // first step of the next launch
  uint64_t raster_n;      // raster entries written since the last drain
  uint32_t spk_cnt[2];    // senders of step t live in slot t & 1
  uint32_t overflow;      // raster capacity exceeded
  uint32_t error;         // a bounded wait of the persistent kernel expired
  uint64_t barrier;       // persistent kernel: arrivals
  uint64_t exit_count;    // persistent kernel: blocks that have left
  uint64_t pad[2];
};

struct DeviceNet {
  uint32_t n_inst = 0;
  uint32_t nquads = 0;          // all instances, padded
  uint32_t ntot = 0;            // 4 * nquads = ring row stride
  uint32_t nwin_max = 1;
  uint32_t syn_format = SNN_SYN_PLAIN8;
  const InstDev *inst = nullptr;
  const uint32_t *qinfo = nullptr;  // per quad: instance << 24 | local quad
  const uint32_t *thr = nullptr;
  float *U = nullptr, *I = nullptr;
  uint32_t *R4 = nullptr;           // 4 refractory counters per quad (bytes)
  int32_t *W = nullptr;             // [64][ntot]
  const uint64_t *seg_ptr = nullptr;
  const uint64_t *rec8 = nullptr;
  const uint16_t *tgt16 = nullptr;
  const int16_t *w16 = nullptr;
  const uint8_t *d8 = nullptr;
  uint32_t *spk_list = nullptr;     // [2][ntot]
  uint64_t *raster = nullptr;       // (step << 32) | global id
  uint64_t raster_cap = 0;
  int64_t *wave_ctr = nullptr;      // [nquads / 64][4]: spikes, thalamic, consumed
  uint64_t *events = nullptr;       // [n_inst]
  DevConsts *consts = nullptr;
  Control *ctl = nullptr;
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

}  // namespace snn
