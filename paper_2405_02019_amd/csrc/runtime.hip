// runtime.hip -- the C ABI of include/snn.h: network upload, device memory
// (caller allocator or hipMalloc), the HIP stream, captured step chunks, raster
// drains and state readback.
#include <algorithm>
#include <cmath>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "engine.hpp"

using namespace snn;

namespace {
thread_local std::string g_build_error;

struct InstMeta {
  uint32_t n = 0, gbase = 0, npad = 0;
  uint32_t win0 = 0, nwin = 0, wlen = 0;   // LDS engine: windows and their length (neurons)
  uint32_t pop_off[9] = {};
  uint64_t nsyn = 0;
  double w_f = 0.0;
  int32_t w_ext_q = 0;
};
}  // namespace

struct snn_net {
  snn_config cfg{};
  std::vector<InstMeta> im;
  DeviceNet d;
  LaunchShape shape;
  uint32_t engine = SNN_ENGINE_STEPWISE;
  uint32_t chunk = 100;
  uint64_t n_real = 0;              // neurons without padding
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<void *> allocs;
  size_t device_bytes = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  std::vector<uint64_t> raster;     // drained; sorted by (step, global id) up to raster_sorted
  uint64_t *staging = nullptr;      // pinned host buffer for raster drains
  uint64_t *raster_alt = nullptr;   // second device raster (engines without a captured graph):
                                    // the step loop swaps to it at a drain and reads the
                                    // other back while the next chunk runs
  size_t staging_cap = 0;           // its capacity in entries
  size_t raster_sorted = 0;         // later drains hold later steps: only the tail needs sorting
  uint64_t raster_version = 0;      // bumped whenever the stored raster changes
  std::vector<uint64_t> by_inst;    // several instances: the sorted raster grouped by instance
  std::vector<size_t> by_inst_off;  // [n_instances + 1] into by_inst
  uint64_t by_inst_version = ~0ull; // raster version by_inst was built from
  uint64_t t = 0;
  uint64_t pending = 0;             // worst-case raster entries since the last drain
  bool overflowed = false;
  bool dead = false;
  std::vector<uint2> lds_groups;    // LDS engine: launches (first window, windows)
  uint32_t band_variant = 0;        // banded engine: kernel variant (kBandVariants)
  int device = 0;                   // the GPU the handle lives on
  std::string err;
  double build_seconds = 0.0;
};

namespace {

int fail(snn_net *h, int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (h)
    h->err = buf;
  else
    g_build_error = buf;
  return code;
}

#define HIP_OK(h, expr)                                                                    \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail((h), SNN_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

int dalloc(snn_net *h, void **p, size_t bytes) {
  bytes = std::max<size_t>(256, (bytes + 255) & ~size_t(255));
  void *q = nullptr;
  if (h->cfg.dev_alloc) {
    q = h->cfg.dev_alloc(bytes, h->cfg.alloc_ctx);
  } else if (hipMalloc(&q, bytes) != hipSuccess) {
    q = nullptr;
  }
  if (!q) return fail(h, SNN_E_NOMEM, "device allocation of %zu bytes failed", bytes);
  h->allocs.push_back(q);
  h->device_bytes += bytes;
  *p = q;
  return SNN_OK;
}

template <class T>
int dalloc_n(snn_net *h, T **p, size_t n) {
  void *q = nullptr;
  int rc = dalloc(h, &q, n * sizeof(T));
  *p = static_cast<T *>(q);
  return rc;
}

void release(snn_net *h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  for (void *p : h->allocs) {
    if (h->cfg.dev_free)
      h->cfg.dev_free(p, h->cfg.alloc_ctx);
    else
      (void)hipFree(p);
  }
  h->allocs.clear();
  if (h->staging) (void)hipHostFree(h->staging);
  h->staging = nullptr;
  h->staging_cap = 0;
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  h->stream = nullptr;
}

// Appends m entries of a device raster buffer to the host store, through a
// pinned buffer (a copy into pageable memory is staged by the runtime in
// small pieces).  The buffer grows to twice what is needed: freeing pinned
// memory waits for the device, which would leave it idle until the next
// chunk is queued.
int store_raster(snn_net *h, const uint64_t *src, uint64_t m) {
  if (m > h->staging_cap) {
    if (h->staging) (void)hipHostFree(h->staging);
    h->staging = nullptr;
    h->staging_cap = 0;
    const size_t cap = std::max<size_t>(2 * m, size_t(1) << 21);
    HIP_OK(h, hipHostMalloc(reinterpret_cast<void **>(&h->staging), cap * sizeof(uint64_t),
                            hipHostMallocDefault));
    h->staging_cap = cap;
  }
  HIP_OK(h, hipMemcpy(h->staging, src, m * sizeof(uint64_t), hipMemcpyDeviceToHost));
  h->raster.insert(h->raster.end(), h->staging, h->staging + m);
  ++h->raster_version;
  return SNN_OK;
}

// Waits for the queued steps and reads the control words: the entries in
// the device raster (*m), a device error, an overflow.
int settle(snn_net *h, uint64_t *m, bool *reset) {
  HIP_OK(h, hipStreamSynchronize(h->stream));
  Control c{};
  HIP_OK(h, hipMemcpy(&c, h->d.ctl, sizeof c, hipMemcpyDeviceToHost));
  if (c.error) {
    h->dead = true;
    return fail(h, SNN_E_DEVICE, "a bounded device wait expired (code %u)", c.error);
  }
  if (c.overflow) h->overflowed = true;
  *m = std::min<uint64_t>(c.raster_n, h->d.raster_cap);
  *reset = c.raster_n || c.overflow;
  return SNN_OK;
}

// Copy the device raster to the host store and reset it.
int drain(snn_net *h) {
  uint64_t m = 0;
  bool reset = false;
  if (int rc = settle(h, &m, &reset)) return rc;
  if (m) {
    if (int rc = store_raster(h, h->d.raster, m)) return rc;
  }
  if (reset) HIP_OK(h, launch_reset_raster(h->d, h->stream));
  h->pending = 0;
  return SNN_OK;
}

// The step loop's drain: the next steps write into the other raster buffer,
// so they can be queued before the full one (*old, *m entries) is read back.
int swap_raster(snn_net *h, const uint64_t **old, uint64_t *m) {
  bool reset = false;
  if (int rc = settle(h, m, &reset)) return rc;
  *old = h->d.raster;
  std::swap(h->d.raster, h->raster_alt);
  if (reset) HIP_OK(h, launch_reset_raster(h->d, h->stream));
  h->pending = 0;
  return SNN_OK;
}

// Sorts raster entries (step << 32 | id) from index `from` on: a counting
// sort by step (the entries of the tail span few steps), then each step's
// handful of ids.
void sort_raster_tail(std::vector<uint64_t> &r, size_t from) {
  const size_t n = r.size() - from;
  if (n < 2) return;
  uint64_t lo = ~0ull, hi = 0;
  for (size_t i = from; i < r.size(); ++i) {
    lo = std::min(lo, r[i] >> 32);
    hi = std::max(hi, r[i] >> 32);
  }
  const uint64_t span = hi - lo + 1;
  if (span > 4 * n + 1024) {   // sparse in time: a comparison sort is cheaper
    std::sort(r.begin() + from, r.end());
    return;
  }
  std::vector<size_t> start(span + 1, 0);
  for (size_t i = from; i < r.size(); ++i) ++start[(r[i] >> 32) - lo + 1];
  for (uint64_t k = 0; k < span; ++k) start[k + 1] += start[k];
  std::vector<uint64_t> out(n);
  for (size_t i = from; i < r.size(); ++i) out[start[(r[i] >> 32) - lo]++] = r[i];
  size_t a = 0;
  for (uint64_t k = 0; k < span; ++k) {   // start[k] is now the end of step lo + k
    std::sort(out.begin() + a, out.begin() + start[k]);
    a = start[k];
  }
  std::copy(out.begin(), out.end(), r.begin() + from);
}

// The LDS engine's raster: a block stages its spikes in (step, id) order and
// flushes them as one contiguous run, and blocks own disjoint windows of ids
// in window order.  Taking the runs window by window (drain order within a
// window), a stable counting sort by step leaves every step's ids ascending
// with no sort within steps.  Returns false where a comparison sort is the
// better choice (entries sparse in time).
bool sort_raster_tail_windows(std::vector<uint64_t> &r, size_t from,
                              const std::vector<InstMeta> &im) {
  const size_t n = r.size() - from;
  if (n < 2) return true;
  uint64_t lo = ~0ull, hi = 0;
  for (size_t i = from; i < r.size(); ++i) {
    lo = std::min(lo, r[i] >> 32);
    hi = std::max(hi, r[i] >> 32);
  }
  const uint64_t span = hi - lo + 1;
  if (span > 4 * n + 1024) return false;
  const uint32_t nwin = im.back().win0 + im.back().nwin;
  auto window_of = [&](uint32_t g) {
    size_t a = 0, b = im.size();   // last instance with gbase <= g
    while (b - a > 1) {
      const size_t c = (a + b) / 2;
      if (im[c].gbase <= g) a = c; else b = c;
    }
    return im[a].win0 + (g - im[a].gbase) / im[a].wlen;
  };
  std::vector<uint32_t> run_at, run_win;   // runs of one window: first entry, window
  uint32_t prev = ~0u;
  for (size_t i = 0; i < n; ++i) {
    const uint32_t w = window_of(uint32_t(r[from + i]));
    if (w != prev) {
      run_at.push_back(uint32_t(i));
      run_win.push_back(w);
      prev = w;
    }
  }
  const size_t nruns = run_at.size();
  run_at.push_back(uint32_t(n));
  std::vector<uint32_t> first(size_t(nwin) + 1, 0), order(nruns);
  for (size_t k = 0; k < nruns; ++k) ++first[run_win[k] + 1];
  for (uint32_t w = 0; w < nwin; ++w) first[w + 1] += first[w];
  for (size_t k = 0; k < nruns; ++k) order[first[run_win[k]]++] = uint32_t(k);
  std::vector<uint32_t> at(span + 1, 0);
  for (size_t i = from; i < r.size(); ++i) ++at[(r[i] >> 32) - lo + 1];
  for (uint64_t k = 0; k < span; ++k) at[k + 1] += at[k];
  std::vector<uint64_t> out(n);
  for (const uint32_t k : order)
    for (uint32_t i = run_at[k]; i < run_at[k + 1]; ++i) {
      const uint64_t v = r[from + i];
      out[at[(v >> 32) - lo]++] = v;
    }
  std::copy(out.begin(), out.end(), r.begin() + from);
  return true;
}

// Orders the raster entries drained since the last call.
void sort_drained(snn_net *h) {
  if (h->raster_sorted >= h->raster.size()) return;
  const bool windows = h->engine == SNN_ENGINE_LDS || h->engine == SNN_ENGINE_BAND;
  if (!windows || !sort_raster_tail_windows(h->raster, h->raster_sorted, h->im))
    sort_raster_tail(h->raster, h->raster_sorted);
  h->raster_sorted = h->raster.size();
  ++h->raster_version;
}

uint64_t spike_bound(const snn_net *h, uint64_t steps) {
  // A neuron spikes at most once per 21 steps (20 refractory steps).
  return h->n_real * ((steps + kRefSteps) / (kRefSteps + 1));
}

// LDS engine plan.  Instance k's nq quads are cut into nwin windows of at
// most L neurons (balanced: every window has ceil(nq / nwin) quads but the
// last); a block owns one window and its 64 ring rows in LDS.  Windows are
// numbered instance by instance, and consecutive instances are launched
// together while their windows fit the co-resident grid (one block per CU).
// Automatic choice: the shortest window (at least 256 neurons) that puts the
// whole network into one launch, else 512-neuron windows in several
// launches.  A requested grid size fixes the number of windows.
struct LdsPlan {
  uint32_t wn = 0;   // kernel window capacity: 320 or 512
  uint32_t total = 0;
  std::vector<uint32_t> nwin, wq;
  std::vector<uint2> groups;
};

uint32_t quads_of(const InstMeta &m) { return (m.n + 3) / 4; }

uint32_t windows_for(uint32_t nq, uint32_t L) { return (nq + L / 4 - 1) / (L / 4); }

// Ls: the window length of each instance.
bool make_plan(const std::vector<InstMeta> &im, const std::vector<uint32_t> &Ls, uint32_t wn,
               uint32_t maxg, LdsPlan &p) {
  p = LdsPlan();
  p.wn = wn;
  uint32_t g0 = 0, gsize = 0;
  for (size_t k = 0; k < im.size(); ++k) {
    const InstMeta &m = im[k];
    const uint32_t L = Ls[k];
    if (L < 4 || L > wn) return false;
    const uint32_t nq = quads_of(m);
    const uint32_t nw0 = windows_for(nq, L);
    if (nw0 == 0) return false;
    const uint32_t wq = (nq + nw0 - 1) / nw0;
    const uint32_t nw = (nq + wq - 1) / wq;   // can be below nw0 after balancing
    if (nw > maxg || 4 * wq > wn) return false;
    p.nwin.push_back(nw);
    p.wq.push_back(wq);
    if (gsize + nw > maxg) {
      p.groups.push_back(make_uint2(g0, gsize));
      g0 += gsize;
      gsize = 0;
    }
    gsize += nw;
    p.total += nw;
  }
  p.groups.push_back(make_uint2(g0, gsize));
  return true;
}

bool make_plan(const std::vector<InstMeta> &im, uint32_t L, uint32_t wn, uint32_t maxg,
               LdsPlan &p) {
  return make_plan(im, std::vector<uint32_t>(im.size(), L), wn, maxg, p);
}

// Window lengths that even out the synaptic events a block delivers per step
// (the destination classes of Sec. 3.6 sized by load): instance k, with w[k]
// events per neuron and step, gets windows of about T / w[k] neurons (at most
// wn, the kernel's capacity; silent instances get wn), for the smallest T
// whose windows fit maxg blocks.  False when even wn-neuron windows do not.
bool balanced_lengths(const std::vector<InstMeta> &im, const std::vector<double> &w, uint32_t wn,
                      uint32_t maxg, std::vector<uint32_t> &L) {
  const size_t n = im.size();
  L.assign(n, wn);
  auto lengths = [&](double T, std::vector<uint32_t> &out) {
    uint64_t total = 0;
    for (size_t k = 0; k < n; ++k) {
      uint32_t l = wn;
      if (w[k] > 0.0 && T / w[k] < double(wn)) l = std::max(4u, uint32_t(T / w[k]) & ~3u);
      out[k] = l;
      total += windows_for(quads_of(im[k]), l);
    }
    return total;
  };
  double wmax = 0.0;
  for (double x : w) wmax = std::max(wmax, x);
  std::vector<uint32_t> tmp(n);
  if (lengths(wmax * wn, L) > maxg) return false;
  if (wmax <= 0.0) return true;
  double lo = 0.0, hi = wmax * wn;
  for (int it = 0; it < 64; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (lengths(mid, tmp) <= maxg) hi = mid; else lo = mid;
  }
  lengths(hi, L);
  return true;
}

int plan_lds(const std::vector<InstMeta> &im, uint32_t block, uint32_t grid, uint32_t want_L,
             const uint32_t *each_L, bool allow_groups, LdsPlan &p, std::string &why) {
  if (block && block != 256) {
    why = "the LDS engine runs 256-thread blocks";
    return SNN_E_INVAL;
  }
  const int g320 = lds_max_grid(320), g512 = lds_max_grid(512);
  if (g320 <= 0 || g512 <= 0) {
    why = "the LDS kernel cannot be made co-resident on this device";
    return SNN_E_RANGE;
  }
  if (each_L) {   // one window length per instance
    const std::vector<uint32_t> Ls(each_L, each_L + im.size());
    const uint32_t Lmax = *std::max_element(Ls.begin(), Ls.end());
    const uint32_t wn = Lmax <= 320 ? 320 : 512;
    const uint32_t maxg = uint32_t(wn == 320 ? g320 : g512);
    if (Lmax <= 512 && make_plan(im, Ls, wn, maxg, p) && p.groups.size() == 1 &&
        (!grid || p.total == grid))
      return SNN_OK;
    why = "the per-instance window lengths do not fit one launch of the LDS engine";
    return SNN_E_RANGE;
  }
  if (want_L) {   // the requested window length
    const uint32_t L = want_L & ~3u;
    const uint32_t wn = L <= 320 ? 320 : 512;
    const uint32_t maxg = uint32_t(wn == 320 ? g320 : g512);
    if (L >= 4 && L <= 512 && make_plan(im, L, wn, maxg, p) && p.groups.size() == 1 &&
        (!grid || p.total == grid))
      return SNN_OK;
    why = "the requested window length does not fit one launch of the LDS engine";
    return SNN_E_RANGE;
  }
  if (grid) {   // exactly `grid` windows in one launch
    for (uint32_t L = 512; L >= 4; L -= 4) {
      const uint32_t wn = L <= 320 ? 320 : 512;
      const uint32_t maxg = uint32_t(wn == 320 ? g320 : g512);
      if (make_plan(im, L, wn, maxg, p) && p.groups.size() == 1 && p.total == grid) return SNN_OK;
    }
    why = "no window length gives the requested number of blocks in one launch";
    return SNN_E_RANGE;
  }
  uint64_t nq = 0;
  for (const InstMeta &m : im) nq += quads_of(m);
  for (uint32_t L = 256; L <= 512; L += 4) {
    const uint32_t wn = L <= 320 ? 320 : 512;
    const uint32_t maxg = uint32_t(wn == 320 ? g320 : g512);
    if (4 * nq > uint64_t(maxg) * L) continue;
    if (make_plan(im, L, wn, maxg, p) && p.groups.size() == 1) return SNN_OK;
  }
  // Networks beyond one co-resident grid: groups of whole instances at
  // 512-neuron windows, launched one after another (only when the LDS engine
  // is requested; the automatic choice prefers the banded engine's single
  // launch).
  if (allow_groups && make_plan(im, 512, 512, uint32_t(g512), p)) return SNN_OK;
  why = "the network needs more windows than one co-resident launch of the LDS engine holds";
  return SNN_E_RANGE;
}

// Banded engine plan: the first kernel variant (by window capacity) and the
// shortest window (at least 256 neurons) that put every instance into one
// co-resident launch; a requested grid size fixes the number of windows.
int plan_band(const std::vector<InstMeta> &im, uint32_t block, uint32_t grid, uint32_t want_L,
              const uint32_t *each_L, LdsPlan &p, uint32_t &variant, std::string &why) {
  uint64_t nq = 0;
  for (const InstMeta &m : im) nq += quads_of(m);
  for (uint32_t v = 0; v < kNumBandVariants; ++v) {
    const BandVariant &bv = kBandVariants[v];
    if (block && block != bv.block) continue;
    const int g = band_max_grid(v);
    if (g <= 0) continue;
    const uint32_t maxg = uint32_t(g);
    if (each_L) {   // one window length per instance, the first variant holding them
      const std::vector<uint32_t> Ls(each_L, each_L + im.size());
      if (make_plan(im, Ls, bv.wn, maxg, p) && p.groups.size() == 1 && (!grid || p.total == grid)) {
        variant = v;
        return SNN_OK;
      }
      continue;
    }
    if (want_L) {   // the requested window length, with the first variant holding it
      const uint32_t L = want_L & ~3u;
      if (L >= 4 && L <= bv.wn && make_plan(im, L, bv.wn, maxg, p) && p.groups.size() == 1 &&
          (!grid || p.total == grid)) {
        variant = v;
        return SNN_OK;
      }
      continue;
    }
    if (grid) {
      for (uint32_t L = bv.wn; L >= 4; L -= 4)
        if (make_plan(im, L, bv.wn, maxg, p) && p.groups.size() == 1 && p.total == grid) {
          variant = v;
          return SNN_OK;
        }
      continue;
    }
    for (uint32_t L = 256; L <= bv.wn; L += 4) {
      if (4 * nq > uint64_t(maxg) * L) continue;
      if (make_plan(im, L, bv.wn, maxg, p) && p.groups.size() == 1) {
        variant = v;
        return SNN_OK;
      }
    }
  }
  why = each_L ? "no banded kernel holds the per-instance window lengths in one launch"
       : grid   ? "no banded kernel gives the requested number of blocks in one launch"
                : "the network needs more windows than one co-resident launch of the banded engine holds";
  return SNN_E_RANGE;
}

// Persistent grid: 4 neurons per quad, `qpt` quads per thread, at most the
// co-resident block count of the kernel.  Fewer blocks make the per-step grid
// barrier cheaper; more threads give the transfer phase more parallelism.
int choose_persistent_shape(snn_net *h, uint32_t block, uint32_t grid) {
  const DeviceNet &d = h->d;
  const uint32_t blocks[] = {256, 128, 512, 1024};
  for (uint32_t b : blocks) {
    if (block && b != block) continue;
    for (uint32_t q : {1u, 2u, 4u, 8u}) {
      const int maxg = persistent_max_grid(d, b, q);
      if (maxg <= 0) continue;
      uint32_t g = grid ? grid : (d.nquads + b * q - 1) / (b * q);
      if (g == 0 || g > uint32_t(maxg)) continue;
      const uint32_t need = (d.nquads + g * b - 1) / (g * b);
      if (need > q) continue;
      h->shape.block = b;
      h->shape.grid = g;
      h->shape.qpt = need ? need : 1;
      return SNN_OK;
    }
  }
  return fail(h, SNN_E_RANGE, "no co-resident persistent grid fits %u neurons", d.ntot);
}

// One chunk of the LDS engine: the launches of every instance group.
hipError_t launch_lds_chunk(snn_net *h, uint32_t n) {
  const uint32_t ng = uint32_t(h->lds_groups.size());
  for (uint32_t g = 0; g < ng; ++g) {
    const uint2 gr = h->lds_groups[g];
    const hipError_t e = launch_lds(h->d, g, ng, gr.x, gr.y, n, h->stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int queue_steps(snn_net *h, uint32_t n) {
  if (h->engine == SNN_ENGINE_BAND) {
    HIP_OK(h, launch_band(h->d, h->band_variant, n, h->stream));
    return SNN_OK;
  }
  if (h->engine == SNN_ENGINE_LDS) {
    HIP_OK(h, launch_lds_chunk(h, n));
    return SNN_OK;
  }
  if (h->engine == SNN_ENGINE_PERSISTENT) {
    HIP_OK(h, launch_persistent(h->d, h->shape, n, h->stream));
    return SNN_OK;
  }
  if (h->graph_exec && n == h->chunk) {
    HIP_OK(h, hipGraphLaunch(h->graph_exec, h->stream));
    return SNN_OK;
  }
  HIP_OK(h, launch_stepwise(h->d, h->shape, n, h->stream));
  return SNN_OK;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free step call: the per-call state of the LDS
// engines (control words, flag epoch, flag words, sender lists, sender
// history beyond the blocks' LDS) in one file-scope device array.  Every GPU
// the library runs on holds its own copy until the process ends; host code
// uses the address hipGetSymbolAddress returns for the current device, never
// the array's name.  Calls that overlap on one GPU share it and race.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(32) << 20;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's scratch (looked up once per device).
int scratch_address(int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(nullptr, SNN_E_INVAL, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(nullptr, SNN_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SNN_OK;
}

// Start of an allocation-free call: the scratch control block takes the
// handle's step origin and clears the rest; flag words and the flag epoch
// start at zero.  A kernel, not a memset, so the call can be captured.
__global__ void k_noalloc_begin(Control *ctl, const Control *own, uint64_t *flags, uint32_t nflags,
                                uint2 *lgroup) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    Control c{};
    c.t_base = own->t_base;
    *ctl = c;
    *lgroup = make_uint2(0, 0);
  }
  for (uint32_t k = i; k < nflags; k += gridDim.x * blockDim.x) flags[k] = 0;
}

// End of an allocation-free call: the handle's step origin advances and the
// caller's status words receive the raster entries written and the error
// code of the bounded waits.
__global__ void k_noalloc_end(Control *own, const Control *ctl, uint64_t *status) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    own->t_base = ctl->t_base;
    status[0] = ctl->raster_n;
    status[1] = uint64_t(ctl->error) | (uint64_t(ctl->overflow) << 32);
  }
}

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

extern "C" {

void snn_instance_default(snn_instance_cfg *c) {
  if (!c) return;
  std::memset(c, 0, sizeof *c);
  c->seed = 1;
  c->scale = 1.0;
  c->indegree_mode = 0;
  c->count_rule = 0;
  c->rows_are_sources = 0;
  c->g = -4.0;
  c->bg_rate_hz = 8.0;
  c->psp_ext_mv = 0.15;
  c->bg_const_T = -1;
  c->conn = nullptr;
}

void snn_config_default(snn_config *c) {
  if (!c) return;
  std::memset(c, 0, sizeof *c);
  c->abi_version = SNN_ABI_VERSION;
  c->n_instances = 1;
  c->inst = nullptr;
  c->syn_format = SNN_SYN_PLAIN8;
  c->engine = SNN_ENGINE_AUTO;
  c->chunk_steps = 100;
  c->use_graphs = 1;
}

const char *snn_last_error(const snn_net *h) {
  return h ? h->err.c_str() : g_build_error.c_str();
}

void snn_destroy(snn_net *h) {
  if (!h) return;
  release(h);
  delete h;
}

int snn_build(const snn_config *cfg, snn_net **out) {
  if (!out) return fail(nullptr, SNN_E_INVAL, "out is NULL");
  *out = nullptr;
  if (!cfg) return fail(nullptr, SNN_E_INVAL, "cfg is NULL");
  if (cfg->abi_version != SNN_ABI_VERSION)
    return fail(nullptr, SNN_E_INVAL, "ABI version %u, library has %u", cfg->abi_version,
                SNN_ABI_VERSION);
  if (cfg->n_instances < 1 || cfg->n_instances > kMaxInstances || !cfg->inst)
    return fail(nullptr, SNN_E_INVAL, "need 1..%u instances", kMaxInstances);
  if (cfg->syn_format > SNN_SYN_DEV8)
    return fail(nullptr, SNN_E_INVAL, "unknown synapse format %u", cfg->syn_format);
  if (cfg->syn_format == SNN_SYN_DEV8 && cfg->engine != SNN_ENGINE_AUTO &&
      cfg->engine != SNN_ENGINE_LDS && cfg->engine != SNN_ENGINE_BAND)
    return fail(nullptr, SNN_E_INVAL, "the deviation format runs on the LDS and banded engines only");
  if (cfg->engine > SNN_ENGINE_BAND)
    return fail(nullptr, SNN_E_INVAL, "unknown engine %u", cfg->engine);
  if (cfg->inst_window_neurons) {
    if (cfg->window_neurons)
      return fail(nullptr, SNN_E_INVAL, "window_neurons and per-instance window lengths are exclusive");
    if (cfg->engine != SNN_ENGINE_LDS && cfg->engine != SNN_ENGINE_BAND)
      return fail(nullptr, SNN_E_INVAL, "per-instance window lengths need the LDS or banded engine");
    for (uint32_t k = 0; k < cfg->n_instances; ++k) {
      const uint32_t L = cfg->inst_window_neurons[k];
      if (L < 4 || L % 4)
        return fail(nullptr, SNN_E_INVAL, "instance %u: window length %u (a positive multiple of 4)", k, L);
    }
  }
  const auto t_start = std::chrono::steady_clock::now();

  snn_net *h = new snn_net();
  h->cfg = *cfg;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return fail(nullptr, SNN_E_HIP, "no current HIP device");
  }
  h->cfg.inst = nullptr;
  h->cfg.inst_window_neurons = nullptr;
  h->chunk = cfg->chunk_steps ? cfg->chunk_steps : 100;
  auto bail = [&](int rc) {
    g_build_error = h->err;
    snn_destroy(h);
    return rc;
  };

  // ---- placement (before sampling: the storage layout depends on it) ----
  const uint32_t ni = cfg->n_instances;
  h->im.resize(ni);
  uint32_t gbase = 0;
  for (uint32_t k = 0; k < ni; ++k) {
    InstMeta &m = h->im[k];
    m.n = instance_neurons(cfg->inst[k]);
    if (m.n == 0 || m.n >= (1u << 26)) {
      fail(h, SNN_E_INVAL, "instance %u: scale %g gives %u neurons", k, cfg->inst[k].scale, m.n);
      return bail(SNN_E_INVAL);
    }
    m.npad = (m.n + kInstAlign - 1) / kInstAlign * kInstAlign;
    m.gbase = gbase;
    if (uint64_t(gbase) + m.npad >= (1ull << 26)) {
      fail(h, SNN_E_RANGE, "more than 2^26 neurons in total");
      return bail(SNN_E_RANGE);
    }
    gbase += m.npad;
  }
  const uint32_t ntot = gbase;

  // ---- engine: the LDS-resident ring needs its whole network in the
  // aggregate LDS (one 512- or 256-neuron window per co-resident block) ----
  // AUTO: the LDS engine when the network's 64-row ring fits the chip's LDS,
  // else the banded engine (fewer ring rows in LDS), else the persistent one.
  h->engine = cfg->engine == SNN_ENGINE_AUTO ? SNN_ENGINE_LDS : cfg->engine;
  uint32_t lds_window = 0;   // LDS or banded engine: kernel window capacity
  LdsPlan plan;
  uint32_t tab = 0;
  for (uint32_t k = 0; k < ni; ++k) tab = std::max(tab, thalamic_table_max(cfg->inst[k]));
  for (int attempt = 0; attempt < 2; ++attempt) {
    if (h->engine != SNN_ENGINE_LDS && h->engine != SNN_ENGINE_BAND) break;
    std::string why;
    int prc = SNN_E_RANGE;
    if (tab > kLdsTab) {
      char b[128];
      std::snprintf(b, sizeof b, "the LDS engines hold thalamic tables of at most %u entries (need %u)",
                    kLdsTab, tab);
      why = b;
    } else if (h->engine == SNN_ENGINE_LDS) {
      prc = plan_lds(h->im, cfg->block_size, cfg->grid_blocks, cfg->window_neurons,
                     cfg->inst_window_neurons, cfg->engine == SNN_ENGINE_LDS, plan, why);
    } else {
      prc = plan_band(h->im, cfg->block_size, cfg->grid_blocks, cfg->window_neurons,
                      cfg->inst_window_neurons, plan, h->band_variant, why);
    }
    if (prc == SNN_OK) {
      lds_window = plan.wn;
      uint32_t w0 = 0;
      for (uint32_t k = 0; k < ni; ++k) {
        h->im[k].win0 = w0;
        h->im[k].nwin = plan.nwin[k];
        h->im[k].wlen = 4 * plan.wq[k];
        w0 += plan.nwin[k];
      }
      h->lds_groups = plan.groups;
      break;
    }
    // The deviation format has no layout for the persistent engine.
    const bool dev_end = cfg->syn_format == SNN_SYN_DEV8 && h->engine == SNN_ENGINE_BAND;
    if (cfg->engine != SNN_ENGINE_AUTO || dev_end) {
      fail(h, prc, "%s%s", dev_end ? "the deviation format needs the LDS or banded engine: " : "",
           why.c_str());
      return bail(prc);
    }
    h->engine = h->engine == SNN_ENGINE_LDS ? SNN_ENGINE_BAND : SNN_ENGINE_PERSISTENT;
    if (h->engine == SNN_ENGINE_PERSISTENT) break;
  }
  if (!lds_window && (h->engine == SNN_ENGINE_LDS || h->engine == SNN_ENGINE_BAND))
    h->engine = SNN_ENGINE_PERSISTENT;
  const bool banded = h->engine == SNN_ENGINE_BAND;
  const uint32_t band_h = banded ? kBandVariants[h->band_variant].h : 0u;
  const uint32_t nband = banded ? band_count(band_h) : 1u;

  // ---- sample every instance on the host ----
  std::vector<HostInstance> hi(ni);
  uint32_t nwin_max = 1;
  uint64_t nseg_tot = 0, nrec_tot = 0, nthr = 0;
  for (uint32_t k = 0; k < ni; ++k) {
    InstMeta &m = h->im[k];
    uint32_t wsize = kNoWindows, worigin = 0;
    if (lds_window) {
      wsize = m.wlen;
    } else if (cfg->syn_format == SNN_SYN_COMPRESSED5) {
      wsize = 1u << kTargetBlockBits;
    }
    std::string e;
    int rc = banded ? sample_instance_banded(cfg->inst[k], cfg->syn_format, wsize, band_h,
                                             cfg->host_threads, hi[k], e)
                    : sample_instance(cfg->inst[k], cfg->syn_format, wsize, worigin, lds_window != 0,
                                      cfg->host_threads, hi[k], e);
    if (rc) {
      fail(h, rc, "instance %u: %s", k, e.c_str());
      return bail(rc);
    }
    if (lds_window && hi[k].nwin != m.nwin) {
      fail(h, SNN_E_RANGE, "instance %u: %u windows sampled, %u planned", k, hi[k].nwin, m.nwin);
      return bail(SNN_E_RANGE);
    }
    std::memcpy(m.pop_off, hi[k].pop_off, sizeof m.pop_off);
    m.nsyn = hi[k].nsyn;
    m.w_f = hi[k].w_f;
    m.w_ext_q = hi[k].w_ext_q;
    nwin_max = std::max(nwin_max, hi[k].nwin);
    if (!hi[k].padded) nseg_tot += uint64_t(m.n) * hi[k].nwin;
    nrec_tot += hi[k].nrec;
    for (int p = 0; p < 8; ++p) nthr += hi[k].thr_len[p];
    h->n_real += m.n;
  }
  DeviceNet &d = h->d;
  d.n_inst = ni;
  d.ntot = ntot;
  d.nquads = ntot / 4;
  d.lds_window = lds_window;
  d.band_h = band_h;
  d.n_lwin = plan.total;
  d.nwin_max = nwin_max;
  d.syn_format = cfg->syn_format;

  // ---- stream ----
  if (cfg->hip_stream) {
    h->stream = static_cast<hipStream_t>(cfg->hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) {
      fail(h, SNN_E_HIP, "hipStreamCreate failed");
      return bail(SNN_E_HIP);
    }
    h->own_stream = true;
  }

  // ---- device memory ----
  InstDev *d_inst;
  uint32_t *d_qinfo, *d_thr;
  uint2 *d_pmeta;
  uint64_t *d_seg, *d_rec8 = nullptr;
  uint16_t *d_tgt16 = nullptr;
  uint32_t *d_rec4 = nullptr;
  int16_t *d_w16 = nullptr;
  uint8_t *d_d8 = nullptr;
  uint16_t *d_rec2 = nullptr;
  int8_t *d_dev8 = nullptr;
  const bool comp = cfg->syn_format == SNN_SYN_COMPRESSED5;
  const bool devf = cfg->syn_format == SNN_SYN_DEV8;
  uint64_t cap = cfg->raster_capacity;
  // Default: room for the worst case of about 20,000 steps (a neuron spikes
  // at most every 21 steps), so that drains -- a stream synchronisation each
  // -- are rare; at most 2^30 entries.
  if (!cap)
    cap = std::min<uint64_t>(uint64_t(1) << 30,
                             std::max<uint64_t>(uint64_t(1) << 20, uint64_t(1024) * d.ntot));
  cap = std::max<uint64_t>(cap, 2 * h->n_real + 64);
  d.raster_cap = cap;
  int rc = SNN_OK;
#define ALLOC(ptr, n)                           \
  do {                                          \
    rc = dalloc_n(h, &(ptr), (n));              \
    if (rc) return bail(rc);                    \
  } while (0)
  ALLOC(d_inst, ni);
  ALLOC(d_qinfo, d.nquads);
  ALLOC(d_thr, nthr + 8);
  ALLOC(d_pmeta, size_t(ni) * 8);
  ALLOC(d.U, d.ntot);
  ALLOC(d.I, d.ntot);
  ALLOC(d.R4, d.nquads);
  ALLOC(d.W, size_t(kRing) * d.ntot);
  ALLOC(d_seg, nseg_tot + 1);
  if (devf) {
    ALLOC(d_rec2, std::max<uint64_t>(1, nrec_tot));
    ALLOC(d_dev8, std::max<uint64_t>(1, nrec_tot));
  } else if (comp && lds_window) {
    ALLOC(d_rec4, std::max<uint64_t>(1, nrec_tot));
  } else if (comp) {
    ALLOC(d_tgt16, std::max<uint64_t>(1, nrec_tot));
    ALLOC(d_w16, std::max<uint64_t>(1, nrec_tot));
    ALLOC(d_d8, std::max<uint64_t>(1, nrec_tot));
  } else {
    ALLOC(d_rec8, std::max<uint64_t>(1, nrec_tot));
  }
  ALLOC(d.spk_list, 2 * size_t(d.ntot));
  ALLOC(d.raster, cap);
  // A captured graph holds the raster's address: only the other engines swap.
  if (!(cfg->use_graphs && h->engine == SNN_ENGINE_STEPWISE)) ALLOC(h->raster_alt, cap);
  ALLOC(d.wave_ctr, 4 * size_t(d.nquads / 64));
  ALLOC(d.events, ni);
  ALLOC(d.consts, 1);
  ALLOC(d.ctl, 1);
  if (h->engine == SNN_ENGINE_PERSISTENT) ALLOC(d.seg_list, 3 * size_t(d.ntot) * nwin_max);
  const uint32_t nwin_lds = lds_window ? plan.total : 0;
  WinClass *d_wcls = nullptr;
  uint2 *d_wrel = nullptr;
  uint4 *d_lwin = nullptr;
  uint32_t *d_outdeg = nullptr;
  if (banded) {
    ALLOC(d.ghist, size_t(64) * d.ntot);
    if (kBandVariants[h->band_variant].block < 1024)
      ALLOC(d.phist, size_t(nwin_lds) * 64 * kBandPrivHist);
  }
  if (lds_window) {
    ALLOC(d_wcls, size_t(nwin_lds) * nband * kWinClasses);
    ALLOC(d_wrel, nwin_lds);
    ALLOC(d_lwin, nwin_lds);
    ALLOC(d_outdeg, d.ntot);
    ALLOC(d.lflags, kSlots * size_t(nwin_lds));
    ALLOC(d.llist, kSlots * size_t(d.ntot));
    ALLOC(d.blk_ctr, 4 * size_t(nwin_lds));
    ALLOC(d.lgroup, plan.groups.size());
  }
#undef ALLOC

  // ---- host staging and upload ----
  std::vector<InstDev> hinst(ni);
  std::vector<uint32_t> qinfo(d.nquads, 0);
  std::vector<uint32_t> thr;
  std::vector<uint2> pmeta(size_t(ni) * 8);
  std::vector<float> u0(d.ntot, 0.0f);
  std::vector<uint64_t> seg;
  seg.reserve(nseg_tot + 1);
  uint64_t syn_base = 0;
  for (uint32_t k = 0; k < ni; ++k) {
    const HostInstance &x = hi[k];
    const InstMeta &m = h->im[k];
    InstDev &v = hinst[k];
    std::memset(&v, 0, sizeof v);
    v.seed = x.cfg.seed;
    v.gbase = m.gbase;
    v.n = m.n;
    v.npad = m.npad;
    v.w_ext_q = x.w_ext_q;
    std::memcpy(v.pop_off, x.pop_off, sizeof v.pop_off);
    for (int p = 0; p < 8; ++p) {
      v.thr_off[p] = uint32_t(thr.size());
      v.thr_len[p] = x.thr_len[p];
      pmeta[size_t(k) * 8 + p] = make_uint2(v.thr_off[p], v.thr_len[p]);
      thr.insert(thr.end(), x.thr[p], x.thr[p] + x.thr_len[p]);
    }
    v.seg_base = uint32_t(seg.size());
    v.nwin = x.nwin;
    v.win_first = x.win_first;
    v.win_size = x.win_size;
    v.tbase0 = uint32_t(uint64_t(m.gbase) + uint64_t(x.win_first) * x.win_size - x.win_origin);
    std::memcpy(v.dev_mq, x.dev_mq, sizeof v.dev_mq);
    std::memcpy(v.dev_sq, x.dev_sq, sizeof v.dev_sq);
    for (uint32_t lq = 0; lq < m.npad / 4; ++lq) qinfo[m.gbase / 4 + lq] = (k << 24) | lq;
    std::copy(x.u0.begin(), x.u0.end(), u0.begin() + m.gbase);
    for (uint64_t s = 0; s + 1 < x.seg_ptr.size(); ++s) seg.push_back(syn_base + x.seg_ptr[s]);
    syn_base += x.nrec;
  }
  seg.push_back(syn_base);
  thr.resize(thr.size() + 8, 0xFFFFFFFFu);  // padding read by the 8-wide table scan
  if (seg.size() >= (uint64_t(1) << 32)) {
    fail(h, SNN_E_RANGE, "too many storage segments");
    return bail(SNN_E_RANGE);
  }
#define UPLOAD(dst, src, bytes)                                                     \
  do {                                                                              \
    if (bytes) {                                                                    \
      const hipError_t ue = hipMemcpy((dst), (src), (bytes), hipMemcpyHostToDevice); \
      if (ue != hipSuccess) {                                                       \
        fail(h, SNN_E_HIP, "upload of %s failed: %s", #src, hipGetErrorString(ue)); \
        return bail(SNN_E_HIP);                                                     \
      }                                                                             \
    }                                                                               \
  } while (0)
  UPLOAD(d_inst, hinst.data(), ni * sizeof(InstDev));
  UPLOAD(d_qinfo, qinfo.data(), qinfo.size() * sizeof(uint32_t));
  UPLOAD(d_thr, thr.data(), thr.size() * sizeof(uint32_t));
  UPLOAD(d_pmeta, pmeta.data(), pmeta.size() * sizeof(uint2));
  UPLOAD(d.U, u0.data(), u0.size() * sizeof(float));
  UPLOAD(d_seg, seg.data(), seg.size() * sizeof(uint64_t));
  if (lds_window) {
    // Per window: its neurons, the sender classes of its instance, and the
    // windows of that instance (the only ones whose senders reach it).
    std::vector<WinClass> wcls(size_t(nwin_lds) * nband * kWinClasses);
    std::vector<uint2> wrel(nwin_lds);
    std::vector<uint4> lwin(nwin_lds);
    std::vector<uint32_t> outdeg(d.ntot, 0);
    uint64_t rb = 0;
    for (uint32_t k = 0; k < ni; ++k) {
      const HostInstance &x = hi[k];
      const InstMeta &m = h->im[k];
      const uint32_t span = 4 * quads_of(m);
      for (uint32_t w = 0; w < m.nwin; ++w) {
        const uint32_t gw = m.win0 + w;
        const uint32_t first = w * m.wlen;
        lwin[gw] = make_uint4(m.gbase + first, std::min(m.wlen, span - first), k, 0);
        wrel[gw] = make_uint2(m.win0, m.win0 + m.nwin);
        // [window][band][class]; the LDS engine has one band.
        for (uint32_t b = 0; b < nband; ++b)
          for (int c = 0; c < 8; ++c) {
            const size_t src = (size_t(w) * nband + b) * 8 + c;
            WinClass &e = wcls[(size_t(gw) * nband + b) * kWinClasses + c];
            e.base = rb + x.cls_base[src];
            e.first = m.gbase + x.pop_off[c];
            e.n = x.pop_off[c + 1] - x.pop_off[c];
            e.cap = x.cls_cap[src];
          }
      }
      std::copy(x.outdeg.begin(), x.outdeg.end(), outdeg.begin() + m.gbase);
      rb += x.nrec;
    }
    UPLOAD(d_wcls, wcls.data(), wcls.size() * sizeof(WinClass));
    UPLOAD(d_wrel, wrel.data(), wrel.size() * sizeof(uint2));
    UPLOAD(d_lwin, lwin.data(), lwin.size() * sizeof(uint4));
    UPLOAD(d_outdeg, outdeg.data(), outdeg.size() * sizeof(uint32_t));
  }
  syn_base = 0;
  for (uint32_t k = 0; k < ni; ++k) {
    HostInstance &x = hi[k];
    if (devf) {
      UPLOAD(d_rec2 + syn_base, x.rec2.data(), x.nrec * sizeof(uint16_t));
      UPLOAD(d_dev8 + syn_base, x.dev8.data(), x.nrec * sizeof(int8_t));
    } else if (comp && lds_window) {
      UPLOAD(d_rec4 + syn_base, x.rec4.data(), x.nrec * sizeof(uint32_t));
    } else if (comp) {
      UPLOAD(d_tgt16 + syn_base, x.tgt16.data(), x.nrec * sizeof(uint16_t));
      UPLOAD(d_w16 + syn_base, x.w16.data(), x.nrec * sizeof(int16_t));
      UPLOAD(d_d8 + syn_base, x.d8.data(), x.nrec * sizeof(uint8_t));
    } else {
      if (h->im[k].gbase) {  // targets become global ids
        const uint64_t add = uint64_t(h->im[k].gbase) << 38;
        for (auto &r : x.rec8) r += add;
      }
      UPLOAD(d_rec8 + syn_base, x.rec8.data(), x.nrec * sizeof(uint64_t));
    }
    syn_base += x.nrec;
    x = HostInstance();  // release host copies early
  }
#undef UPLOAD
  d.inst = d_inst;
  d.qinfo = d_qinfo;
  d.thr = d_thr;
  d.pmeta = d_pmeta;
  d.nthr = uint32_t(nthr);
  d.thr_lds = (nthr <= kThrLds && size_t(ni) * 8 <= kMetaLds) ? 1u : 0u;
  d.seg_ptr = d_seg;
  d.rec8 = d_rec8;
  d.rec4 = d_rec4;
  d.rec2 = d_rec2;
  d.dev8 = d_dev8;
  d.tgt16 = d_tgt16;
  d.w16 = d_w16;
  d.d8 = d_d8;
  d.wcls = d_wcls;
  d.wrel = d_wrel;
  d.lwin = d_lwin;
  d.outdeg = d_outdeg;
  if (hipMemset(d.I, 0, d.ntot * sizeof(float)) != hipSuccess ||
      hipMemset(d.R4, 0, d.nquads * sizeof(uint32_t)) != hipSuccess ||
      hipMemset(d.W, 0, size_t(kRing) * d.ntot * sizeof(int32_t)) != hipSuccess ||
      hipMemset(d.spk_list, 0, 2 * size_t(d.ntot) * sizeof(uint32_t)) != hipSuccess ||
      hipMemset(d.wave_ctr, 0, 4 * size_t(d.nquads / 64) * sizeof(int64_t)) != hipSuccess ||
      hipMemset(d.events, 0, ni * sizeof(uint64_t)) != hipSuccess ||
      hipMemset(d.ctl, 0, sizeof(Control)) != hipSuccess ||
      (d.lflags && hipMemset(d.lflags, 0, kSlots * size_t(nwin_lds) * sizeof(uint64_t)) != hipSuccess) ||
      (d.blk_ctr && hipMemset(d.blk_ctr, 0, 4 * size_t(nwin_lds) * sizeof(int64_t)) != hipSuccess) ||
      (d.lgroup && hipMemset(d.lgroup, 0, plan.groups.size() * sizeof(uint2)) != hipSuccess) ||
      (d.ghist && hipMemset(d.ghist, 0, size_t(64) * d.ntot * sizeof(uint32_t)) != hipSuccess)) {
    fail(h, SNN_E_HIP, "device memset failed");
    return bail(SNN_E_HIP);
  }
  if (launch_propagators(d, h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess) {
    fail(h, SNN_E_HIP, "propagator kernel failed");
    return bail(SNN_E_HIP);
  }

  // ---- engine ----
  h->shape.block = 256;
  h->shape.scatter_blocks = 1024;
  if (h->engine == SNN_ENGINE_LDS || h->engine == SNN_ENGINE_BAND) {
    h->shape.block = banded ? kBandVariants[h->band_variant].block : 256;
    h->shape.grid = plan.total;
    h->shape.qpt = 1;
  } else if (h->engine == SNN_ENGINE_PERSISTENT) {
    int rc2 = choose_persistent_shape(h, cfg->block_size, cfg->grid_blocks);
    if (rc2 != SNN_OK) {
      if (cfg->engine == SNN_ENGINE_PERSISTENT) return bail(rc2);
      h->engine = SNN_ENGINE_STEPWISE;
    }
  }
  if (h->engine == SNN_ENGINE_STEPWISE) {
    if (cfg->block_size && cfg->block_size != 256) {
      fail(h, SNN_E_INVAL, "the stepwise engine runs 256-thread blocks");
      return bail(SNN_E_INVAL);
    }
    if (cfg->grid_blocks) h->shape.scatter_blocks = cfg->grid_blocks;
  }
  // The LDS engine launches its chunks directly: a captured kernel node does
  // not carry the cooperative launch's co-residency guarantee.
  if (cfg->use_graphs && h->engine == SNN_ENGINE_STEPWISE) {
    if (hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      fail(h, SNN_E_HIP, "stream capture failed to start");
      return bail(SNN_E_HIP);
    }
    hipError_t le = launch_stepwise(d, h->shape, h->chunk, h->stream);
    hipError_t ce = hipStreamEndCapture(h->stream, &h->graph);
    if (le != hipSuccess || ce != hipSuccess ||
        hipGraphInstantiate(&h->graph_exec, h->graph, nullptr, nullptr, 0) != hipSuccess) {
      fail(h, SNN_E_HIP, "graph capture of a %u-step chunk failed", h->chunk);
      return bail(SNN_E_HIP);
    }
  }
  h->build_seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  *out = h;
  return SNN_OK;
}

int snn_step_n(snn_net *h, uint64_t n_steps) {
  if (!h) return fail(nullptr, SNN_E_INVAL, "handle is NULL");
  if (h->dead) return fail(h, SNN_E_DEVICE, "the handle is unusable after a device failure");
  while (n_steps) {
    uint64_t piece = std::min<uint64_t>(n_steps, h->chunk);
    while (piece > 1 && spike_bound(h, piece) > h->d.raster_cap) piece /= 2;
    const uint64_t *old = nullptr;
    uint64_t m_old = 0;
    if (h->pending + spike_bound(h, piece) > h->d.raster_cap) {
      int rc = h->raster_alt ? swap_raster(h, &old, &m_old) : drain(h);
      if (rc) return rc;
    }
    int rc = queue_steps(h, uint32_t(piece));
    // The full buffer is read back while the device runs the chunk just
    // queued (it is not written again before the next drain).
    if (m_old) {
      const int rs = store_raster(h, old, m_old);
      if (!rc) rc = rs;
    }
    if (rc) return rc;
    h->pending += spike_bound(h, piece);
    h->t += piece;
    n_steps -= piece;
    sort_drained(h);   // while the device runs the chunk just queued
  }
  return SNN_OK;
}

int snn_step_n_noalloc(snn_net *h, uint64_t n_steps, uint64_t *d_raster, uint64_t raster_cap,
                       uint64_t *d_status) {
  if (!h) return fail(nullptr, SNN_E_INVAL, "handle is NULL");
  if (h->dead) return fail(h, SNN_E_DEVICE, "the handle is unusable after a device failure");
  if (h->engine != SNN_ENGINE_LDS && h->engine != SNN_ENGINE_BAND)
    return fail(h, SNN_E_INVAL, "the allocation-free call runs the LDS and banded engines only");
  if (h->lds_groups.size() != 1) return fail(h, SNN_E_INVAL, "one launch per chunk is required");
  if (!d_raster || !d_status) return fail(h, SNN_E_INVAL, "NULL raster or status");
  if (n_steps == 0) return SNN_OK;
  if (spike_bound(h, n_steps) > raster_cap)
    return fail(h, SNN_E_RANGE, "%llu steps may emit %llu spikes, the raster holds %llu",
                (unsigned long long)n_steps, (unsigned long long)spike_bound(h, n_steps),
                (unsigned long long)raster_cap);
  int dev = -1;
  HIP_OK(h, hipGetDevice(&dev));
  if (dev != h->device) return fail(h, SNN_E_INVAL, "the handle's device %d is not current", h->device);
  const DeviceNet &d = h->d;
  const size_t nflags = size_t(kSlots) * d.n_lwin;
  const size_t b_ctl = round256(sizeof(Control)), b_grp = 256, b_flags = round256(nflags * 8),
               b_list = round256(size_t(kSlots) * d.ntot * 4),
               b_hist = d.ghist ? round256(size_t(64) * d.ntot * 4) : 0,
               b_phist = d.phist ? round256(size_t(d.n_lwin) * 64 * kBandPrivHist * 4) : 0;
  const size_t need = b_ctl + b_grp + b_flags + b_list + b_hist + b_phist;
  if (need > kScratchBytes)
    return fail(h, SNN_E_RANGE, "the network needs %zu bytes of scratch, the static area holds %zu",
                need, kScratchBytes);
  void *base = nullptr;
  const int rc = scratch_address(dev, &base);
  if (rc) return fail(h, rc, "%s", snn_last_error(nullptr));
  unsigned char *p = static_cast<unsigned char *>(base);
  DeviceNet dv = d;
  dv.ctl = reinterpret_cast<Control *>(p);
  dv.lgroup = reinterpret_cast<uint2 *>(p + b_ctl);
  dv.lflags = reinterpret_cast<uint64_t *>(p + b_ctl + b_grp);
  dv.llist = reinterpret_cast<uint32_t *>(p + b_ctl + b_grp + b_flags);
  dv.ghist = d.ghist ? reinterpret_cast<uint32_t *>(p + b_ctl + b_grp + b_flags + b_list) : nullptr;
  dv.phist = d.phist ? reinterpret_cast<uint32_t *>(p + b_ctl + b_grp + b_flags + b_list + b_hist)
                     : nullptr;
  dv.raster = d_raster;
  dv.raster_cap = raster_cap;
  hipLaunchKernelGGL(k_noalloc_begin, dim3(1), dim3(256), 0, h->stream, dv.ctl, d.ctl, dv.lflags,
                     uint32_t(nflags), dv.lgroup);
  HIP_OK(h, hipGetLastError());
  for (uint64_t left = n_steps; left;) {
    const uint32_t piece = uint32_t(std::min<uint64_t>(left, h->chunk));
    if (h->engine == SNN_ENGINE_BAND) {
      HIP_OK(h, launch_band(dv, h->band_variant, piece, h->stream));
    } else {
      const uint2 gr = h->lds_groups[0];
      HIP_OK(h, launch_lds(dv, 0, 1, gr.x, gr.y, piece, h->stream));
    }
    left -= piece;
  }
  hipLaunchKernelGGL(k_noalloc_end, dim3(1), dim3(64), 0, h->stream, d.ctl, dv.ctl, d_status);
  HIP_OK(h, hipGetLastError());
  h->t += n_steps;
  return SNN_OK;
}

int snn_read_spikes(snn_net *h, uint32_t inst, uint64_t t0, uint64_t t1, uint32_t *steps,
                    uint32_t *ids, uint64_t cap, uint64_t *n_out) {
  if (!h || !n_out) return fail(h, SNN_E_INVAL, "NULL argument");
  if (inst >= h->im.size()) return fail(h, SNN_E_INVAL, "instance %u out of range", inst);
  int rc = drain(h);
  if (rc) return rc;
  if (h->overflowed) return fail(h, SNN_E_OVERFLOW, "the device raster overflowed");
  const InstMeta &m = h->im[inst];
  t0 = std::min<uint64_t>(t0, 0xFFFFFFFFull);
  t1 = std::min<uint64_t>(t1, 0x100000000ull);
  sort_drained(h);
  // The entries of one instance, sorted by (step, id): the whole raster for
  // one instance, else its part of the raster grouped by instance (built
  // once per raster version by a stable counting sort on the instance).
  const uint64_t *first = h->raster.data(), *last = h->raster.data() + h->raster.size();
  if (h->im.size() > 1) {
    if (h->by_inst_version != h->raster_version) {
      const size_t ni = h->im.size();
      std::vector<uint32_t> which(h->raster.size());
      h->by_inst_off.assign(ni + 1, 0);
      for (size_t i = 0; i < h->raster.size(); ++i) {
        const uint32_t g = uint32_t(h->raster[i]);
        size_t a = 0, b = ni;   // last instance with gbase <= g
        while (b - a > 1) {
          const size_t c = (a + b) / 2;
          if (h->im[c].gbase <= g) a = c; else b = c;
        }
        which[i] = uint32_t(a);
        ++h->by_inst_off[a + 1];
      }
      for (size_t k = 0; k < ni; ++k) h->by_inst_off[k + 1] += h->by_inst_off[k];
      std::vector<size_t> at(h->by_inst_off.begin(), h->by_inst_off.end() - 1);
      h->by_inst.resize(h->raster.size());
      for (size_t i = 0; i < h->raster.size(); ++i) h->by_inst[at[which[i]]++] = h->raster[i];
      h->by_inst_version = h->raster_version;
    }
    first = h->by_inst.data() + h->by_inst_off[inst];
    last = h->by_inst.data() + h->by_inst_off[inst + 1];
  }
  const uint64_t *lo = std::lower_bound(first, last, t0 << 32);
  const uint64_t *hi = t1 >= 0x100000000ull ? last : std::lower_bound(first, last, t1 << 32);
  const uint64_t cnt = uint64_t(hi - lo);
  *n_out = cnt;
  if (!steps && !ids) return SNN_OK;
  if (cnt > cap) return fail(h, SNN_E_RANGE, "%llu spikes, buffer holds %llu",
                             (unsigned long long)cnt, (unsigned long long)cap);
  uint64_t k = 0;
  for (const uint64_t *it = lo; it < hi; ++it, ++k) {
    if (steps) steps[k] = uint32_t(*it >> 32);
    if (ids) ids[k] = uint32_t(*it) - m.gbase;
  }
  return SNN_OK;
}

int snn_discard_spikes(snn_net *h, uint64_t t_before) {
  if (!h) return fail(nullptr, SNN_E_INVAL, "handle is NULL");
  int rc = drain(h);
  if (rc) return rc;
  sort_drained(h);
  const uint64_t key = std::min<uint64_t>(t_before, 0x100000000ull);
  auto end = key >= 0x100000000ull ? h->raster.end()
                                   : std::lower_bound(h->raster.begin(), h->raster.end(), key << 32);
  const size_t n = size_t(end - h->raster.begin());
  h->raster.erase(h->raster.begin(), end);
  h->raster_sorted -= std::min(h->raster_sorted, n);
  ++h->raster_version;
  if (h->raster.capacity() > 4 * h->raster.size() + (size_t(1) << 20)) h->raster.shrink_to_fit();
  return SNN_OK;
}

int snn_read_state(snn_net *h, uint32_t inst, snn_state *out) {
  if (!h || !out) return fail(h, SNN_E_INVAL, "NULL argument");
  if (inst >= h->im.size()) return fail(h, SNN_E_INVAL, "instance %u out of range", inst);
  HIP_OK(h, hipStreamSynchronize(h->stream));
  const InstMeta &m = h->im[inst];
  const DeviceNet &d = h->d;
  if (out->U) HIP_OK(h, hipMemcpy(out->U, d.U + m.gbase, m.n * sizeof(float), hipMemcpyDeviceToHost));
  if (out->I) HIP_OK(h, hipMemcpy(out->I, d.I + m.gbase, m.n * sizeof(float), hipMemcpyDeviceToHost));
  if (out->R) {
    std::vector<uint32_t> r4(m.npad / 4);
    HIP_OK(h, hipMemcpy(r4.data(), d.R4 + m.gbase / 4, r4.size() * sizeof(uint32_t),
                        hipMemcpyDeviceToHost));
    for (uint32_t i = 0; i < m.n; ++i) out->R[i] = int32_t((r4[i / 4] >> (8 * (i % 4))) & 0xFFu);
  }
  if (out->W) {
    HIP_OK(h, hipMemcpy2D(out->W, m.n * sizeof(int32_t), d.W + m.gbase, size_t(d.ntot) * sizeof(int32_t),
                          m.n * sizeof(int32_t), kRing, hipMemcpyDeviceToHost));
  }
  std::vector<int64_t> wc(4 * size_t(m.npad / 256));
  HIP_OK(h, hipMemcpy(wc.data(), d.wave_ctr + 4 * size_t(m.gbase / 256), wc.size() * sizeof(int64_t),
                      hipMemcpyDeviceToHost));
  int64_t sp = 0, po = 0, co = 0, ev_slots = 0;
  for (size_t w = 0; w < wc.size() / 4; ++w) {
    sp += wc[4 * w];
    po += wc[4 * w + 1];
    co += wc[4 * w + 2];
    ev_slots += wc[4 * w + 3];
  }
  if (d.blk_ctr && m.nwin) {   // LDS engine: one counter set per window
    std::vector<int64_t> bc(4 * size_t(m.nwin));
    HIP_OK(h, hipMemcpy(bc.data(), d.blk_ctr + 4 * size_t(m.win0), bc.size() * sizeof(int64_t),
                        hipMemcpyDeviceToHost));
    for (size_t w = 0; w < m.nwin; ++w) {
      sp += bc[4 * w];
      po += bc[4 * w + 1];
      co += bc[4 * w + 2];
      ev_slots += bc[4 * w + 3];
    }
  }
  uint64_t ev = 0;
  HIP_OK(h, hipMemcpy(&ev, d.events + inst, sizeof ev, hipMemcpyDeviceToHost));
  ev += uint64_t(ev_slots);
  DevConsts kc{};
  HIP_OK(h, hipMemcpy(&kc, d.consts, sizeof kc, hipMemcpyDeviceToHost));
  out->t = h->t;
  out->n_neurons = m.n;
  out->n_synapses = m.nsyn;
  out->spikes = uint64_t(sp);
  out->events = ev;
  out->poisson = uint64_t(po);
  out->consumed = co;
  out->p11 = kc.p11;
  out->p21 = kc.p21;
  out->p22 = kc.p22;
  out->w_ext_q = m.w_ext_q;
  out->w_f = m.w_f;
  return SNN_OK;
}

int snn_get_info(const snn_net *h, snn_info *out) {
  if (!h || !out) return SNN_E_INVAL;
  std::memset(out, 0, sizeof *out);
  out->engine = h->engine;
  out->block_size = h->shape.block;
  out->grid_blocks = h->engine == SNN_ENGINE_STEPWISE ? h->shape.scatter_blocks : h->shape.grid;
  out->quads_per_thread = h->shape.qpt;
  out->chunk_steps = h->chunk;
  out->n_neurons_total = h->d.ntot;
  uint64_t s = 0;
  for (const auto &m : h->im) s += m.nsyn;
  out->n_synapses_total = s;
  out->device_bytes = h->device_bytes;
  out->build_seconds = h->build_seconds;
  out->graphs = h->graph_exec ? 1u : 0u;
  out->ring_rows = h->engine == SNN_ENGINE_BAND ? h->d.band_h : uint32_t(kRing);
  if (h->engine == SNN_ENGINE_LDS || h->engine == SNN_ENGINE_BAND) {
    out->launches_per_chunk = uint32_t(h->lds_groups.size());
    for (const auto &m : h->im) out->window_neurons = std::max(out->window_neurons, m.wlen);
  } else {
    out->launches_per_chunk = h->engine == SNN_ENGINE_PERSISTENT ? 1u : 2u * h->chunk;
  }
  return SNN_OK;
}

int snn_autotune(snn_net *h, uint32_t trial_steps, snn_tune_report *out) {
  if (!h || !out) return fail(h, SNN_E_INVAL, "NULL argument");
  if (!trial_steps) return fail(h, SNN_E_INVAL, "trial_steps must be positive");
  if (h->dead) return fail(h, SNN_E_DEVICE, "the handle is unusable after a device failure");
  std::memset(out, 0, sizeof *out);
  out->engine = h->engine;
  auto timed = [&](double *us) -> int {
    double ms = 0.0;
    const int rc = snn_time_steps(h, trial_steps, &ms);
    *us = 1000.0 * ms / trial_steps;
    return rc;
  };
  // Stepwise: the chunk graph bakes the transfer grid in; capture it again.
  auto recapture = [&]() -> int {
    if (!h->graph_exec) return SNN_OK;
    (void)hipGraphExecDestroy(h->graph_exec);
    (void)hipGraphDestroy(h->graph);
    h->graph_exec = nullptr;
    h->graph = nullptr;
    HIP_OK(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    const hipError_t le = launch_stepwise(h->d, h->shape, h->chunk, h->stream);
    const hipError_t ce = hipStreamEndCapture(h->stream, &h->graph);
    if (le != hipSuccess || ce != hipSuccess ||
        hipGraphInstantiate(&h->graph_exec, h->graph, nullptr, nullptr, 0) != hipSuccess)
      return fail(h, SNN_E_HIP, "graph capture of a %u-step chunk failed", h->chunk);
    return SNN_OK;
  };
  std::vector<LaunchShape> cands;
  const LaunchShape first = h->shape;
  cands.push_back(first);
  if (h->engine == SNN_ENGINE_PERSISTENT) {
    for (uint32_t b : {128u, 256u, 512u, 1024u})
      for (uint32_t q : {1u, 2u, 4u, 8u}) {
        const int maxg = persistent_max_grid(h->d, b, q);
        const uint32_t g = (h->d.nquads + b * q - 1) / (b * q);
        if (maxg <= 0 || g == 0 || g > uint32_t(maxg)) continue;
        LaunchShape s = first;
        s.block = b;
        s.grid = g;
        s.qpt = (h->d.nquads + g * b - 1) / (g * b);
        if (s.block != first.block || s.grid != first.grid || s.qpt != first.qpt) cands.push_back(s);
      }
  } else if (h->engine == SNN_ENGINE_STEPWISE) {
    for (uint32_t sb : {256u, 512u, 1024u, 2048u, 4096u})
      if (sb != first.scatter_blocks) {
        LaunchShape s = first;
        s.scatter_blocks = sb;
        cands.push_back(s);
      }
  }
  double best = 0.0;
  size_t bi = 0;
  for (size_t i = 0; i < cands.size(); ++i) {
    h->shape = cands[i];
    int rc = h->engine == SNN_ENGINE_STEPWISE ? recapture() : SNN_OK;
    double us = 0.0;
    if (!rc) rc = timed(&us);
    if (rc) {
      h->shape = first;
      return rc;
    }
    if (i == 0) out->us_per_step_first = us;
    if (i == 0 || us < best) {
      best = us;
      bi = i;
    }
  }
  h->shape = cands[bi];
  if (h->engine == SNN_ENGINE_STEPWISE) {
    const int rc = recapture();
    if (rc) return rc;
  }
  out->candidates = uint32_t(cands.size());
  out->block_size = h->shape.block;
  out->grid_blocks = h->engine == SNN_ENGINE_STEPWISE ? h->shape.scatter_blocks : h->shape.grid;
  out->quads_per_thread = h->shape.qpt;
  for (const auto &m : h->im) out->window_neurons = std::max(out->window_neurons, m.wlen);
  out->us_per_step_best = best;
  return SNN_OK;
}

}  // extern "C"

namespace {

struct TuneCand {
  uint32_t engine, L;
  std::vector<uint32_t> each;   // per-instance window lengths (L = 0), or empty
};

// Candidate layouts of the LDS engines for a configuration: per engine the
// shortest window that fills one launch, and longer ones (x 1.25, x 1.6) as
// far as a kernel variant holds them.
std::vector<TuneCand> tune_candidates(const snn_config *cfg) {
  std::vector<InstMeta> im(cfg->n_instances);
  for (uint32_t k = 0; k < cfg->n_instances; ++k) im[k].n = instance_neurons(cfg->inst[k]);
  std::vector<TuneCand> out;
  auto family = [&](uint32_t eng) {
    LdsPlan p;
    std::string why;
    uint32_t v = 0;
    const int rc = eng == SNN_ENGINE_LDS
                       ? plan_lds(im, cfg->block_size, cfg->grid_blocks, 0, nullptr, false, p, why)
                       : plan_band(im, cfg->block_size, cfg->grid_blocks, 0, nullptr, p, v, why);
    if (rc) return;
    uint32_t L0 = 0;
    for (uint32_t wq : p.wq) L0 = std::max(L0, 4 * wq);
    std::vector<uint32_t> seen;
    for (double f : {1.0, 1.25, 1.6}) {
      const uint32_t L = uint32_t(L0 * f + 3.0) & ~3u;
      const int ok = eng == SNN_ENGINE_LDS
                         ? plan_lds(im, cfg->block_size, cfg->grid_blocks, L, nullptr, false, p, why)
                         : plan_band(im, cfg->block_size, cfg->grid_blocks, L, nullptr, p, v, why);
      if (ok != SNN_OK || std::find(seen.begin(), seen.end(), p.total) != seen.end()) continue;
      seen.push_back(p.total);
      out.push_back({eng, L, {}});
    }
  };
  if (cfg->engine == SNN_ENGINE_AUTO || cfg->engine == SNN_ENGINE_LDS) family(SNN_ENGINE_LDS);
  if (cfg->engine == SNN_ENGINE_AUTO || cfg->engine == SNN_ENGINE_BAND) family(SNN_ENGINE_BAND);
  return out;
}

// FNV-1a digest of everything in a configuration that shapes the network and
// its step loop.
uint64_t config_digest(const snn_config *cfg) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void *p, size_t n) {
    const unsigned char *b = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
  };
  mix(&cfg->n_instances, 4);
  mix(&cfg->syn_format, 4);
  mix(&cfg->engine, 4);
  mix(&cfg->block_size, 4);
  mix(&cfg->grid_blocks, 4);
  mix(&cfg->chunk_steps, 4);
  for (uint32_t k = 0; k < cfg->n_instances; ++k) {
    const snn_instance_cfg &c = cfg->inst[k];
    mix(&c.seed, 8);
    mix(&c.scale, 8);
    mix(&c.indegree_mode, 4);
    mix(&c.count_rule, 4);
    mix(&c.rows_are_sources, 4);
    mix(&c.g, 8);
    mix(&c.bg_rate_hz, 8);
    mix(&c.psp_ext_mv, 8);
    mix(&c.bg_const_T, 4);
    if (c.conn) mix(c.conn, 64 * sizeof(double));
  }
  return h;
}

}  // namespace

extern "C" {

int snn_build_tuned(const snn_config *cfg, uint32_t trial_steps, const char *cache_path,
                    snn_net **out, snn_tune_report *rep) {
  if (!out || !rep) return fail(nullptr, SNN_E_INVAL, "NULL argument");
  *out = nullptr;
  std::memset(rep, 0, sizeof *rep);
  if (!trial_steps) return fail(nullptr, SNN_E_INVAL, "trial_steps must be positive");
  if (!cfg || !cfg->inst || cfg->n_instances < 1 || cfg->n_instances > kMaxInstances)
    return fail(nullptr, SNN_E_INVAL, "bad configuration");
  const uint32_t ni = cfg->n_instances;
  snn_config c = *cfg;
  std::vector<TuneCand> cands = cfg->window_neurons || cfg->inst_window_neurons
                                    ? std::vector<TuneCand>()
                                    : tune_candidates(cfg);
  if (cands.empty()) return snn_build(cfg, out);   // nothing to choose
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return fail(nullptr, SNN_E_HIP, "no current HIP device");
  char key[160];
  std::snprintf(key, sizeof key, "%s %016llx", prop.gcnArchName,
                (unsigned long long)config_digest(cfg));
  TuneCand best{0, 0, {}};
  double best_us = 0.0, first_us = 0.0;
  uint32_t n_timed = 0;
  bool cached = false;
  if (cache_path) {   // last matching line wins
    if (FILE *f = std::fopen(cache_path, "r")) {
      std::vector<char> line(16384);
      char arch[96], dig[32];
      unsigned e = 0, L = 0;
      double us = 0.0, us0 = 0.0;
      int used = 0;
      while (std::fgets(line.data(), int(line.size()), f))
        if (std::sscanf(line.data(), "%95s %31s %u %u %lf %lf%n", arch, dig, &e, &L, &us, &us0,
                        &used) == 6 &&
            std::strlen(key) == std::strlen(arch) + 1 + std::strlen(dig) &&
            std::strncmp(key, arch, std::strlen(arch)) == 0 &&
            std::strcmp(key + std::strlen(arch) + 1, dig) == 0) {
          // An optional seventh field: the per-instance window lengths.
          std::vector<uint32_t> each;
          const char *q = line.data() + used;
          while (*q == ' ') ++q;
          while (*q >= '0' && *q <= '9') {
            char *end = nullptr;
            each.push_back(uint32_t(std::strtoul(q, &end, 10)));
            q = end;
            if (*q == ',') ++q;
          }
          if (!each.empty() && each.size() != ni) continue;   // not this configuration's
          best = {e, each.empty() ? L : 0u, each};
          best_us = us;
          first_us = us0;
          cached = true;
        }
      std::fclose(f);
    }
  }
  if (!cached) {
    // Times one candidate; on the first, also measures the synaptic events
    // per neuron and step of every instance (the same for every layout).
    std::vector<double> load;
    auto time_cand = [&](const TuneCand &cd, bool measure, double &us) -> int {
      c.engine = cd.engine;
      c.window_neurons = cd.L;
      c.inst_window_neurons = cd.each.empty() ? nullptr : cd.each.data();
      snn_net *h = nullptr;
      int rc = snn_build(&c, &h);
      if (rc) return rc;
      std::vector<uint64_t> e0(ni, 0);
      auto events = [&](std::vector<uint64_t> &ev) {
        for (uint32_t k = 0; k < ni && rc == SNN_OK; ++k) {
          snn_state st{};
          rc = snn_read_state(h, k, &st);
          ev[k] = st.events;
        }
      };
      double ms = 0.0;
      rc = snn_step_n(h, std::max(1u, trial_steps / 4));
      if (!rc && measure) events(e0);
      if (!rc) rc = snn_time_steps(h, trial_steps, &ms);
      if (!rc && measure) {
        std::vector<uint64_t> e1(ni, 0);
        events(e1);
        load.assign(ni, 0.0);
        for (uint32_t k = 0; k < ni; ++k)
          load[k] = double(e1[k] - e0[k]) / (double(h->im[k].n) * trial_steps);
      }
      if (rc) {
        g_build_error = h->err;
        snn_destroy(h);
        return rc;
      }
      snn_destroy(h);
      us = 1000.0 * ms / trial_steps;
      ++n_timed;
      return SNN_OK;
    };
    auto consider = [&](const TuneCand &cd, bool first) -> int {
      double us = 0.0;
      const int rc = time_cand(cd, first, us);
      if (rc) return rc;
      if (first) first_us = us;
      if (first || us < best_us) {
        best_us = us;
        best = cd;
      }
      return SNN_OK;
    };
    for (size_t i = 0; i < cands.size(); ++i)
      if (int rc = consider(cands[i], i == 0)) return rc;
    // Several instances: the winner's kernel and number of blocks again,
    // with each instance's windows sized by its measured load.
    double lmax = 0.0;
    for (double x : load) lmax = std::max(lmax, x);
    if (ni > 1 && lmax > 0.0) {
      std::vector<InstMeta> im(ni);
      for (uint32_t k = 0; k < ni; ++k) im[k].n = instance_neurons(cfg->inst[k]);
      LdsPlan p;
      std::string why;
      uint32_t v = 0, wn = 0;
      if (best.engine == SNN_ENGINE_LDS) {
        if (plan_lds(im, cfg->block_size, cfg->grid_blocks, best.L, nullptr, false, p, why) == SNN_OK)
          wn = p.wn;
      } else if (plan_band(im, cfg->block_size, cfg->grid_blocks, best.L, nullptr, p, v, why) == SNN_OK) {
        wn = kBandVariants[v].wn;
      }
      std::vector<uint32_t> Ls;
      if (wn && balanced_lengths(im, load, wn, p.total, Ls)) {
        const int ok = best.engine == SNN_ENGINE_LDS
                           ? plan_lds(im, cfg->block_size, cfg->grid_blocks, 0, Ls.data(), false, p, why)
                           : plan_band(im, cfg->block_size, cfg->grid_blocks, 0, Ls.data(), p, v, why);
        if (ok == SNN_OK) {
          cands.push_back({best.engine, 0u, Ls});
          if (int rc = consider(cands.back(), false)) return rc;
        }
      }
    }
    if (cache_path) {
      if (FILE *f = std::fopen(cache_path, "a")) {
        std::fprintf(f, "%s %u %u %.4f %.4f", key, best.engine, best.L, best_us, first_us);
        for (size_t k = 0; k < best.each.size(); ++k)
          std::fprintf(f, "%c%u", k ? ',' : ' ', best.each[k]);
        std::fprintf(f, "\n");
        std::fclose(f);
      }
    }
  }
  c.engine = best.engine;
  c.window_neurons = best.L;
  c.inst_window_neurons = best.each.empty() ? nullptr : best.each.data();
  const int rc = snn_build(&c, out);
  if (rc) return rc;
  const snn_net *h = *out;
  rep->engine = h->engine;
  rep->candidates = cached ? 0u : n_timed;
  rep->block_size = h->shape.block;
  rep->grid_blocks = h->shape.grid;
  rep->quads_per_thread = h->shape.qpt;
  for (const auto &m : h->im) rep->window_neurons = std::max(rep->window_neurons, m.wlen);
  rep->us_per_step_first = first_us;
  rep->us_per_step_best = best_us;
  return SNN_OK;
}

int snn_time_steps(snn_net *h, uint64_t n_steps, double *elapsed_ms) {
  if (!h || !elapsed_ms) return fail(h, SNN_E_INVAL, "NULL argument");
  hipEvent_t a = nullptr, b = nullptr;
  // Both events are released on every path, the error paths included.
  struct Events {
    hipEvent_t *a, *b;
    ~Events() {
      if (*a) (void)hipEventDestroy(*a);
      if (*b) (void)hipEventDestroy(*b);
    }
  } guard{&a, &b};
  HIP_OK(h, hipEventCreate(&a));
  HIP_OK(h, hipEventCreate(&b));
  HIP_OK(h, hipEventRecord(a, h->stream));
  const int rc = snn_step_n(h, n_steps);
  if (rc) return rc;
  HIP_OK(h, hipEventRecord(b, h->stream));
  HIP_OK(h, hipEventSynchronize(b));
  float ms = 0.0f;
  HIP_OK(h, hipEventElapsedTime(&ms, a, b));
  *elapsed_ms = ms;
  return SNN_OK;
}

int snn_sample_network(const snn_instance_cfg *inst, uint32_t syn_format, int32_t host_threads,
                       snn_host_network **out) {
  return snn_sample_network_windows(inst, syn_format, 0, host_threads, out);
}

}  // extern "C"

namespace {

// Rows of a sampled instance read back from its storage layout, in storage
// order (by target window, then band, then segment order).
int read_back(const HostInstance &x, uint32_t syn_format, snn_host_network **out) {
  snn_host_network *n = static_cast<snn_host_network *>(std::calloc(1, sizeof(snn_host_network)));
  if (!n) return fail(nullptr, SNN_E_NOMEM, "host allocation failed");
  n->n_neurons = x.n;
  n->n_synapses = x.nsyn;
  std::memcpy(n->pop_offset, x.pop_off, sizeof n->pop_offset);
  n->row_ptr = static_cast<uint64_t *>(std::malloc((x.n + 1) * sizeof(uint64_t)));
  n->post = static_cast<uint32_t *>(std::malloc(std::max<uint64_t>(1, x.nsyn) * sizeof(uint32_t)));
  n->delay = static_cast<uint8_t *>(std::malloc(std::max<uint64_t>(1, x.nsyn)));
  n->w_q = static_cast<int32_t *>(std::malloc(std::max<uint64_t>(1, x.nsyn) * sizeof(int32_t)));
  n->u0 = static_cast<float *>(std::malloc(x.n * sizeof(float)));
  if (!n->row_ptr || !n->post || !n->delay || !n->w_q || !n->u0) {
    snn_free_network(n);
    return fail(nullptr, SNN_E_NOMEM, "host allocation failed");
  }
  std::memcpy(n->u0, x.u0.data(), x.n * sizeof(float));
  const bool comp = syn_format == SNN_SYN_COMPRESSED5;
  const uint32_t nb = x.nband;
  const uint32_t ob = x.band_h ? band_offset_bits(x.band_h) : 0u;
  uint64_t o = 0;
  for (uint32_t i = 0; i < x.n; ++i) {
    n->row_ptr[i] = o;
    uint32_t c = 0;
    while (x.padded && i >= x.pop_off[c + 1]) ++c;
    for (uint32_t w = 0; w < x.nwin; ++w) {
      for (uint32_t b = 0; b < (x.padded ? nb : 1u); ++b) {
        uint64_t lo = 0, hi = 0;
        if (x.padded) {
          const size_t k = (size_t(w) * nb + b) * 8 + c;
          const uint32_t cap = x.cls_cap[k];
          lo = x.cls_base[k] + uint64_t(i - x.pop_off[c]) * cap;
          hi = lo + cap;
        } else {
          const uint64_t s = uint64_t(i) * x.nwin + w;
          lo = x.seg_ptr[s];
          hi = x.seg_ptr[s + 1];
        }
        for (uint64_t e2 = lo; e2 < hi; ++e2) {
          uint32_t post, dl;
          int32_t wq;
          bool unused;
          if (syn_format == SNN_SYN_DEV8 && x.band_h) {
            // banded: doubled << 15 | (delay - band_lo) << od | offset, deviation (-128: unused)
            const uint32_t od = band_dev_offset_bits(x.band_h);
            const uint32_t r = x.rec2[e2];
            const int di = int(2 * c + (r >> 15));
            post = w * x.win_size + (r & ((1u << od) - 1u));
            dl = band_lo(b, x.band_h) + ((r >> od) & (x.band_h - 1u));
            wq = x.dev_mq[di] + int32_t(x.dev8[e2]) * x.dev_sq[di];
            unused = x.dev8[e2] == -128;
          } else if (syn_format == SNN_SYN_DEV8) {   // doubled << 15 | delay << 9 | offset, deviation
            const uint32_t r = x.rec2[e2];
            const int di = int(2 * c + (r >> 15));
            post = (x.win_first + w) * x.win_size + (r & 511u) - x.win_origin;
            dl = (r >> 9) & 63u;
            wq = x.dev_mq[di] + int32_t(x.dev8[e2]) * x.dev_sq[di];
            unused = dl == 0;
          } else if (comp && x.band_h) {   // banded: weight << 16 | (delay - band_lo) << ob | offset
            const uint32_t r = x.rec4[e2];
            post = w * x.win_size + (r & ((1u << ob) - 1u));
            dl = band_lo(b, x.band_h) + ((r & 0xFFFFu) >> ob);
            wq = int32_t(int16_t(uint16_t(r >> 16))) * 8;
            unused = wq == 0;
          } else if (comp && x.padded) {
            const uint32_t r = x.rec4[e2];
            post = (x.win_first + w) * x.win_size + (r & 1023u) - x.win_origin;
            dl = (r >> 10) & 63u;
            wq = int32_t(int16_t(uint16_t(r >> 16))) * 8;
            unused = dl == 0;
          } else if (comp) {
            post = (x.win_first + w) * x.win_size + x.tgt16[e2] - x.win_origin;
            dl = x.d8[e2];
            wq = int32_t(x.w16[e2]) * 8;
            unused = false;
          } else {
            const uint32_t hiw = uint32_t(x.rec8[e2] >> 32);
            post = hiw >> 6;
            dl = hiw & 63u;
            wq = int32_t(uint32_t(x.rec8[e2]));
            unused = dl == 0;
          }
          if (unused) continue;  // an unused slot of a padded segment
          if (o >= x.nsyn) {
            snn_free_network(n);
            return fail(nullptr, SNN_E_RANGE, "storage holds more synapses than sampled");
          }
          n->post[o] = post;
          n->delay[o] = uint8_t(dl);
          n->w_q[o] = wq;
          ++o;
        }
      }
    }
  }
  n->row_ptr[x.n] = o;
  if (o != x.nsyn) {
    snn_free_network(n);
    return fail(nullptr, SNN_E_RANGE, "storage holds %llu of %llu synapses", (unsigned long long)o,
                (unsigned long long)x.nsyn);
  }
  *out = n;
  return SNN_OK;
}

}  // namespace

extern "C" {

int snn_sample_network_windows(const snn_instance_cfg *inst, uint32_t syn_format, uint32_t window,
                               int32_t host_threads, snn_host_network **out) {
  if (!inst || !out) return fail(nullptr, SNN_E_INVAL, "NULL argument");
  *out = nullptr;
  if (window != 0 && window != 256 && window != 512)
    return fail(nullptr, SNN_E_INVAL, "window must be 0, 256 or 512");
  HostInstance x;
  std::string e;
  uint32_t wsize = syn_format == SNN_SYN_COMPRESSED5 ? (1u << kTargetBlockBits) : kNoWindows;
  if (window) wsize = window;
  int rc = sample_instance(*inst, syn_format, wsize, 0, window != 0, host_threads, x, e);
  if (rc) return fail(nullptr, rc, "%s", e.c_str());
  return read_back(x, syn_format, out);
}

int snn_balanced_windows(uint32_t n_instances, const uint32_t *n_neurons, const double *load,
                         uint32_t max_window, uint32_t max_blocks, uint32_t *window_out) {
  if (!n_instances || !n_neurons || !load || !window_out)
    return fail(nullptr, SNN_E_INVAL, "NULL array or no instances");
  if (max_window < 4 || max_window % 4)
    return fail(nullptr, SNN_E_INVAL, "max_window must be a positive multiple of 4");
  std::vector<InstMeta> im(n_instances);
  std::vector<double> w(n_instances);
  for (uint32_t k = 0; k < n_instances; ++k) {
    if (!(load[k] >= 0.0) || !std::isfinite(load[k]))
      return fail(nullptr, SNN_E_INVAL, "instance %u: load must be finite and >= 0", k);
    im[k].n = n_neurons[k];
    w[k] = load[k];
  }
  std::vector<uint32_t> L;
  if (!balanced_lengths(im, w, max_window, max_blocks, L))
    return fail(nullptr, SNN_E_RANGE, "%u-neuron windows need more than %u blocks", max_window,
                max_blocks);
  std::copy(L.begin(), L.end(), window_out);
  return SNN_OK;
}

int snn_sample_network_bands(const snn_instance_cfg *inst, uint32_t syn_format, uint32_t window,
                             uint32_t ring_rows, int32_t host_threads, snn_host_network **out) {
  if (!inst || !out) return fail(nullptr, SNN_E_INVAL, "NULL argument");
  *out = nullptr;
  if (window < 4 || window > 4096 || window % 4)
    return fail(nullptr, SNN_E_INVAL, "window must be a multiple of 4 in [4, 4096]");
  if (ring_rows != 64 && ring_rows != 32 && ring_rows != 16 && ring_rows != 8)
    return fail(nullptr, SNN_E_INVAL, "ring_rows must be 64, 32, 16 or 8");
  HostInstance x;
  std::string e;
  int rc = sample_instance_banded(*inst, syn_format, window, ring_rows, host_threads, x, e);
  if (rc) return fail(nullptr, rc, "%s", e.c_str());
  return read_back(x, syn_format, out);
}

void snn_free_network(snn_host_network *n) {
  if (!n) return;
  std::free(n->row_ptr);
  std::free(n->post);
  std::free(n->delay);
  std::free(n->w_q);
  std::free(n->u0);
  std::free(n);
}

}  // extern "C"
