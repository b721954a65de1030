// band.hip -- the banded LDS engine: horizon-based spike transfer (Sec. 3.4,
// lst:horizon2) over destination-partitioned synapse classes (Sec. 3.6), so
// that networks whose 64-row ring does not fit the chip's LDS still keep their
// ring on chip, and so that only the one-step delays sit on the step's
// dependent chain.
//
// Block b owns the neurons of window b and H rows of their ring buffer in LDS
// (H = 64, 16 or 8), the live rows [t, t + H) of step t.  Synapses are stored
// per (sender, window, delay band) in fixed-capacity segments whose address
// follows from the sender's id: band 0 holds delay 1, slow band j >= 1 the
// delays [2 + (j-1) H, 1 + j H].  The spikes of step s are delivered band by
// band: band 0 right after their flags arrive (iteration s + 1, rows s + 1),
// slow band j at iteration s + lo_j (rows [s + lo_j, s + lo_j + H)), i.e.
// while the block waits for the next flags.  lst:horizon2 delivers a band of
// H delays per spike every H steps in the same way; here the first band is
// cut to the single delay the next decision depends on.
//
// The sender ids of past steps are kept per block: an LDS history of HC ids
// per step, then (below 1,024 threads) 192 more in device memory private to
// the block, the rest in device memory shared by the instance's blocks, which
// all write the same ids there.  Between launches the 64-row ring in device memory is
// complete: a launch loads rows [t0, t0 + H) and pulls rows t0 + H .. t0 + 63
// as they enter the horizon, and at its end delivers every slow band still
// pending -- into LDS rows inside the horizon, with device atomics beyond it
// -- and writes its H live rows back.
//
// Blocks exchange senders through one 64-bit flag word per block and step
// (epoch, spike count, the window offsets of its first spikes) and a list in
// device memory for the others, as the LDS engine of kernels.hip does.
#include "device.hpp"

namespace snn {
namespace {

// Flag word: bits 0-15 epoch (mod 2^16), then the spike count (CB bits),
// then the window offsets of the first NI spikes (OB bits each).
template <int WN>
struct FlagFmt {
  static constexpr uint32_t CB = WN <= 512 ? 10u : 12u;
  static constexpr uint32_t OB = WN <= 512 ? 9u : 12u;
  static constexpr uint32_t NI = (64u - 16u - CB) / OB;
  static_assert(uint32_t(WN) < (1u << CB) && uint32_t(WN) <= (1u << OB), "window too large");
  __device__ static uint32_t count(uint64_t f) { return uint32_t(f >> 16) & ((1u << CB) - 1u); }
  __device__ static uint32_t local(uint64_t f, uint32_t k) {
    return uint32_t(f >> (16u + CB + OB * k)) & ((1u << OB) - 1u);
  }
  __device__ static uint64_t word(uint32_t ep, uint32_t cnt) {
    return uint64_t(ep & 0xFFFFu) | (uint64_t(cnt) << 16);
  }
  __device__ static uint64_t inline_sender(uint32_t k, uint32_t loc) {
    return uint64_t(loc) << (16u + CB + OB * k);
  }
};

constexpr uint32_t kSBH = 128;   // senders a polling wave expands into s_sid

// Sender j of step t-1's set, as a global id: from the expanded list s_sid
// (the first kSBH senders of a polling wave's half; list markers are
// 1 << 31 | relative window << 12 | index), else by search over the windows
// with senders (s_nzf / s_nzp / s_nzb); senders past a window's first NI come
// from its list in device memory.
template <class F>
__device__ __forceinline__ uint32_t band_sender_gid(const uint32_t *llist, uint32_t ntot, uint32_t j,
                                                    uint32_t nnz, uint32_t lslot, const uint32_t *s_sid,
                                                    const uint64_t *s_nzf, const uint32_t *s_nzp,
                                                    const uint16_t *s_nzb, const uint32_t *s_wstart) {
  uint32_t src, kk;
  if (j < kSBH) {
    const uint32_t v = s_sid[j];
    if (!(v >> 31)) return v;
    src = (v >> 12) & 0x7FFFFu;
    kk = v & 4095u;
  } else {
    uint32_t lo = 0, hi = nnz;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (s_nzp[mid] <= j) lo = mid; else hi = mid;
    }
    kk = j - s_nzp[lo];
    src = s_nzb[lo];
    if (kk < F::NI) return s_wstart[src] + F::local(s_nzf[lo], kk);
  }
  const uint32_t w0 = s_wstart[src];
  return w0 + ld_ag(llist + size_t(lslot) * ntot + w0 + kk);
}

// Record formats of the banded layout: plain (8 bytes), compressed (4
// bytes), deviation (a 2-byte locator and a 1-byte deviation from the mean
// of the sender's population pair).
constexpr int kBandPlain = 0, kBandComp = 1, kBandDev = 2;

// Decoded record: the weight (0 for an unused slot), the row it adds to
// (absolute step, low 32 bits) and its offset in the window.  Deviation
// format: loc2 the locator, dv the deviation, pc the sender's population, dq
// and dsq the mean and step of each (population, doubled) pair.
template <int FMT, int H>
__device__ __forceinline__ void decode(uint64_t rec8, uint32_t rec4, uint32_t loc2, int32_t dv,
                                       uint32_t pc, const int32_t *dq, const int32_t *dsq,
                                       uint32_t rb, uint32_t wb0, int32_t &w, uint32_t &row,
                                       uint32_t &loc) {
  if (FMT == kBandComp) {
    constexpr uint32_t OB = band_offset_bits(H);
    w = int32_t(int16_t(uint16_t(rec4 >> 16))) * 8;
    row = rb + ((rec4 & 0xFFFFu) >> OB);
    loc = rec4 & ((1u << OB) - 1u);
  } else if (FMT == kBandDev) {
    constexpr uint32_t OD = band_dev_offset_bits(H);
    const uint32_t di = 2u * pc + (loc2 >> 15);
    w = dv == -128 ? 0 : dq[di] + dv * dsq[di];
    row = rb + ((loc2 >> OD) & uint32_t(H - 1));
    loc = loc2 & ((1u << OD) - 1u);
  } else {
    const uint32_t hiw = uint32_t(rec8 >> 32);
    w = int32_t(uint32_t(rec8));
    row = rb + (hiw & 63u);
    loc = (hiw >> 6) - wb0;
  }
}

// Delivery of one batch of segments, one per lane of the wave: lane l holds
// the segment (base, capacity) of the wave's sender l and its row base rb
// (step of the spike, plus the band's first delay for compressed records,
// whose delays are stored relative to it).  Three ways to cut the batch into
// loads of 64 lanes:
//  * grouped: with every capacity at most G <= 64 (a power of two, the
//    band's largest capacity rounded up) the senders are packed 64 / G to a
//    load, G lanes each;
//  * pieces: every sender is cut into 64-record pieces, one load each;
//  * packed: the segments are laid back to back and each load takes 64
//    consecutive slots; slot k belongs to the last lane whose exclusive
//    prefix of capacities is <= k (a binary search over the lanes).
// Capacities of one band differ by up to two orders of magnitude between
// populations, so the first two can leave most lanes empty; the packed walk
// has the fewest loads but its search lengthens each load's address.  PACK
// selects the packed walk for every batch; it is set only where that was
// measured to pay (the 512-thread variant with 16 ring rows, whose slow bands
// otherwise take several rounds of loads; elsewhere the other two fit one
// round and are faster).  UR loads are in flight per lane.
template <int FMT, int UR, int H, bool PACK>
struct BandWalk {
  uint64_t rec[FMT == kBandPlain ? UR : 1];
  uint32_t r4[FMT == kBandComp ? UR : 1];
  uint32_t r2[FMT == kBandDev ? UR : 1];    // deviation format: locator
  int32_t dv[FMT == kBandDev ? UR : 1];     // and deviation (-128: unused slot)
  uint32_t pcv[FMT == kBandDev ? UR : 1];   // and the sender's population
  uint32_t rbv[UR];
  uint64_t base_l;
  uint32_t cap_l, rb_l, cls_l;
  uint32_t G;        // lanes per sender (grouped), or 64 with pieces
  uint32_t mode;     // 0 grouped, 1 pieces, 2 packed (wave-uniform)
  uint32_t p_l;      // pieces: the lane's first piece; packed: its first slot
  uint32_t total;    // packed: slots of the batch
  uint32_t nu;       // units (loads of 64 lanes) of the batch, wave-uniform
  uint32_t u0;       // next unit
  uint32_t nv;       // slots filled by the last load()

  // cls: the lane's sender population (read by the deviation format only).
  __device__ __forceinline__ void begin(uint64_t base, uint32_t cap, uint32_t rb, uint32_t nsend,
                                        uint32_t gmax, uint32_t cls) {
    base_l = base;
    cap_l = cap;
    rb_l = rb;
    cls_l = cls;
    u0 = 0;
    total = 0;
    if (PACK) {
      mode = 2;
      G = 64;
      p_l = wave_prefix(cap, total);
      nu = (total + 63u) >> 6;
    } else if (gmax <= 64u) {
      mode = 0;
      G = gmax;
      const uint32_t per = 64u / G;
      nu = (nsend + per - 1u) / per;
      p_l = 0;
    } else {
      mode = 1;
      G = 64;
      p_l = wave_prefix((cap + 63u) >> 6, nu);
    }
  }
  __device__ __forceinline__ bool more() const { return u0 < nu; }

  // Slot u holds nothing (decodes to weight 0).
  __device__ __forceinline__ void clear(int u) {
    if (FMT == kBandComp) r4[u] = 0u;
    if (FMT == kBandPlain) rec[u] = 0ull;
    if (FMT == kBandDev) {
      r2[u] = 0u;
      dv[u] = -128;
      pcv[u] = 0u;
    }
  }
  // Loads slot u from record address addr when ok.
  __device__ __forceinline__ void fetch(const DeviceNet &d, int u, uint64_t addr, bool ok) {
    if (!ok) return;
    if (FMT == kBandComp) r4[u] = __builtin_nontemporal_load(d.rec4 + addr);
    if (FMT == kBandPlain) rec[u] = __builtin_nontemporal_load(d.rec8 + addr);
    if (FMT == kBandDev) {
      r2[u] = uint32_t(__builtin_nontemporal_load(d.rec2 + addr));
      dv[u] = int32_t(__builtin_nontemporal_load(d.dev8 + addr));
    }
  }

  __device__ __forceinline__ void load(const DeviceNet &d) {
    if constexpr (PACK) {
      load_packed(d);
      return;
    }
    const uint32_t lane = __lane_id();
#pragma unroll
    for (int u = 0; u < UR; ++u) {
      const uint32_t U = u0 + uint32_t(u);
      clear(u);
      rbv[u] = 0;
      if (U >= nu) continue;   // wave-uniform
      uint64_t addr;
      bool ok;
      if (!PACK && mode == 0) {
        const uint32_t per = 64u / G;
        const uint32_t k = U * per + lane / G;   // sender (lane of the batch)
        const uint32_t off = lane & (G - 1u);
        const uint32_t blo = __shfl(uint32_t(base_l), int(k & 63u));
        const uint32_t bhi = __shfl(uint32_t(base_l >> 32), int(k & 63u));
        uint32_t cap = __shfl(cap_l, int(k & 63u));
        rbv[u] = __shfl(rb_l, int(k & 63u));
        if (FMT == kBandDev) pcv[u] = __shfl(cls_l, int(k & 63u));
        cap = k < 64u ? cap : 0u;
        addr = join64(bhi, blo) + off;
        ok = off < cap;
      } else if (!PACK) {
        // The piece's sender is the last lane whose first piece is <= U
        // (lanes past the last sender have p_l = nu > U).
        const uint32_t s = uint32_t(__popcll(__ballot(int(p_l <= U)))) - 1u;
        const uint32_t k = U - __builtin_amdgcn_readlane(p_l, s);
        const uint32_t cap = __builtin_amdgcn_readlane(cap_l, s);
        rbv[u] = __builtin_amdgcn_readlane(rb_l, s);
        if (FMT == kBandDev) pcv[u] = __builtin_amdgcn_readlane(cls_l, s);
        const uint32_t off = 64u * k + lane;
        addr = join64(uint32_t(__builtin_amdgcn_readlane(uint32_t(base_l >> 32), s)),
                      uint32_t(__builtin_amdgcn_readlane(uint32_t(base_l), s))) + off;
        ok = off < cap;
      } else {
        addr = 0;
        ok = false;
      }
      fetch(d, u, addr, ok);
    }
    nv = min(nu - u0, uint32_t(UR));
    u0 += UR;
  }

  // Packed walk: slot 64 U + lane of the batch belongs to the largest lane
  // s with p_s <= slot (a slot below the total lies in a segment of positive
  // capacity, so s is a real sender and the slot's offset in it is below its
  // capacity).  The six-level binary searches of PG units run interleaved:
  // each level is a cross-lane read whose latency the other units' reads
  // hide.  The first level compares with lane 32 for every slot.
  __device__ __forceinline__ void load_packed(const DeviceNet &d) {
    constexpr int PG = 2;
    static_assert(UR % PG == 0, "units per round: a multiple of the search group");
    const uint32_t lane = __lane_id();
    const uint32_t p32 = uint32_t(__builtin_amdgcn_readlane(p_l, 32));
#pragma unroll
    for (int g = 0; g < UR; g += PG) {
#pragma unroll
      for (int v = 0; v < PG; ++v) {
        clear(g + v);
        rbv[g + v] = 0;
      }
      if (u0 + uint32_t(g) >= nu) continue;   // wave-uniform
      uint32_t sv[PG], ps[PG], slot[PG];
#pragma unroll
      for (int v = 0; v < PG; ++v) {
        slot[v] = 64u * (u0 + uint32_t(g + v)) + lane;
        const bool le = p32 <= slot[v];
        sv[v] = le ? 32u : 0u;
        ps[v] = le ? p32 : 0u;
      }
#pragma unroll
      for (uint32_t step = 16; step; step >>= 1) {
        uint32_t pc[PG];
#pragma unroll
        for (int v = 0; v < PG; ++v) pc[v] = __shfl(p_l, int(sv[v] + step));
#pragma unroll
        for (int v = 0; v < PG; ++v) {
          const bool le = pc[v] <= slot[v];
          sv[v] = le ? sv[v] + step : sv[v];
          ps[v] = le ? pc[v] : ps[v];
        }
      }
#pragma unroll
      for (int v = 0; v < PG; ++v) {
        const uint32_t blo = __shfl(uint32_t(base_l), int(sv[v]));
        const uint32_t bhi = __shfl(uint32_t(base_l >> 32), int(sv[v]));
        rbv[g + v] = __shfl(rb_l, int(sv[v]));
        if (FMT == kBandDev) pcv[g + v] = __shfl(cls_l, int(sv[v]));
        const uint64_t addr = join64(bhi, blo) + (slot[v] - ps[v]);
        fetch(d, g + v, addr, slot[v] < total);
      }
    }
    nv = min(nu - u0, uint32_t(UR));
    u0 += UR;
  }

  // Adds the loaded records into the LDS ring (rows mod H).
  template <int WN>
  __device__ __forceinline__ void apply(int32_t *s_ring, uint32_t wb0, const int32_t *dq,
                                        const int32_t *dsq) const {
#pragma unroll
    for (int u = 0; u < UR; ++u) {
      if (uint32_t(u) >= nv) {   // wave-uniform; past 8 slots the compiler unrolls
        if (UR > 8) continue;    // only a loop without an early exit
        break;
      }
      int32_t w;
      uint32_t row, loc;
      decode<FMT, H>(FMT == kBandPlain ? rec[u] : 0ull, FMT == kBandComp ? r4[u] : 0u,
                     FMT == kBandDev ? r2[u] : 0u, FMT == kBandDev ? dv[u] : 0,
                     FMT == kBandDev ? pcv[u] : 0u, dq, dsq, rbv[u], wb0, w, row, loc);
      if (w) atomicAdd(&s_ring[(row & (H - 1u)) * WN + loc], w);
    }
  }

  // End of a launch: rows inside the horizon [t_end, t_end + H) go to the
  // LDS ring, rows beyond it to the ring in device memory (device atomics on
  // the block's own window only).
  template <int WN>
  __device__ __forceinline__ void apply_flush(int32_t *s_ring, int32_t *W, uint32_t ntot, uint32_t wb0,
                                              uint32_t t_end, const int32_t *dq,
                                              const int32_t *dsq) const {
#pragma unroll
    for (int u = 0; u < UR; ++u) {
      if (uint32_t(u) >= nv) {   // wave-uniform; past 8 slots the compiler unrolls
        if (UR > 8) continue;    // only a loop without an early exit
        break;
      }
      int32_t w;
      uint32_t row, loc;
      decode<FMT, H>(FMT == kBandPlain ? rec[u] : 0ull, FMT == kBandComp ? r4[u] : 0u,
                     FMT == kBandDev ? r2[u] : 0u, FMT == kBandDev ? dv[u] : 0,
                     FMT == kBandDev ? pcv[u] : 0u, dq, dsq, rbv[u], wb0, w, row, loc);
      if (!w) continue;
      if (row - t_end < uint32_t(H))
        atomicAdd(&s_ring[(row & (H - 1u)) * WN + loc], w);
      else
        atomicAdd(W + size_t(row & 63u) * ntot + wb0 + loc, w);
    }
  }
};

template <int BS, int WN, int H, int HC, int FMT>
__global__ __launch_bounds__(BS) void k_band(DeviceNet d, uint32_t n_steps, uint32_t spin_limit) {
  using F = FlagFmt<WN>;
  constexpr uint32_t NW = BS / 64;
  constexpr uint32_t NQ = WN / 4;              // quads a window can hold
  constexpr uint32_t Q0 = BS - NQ;             // threads Q0.. own one quad each
  constexpr uint32_t NB = band_count(H);       // band 0 (delay 1) and the slow bands
  constexpr uint32_t LOMAX = band_lo(NB - 1, H);
  constexpr uint32_t NSLOT = H == 64 ? 4u : 64u;   // steps of sender history kept
  constexpr uint32_t TS = kLdsTab + 8;         // stride of an LDS thalamic table
  constexpr uint32_t NZ = kLdsMaxGrid;         // windows of one instance, at most
  constexpr int NJ = NZ / 128;                 // flags per lane of a polling wave
  constexpr uint32_t NZH = NZ / 2;             // windows polled by one wave
  constexpr uint32_t RC = 640;                 // raster staging entries
  constexpr uint32_t SB = 64 * NW;             // senders resolved per round
  // Loads in flight per lane.  The 1,024-thread variant keeps 12 although
  // its registers then spill part of them to scratch: fewer in flight leave
  // it waiting on the memory latency (measured: 4 and 8 slower, 16 too).
  constexpr int UR = BS >= 1024 ? 12 : (BS == 512 ? 16 : 8);
  constexpr bool PACK = BS == 512;             // packed walk (the variant of the widest bands)
  static_assert(Q0 >= 128, "waves 0 and 1 own no quad");
  static_assert(NSLOT > LOMAX, "the history must reach the last slow band");
  static_assert((H & (H - 1)) == 0 && H >= 8 && H <= 64, "ring rows: a power of two in [8, 64]");
  __shared__ __align__(16) int32_t s_ring[H * WN];
  __shared__ __align__(16) uint32_t s_thr[8 * TS];
  __shared__ uint32_t s_tlen[8];
  __shared__ uint32_t s_cf[8], s_cn[8];        // sender classes: first id, count
  __shared__ int32_t s_dq[16], s_ds[16];       // deviation format: mean and step per (class, doubled)
  __shared__ uint32_t s_ccap[NB * 8];          // per band and class: slots per sender
  __shared__ uint64_t s_cbase[NB * 8];
  __shared__ uint32_t s_gmax[NB];              // per band: group width (<= 64), or 65
  __shared__ uint32_t s_wstart[NZ];            // first neuron of each window of the instance
  __shared__ uint32_t s_sid[2 * kSBH];         // senders of step t-1 (gid or list marker)
  __shared__ uint64_t s_nzf[NZ];
  __shared__ uint32_t s_nzp[NZ];
  __shared__ uint16_t s_nzb[NZ];
  __shared__ uint32_t s_hist[NSLOT * HC];      // sender ids of past steps
  __shared__ uint32_t s_hn[NSLOT];             // senders of each past step
  __shared__ uint64_t s_rast[RC];
  __shared__ uint32_t s_wave[NW], s_inl[F::NI];
  __shared__ uint32_t s_flag[2], s_n[2], s_nnz[2];
  __shared__ unsigned long long s_rbase;
  __shared__ long long s_ctr[4];

  const uint32_t GT = d.n_lwin, blk = blockIdx.x;
  const uint64_t t0 = d.ctl->t_base;
  const uint64_t t_end = t0 + n_steps;
  const uint32_t ep0 = d.lgroup[0].x;
  const uint32_t tid = threadIdx.x, lane = __lane_id();
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint4 wi = d.lwin[blk];                // (first neuron, neurons, instance, -)
  const uint32_t wb0 = wi.x, wlen = wi.y, inst = wi.z;
  const uint32_t oq = tid - Q0;                // owned quad in the window
  const uint32_t q = wb0 / 4 + oq;
  const bool owner = tid >= Q0 && oq < wlen / 4;
  const InstDev *ip = d.inst + inst;
  const uint2 rel = d.wrel[blk];               // windows whose senders can reach this one
  uint64_t *const flags = d.lflags;

  // Live rows [t0, t0 + H) into LDS (LDS row r & (H-1) holds row r).  With
  // H < 64 the rows are consumed here, so their device copies are cleared.
  for (uint32_t i = tid; i < uint32_t(H) * WN; i += BS) {
    const uint32_t lr = i / WN, c = i % WN;
    const uint64_t a = t0 + ((uint64_t(lr) - t0) & uint64_t(H - 1));
    int32_t *g = d.W + size_t(a & 63u) * d.ntot + wb0 + c;
    int32_t v = 0;
    if (c < wlen) {
      v = *g;
      if (H < 64) *g = 0;
    }
    s_ring[i] = v;
  }
  if (tid < 8u) {
    const WinClass c = d.wcls[size_t(blk) * NB * 8 + tid];
    s_cf[tid] = c.first;
    s_cn[tid] = c.n;
  }
  for (uint32_t i = tid; i < NB * 8; i += BS) {
    const WinClass c = d.wcls[size_t(blk) * NB * 8 + i];
    s_ccap[i] = c.cap;
    s_cbase[i] = c.base;
  }
  if (tid < 4u) s_ctr[tid] = 0;
  if (tid < NSLOT) s_hn[tid] = 0;
  if (FMT == kBandDev && tid < 16u) {
    s_dq[tid] = ip->dev_mq[tid];
    s_ds[tid] = ip->dev_sq[tid];
  }
  for (uint32_t i = tid; i < rel.y - rel.x; i += BS) s_wstart[i] = d.lwin[rel.x + i].x;
  // Thalamic tables of the window's instance.
  if (tid < 8u) {
    const uint2 m = d.pmeta[inst * 8 + tid];
    const uint32_t off = tid * TS;
    for (uint32_t kk = 0; kk < TS; ++kk) s_thr[off + kk] = kk < m.y ? d.thr[m.x + kk] : 0xFFFFFFFFu;
    s_tlen[tid] = m.y;
  }
  __syncthreads();

  if (tid < NB) {   // group width of each band: the next power of two of its largest capacity
    uint32_t mx = 0;
    for (int c = 0; c < 8; ++c) mx = max(mx, s_cn[c] ? s_ccap[tid * 8 + c] : 0u);
    uint32_t g = 1;
    while (g < mx && g <= 64u) g <<= 1;
    s_gmax[tid] = mx > 64u ? 65u : g;
  }

  float U[4] = {0, 0, 0, 0}, I[4] = {0, 0, 0, 0};
  uint32_t R = 0, c_spk = 0, c_poi = 0, dcode = 0, Tp = 0;
  uint32_t OD[4] = {0, 0, 0, 0};
  int64_t c_con = 0;
  uint64_t c_ev = 0;
  const uint32_t lq = q - ip->gbase / 4;       // quad index in the instance
  if (owner) {
    const float4 uv = ld4(d.U + 4 * size_t(q));
    const float4 iv = ld4(d.I + 4 * size_t(q));
    U[0] = uv.x; U[1] = uv.y; U[2] = uv.z; U[3] = uv.w;
    I[0] = iv.x; I[1] = iv.y; I[2] = iv.z; I[3] = iv.w;
    R = d.R4[q];
    dcode = quad_code(ip, lq);
    const uint4 od = *reinterpret_cast<const uint4 *>(d.outdeg + 4 * size_t(q));
    OD[0] = od.x; OD[1] = od.y; OD[2] = od.z; OD[3] = od.w;
  }
  // Block-uniform values used only by vector arithmetic, and the pointers of
  // rare paths, live in vector registers and leave scalar registers to the
  // loop.
  uint64_t seed = ip->seed;
  Props k{d.consts->p11, d.consts->p22, d.consts->p21};
  int32_t wext = ip->w_ext_q;
  uint32_t wb0v = wb0;
  asm volatile("" : "+v"(seed), "+v"(k.p11), "+v"(k.p22), "+v"(k.p21), "+v"(wext), "+v"(wb0v));
  uint32_t *llist_v = d.llist;
  uint32_t *ghist_v = d.ghist;
  // The 1,024-thread variant (windows of small instances, rarely more than
  // HC senders a step) keeps no private history: its registers are spent.
  constexpr uint32_t PH = BS >= 1024 ? 0u : kBandPrivHist;
  uint32_t *phist_v = PH ? d.phist + size_t(blk) * 64u * PH : nullptr;
  if constexpr (PH > 0) asm volatile("" : "+v"(phist_v));
  uint64_t *raster_v = d.raster;
  Control *ctl_v = d.ctl;
  uint64_t rcap_v = d.raster_cap;
  uint32_t ntot_v = d.ntot;
  uint32_t gbase_v = ip->gbase;
  int32_t *W_v = d.W;
  asm volatile("" : "+v"(llist_v), "+v"(ghist_v), "+v"(raster_v), "+v"(ctl_v), "+v"(rcap_v),
               "+v"(ntot_v), "+v"(gbase_v), "+v"(W_v));
  // Waves 0 and 1 poll the flags, each of half of the windows that can reach
  // this one: flag index read by lane l in poll slot j (~0 past the windows
  // of the instance) and that window's first neuron.
  const bool poller = wave < 2u;
  const uint32_t h = wave & 1u;
  uint32_t pb[NJ], wst[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const uint32_t bb = rel.x + NZH * h + lane + 64u * uint32_t(j);
    pb[j] = bb < rel.y ? bb : ~0u;
    wst[j] = bb < rel.y ? d.lwin[bb].x : 0u;
  }
  __syncthreads();

  // Flushes the staged raster entries to the device raster.
  uint32_t rn = 0;
  auto flush = [&]() {
    if (tid == 0)
      s_rbase = atomicAdd(reinterpret_cast<unsigned long long *>(&ctl_v->raster_n),
                          (unsigned long long)rn);
    __syncthreads();
    for (uint32_t i = tid; i < rn; i += BS) {
      const uint64_t pos = s_rbase + i;
      if (pos < rcap_v)
        raster_v[pos] = s_rast[i];
      else
        ctl_v->overflow = 1;
    }
    __syncthreads();
    rn = 0;
  };

  // Thalamic counts T_t of the owner's quad (Sec. 2.2: T ~ Poisson(v_th K
  // dt)), one byte per neuron: one Philox4x32-10 block per quad and step,
  // each word turned into a count by its population's inverse-CDF table.
  auto draw = [&](uint64_t t) -> uint32_t {
    // The key, the counter word and the population codes pass through opaque
    // copies at every draw, so that the round keys, the first round's product
    // and the table addresses are formed here instead of being hoisted out of
    // the step loop (about thirty registers held across the loop, spilled to
    // scratch in the 1,024-thread variant).
    uint32_t k0 = uint32_t(seed), k1 = uint32_t(seed >> 32), c0 = lq, dc = dcode;
    asm volatile("" : "+v"(k0), "+v"(k1), "+v"(c0), "+v"(dc));
    if (!(dc >> 12)) return 0u;   // no real neuron in the quad
    const Philox4 x = philox4x32_10(c0, uint32_t(t), uint32_t(t >> 32), kStreamThalamic, k0, k1);
    uint32_t tp = 0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const uint32_t pm = (dc >> (3 * m)) & 7u;
      const uint4 *tb = reinterpret_cast<const uint4 *>(s_thr + pm * TS);
      const uint4 lo = tb[0], hi = tb[1];
      const uint32_t len = s_tlen[pm];
      const uint32_t u = x.v[m];
      // Entries past a table's length hold ~0, which no word below ~0
      // reaches; the word ~0 reaches every entry, so its count is the length.
      const uint32_t v[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
      uint32_t c = 0;
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) c += u >= v[kk] ? 1u : 0u;
      c = u == ~0u ? len : c;
      if (c == 8u) {   // rare: the count continues in the table
        const uint32_t *tab = s_thr + pm * TS;
        while (c < len && u >= tab[c]) ++c;
      }
      tp |= (((dc >> (12 + m)) & 1u) ? c : 0u) << (8 * m);
    }
    return tp;
  };

  // Class of a sender id: populations are contiguous and in order, so it is
  // the last non-empty class starting at or before gid.
  auto sender_class = [&](uint32_t gid) -> uint32_t {
    uint32_t ci = 0;
#pragma unroll
    for (int c = 1; c < 8; ++c)
      if (gid >= s_cf[c] && s_cn[c]) ci = uint32_t(c);
    return ci;
  };
  // Sender k of step s from the history: the first HC in LDS, the next PH
  // in the block's own device memory (written and read by this block only,
  // ordered by its barriers), the rest in the instance's shared history.
  auto hist = [&](uint64_t s, uint32_t kk) -> uint32_t {
    if (kk < uint32_t(HC)) return s_hist[uint32_t(s % NSLOT) * HC + kk];
    if (kk < uint32_t(HC) + PH) return phist_v[(size_t(s & 63u)) * PH + (kk - uint32_t(HC))];
    return ld_ag(ghist_v + size_t(s & 63u) * ntot_v + gbase_v + kk);
  };

  bool alive = true;
  for (uint32_t it = 0; it <= n_steps; ++it) {
    const uint64_t t = t0 + it;
    const bool decide = it < n_steps;
    const uint32_t ep = ep0 + it + 1;          // epoch of step t's flags
    const uint32_t epp = ep - 1;               // epoch of step t-1's flags
    const uint64_t *fs = flags + size_t(epp % kSlots) * GT;

    // The polling waves issue the flag loads of step t-1 now; they are
    // checked after the slow bands.
    uint64_t fv[NJ];
    if (poller && it > 0) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) fv[j] = pb[j] != ~0u ? ld_ag(fs + pb[j]) : 0ull;
    }
    // Row t + H - 1 enters the horizon in this iteration; in the first 64 - H
    // iterations of a launch it may hold deliveries made before the launch.
    const bool pulling = H < 64 && it > 0 && it <= 64u - uint32_t(H);
    int4 pull = make_int4(0, 0, 0, 0);
    int4 *prow = nullptr;
    if (pulling && owner) {
      prow = reinterpret_cast<int4 *>(W_v + size_t((t + H - 1) & 63u) * ntot_v + wb0v + 4 * oq);
      pull = *prow;
    }

    // (a) complete step t-1 from ring row t-1 and T_{t-1}; the LDS row then
    // becomes row t + H - 1.
    if (it > 0 && owner) {
      int4 *row = reinterpret_cast<int4 *>(s_ring + uint32_t((t - 1) & (H - 1)) * WN + 4 * oq);
      const int4 wv = *row;
      *row = pull;
      if (pulling) *prow = make_int4(0, 0, 0, 0);
      const int32_t W4[4] = {wv.x, wv.y, wv.z, wv.w};
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int32_t T = int32_t((Tp >> (8 * m)) & 0xFFu);
        I[m] = next_current(I[m], T, wext, W4[m], k.p11);
      }
      c_con += int64_t(W4[0]) + W4[1] + W4[2] + W4[3];
      c_poi += __builtin_amdgcn_sad_u8(Tp, 0u, 0u);
    }

    // (b) decide step t and publish its senders: raster entries, the window
    // offsets of the first NI spikes in the flag word, list entries for the
    // others, then the flag.
    if (decide) {
      const uint32_t fl = owner ? lif_quad_padded(k, U, I, R) : 0u;
      uint32_t lo, tot;
      wave_compact(fl, lo, tot);
      if (lane == 0) s_wave[wave] = tot;
      __syncthreads();
      uint32_t before = 0, cnt = 0;
#pragma unroll
      for (uint32_t w = 0; w < NW; ++w) {
        const uint32_t c = __builtin_amdgcn_readfirstlane(s_wave[w]);
        before += w < wave ? c : 0u;
        cnt += c;
      }
      if (rn + cnt > RC) flush();              // block-uniform
      const bool direct = cnt > RC;            // a burst larger than the staging area
      if (direct) {
        if (tid == 0)
          s_rbase = atomicAdd(reinterpret_cast<unsigned long long *>(&ctl_v->raster_n),
                              (unsigned long long)cnt);
        __syncthreads();
      }
      if (fl) {
        uint32_t p = before + lo;
        uint32_t *lst = llist_v + size_t(ep % kSlots) * ntot_v + wb0;
        c_spk += __popc(fl);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          if (!((fl >> m) & 1u)) continue;
          const uint32_t loc = 4 * oq + uint32_t(m);
          if (p < F::NI)
            s_inl[p] = loc;
          else
            st_ag(lst + p, loc);
          const uint64_t e = (t << 32) | (wb0 + loc);
          if (!direct) {
            s_rast[rn + p] = e;
          } else {
            const uint64_t pos = s_rbase + p;
            if (pos < rcap_v)
              raster_v[pos] = e;
            else
              ctl_v->overflow = 1;
          }
          uint32_t od = OD[m];   // opaque: keeps the 64-bit widening out of the loop
          asm volatile("" : "+v"(od));
          c_ev += od;
          ++p;
        }
      }
      if (cnt) {   // block-uniform
        // List entries must be performed before the flag that announces them.
        if (cnt > F::NI) __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
        __syncthreads();
      }
      // Wave 2 stores the flag: a wave's vector memory operations complete in
      // order, so a polling wave would otherwise wait for the store's
      // acknowledgement before it could read any flag.
      if (tid == 128) {
        uint64_t f = F::word(ep, cnt);
        for (uint32_t kk = 0; kk < F::NI && kk < cnt; ++kk) f |= F::inline_sender(kk, s_inl[kk]);
        st_ag(flags + size_t(ep % kSlots) * GT + blk, f);
      }
      if (!direct) rn += cnt;
    }

    if (it == 0) {   // nothing to deliver yet
      if (decide && owner) Tp = draw(t);     // T_t, used when step t completes
      __syncthreads();
      continue;
    }
    // Deliveries may land in the row (a) has just turned over.
    if (!decide) __syncthreads();

    // (c1) slow bands: band j of the senders of step t - lo_j, decided in
    // this launch (earlier steps' bands were delivered when their launch
    // ended).  The bands' senders are concatenated; sender m of the batch
    // goes to wave m mod NW.
    {
      uint32_t nj[NB], total = 0;
#pragma unroll
      for (uint32_t j = 1; j < NB; ++j) {
        const uint32_t lo_j = band_lo(j, H);
        nj[j] = it >= lo_j ? s_hn[uint32_t((t - lo_j) % NSLOT)] : 0u;
        total += nj[j];
      }
      uint32_t gs = 1;
#pragma unroll
      for (uint32_t j = 1; j < NB; ++j) gs = max(gs, s_gmax[j]);
      for (uint32_t m0 = 0; m0 < total; m0 += SB) {
        const uint32_t nb = min(SB, total - m0);
        const uint32_t n_l = nb > wave ? (nb - wave + NW - 1u) / NW : 0u;
        uint64_t base = 0;
        uint32_t cap = 0, rb = 0, cl = 0;
        if (lane < n_l) {
          uint32_t m = m0 + wave + NW * lane, j = 1;
#pragma unroll
          for (uint32_t jj = 1; jj + 1 < NB; ++jj)
            if (j == jj && m >= nj[jj]) {
              m -= nj[jj];
              j = jj + 1;
            }
          const uint64_t s = t - band_lo(j, H);
          const uint32_t gid = hist(s, m);
          const uint32_t ci = sender_class(gid);
          cap = gid - s_cf[ci] < s_cn[ci] ? s_ccap[j * 8 + ci] : 0u;
          base = s_cbase[j * 8 + ci] + uint64_t(gid - s_cf[ci]) * cap;
          rb = uint32_t(s) + (FMT != kBandPlain ? band_lo(j, H) : 0u);
          cl = ci;
        }
        BandWalk<FMT, UR, H, PACK> bw;
        bw.begin(base, cap, rb, n_l, gs, cl);
        while (bw.more()) {
          bw.load(d);
          bw.template apply<WN>(s_ring, wb0v, s_dq, s_ds);
        }
      }
    }

    // (c2) waves 0 and 1 wait for step t-1's flags of their windows and
    // stage their senders; the quad owners draw T_t meanwhile.
    if (poller) {
      uint32_t spins = 0;
      bool ok = true;
      for (;;) {
        bool mine = true;
#pragma unroll
        for (int j = 0; j < NJ; ++j)
          mine = mine && (pb[j] == ~0u || (uint32_t(fv[j]) & 0xFFFFu) == (epp & 0xFFFFu));
        if (__all(mine)) break;
        __builtin_amdgcn_s_sleep(1);
#pragma unroll
        for (int j = 0; j < NJ; ++j)   // reload every flag of the lane: one round trip
          if (pb[j] != ~0u) fv[j] = ld_ag(fs + pb[j]);
        if ((++spins & 63u) == 0 && (ld_ag(&ctl_v->error) != 0 || spins > spin_limit)) {
          if (lane == 0) st_ag(&ctl_v->error, 2u);
          ok = false;
          break;
        }
      }
      // Number of each lane's first sender in this wave's sender set.
      uint32_t sc = 0;
#pragma unroll
      for (int j = 0; j < NJ; ++j) sc += F::count(fv[j]);
      uint32_t all_s, all_nz = 0;
      const uint32_t ps0 = wave_prefix(sc, all_s);
      uint32_t *const sid = s_sid + kSBH * h;
      if (all_s > kSBH) {   // wave-uniform
        // Senders past the first kSBH are found by search over the windows
        // with senders, in window order, with their first sender's number.
        uint32_t nzc = 0;
#pragma unroll
        for (int j = 0; j < NJ; ++j) nzc += F::count(fv[j]) ? 1u : 0u;
        uint32_t pz = wave_prefix(nzc, all_nz);
        uint32_t ps = ps0;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          const uint32_t c = F::count(fv[j]);
          if (c) {
            s_nzf[NZH * h + pz] = fv[j];
            s_nzp[NZH * h + pz] = ps;
            s_nzb[NZH * h + pz] = uint16_t(NZH * h + lane + 64u * uint32_t(j));
            ++pz;
            ps += c;
          }
        }
      }
      // The first kSBH senders, expanded: gid for inline ones, else a list
      // marker.
      uint32_t ps = ps0;
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const uint32_t c = F::count(fv[j]);
        const uint32_t src = NZH * h + lane + 64u * uint32_t(j);
        for (uint32_t kk = 0; kk < c && ps < kSBH; ++kk, ++ps)
          sid[ps] = kk < F::NI ? wst[j] + F::local(fv[j], kk) : (1u << 31) | (src << 12) | kk;
      }
      if (lane == 0) {
        s_nnz[h] = all_nz;
        s_n[h] = all_s;
        s_flag[h] = ok ? 1u : 0u;
      }
    } else if (decide && owner) {
      // The other waves draw T_t meanwhile (used when step t completes).
      Tp = draw(t);
    }
    __syncthreads();

    if (!__builtin_amdgcn_readfirstlane(s_flag[0] & s_flag[1])) {
      alive = false;
      break;
    }
    // (c3) band 0 of step t-1's senders; their ids go to the history.
    const uint32_t n0 = __builtin_amdgcn_readfirstlane(s_n[0]);
    const uint32_t n_prev = n0 + __builtin_amdgcn_readfirstlane(s_n[1]);
    const uint32_t g0 = s_gmax[0];
    const uint64_t tsrc = t - 1;
    const uint32_t hslot = uint32_t(tsrc % NSLOT);
    if (tid == 0) s_hn[hslot] = n_prev;
    for (uint32_t j0 = 0; j0 < n_prev; j0 += SB) {
      const uint32_t nb = min(SB, n_prev - j0);
      const uint32_t n_l = nb > wave ? (nb - wave + NW - 1u) / NW : 0u;
      uint64_t base = 0;
      uint32_t cap = 0, cl = 0;
      if (lane < n_l) {
        // Senders of polling wave 0 come first, then those of wave 1.
        const uint32_t j = j0 + wave + NW * lane;
        const uint32_t hs = j < n0 ? 0u : 1u;
        const uint32_t gid = band_sender_gid<F>(llist_v, ntot_v, j - (hs ? n0 : 0u), s_nnz[hs],
                                                epp % kSlots, s_sid + kSBH * hs, s_nzf + NZH * hs,
                                                s_nzp + NZH * hs, s_nzb + NZH * hs, s_wstart);
        if (j < uint32_t(HC))
          s_hist[hslot * HC + j] = gid;
        else if (j < uint32_t(HC) + PH)
          phist_v[size_t(tsrc & 63u) * PH + (j - uint32_t(HC))] = gid;
        else
          st_ag(ghist_v + size_t(tsrc & 63u) * ntot_v + gbase_v + j, gid);
        const uint32_t ci = sender_class(gid);
        cap = gid - s_cf[ci] < s_cn[ci] ? s_ccap[ci] : 0u;
        base = s_cbase[ci] + uint64_t(gid - s_cf[ci]) * cap;
        cl = ci;
      }
      BandWalk<FMT, UR, H, PACK> bw;
      bw.begin(base, cap, uint32_t(tsrc) + (FMT != kBandPlain ? 1u : 0u), n_l, g0, cl);
      while (bw.more()) {
        bw.load(d);
        bw.template apply<WN>(s_ring, wb0v, s_dq, s_ds);
      }
    }
    __syncthreads();
  }

  // End of the launch: the slow bands still pending -- band j of step s with
  // s + lo_j > t_end -- are delivered now (into LDS rows inside the horizon,
  // device rows beyond it).  Pairs (s, j) go to waves round robin.
  __syncthreads();
  if (alive) {
    uint32_t pair = 0;
#pragma unroll 1
    for (uint32_t j = 1; j < NB; ++j) {
      const uint32_t lo_j = band_lo(j, H);
      const uint64_t s_first = t_end >= lo_j - 1 + t0 ? t_end - (lo_j - 1) : t0;
#pragma unroll 1
      for (uint64_t s = s_first; s < t_end; ++s, ++pair) {
        if (pair % NW != wave) continue;
        const uint32_t n = s_hn[uint32_t(s % NSLOT)];
        const uint32_t gj = s_gmax[j];
        for (uint32_t k0 = 0; k0 < n; k0 += 64) {
          const uint32_t n_l = min(64u, n - k0);
          uint64_t base = 0;
          uint32_t cap = 0, cl = 0;
          if (lane < n_l) {
            const uint32_t gid = hist(s, k0 + lane);
            const uint32_t ci = sender_class(gid);
            cap = gid - s_cf[ci] < s_cn[ci] ? s_ccap[j * 8 + ci] : 0u;
            base = s_cbase[j * 8 + ci] + uint64_t(gid - s_cf[ci]) * cap;
            cl = ci;
          }
          BandWalk<FMT, UR, H, PACK> bw;
          bw.begin(base, cap, uint32_t(s) + (FMT != kBandPlain ? lo_j : 0u), n_l, gj, cl);
          while (bw.more()) {
            bw.load(d);
            bw.template apply_flush<WN>(s_ring, W_v, ntot_v, wb0v, uint32_t(t_end), s_dq, s_ds);
          }
        }
      }
    }
  }
  __syncthreads();

  // Raster, live ring rows, state and counters back to memory.
  if (rn) flush();
  for (uint32_t i = tid; i < uint32_t(H) * WN; i += BS) {
    const uint32_t lr = i / WN, c = i % WN;
    const uint64_t a = t_end + ((uint64_t(lr) - t_end) & uint64_t(H - 1));
    if (c < wlen) d.W[size_t(a & 63u) * d.ntot + wb0 + c] = s_ring[i];
  }
  if (owner) {
    *reinterpret_cast<float4 *>(d.U + 4 * size_t(q)) = make_float4(U[0], U[1], U[2], U[3]);
    *reinterpret_cast<float4 *>(d.I + 4 * size_t(q)) = make_float4(I[0], I[1], I[2], I[3]);
    d.R4[q] = R;
  }
  {
    uint64_t sp = c_spk, po = c_poi, ev = c_ev;
    int64_t co = c_con;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      sp += __shfl_xor(sp, o);
      po += __shfl_xor(po, o);
      ev += __shfl_xor(ev, o);
      co += __shfl_xor(co, o);
    }
    if (lane == 0 && wave >= Q0 / 64) {
      atomicAdd(reinterpret_cast<unsigned long long *>(&s_ctr[0]), (unsigned long long)sp);
      atomicAdd(reinterpret_cast<unsigned long long *>(&s_ctr[1]), (unsigned long long)po);
      atomicAdd(reinterpret_cast<unsigned long long *>(&s_ctr[2]), (unsigned long long)co);
      atomicAdd(reinterpret_cast<unsigned long long *>(&s_ctr[3]), (unsigned long long)ev);
    }
  }
  __syncthreads();
  if (tid < 4u) d.blk_ctr[size_t(blk) * 4 + tid] += s_ctr[tid];
  __builtin_amdgcn_s_waitcnt(0x0F70);
  __syncthreads();
  if (tid == 0) {
    unsigned int *exits = &d.lgroup[0].y;
    const uint32_t done = __hip_atomic_fetch_add(exits, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (done == gridDim.x - 1) {
      st_ag(exits, 0u);
      st_ag(&d.lgroup[0].x, ep0 + n_steps);
      st_ag(&d.ctl->t_base, t_end);
    }
  }
}

using BandFn = void (*)(DeviceNet, uint32_t, uint32_t);

template <int FMT>
BandFn band_fn_of(uint32_t v) {
  switch (v) {
    case 0: return k_band<256, 320, 64, 512, FMT>;
    case 1: return k_band<256, 512, 64, 256, FMT>;
    case 2: return k_band<512, 1536, 16, 128, FMT>;
    case 3: return k_band<1024, 3584, 8, 32, FMT>;
    default: return nullptr;
  }
}

}  // namespace

const BandVariant kBandVariants[kNumBandVariants] = {
    {256, 320, 64, 512}, {256, 512, 64, 256}, {512, 1536, 16, 128}, {1024, 3584, 8, 32}};

int band_max_grid(uint32_t variant) {
  BandFn fn = band_fn_of<kBandPlain>(variant);
  if (!fn) return 0;
  int per_cu = 0, dev = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(fn),
                                                   int(kBandVariants[variant].block), 0) != hipSuccess)
    return 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
  return std::min<int>(std::min(per_cu, 1) * prop.multiProcessorCount, int(kLdsMaxGrid));
}

hipError_t launch_band(const DeviceNet &d, uint32_t variant, uint32_t n, hipStream_t s) {
  BandFn fn = d.syn_format == SNN_SYN_COMPRESSED5 ? band_fn_of<kBandComp>(variant)
             : d.syn_format == SNN_SYN_DEV8      ? band_fn_of<kBandDev>(variant)
                                                 : band_fn_of<kBandPlain>(variant);
  if (!fn || d.n_lwin == 0 || d.n_lwin > kLdsMaxGrid || d.band_h != kBandVariants[variant].h)
    return hipErrorInvalidConfiguration;
  DeviceNet dv = d;
  uint32_t steps = n;
  uint32_t spin = 1u << 24;
  void *args[] = {&dv, &steps, &spin};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(fn), dim3(d.n_lwin),
                                    dim3(kBandVariants[variant].block), args, 0, s);
}

}  // namespace snn
