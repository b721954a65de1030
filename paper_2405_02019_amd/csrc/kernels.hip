// kernels.hip -- CDNA4 (gfx950) kernels of the clock-driven microcircuit
// simulation: FP64 propagators, the neuron update with Philox thalamic drive
// and wave-ballot spike compaction, and the push transfer of every spike's
// synapses into the int32 delay ring buffer.
//
// Numerics: FP32 state, every product and sum rounded on its own (the file is
// compiled with -ffp-contract=off, denormals kept), synaptic input summed as
// exact int32 in 2^-8 pA, so the order in which atomics land cannot change
// the result.
//
// Latency, not bandwidth, bounds one microcircuit step (a few hundred KB of
// traffic), so the kernels are built to keep every memory round trip off the
// dependent chain: thalamic tables sit in LDS and are scanned eight entries at
// a time, and each thread issues the record loads of all its synapses before
// any of their atomics.
#include "device.hpp"

namespace snn {

// ---------------------------------------------------------------------------
// Propagators (Sec. 2.2, eqn:p11p22, eqn:p21), FP64 on the device.
// ---------------------------------------------------------------------------
__global__ void k_propagators(double cm, double tau_m, double tau_s, double h, DevConsts *out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const double p11 = exp(-h / tau_s);
  const double p22 = exp(-h / tau_m);
  const double beta = tau_s * tau_m / (tau_m - tau_s);
  const double p21 = p11 * (beta / cm) * (exp(h / beta) - 1.0);
  out->p11d = p11;
  out->p22d = p22;
  out->p21d = p21;
  out->padd = 0.0;
  out->p11 = float(p11);
  out->p22 = float(p22);
  out->p21 = float(p21);
  out->pad = 0.0f;
}

hipError_t launch_propagators(const DeviceNet &d, hipStream_t s) {
  hipLaunchKernelGGL(k_propagators, dim3(1), dim3(64), 0, s, 250.0, 10.0, 0.5, 0.1, d.consts);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Shared pieces of the neuron update.
// ---------------------------------------------------------------------------
// Thalamic tables in LDS (or straight from global memory when the batch's
// tables are too large); copied by the whole block.
struct ThrTables {
  uint32_t thr[kThrLds + 8];
  uint2 meta[kMetaLds];
};

template <bool LDS>
__device__ __forceinline__ void stage_tables(const DeviceNet &d, ThrTables &s) {
  if (!LDS) return;
  for (uint32_t i = threadIdx.x; i < d.nthr + 8; i += blockDim.x) s.thr[i] = d.thr[i];
  for (uint32_t i = threadIdx.x; i < d.n_inst * 8; i += blockDim.x) s.meta[i] = d.pmeta[i];
}

// T = #{k < len : u >= thr[off + k]} for a sorted table (m = (off, len)).
// The first eight entries are read unconditionally (tables are padded by 8),
// so the loads do not depend on each other; longer counts (P ~ 1e-4 at the
// model's rates) continue one entry at a time.
__device__ __forceinline__ uint32_t thalamic_count(const uint32_t *tab, uint2 m, uint32_t u) {
  uint32_t T = 0;
#pragma unroll
  for (uint32_t k = 0; k < 8; ++k) {
    const uint32_t v = tab[m.x + k];
    T += (k < m.y && u >= v) ? 1u : 0u;
  }
  if (T == 8u) {
    while (T < m.y && u >= tab[m.x + T]) ++T;
  }
  return T;
}

// eqn:mem and eqn:ref for step t: the membrane update of the quad's real
// neurons (bit 12 + m of code).  Returns a 4-bit spike mask.
__device__ __forceinline__ uint32_t lif_quad(uint32_t code, Props k, float (&u)[4],
                                             const float (&i)[4], uint32_t &r4) {
  uint32_t flags = 0, rout = 0;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    uint32_t r = (r4 >> (8 * m)) & 0xFFu;
    if ((code >> (12 + m)) & 1u) {
      if (r == 0) {
        const float a = k.p22 * u[m];
        const float b = k.p21 * i[m];
        float xm = a + b;
        if (xm >= kTheta) {
          flags |= 1u << m;
          xm = 0.0f;
          r = kRefSteps;
        }
        u[m] = xm;
      } else {
        u[m] = 0.0f;
        r -= 1;
      }
    }
    rout |= r << (8 * m);
  }
  r4 = rout;
  return flags;
}

// Step t of a quad: the thalamic counts T_t (packed one byte per neuron into
// tp, their sum added to tsum) and the membrane update.  tab/meta hold the
// thalamic tables; meta[mbase + population] = (offset, length).
__device__ __forceinline__ uint32_t decide_quad(const uint32_t *tab, const uint2 *meta,
                                                uint32_t mbase, uint64_t seed, uint32_t lq,
                                                uint32_t code, uint64_t t, Props k,
                                                float (&u)[4], const float (&i)[4], uint32_t &r4,
                                                uint32_t &tp, uint32_t &tsum) {
  const Philox4 x = philox4x32_10(lq, uint32_t(t), uint32_t(t >> 32), kStreamThalamic,
                                  uint32_t(seed), uint32_t(seed >> 32));
  uint32_t tpk = 0;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    if ((code >> (12 + m)) & 1u) {
      const uint2 mt = meta[mbase + ((code >> (3 * m)) & 7u)];
      const uint32_t T = thalamic_count(tab, mt, x.v[m]);
      tpk |= T << (8 * m);
      tsum += T;
    }
  }
  tp = tpk;
  return lif_quad(code, k, u, i, r4);
}

template <int BS>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *s_tmp,
                                                         uint32_t &total) {
  constexpr int NW = BS / 64;
  const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o);
    if (lane >= uint32_t(o)) x += y;
  }
  if (lane == 63) s_tmp[wave] = x;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const uint32_t c = s_tmp[w];
    before += uint32_t(w) < wave ? c : 0u;
    all += c;
  }
  __syncthreads();
  total = all;
  return before + x - v;
}

// ---------------------------------------------------------------------------
// Push transfer of one batch of staged segments (lst:push2): synapse e of the
// concatenated segments goes to thread e mod TT.  Each thread first locates
// and loads up to 8 of its records, then issues their atomics, so one record
// round trip covers them all.  Delay d lands in row (t_src + d) mod 64.
// ---------------------------------------------------------------------------
struct SegStage {
  uint64_t start;
  uint32_t len;
  uint32_t tbase;
};

template <bool COMP>
__device__ __forceinline__ void deliver_batch(const DeviceNet &d, uint64_t t_src,
                                              const SegStage *s_seg, const uint32_t *s_excl,
                                              uint32_t nb, uint32_t total, uint32_t gt,
                                              uint32_t TT) {
  constexpr int U = 8;
  for (uint32_t e0 = gt; e0 < total; e0 += TT * U) {
    uint64_t idx[U];
    uint32_t tb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t e = e0 + uint32_t(u) * TT;
      idx[u] = ~0ull;
      tb[u] = 0;
      if (e < total) {
        uint32_t lo = 0, hi = nb;
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) >> 1;
          if (s_excl[mid] <= e) lo = mid; else hi = mid;
        }
        idx[u] = s_seg[lo].start + (e - s_excl[lo]);
        tb[u] = s_seg[lo].tbase;
      }
    }
    uint32_t tgt[U], dl[U];
    int32_t wq[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      tgt[u] = 0;
      dl[u] = 0;
      wq[u] = 0;
      if (idx[u] != ~0ull) {
        if (COMP) {
          tgt[u] = tb[u] + d.tgt16[idx[u]];
          wq[u] = int32_t(d.w16[idx[u]]) * 8;
          dl[u] = d.d8[idx[u]];
        } else {
          const uint64_t rec = d.rec8[idx[u]];
          const uint32_t hiw = uint32_t(rec >> 32);
          wq[u] = int32_t(uint32_t(rec));
          tgt[u] = hiw >> 6;
          dl[u] = hiw & 63u;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (idx[u] != ~0ull)
        atomicAdd(d.W + size_t((t_src + dl[u]) & (kRing - 1)) * d.ntot + tgt[u], wq[u]);
  }
}

// ---------------------------------------------------------------------------
// Stepwise engine, kernel 1 of 2: update every neuron for step t, read and
// clear ring row t, append spikes to the step's sender list and the raster.
// ---------------------------------------------------------------------------
template <int BS, bool LDS>
__global__ __launch_bounds__(BS) void k_update(DeviceNet d, uint32_t k_step) {
  constexpr int NW = BS / 64;
  __shared__ ThrTables s_tab;
  __shared__ uint32_t s_wave[NW];
  __shared__ uint32_t s_base;
  __shared__ unsigned long long s_rbase;
  stage_tables<LDS>(d, s_tab);
  const uint64_t t = d.ctl->t_base + k_step;
  const uint32_t slot = uint32_t(t & 1u);
  const uint32_t q = blockIdx.x * BS + threadIdx.x;
  const uint32_t wave = threadIdx.x >> 6;
  if (blockIdx.x == 0 && threadIdx.x == 0) d.ctl->spk_cnt[slot ^ 1u] = 0;
  __syncthreads();

  uint32_t flags = 0, tsum = 0, gid0 = 0;
  int64_t consumed = 0;
  if (q < d.nquads) {
    const uint32_t qi = d.qinfo[q];
    const uint32_t inst = __builtin_amdgcn_readfirstlane(qi >> 24);
    const InstDev *ip = d.inst + inst;
    const uint32_t lq = qi & 0xFFFFFFu;
    const DevConsts *kc = d.consts;
    const Props k{kc->p11, kc->p22, kc->p21};
    int32_t *wrow = d.W + size_t(t & (kRing - 1)) * d.ntot;
    const int4 w4 = reinterpret_cast<const int4 *>(wrow)[q];
    reinterpret_cast<int4 *>(wrow)[q] = make_int4(0, 0, 0, 0);
    const float4 uv = ld4(d.U + 4 * size_t(q));
    const float4 iv = ld4(d.I + 4 * size_t(q));
    float u[4] = {uv.x, uv.y, uv.z, uv.w};
    float i[4] = {iv.x, iv.y, iv.z, iv.w};
    const int32_t w[4] = {w4.x, w4.y, w4.z, w4.w};
    uint32_t r4 = d.R4[q], tp = 0;
    const uint32_t code = quad_code(ip, lq);
    flags = decide_quad(LDS ? s_tab.thr : d.thr, LDS ? s_tab.meta : d.pmeta, inst * 8u, ip->seed,
                        lq, code, t, k, u, i, r4, tp, tsum);
    const int32_t wext = ip->w_ext_q;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      if ((code >> (12 + m)) & 1u) {
        i[m] = next_current(i[m], int32_t((tp >> (8 * m)) & 0xFFu), wext, w[m], k.p11);
        consumed += w[m];
      }
    }
    *reinterpret_cast<float4 *>(d.U + 4 * size_t(q)) = make_float4(u[0], u[1], u[2], u[3]);
    *reinterpret_cast<float4 *>(d.I + 4 * size_t(q)) = make_float4(i[0], i[1], i[2], i[3]);
    d.R4[q] = r4;
    gid0 = 4 * q;
  }

  // Per-wave counters: one slot per 64 quads (a wave never spans instances).
  uint32_t lane_off, wtot;
  wave_compact(flags, lane_off, wtot);
  {
    uint64_t ts = tsum;
    int64_t cs = consumed;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      ts += __shfl_xor(ts, o);
      cs += __shfl_xor(cs, o);
    }
    if (__lane_id() == 0 && (q >> 6) < (d.nquads >> 6)) {
      int64_t *c = d.wave_ctr + 4 * size_t(q >> 6);
      c[0] += wtot;
      c[1] += int64_t(ts);
      c[2] += cs;
    }
  }
  if (__lane_id() == 0) s_wave[wave] = wtot;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int w = 0; w < NW; ++w) {
      const uint32_t c = s_wave[w];
      s_wave[w] = run;
      run += c;
    }
    if (run) {
      s_base = atomicAdd(&d.ctl->spk_cnt[slot], run);
      s_rbase = atomicAdd(reinterpret_cast<unsigned long long *>(&d.ctl->raster_n),
                          (unsigned long long)run);
    }
  }
  __syncthreads();
  if (flags) {
    uint32_t o = s_wave[wave] + lane_off;
    for (int j = 0; j < 4; ++j) {
      if (!((flags >> j) & 1u)) continue;
      const uint32_t gid = gid0 + uint32_t(j);
      d.spk_list[size_t(slot) * d.ntot + s_base + o] = gid;
      const uint64_t pos = s_rbase + o;
      if (pos < d.raster_cap)
        d.raster[pos] = (t << 32) | gid;
      else
        d.ctl->overflow = 1;
      ++o;
    }
  }
}

// ---------------------------------------------------------------------------
// Stepwise engine, kernel 2 of 2: push transfer of the senders of step t.
// Every block stages the senders' storage segments in LDS with an exclusive
// prefix over their lengths, then the whole grid shares the concatenated
// synapse range (deliver_batch).
// ---------------------------------------------------------------------------
constexpr int kSegCap = 1024;

template <int BS, bool COMP>
__global__ __launch_bounds__(BS) void k_transfer(DeviceNet d, uint32_t k_step) {
  constexpr int IPT = kSegCap / BS;
  __shared__ SegStage s_seg[kSegCap];
  __shared__ uint32_t s_excl[kSegCap];
  __shared__ uint32_t s_tmp[BS / 64];
  const uint64_t t = d.ctl->t_base + k_step;
  const uint32_t slot = uint32_t(t & 1u);
  const uint32_t n = d.ctl->spk_cnt[slot];
  if (n == 0) return;
  const uint32_t nwin = d.nwin_max;
  const uint32_t per_batch = kSegCap / nwin;
  const uint32_t *list = d.spk_list + size_t(slot) * d.ntot;

  for (uint32_t b0 = 0; b0 < n; b0 += per_batch) {
    const uint32_t nb = min(per_batch, n - b0);
    const uint32_t nseg = nb * nwin;
    uint32_t len[IPT];
    uint32_t mysum = 0;
#pragma unroll
    for (int m = 0; m < IPT; ++m) {
      const uint32_t s = threadIdx.x * IPT + m;
      len[m] = 0;
      if (s < nseg) {
        const uint32_t sp = s / nwin, win = s - sp * nwin;
        const uint32_t gid = list[b0 + sp];
        const uint32_t inst = d.qinfo[gid >> 2] >> 24;
        const InstDev *ip = d.inst + inst;
        const uint32_t local = gid - ip->gbase;
        const uint32_t inw = ip->nwin;
        uint64_t st = 0;
        if (win < inw) {
          const uint64_t sg = uint64_t(ip->seg_base) + uint64_t(local) * inw + win;
          st = d.seg_ptr[sg];
          len[m] = uint32_t(d.seg_ptr[sg + 1] - st);
          if (blockIdx.x == 0 && win == 0) {
            const uint64_t row = d.seg_ptr[sg + inw] - st;
            atomicAdd(reinterpret_cast<unsigned long long *>(d.events + inst),
                      (unsigned long long)row);
          }
        }
        s_seg[s].start = st;
        s_seg[s].len = len[m];
        s_seg[s].tbase = ip->tbase0 + win * ip->win_size;
      }
      mysum += len[m];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan<BS>(mysum, s_tmp, total);
#pragma unroll
    for (int m = 0; m < IPT; ++m) {
      const uint32_t s = threadIdx.x * IPT + m;
      if (s < nseg) s_excl[s] = run;
      run += len[m];
    }
    __syncthreads();
    deliver_batch<COMP>(d, t, s_seg, s_excl, nseg, total, blockIdx.x * BS + threadIdx.x,
                        gridDim.x * BS);
    __syncthreads();
  }
}

__global__ void k_advance(Control *ctl, uint32_t n) {
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->t_base += n;
}

__global__ void k_reset_raster(Control *ctl) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->raster_n = 0;
    ctl->overflow = 0;
  }
}

hipError_t launch_reset_raster(const DeviceNet &d, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_raster, dim3(1), dim3(64), 0, s, d.ctl);
  return hipGetLastError();
}

hipError_t launch_stepwise(const DeviceNet &d, const LaunchShape &sh, uint32_t n, hipStream_t s) {
  constexpr int BS = 256;
  const uint32_t ublocks = (d.nquads + BS - 1) / BS;
  for (uint32_t k = 0; k < n; ++k) {
    if (d.thr_lds)
      hipLaunchKernelGGL((k_update<BS, true>), dim3(ublocks), dim3(BS), 0, s, d, k);
    else
      hipLaunchKernelGGL((k_update<BS, false>), dim3(ublocks), dim3(BS), 0, s, d, k);
    if (d.syn_format == SNN_SYN_COMPRESSED5)
      hipLaunchKernelGGL((k_transfer<BS, true>), dim3(sh.scatter_blocks), dim3(BS), 0, s, d, k);
    else
      hipLaunchKernelGGL((k_transfer<BS, false>), dim3(sh.scatter_blocks), dim3(BS), 0, s, d, k);
  }
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, d.ctl, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Persistent engine: one cooperative launch runs a chunk of steps with one
// grid-wide barrier per step.
//
// Iteration `it` (step t = t0 + it) of every block:
//   (a) completes step t-1 for the block's neurons: reads and clears ring row
//       t-1 with device-coherent loads and stores, I_t = p11 I + (T w + W) 2^-8;
//   (b) decides step t (eqn:mem / eqn:ref) and publishes the storage
//       segments of its senders to the rotating segment list of step t;
//   (c) delivers the senders of step t-1 (published in the previous
//       iteration) into rows t .. t+62 -- never row t-1, which (a) reads.
// Row t-1 is complete when (a) reads it: its last contributions come from the
// senders of step t-2 with delay 1, delivered in iteration it-1 before the
// barrier.  After the last step one more (a)+(c) pass leaves the state
// canonical (all senders delivered, I of the next step computed).
//
// Everything one block writes and another reads after a barrier goes through
// device-scope atomics (ring adds, list counts) or device-scope atomic loads
// and stores (ring reads and clears, list entries), so the barrier needs no cache
// write-back or invalidation: each wave waits until its own memory operations
// are performed (vmcnt 0), then one thread per block arrives and polls.  Every
// wait is bounded; on expiry the kernel records an error and all blocks leave.
// ---------------------------------------------------------------------------
constexpr uint32_t kSpec = 64;   // list entries fetched together with the count

__device__ __forceinline__ SegStage ld_entry(const SegEntry *e) {
  SegStage r;
  r.start = ld_ag(&e->start);
  const uint64_t lt = ld_ag(reinterpret_cast<const uint64_t *>(&e->len));
  r.len = uint32_t(lt);
  r.tbase = uint32_t(lt >> 32);
  return r;
}
__device__ __forceinline__ void st_entry(SegEntry *e, uint64_t start, uint32_t len, uint32_t tbase) {
  st_ag(&e->start, start);
  st_ag(reinterpret_cast<uint64_t *>(&e->len), uint64_t(len) | (uint64_t(tbase) << 32));
}

__device__ __forceinline__ bool grid_barrier(Control *ctl, uint64_t target, uint32_t spin_limit,
                                             uint32_t *s_flag) {
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's stores and atomics are performed
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(&ctl->barrier, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t ok = 1, spins = 0;
    while (ld_ag(&ctl->barrier) < target) {
      __builtin_amdgcn_s_sleep(1);
      if ((++spins & 255u) == 0 && (ld_ag(&ctl->error) != 0 || spins > spin_limit)) {
        st_ag(&ctl->error, 1u);
        ok = 0;
        break;
      }
    }
    *s_flag = ok;
  }
  __syncthreads();
  return *s_flag != 0;
}

template <int BS, int QMAX, bool COMP, bool LDS>
__global__ __launch_bounds__(BS) void k_persistent(DeviceNet d, uint32_t n_steps, uint32_t qpt,
                                                    uint32_t spin_limit) {
  constexpr int NW = BS / 64;
  constexpr int IPT = kSegCap / BS;
  __shared__ ThrTables s_tab;
  __shared__ SegStage s_seg[kSegCap];
  __shared__ uint32_t s_excl[kSegCap];
  __shared__ uint32_t s_tmp[NW];
  __shared__ uint32_t s_wave[NW];
  __shared__ uint32_t s_base, s_flag, s_n;
  __shared__ unsigned long long s_rbase;

  const uint32_t G = gridDim.x;
  const uint32_t TT = G * BS;
  const uint32_t gt = blockIdx.x * BS + threadIdx.x;
  const uint32_t wave = threadIdx.x >> 6;
  const uint32_t lane = __lane_id();
  const uint64_t t0 = d.ctl->t_base;
  const Props k{d.consts->p11, d.consts->p22, d.consts->p21};
  const uint32_t nwin = d.nwin_max;
  const size_t lstride = size_t(d.ntot) * nwin;
  stage_tables<LDS>(d, s_tab);

  // Owned quads q = gt + j * TT: state, thalamic counts of the last decided
  // step, quad info and population code stay in registers for the chunk.
  float U[QMAX][4], I[QMAX][4];
  uint32_t R[QMAX], Tp[QMAX], QI[QMAX], PC[QMAX], c_spk[QMAX], c_poi[QMAX];
  int64_t c_con[QMAX];
  uint64_t c_ev[QMAX];
#pragma unroll
  for (int j = 0; j < QMAX; ++j) {
    const uint32_t q = gt + uint32_t(j) * TT;
    c_spk[j] = c_poi[j] = 0;
    c_con[j] = 0;
    c_ev[j] = 0;
    Tp[j] = R[j] = QI[j] = PC[j] = 0;
#pragma unroll
    for (int m = 0; m < 4; ++m) U[j][m] = I[j][m] = 0.0f;
    if (uint32_t(j) < qpt && q < d.nquads) {
      const float4 uv = ld4(d.U + 4 * size_t(q));
      const float4 iv = ld4(d.I + 4 * size_t(q));
      U[j][0] = uv.x; U[j][1] = uv.y; U[j][2] = uv.z; U[j][3] = uv.w;
      I[j][0] = iv.x; I[j][1] = iv.y; I[j][2] = iv.z; I[j][3] = iv.w;
      R[j] = d.R4[q];
      QI[j] = d.qinfo[q];
      const InstDev *ip = d.inst + __builtin_amdgcn_readfirstlane(QI[j] >> 24);
      PC[j] = quad_code(ip, QI[j] & 0xFFFFFFu);
    }
  }
  __syncthreads();

  for (uint32_t it = 0; it <= n_steps; ++it) {
    const uint64_t t = t0 + it;
    const bool has_prev = it > 0;
    const bool decide = it < n_steps;
    SegEntry *lcur = d.seg_list + size_t(it % 3) * lstride;
    const SegEntry *lprev = d.seg_list + size_t((it + 2) % 3) * lstride;

    // (c) part 1: the count of step t-1's segments and the first kSpec of them.
    uint32_t nprev = 0;
    SegStage spec{0, 0, 0};
    if (has_prev && wave == 0) {
      nprev = ld_ag(&d.ctl->lcnt[(it + 2) % 3]);
      spec = ld_entry(lprev + lane);
    }
    if (decide && gt == 0) st_ag(&d.ctl->lcnt[(it + 1) % 3], 0u);

    // (a) complete step t-1.  Ring words are read and cleared with
    // device-coherent 8-byte loads and stores (two per quad): no atomic unit
    // is involved, and the row has no other writer in this iteration.
    if (has_prev) {
      int32_t *wrow = d.W + size_t((t - 1) & (kRing - 1)) * d.ntot;
#pragma unroll
      for (int j = 0; j < QMAX; ++j) {
        const uint32_t q = gt + uint32_t(j) * TT;
        if (uint32_t(j) < qpt && q < d.nquads) {
          const InstDev *ip = d.inst + __builtin_amdgcn_readfirstlane(QI[j] >> 24);
          const int32_t wext = ip->w_ext_q;
          uint64_t *wp = reinterpret_cast<uint64_t *>(wrow + 4 * size_t(q));
          const uint64_t w01 = ld_ag(wp), w23 = ld_ag(wp + 1);
          st_ag(wp, 0ull);
          st_ag(wp + 1, 0ull);
          const int32_t w[4] = {int32_t(uint32_t(w01)), int32_t(uint32_t(w01 >> 32)),
                                int32_t(uint32_t(w23)), int32_t(uint32_t(w23 >> 32))};
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            if ((PC[j] >> (12 + m)) & 1u) {
              I[j][m] = next_current(I[j][m], int32_t((Tp[j] >> (8 * m)) & 0xFFu), wext, w[m], k.p11);
              c_con[j] += w[m];
            }
          }
        }
      }
    }

    // (b) decide step t and publish the senders' segments.
    if (decide) {
      uint32_t flags[QMAX];
      uint32_t lane_base[QMAX];
      uint32_t wtot = 0;
#pragma unroll
      for (int j = 0; j < QMAX; ++j) {
        flags[j] = 0;
        const uint32_t q = gt + uint32_t(j) * TT;
        if (uint32_t(j) < qpt && q < d.nquads) {
          const uint32_t inst = __builtin_amdgcn_readfirstlane(QI[j] >> 24);
          const InstDev *ip = d.inst + inst;
          flags[j] = decide_quad(LDS ? s_tab.thr : d.thr, LDS ? s_tab.meta : d.pmeta, inst * 8u,
                                 ip->seed, QI[j] & 0xFFFFFFu, PC[j], t, k, U[j], I[j], R[j], Tp[j],
                                 c_poi[j]);
        }
        uint32_t lo, tot;
        wave_compact(flags[j], lo, tot);
        lane_base[j] = wtot + lo;
        wtot += tot;
      }
      if (lane == 0) s_wave[wave] = wtot;
      __syncthreads();
      if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int w = 0; w < NW; ++w) {
          const uint32_t c = s_wave[w];
          s_wave[w] = run;
          run += c;
        }
        if (run) {
          s_base = atomicAdd(&d.ctl->lcnt[it % 3], run * nwin);
          s_rbase = atomicAdd(reinterpret_cast<unsigned long long *>(&d.ctl->raster_n),
                              (unsigned long long)run);
        }
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < QMAX; ++j) {
        if (!flags[j]) continue;
        const uint32_t q = gt + uint32_t(j) * TT;
        const InstDev *ip = d.inst + (QI[j] >> 24);
        const uint32_t lq = QI[j] & 0xFFFFFFu;
        const uint32_t inw = ip->nwin;
        uint32_t o = s_wave[wave] + lane_base[j];
        c_spk[j] += __popc(flags[j]);
        for (int m = 0; m < 4; ++m) {
          if (!((flags[j] >> m) & 1u)) continue;
          const uint32_t gid = 4 * q + uint32_t(m);
          const uint64_t sg = uint64_t(ip->seg_base) + uint64_t(lq * 4u + uint32_t(m)) * inw;
          const uint64_t row0 = d.seg_ptr[sg];
          c_ev[j] += d.seg_ptr[sg + inw] - row0;
          SegEntry *dst = lcur + size_t(s_base) + size_t(o) * nwin;
          for (uint32_t w = 0; w < nwin; ++w) {
            uint64_t st = 0;
            uint32_t len = 0;
            if (w < inw) {
              st = d.seg_ptr[sg + w];
              len = uint32_t(d.seg_ptr[sg + w + 1] - st);
            }
            st_entry(dst + w, st, len, COMP ? ip->tbase0 + w * ip->win_size : 0u);
          }
          const uint64_t pos = s_rbase + o;
          if (pos < d.raster_cap)
            d.raster[pos] = (t << 32) | gid;
          else
            d.ctl->overflow = 1;
          ++o;
        }
      }
    }

    // (c) part 2: deliver the senders of step t-1 into rows t .. t+62.
    if (has_prev) {
      if (wave == 0 && lane == 0) s_n = nprev;
      __syncthreads();
      const uint32_t n = s_n;
      for (uint32_t b0 = 0; b0 < n; b0 += kSegCap) {
        const uint32_t nb = min(uint32_t(kSegCap), n - b0);
        if (b0 == 0) {
          if (wave == 0 && lane < nb) s_seg[lane] = spec;
          for (uint32_t s2 = kSpec + threadIdx.x; s2 < nb; s2 += BS) s_seg[s2] = ld_entry(lprev + s2);
        } else {
          for (uint32_t s2 = threadIdx.x; s2 < nb; s2 += BS) s_seg[s2] = ld_entry(lprev + b0 + s2);
        }
        __syncthreads();
        uint32_t len[IPT];
        uint32_t mysum = 0;
#pragma unroll
        for (int m = 0; m < IPT; ++m) {
          const uint32_t s2 = threadIdx.x * IPT + m;
          len[m] = s2 < nb ? s_seg[s2].len : 0u;
          mysum += len[m];
        }
        uint32_t total;
        uint32_t run = block_exclusive_scan<BS>(mysum, s_tmp, total);
#pragma unroll
        for (int m = 0; m < IPT; ++m) {
          const uint32_t s2 = threadIdx.x * IPT + m;
          if (s2 < nb) s_excl[s2] = run;
          run += len[m];
        }
        __syncthreads();
        deliver_batch<COMP>(d, t - 1, s_seg, s_excl, nb, total, gt, TT);
        __syncthreads();
      }
    }

    if (it == n_steps) break;
    if (!grid_barrier(d.ctl, uint64_t(it + 1) * G, spin_limit, &s_flag)) break;
  }

  // State back to memory; counters to the per-wave slots.
#pragma unroll
  for (int j = 0; j < QMAX; ++j) {
    const uint32_t q = gt + uint32_t(j) * TT;
    const bool act = uint32_t(j) < qpt && q < d.nquads;
    if (act) {
      *reinterpret_cast<float4 *>(d.U + 4 * size_t(q)) = make_float4(U[j][0], U[j][1], U[j][2], U[j][3]);
      *reinterpret_cast<float4 *>(d.I + 4 * size_t(q)) = make_float4(I[j][0], I[j][1], I[j][2], I[j][3]);
      d.R4[q] = R[j];
    }
    uint64_t sp = c_spk[j], po = c_poi[j], ev = c_ev[j];
    int64_t co = c_con[j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      sp += __shfl_xor(sp, o);
      po += __shfl_xor(po, o);
      ev += __shfl_xor(ev, o);
      co += __shfl_xor(co, o);
    }
    if (lane == 0 && uint32_t(j) < qpt && (q >> 6) < (d.nquads >> 6)) {
      int64_t *c = d.wave_ctr + 4 * size_t(q >> 6);
      c[0] += int64_t(sp);
      c[1] += int64_t(po);
      c[2] += co;
      c[3] += int64_t(ev);
    }
  }
  // The last block to finish resets the shared control words for the next
  // launch and advances the step counter.
  __builtin_amdgcn_s_waitcnt(0x0F70);
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint64_t done =
        __hip_atomic_fetch_add(&d.ctl->exit_count, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (done == G - 1) {
      st_ag(&d.ctl->lcnt[0], 0u);
      st_ag(&d.ctl->lcnt[1], 0u);
      st_ag(&d.ctl->lcnt[2], 0u);
      st_ag(&d.ctl->barrier, 0ull);
      st_ag(&d.ctl->exit_count, 0ull);
      st_ag(&d.ctl->t_base, t0 + n_steps);
    }
  }
}

using PersistentFn = void (*)(DeviceNet, uint32_t, uint32_t, uint32_t);

template <bool COMP, bool LDS>
static PersistentFn pick_persistent(uint32_t block, uint32_t qmax) {
#define SNN_PK(BSV, QV) \
  if (block == BSV && qmax == QV) return k_persistent<BSV, QV, COMP, LDS>;
  SNN_PK(256, 1) SNN_PK(256, 2) SNN_PK(256, 4) SNN_PK(256, 8)
  SNN_PK(128, 1) SNN_PK(128, 2) SNN_PK(128, 4)
  SNN_PK(512, 1) SNN_PK(512, 2)
  SNN_PK(1024, 1)
#undef SNN_PK
  return nullptr;
}

uint32_t persistent_qmax(uint32_t qpt) {
  return qpt <= 1 ? 1 : qpt <= 2 ? 2 : qpt <= 4 ? 4 : qpt <= 8 ? 8 : 0;
}

static PersistentFn persistent_fn(const DeviceNet &d, uint32_t block, uint32_t qpt) {
  const uint32_t qmax = persistent_qmax(qpt);
  if (!qmax) return nullptr;
  const bool comp = d.syn_format == SNN_SYN_COMPRESSED5;
  if (d.thr_lds)
    return comp ? pick_persistent<true, true>(block, qmax) : pick_persistent<false, true>(block, qmax);
  return comp ? pick_persistent<true, false>(block, qmax) : pick_persistent<false, false>(block, qmax);
}

int persistent_max_grid(const DeviceNet &d, uint32_t block, uint32_t qpt) {
  PersistentFn fn = persistent_fn(d, block, qpt);
  if (!fn) return 0;
  int per_cu = 0, dev = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(fn),
                                                   int(block), 0) != hipSuccess)
    return 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
  return per_cu * prop.multiProcessorCount;
}

hipError_t launch_persistent(const DeviceNet &d, const LaunchShape &sh, uint32_t n, hipStream_t s) {
  PersistentFn fn = persistent_fn(d, sh.block, sh.qpt);
  if (!fn || sh.grid == 0) return hipErrorInvalidConfiguration;
  DeviceNet dv = d;
  uint32_t steps = n, qpt = sh.qpt;
  // A bounded wait expires after about 2^24 polls (well over 0.1 s).
  uint32_t spin = 1u << 24;
  void *args[] = {&dv, &steps, &qpt, &spin};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(fn), dim3(sh.grid),
                                    dim3(sh.block), args, 0, s);
}


// ---------------------------------------------------------------------------
// LDS engine: the destination-partitioned form of the persistent loop.
//
// Block b owns the WN neurons [b WN, (b+1) WN) and their 64 ring rows, kept in
// LDS for the whole chunk.  Synapses are stored per (sender, destination
// window) in fixed-capacity segments, so a block finds its segment of any
// sender's row from the sender's id alone -- the paper's disjoint synapse
// classes by destination (Sec. 3.6), one class per block -- and adds it into
// its ring with LDS atomics.
//
// Blocks exchange nothing but their senders.  Per step each block publishes
// one 64-bit flag word: the step's epoch, its spike count and the window
// offsets of its first four spikes (further ones go to a list in memory).
// No atomics are involved.  Since every delay is at least one step, a spike
// of step t first changes a decision at step t+2, so a block needs the
// senders of step t-1 only after it has decided step t: the wait for the
// other blocks' flags of step t-1 comes after the block's own decision of
// step t, and the flags' propagation overlaps a whole step of work.  A block
// reads the flags of the blocks that can reach its window (those of its own
// instances) only; blocks of unrelated instances never wait for each other.
//
// Iteration it (t = t0 + it):
//   (a) complete step t-1 from ring row t-1 and the thalamic counts T_{t-1};
//   (b) decide step t (membrane update only) and publish its flag;
//   (c) waves 0 and 3 wait for the flags of step t-1 (half of the windows
//       each) while waves 1 and 2 finish the thalamic counts T_t; then all
//       waves stage those senders, issue their record loads and add the
//       records into rows t .. t+62.
// ---------------------------------------------------------------------------
constexpr uint32_t kInline = 4;  // senders carried in a flag word

// Flag word: bits 0-15 epoch (mod 2^16), 16-25 spike count, then 9 bits per
// inline sender (its offset in the window).
__device__ __forceinline__ uint32_t flag_count(uint64_t f) { return uint32_t(f >> 16) & 1023u; }
__device__ __forceinline__ uint32_t flag_local(uint64_t f, uint32_t k) {
  return uint32_t(f >> (26 + 9 * k)) & 511u;
}

// Sender j of step t-1's set, as a global id: from the expanded list s_sid
// (the first SB senders), else by search over the windows with senders
// (s_nzf / s_nzp / s_nzb, relative to window rel0; nnz of them); senders past
// a window's fourth come from its list in memory.
template <uint32_t SB>
__device__ __forceinline__ uint32_t sender_gid(const uint32_t *llist, uint32_t ntot, uint32_t j, uint32_t nnz,
                                               uint32_t lslot, const uint32_t *s_sid,
                                               const uint64_t *s_nzf, const uint32_t *s_nzp,
                                               const uint16_t *s_nzb, const uint32_t *s_wstart,
                                               uint32_t rel0) {
  uint32_t src, kk;
  if (j < SB) {
    const uint32_t v = s_sid[j];
    if (!(v >> 31)) return v;
    src = (v >> 10) & 0x1FFFFFu;
    kk = v & 1023u;
  } else {
    uint32_t lo = 0, hi = nnz;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (s_nzp[mid] <= j) lo = mid; else hi = mid;
    }
    kk = j - s_nzp[lo];
    src = s_nzb[lo];
    if (kk < kInline) return s_wstart[src] + flag_local(s_nzf[lo], kk);
  }
  const uint32_t w0 = s_wstart[src];
  return w0 + ld_ag(llist + size_t(lslot) * ntot + w0 + kk);
}

// Record formats of the LDS engine: 8-byte plain records, 4-byte compressed
// records (16-bit weight), and the deviation format's 2-byte locator plus
// 8-bit deviation from the pair's mean (Sec. 5.3).
constexpr int kFmtPlain = 0, kFmtComp = 1, kFmtDev = 2;

// UR record slots per lane.  The wave's senders of a batch are held one per
// lane (segment address and capacity); their segments are cut into 64-record
// pieces, numbered sender by sender.  load() takes the next UR pieces, one per
// slot: the sender of piece P is the last lane whose first piece is <= P (a
// ballot), so a piece's address costs a few scalar operations and no branch.
// apply() adds the loaded records into rows (t_src + delay).  Unused slots and
// empty record slots (delay 0) add nothing.
template <int FMT, int UR>
struct SegmentWalk {
  uint64_t rec[FMT == kFmtPlain ? UR : 1];
  uint32_t r4[FMT == kFmtComp ? UR : 1];
  uint32_t r2[FMT == kFmtDev ? UR : 1];    // deviation format: locator
  int32_t dv[FMT == kFmtDev ? UR : 1];     // and deviation
  uint32_t pc[FMT == kFmtDev ? UR : 1];    // and the piece's sender population (wave-uniform)
  uint64_t base_l;   // lane l: segment of the wave's sender l
  uint32_t cap_l;
  uint32_t cls_l;    // lane l: population of the wave's sender l
  uint32_t p_l;      // lane l: number of the sender's first piece
  uint32_t np;       // pieces of the batch (wave-uniform)
  uint32_t p0;       // next piece
  uint32_t nv;       // slots filled by the last load()

  // Lane l holds the segment of the wave's sender l (capacity 0 past the end).
  __device__ __forceinline__ void begin(uint64_t base_lane, uint32_t cap_lane, uint32_t cls_lane) {
    base_l = base_lane;
    cap_l = cap_lane;
    cls_l = cls_lane;
    p_l = wave_prefix((cap_lane + 63u) >> 6, np);
    p0 = 0;
  }
  __device__ __forceinline__ bool more() const { return p0 < np; }

  __device__ __forceinline__ void load(const DeviceNet &d) {
    const uint32_t lane = __lane_id();
#pragma unroll
    for (int u = 0; u < UR; ++u) {
      const uint32_t P = p0 + uint32_t(u);
      if (P >= np) {   // wave-uniform
        if (FMT == kFmtPlain) rec[u] = 0ull;
        if (FMT == kFmtComp) r4[u] = 0u;
        if (FMT == kFmtDev) {
          r2[u] = 0u;
          dv[u] = 0;
          pc[u] = 0u;
        }
        continue;
      }
      // Lanes past the last sender have p_l = np > P, so they never count.
      const uint32_t s = uint32_t(__popcll(__ballot(int(p_l <= P)))) - 1u;
      const uint32_t k = P - __builtin_amdgcn_readlane(p_l, s);
      const uint32_t cap = __builtin_amdgcn_readlane(cap_l, s);
      const uint64_t base = join64(uint32_t(__builtin_amdgcn_readlane(uint32_t(base_l >> 32), s)),
                                   uint32_t(__builtin_amdgcn_readlane(uint32_t(base_l), s))) + 64u * k;
      const bool ok = 64u * k + lane < cap;
      if (FMT == kFmtPlain) {
        rec[u] = ok ? __builtin_nontemporal_load(d.rec8 + base + lane) : 0ull;
      } else if (FMT == kFmtComp) {
        r4[u] = ok ? __builtin_nontemporal_load(d.rec4 + base + lane) : 0u;
      } else {
        r2[u] = ok ? uint32_t(__builtin_nontemporal_load(d.rec2 + base + lane)) : 0u;
        dv[u] = ok ? int32_t(__builtin_nontemporal_load(d.dev8 + base + lane)) : 0;
        pc[u] = uint32_t(__builtin_amdgcn_readlane(cls_l, s));
      }
    }
    nv = min(np - p0, uint32_t(UR));
    p0 += UR;
  }

  // dq / dsq: the deviation format's mean and step of (population, doubled pair).
  template <int WN>
  __device__ __forceinline__ void apply(int32_t *s_ring, uint64_t t_src, uint32_t wb0,
                                        const int32_t *dq, const int32_t *dsq) const {
#pragma unroll
    for (int u = 0; u < UR; ++u) {
      if (uint32_t(u) >= nv) {   // wave-uniform; past 8 pieces the compiler unrolls
        if (UR > 8) continue;    // only a loop without an early exit
        break;
      }
      uint32_t delay, loc;
      int32_t wq;
      if (FMT == kFmtComp) {
        delay = (r4[u] >> 10) & 63u;
        loc = r4[u] & 1023u;
        wq = int32_t(int16_t(uint16_t(r4[u] >> 16))) * 8;
      } else if (FMT == kFmtDev) {
        delay = (r2[u] >> 9) & 63u;
        loc = r2[u] & 511u;
        const uint32_t di = 2u * pc[u] + (r2[u] >> 15);
        wq = dq[di] + dv[u] * dsq[di];
      } else {
        const uint32_t hiw = uint32_t(rec[u] >> 32);
        delay = hiw & 63u;
        loc = (hiw >> 6) - wb0;
        wq = int32_t(uint32_t(rec[u]));
      }
      if (delay) atomicAdd(&s_ring[((t_src + delay) & (kRing - 1)) * WN + loc], wq);
    }
  }
};

template <int WN, int FMT>
__global__ __launch_bounds__(256) void k_lds(DeviceNet d, uint32_t n_steps, uint32_t group,
                                             uint32_t last_group, uint32_t win0,
                                             uint32_t spin_limit) {
  constexpr uint32_t BS = 256;
  constexpr uint32_t NQ = WN / 4;             // quads a window can hold
  constexpr uint32_t Q0 = BS - NQ;            // threads Q0.. own one quad each
  constexpr uint32_t TS = kLdsTab + 8;        // stride of an LDS thalamic table
  constexpr uint32_t NZ = kLdsMaxGrid;        // windows of one instance, at most
  constexpr int NJ = NZ / 128;                // flags per lane of a polling wave
  constexpr uint32_t NZH = NZ / 2;            // windows polled by one wave
  constexpr uint32_t RC = WN + 128;           // raster staging entries
  constexpr uint32_t SB = BS;                 // senders resolved per batch
  constexpr uint32_t SBH = SB / 2;            // senders staged per polling wave
  // Record pieces in flight per lane (measured at full scale: plain records
  // 3.62 / 3.53 / 3.48 us per step at 8 / 12 / 16; the 4- and 3-byte
  // formats are slower at 16 than at 8).
  constexpr int UR = FMT == kFmtPlain ? 16 : 8;
  static_assert(Q0 >= 128, "waves 0 and 1 own no quad");
  __shared__ __align__(16) int32_t s_ring[kRing * WN];
  __shared__ __align__(16) uint32_t s_thr[8 * TS];
  __shared__ uint2 s_meta[8];
  __shared__ uint32_t s_cf[8], s_cn[8], s_ccap[8];   // sender classes
  __shared__ int32_t s_dq[16], s_ds[16];      // deviation format: mean and step per (class, doubled)
  __shared__ uint64_t s_cbase[8];
  __shared__ uint32_t s_wstart[NZ];           // first neuron of each window of the instance
  __shared__ uint32_t s_sid[SB];              // senders of step t-1 (gid or list marker)
  __shared__ uint64_t s_nzf[NZ];
  __shared__ uint32_t s_nzp[NZ];
  __shared__ uint16_t s_nzb[NZ];
  __shared__ uint64_t s_rast[RC];
  __shared__ uint32_t s_T[2 * NQ];            // T_t of each quad by step parity, a byte per neuron
  __shared__ uint4 s_px[NQ];                  // Philox words of each quad for T_t
  __shared__ uint32_t s_wave[BS / 64], s_inl[kInline];
  __shared__ uint32_t s_flag[2], s_n[2], s_nnz[2];   // per polling wave
  __shared__ unsigned long long s_rbase;
  __shared__ long long s_ctr[4];

  const uint32_t GT = d.n_lwin, blk = win0 + blockIdx.x;
  // Step origin and flag epoch live in device memory, so a chunk's launches
  // can be replayed from a captured graph; the group's last block advances
  // them when it leaves.
  const uint64_t t0 = d.ctl->t_base;
  const uint32_t ep0 = d.lgroup[group].x;
  const uint32_t tid = threadIdx.x, lane = __lane_id();
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint4 wi = d.lwin[blk];               // (first neuron, neurons, instance, -)
  const uint32_t wb0 = wi.x, wlen = wi.y, inst = wi.z;
  const uint32_t oq = tid - Q0;               // owned quad in the window
  const uint32_t q = wb0 / 4 + oq;
  const bool owner = tid >= Q0 && oq < wlen / 4;
  const InstDev *ip = d.inst + inst;
  const Props k_s{d.consts->p11, d.consts->p22, d.consts->p21};
  const uint2 rel = d.wrel[blk];              // windows whose senders can reach this one
  uint64_t *const flags = d.lflags;

  // Ring rows of the window into LDS.
  for (uint32_t i = tid; i < kRing * WN; i += BS) {
    const uint32_t r = i / WN, c = i % WN;
    s_ring[i] = c < wlen ? d.W[size_t(r) * d.ntot + wb0 + c] : 0;
  }
  if (tid < 8u) {
    const WinClass c = d.wcls[size_t(blk) * kWinClasses + tid];
    s_cf[tid] = c.first;
    s_cn[tid] = c.n;
    s_ccap[tid] = c.cap;
    s_cbase[tid] = c.base;
  }
  if (tid < 4u) s_ctr[tid] = 0;
  if (tid < 16u) {
    s_dq[tid] = ip->dev_mq[tid];
    s_ds[tid] = ip->dev_sq[tid];
  }
  for (uint32_t i = tid; i < rel.y - rel.x; i += BS) s_wstart[i] = d.lwin[rel.x + i].x;
  // Thalamic tables of the window's instance.
  if (tid < 8u) {
    const uint2 m = d.pmeta[inst * 8 + tid];
    const uint32_t off = tid * TS;
    for (uint32_t kk = 0; kk < TS; ++kk)
      s_thr[off + kk] = kk < m.y ? d.thr[m.x + kk] : 0xFFFFFFFFu;
    s_meta[tid] = make_uint2(off, m.y);
  }

  float U[4] = {0, 0, 0, 0}, I[4] = {0, 0, 0, 0};
  uint32_t R = 0, c_spk = 0, c_poi = 0;
  uint32_t OD[4] = {0, 0, 0, 0};
  int64_t c_con = 0;
  uint64_t c_ev = 0;
  const int32_t wext_s = ip->w_ext_q;
  if (owner) {
    const float4 uv = ld4(d.U + 4 * size_t(q));
    const float4 iv = ld4(d.I + 4 * size_t(q));
    U[0] = uv.x; U[1] = uv.y; U[2] = uv.z; U[3] = uv.w;
    I[0] = iv.x; I[1] = iv.y; I[2] = iv.z; I[3] = iv.w;
    R = d.R4[q];
    const uint4 od = *reinterpret_cast<const uint4 *>(d.outdeg + 4 * size_t(q));
    OD[0] = od.x; OD[1] = od.y; OD[2] = od.z; OD[3] = od.w;
  }
  uint64_t seed = ip->seed;
  // Block-uniform values used only by vector arithmetic live in vector
  // registers, which are plentiful, and leave scalar registers to the loop.
  Props k = k_s;
  int32_t wext = wext_s;
  uint32_t wb0v = wb0;
  asm volatile("" : "+v"(seed), "+v"(k.p11), "+v"(k.p22), "+v"(k.p21), "+v"(wext), "+v"(wb0v));
  // Pointers of the rare paths (lists, raster flush, errors) likewise.
  uint32_t *llist_v = d.llist;
  uint64_t *raster_v = d.raster;
  Control *ctl_v = d.ctl;
  uint64_t rcap_v = d.raster_cap;
  uint32_t ntot_v = d.ntot;
  asm volatile("" : "+v"(llist_v), "+v"(raster_v), "+v"(ctl_v), "+v"(rcap_v), "+v"(ntot_v));
  // Waves 0 and 3 poll the flags: wave 0 of the first NZH windows that can
  // reach this one (h = 0), wave 3 of the others (h = 1).  Flag index
  // (window) read by lane l in poll slot j, ~0 past the windows that can
  // reach this one, and that window's first neuron.
  const bool poller = wave == 0 || wave == 3;
  const uint32_t h = wave == 3 ? 1u : 0u;
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

  // Thalamic counts T_t into s_T (one byte per neuron), one Philox block per
  // quad (eqn:ref's background drive, Sec. 2.2), in two parts placed where
  // waves are idle: waves 0 and 1 (no quads) compute the Philox words of quad
  // tid while the owners complete and decide the step (draw_words); threads
  // 64 + k of waves 1 and 2 turn the words of quad k into counts while waves
  // 0 and 3 wait for the flags (draw_counts).
  const uint32_t lq0 = (wb0 - ip->gbase) / 4;
  const uint32_t nq_win = wlen / 4;
  auto draw_words = [&](uint64_t t) {
    if (tid >= 128u || tid >= nq_win) return;
    const Philox4 x = philox4x32_10(lq0 + tid, uint32_t(t), uint32_t(t >> 32), kStreamThalamic,
                                    uint32_t(seed), uint32_t(seed >> 32));
    s_px[tid] = make_uint4(x.v[0], x.v[1], x.v[2], x.v[3]);
  };
  const uint32_t dq = tid - 64u;               // quad counted by this thread
  uint32_t dcode = 0;
  if (tid >= 64u && dq < nq_win) dcode = quad_code(ip, lq0 + dq);
  auto draw_counts = [&](uint64_t t) {
    if (!(dcode >> 12)) return;                // no real neuron (or no quad)
    const uint4 xw = s_px[dq];
    const Philox4 x{{xw.x, xw.y, xw.z, xw.w}};
    // All table reads first (16 bytes at a time, population p's table at
    // p TS), then the counts without branches; a count reaching 8 continues
    // in the table (rare).
    uint4 lo[4], hi[4];
    uint32_t len[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const uint32_t pm = (dcode >> (3 * m)) & 7u;
      const uint4 *tb = reinterpret_cast<const uint4 *>(s_thr + pm * TS);
      lo[m] = tb[0];
      hi[m] = tb[1];
      len[m] = s_meta[pm].y;
    }
    // Table entries past a table's length hold ~0, which no word below ~0
    // reaches; the word ~0 reaches every entry, so its count is the length.
    uint32_t T[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const uint32_t u = x.v[m];
      const uint32_t v[8] = {lo[m].x, lo[m].y, lo[m].z, lo[m].w, hi[m].x, hi[m].y, hi[m].z, hi[m].w};
      uint32_t c = 0;
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) c += u >= v[kk] ? 1u : 0u;
      T[m] = u == ~0u ? len[m] : c;
    }
    if (T[0] == 8u || T[1] == 8u || T[2] == 8u || T[3] == 8u) {   // rare
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const uint32_t *tab = s_thr + ((dcode >> (3 * m)) & 7u) * TS;
        if (T[m] == 8u)
          while (T[m] < len[m] && x.v[m] >= tab[T[m]]) ++T[m];
      }
    }
    uint32_t tp = 0;
#pragma unroll
    for (int m = 0; m < 4; ++m) tp |= (((dcode >> (12 + m)) & 1u) ? T[m] : 0u) << (8 * m);
    s_T[(t & 1u) * NQ + dq] = tp;
  };

  for (uint32_t it = 0; it <= n_steps; ++it) {
    const uint64_t t = t0 + it;
    const bool decide = it < n_steps;
    const uint32_t ep = ep0 + it + 1;         // epoch of step t's flags
    const uint32_t epp = ep - 1;              // epoch of step t-1's flags
    const uint64_t *fs = flags + size_t(epp % kSlots) * GT;

    // The polling waves issue the flag loads of step t-1 now; they are
    // checked in (c).
    uint64_t fv[NJ];
    if (poller && it > 0) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) fv[j] = pb[j] != ~0u ? ld_ag(fs + pb[j]) : 0ull;
    }
    if (decide) draw_words(t);   // waves 0 and 1

    // (a) complete step t-1 from ring row t-1 and T_{t-1}.
    if (it > 0 && owner) {
      int4 *row = reinterpret_cast<int4 *>(s_ring + ((t - 1) & (kRing - 1)) * WN + 4 * oq);
      const int4 wv = *row;
      *row = make_int4(0, 0, 0, 0);
      const uint32_t Tp = s_T[((t - 1) & 1u) * NQ + oq];
      // Padding neurons receive no records and no thalamic counts, so their
      // current stays 0 and the update needs no per-neuron test.
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
    // offsets of the first kInline spikes for the flag word, list entries for
    // the others, then the flag.
    if (decide) {
      const uint32_t fl = owner ? lif_quad_padded(k, U, I, R) : 0u;
      uint32_t lo, tot;
      wave_compact(fl, lo, tot);
      if (lane == 0) s_wave[wave] = tot;
      __syncthreads();
      uint32_t before = 0, cnt = 0;
#pragma unroll
      for (uint32_t w = 0; w < BS / 64; ++w) {
        const uint32_t c = __builtin_amdgcn_readfirstlane(s_wave[w]);
        before += w < wave ? c : 0u;
        cnt += c;
      }
      if (fl) {
        uint32_t p = before + lo;
        uint32_t *lst = llist_v + size_t(ep % kSlots) * ntot_v + wb0;
        c_spk += __popc(fl);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          if (!((fl >> m) & 1u)) continue;
          const uint32_t loc = 4 * oq + uint32_t(m);
          if (p < kInline)
            s_inl[p] = loc;
          else
            st_ag(lst + p, loc);
          s_rast[rn + p] = (t << 32) | (wb0 + loc);
          c_ev += OD[m];
          ++p;
        }
      }
      if (cnt) {   // block-uniform
        // List entries must be performed before the flag that announces them.
        if (cnt > kInline) __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
        __syncthreads();
      }
      // Wave 1 stores the flag: vector memory operations of a wave complete
      // in order, so the polling wave 0 would otherwise wait for the store's
      // acknowledgement before it can read any flag.
      if (tid == 64) {
        uint64_t f = uint64_t(ep & 0xFFFFu) | (uint64_t(cnt) << 16);
        for (uint32_t kk = 0; kk < kInline && kk < cnt; ++kk)
          f |= uint64_t(s_inl[kk]) << (26 + 9 * kk);
        st_ag(flags + size_t(ep % kSlots) * GT + blk, f);
      }
      rn += cnt;
      if (rn > RC - WN) flush();
    }

    if (it == 0) {   // nothing to deliver yet
      draw_counts(t);
      __syncthreads();
      continue;
    }

    // (c) waves 0 and 3 wait for step t-1's flags of their windows and stage
    // their senders; waves 1 and 2 draw T_t meanwhile.
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
      for (int j = 0; j < NJ; ++j) sc += flag_count(fv[j]);
      uint32_t all_s, all_nz = 0;
      const uint32_t ps0 = wave_prefix(sc, all_s);
      uint32_t *const sid = s_sid + SBH * h;
      if (all_s > SBH) {   // wave-uniform
        // Senders past the first SBH are found by search over the windows
        // with senders, in window order, with their first sender's number.
        uint32_t nzc = 0;
#pragma unroll
        for (int j = 0; j < NJ; ++j) nzc += flag_count(fv[j]) ? 1u : 0u;
        uint32_t pz = wave_prefix(nzc, all_nz);
        uint32_t ps = ps0;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          const uint32_t c = flag_count(fv[j]);
          if (c) {
            s_nzf[NZH * h + pz] = fv[j];
            s_nzp[NZH * h + pz] = ps;
            s_nzb[NZH * h + pz] = uint16_t(NZH * h + lane + 64u * uint32_t(j));   // window, relative to rel.x
            ++pz;
            ps += c;
          }
        }
      }
      // The first SBH senders, expanded: gid for inline ones, else a list
      // marker (1 << 31 | relative window << 10 | index).
      uint32_t ps = ps0;
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const uint32_t c = flag_count(fv[j]);
        const uint32_t src = NZH * h + lane + 64u * uint32_t(j);
        for (uint32_t kk = 0; kk < c && ps < SBH; ++kk, ++ps)
          sid[ps] = kk < kInline ? wst[j] + flag_local(fv[j], kk)
                                 : (1u << 31) | (src << 10) | kk;
      }
      if (lane == 0) {
        s_nnz[h] = all_nz;
        s_n[h] = all_s;
        s_flag[h] = ok ? 1u : 0u;
      }
    } else if (decide) {
      draw_counts(t);
    }
    __syncthreads();

    if (!__builtin_amdgcn_readfirstlane(s_flag[0] & s_flag[1])) break;
    const uint32_t n0 = __builtin_amdgcn_readfirstlane(s_n[0]);
    const uint32_t n_prev = n0 + __builtin_amdgcn_readfirstlane(s_n[1]);
    const uint64_t tsrc = t - 1;
    for (uint32_t j0 = 0; j0 < n_prev; j0 += SB) {
      // This wave's senders of the batch: j0 + wave + 4 l, one per lane l.
      const uint32_t nb = min(SB, n_prev - j0);
      const uint32_t n_l = nb > wave ? (nb - wave + 3u) / 4u : 0u;
      uint64_t base_lane = 0;
      uint32_t cap_lane = 0, cls_lane = 0;
      if (lane < n_l) {
        // Senders of polling wave 0 come first, then those of wave 3.
        const uint32_t j = j0 + wave + 4u * lane;
        const uint32_t hs = j < n0 ? 0u : 1u;
        const uint32_t gid = sender_gid<SBH>(llist_v, ntot_v, j - (hs ? n0 : 0u), s_nnz[hs], epp % kSlots,
                                             s_sid + SBH * hs, s_nzf + NZH * hs, s_nzp + NZH * hs,
                                             s_nzb + NZH * hs, s_wstart, rel.x);
        // Populations are contiguous and in order: the class is the last
        // non-empty one starting at or before gid.
        uint32_t ci = 0;
#pragma unroll
        for (int c = 1; c < 8; ++c)
          if (gid >= s_cf[c] && s_cn[c]) ci = uint32_t(c);
        cap_lane = gid - s_cf[ci] < s_cn[ci] ? s_ccap[ci] : 0u;
        base_lane = s_cbase[ci] + uint64_t(gid - s_cf[ci]) * cap_lane;
        cls_lane = ci;
      }
      SegmentWalk<FMT, UR> sw;
      sw.begin(base_lane, cap_lane, cls_lane);
      while (sw.more()) {
        sw.load(d);
        sw.template apply<WN>(s_ring, tsrc, wb0v, s_dq, s_ds);
      }
    }
    __syncthreads();
  }

  // Raster, ring rows, state and counters back to memory.
  __syncthreads();
  if (rn) flush();
  for (uint32_t i = tid; i < kRing * WN; i += BS) {
    const uint32_t r = i / WN, c = i % WN;
    if (c < wlen) d.W[size_t(r) * d.ntot + wb0 + c] = s_ring[i];
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
    unsigned int *exits = &d.lgroup[group].y;
    const uint32_t done = __hip_atomic_fetch_add(exits, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (done == gridDim.x - 1) {
      st_ag(exits, 0u);
      st_ag(&d.lgroup[group].x, ep0 + n_steps);
      if (last_group) st_ag(&d.ctl->t_base, t0 + n_steps);
    }
  }
}

using LdsFn = void (*)(DeviceNet, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t);

static LdsFn lds_fn(uint32_t wn, uint32_t syn_format) {
  const int f = syn_format == SNN_SYN_COMPRESSED5 ? kFmtComp
                                                  : (syn_format == SNN_SYN_DEV8 ? kFmtDev : kFmtPlain);
  if (wn == 512) return f == kFmtComp ? k_lds<512, kFmtComp> : (f == kFmtDev ? k_lds<512, kFmtDev> : k_lds<512, kFmtPlain>);
  if (wn == 320) return f == kFmtComp ? k_lds<320, kFmtComp> : (f == kFmtDev ? k_lds<320, kFmtDev> : k_lds<320, kFmtPlain>);
  return nullptr;
}

int lds_max_grid(uint32_t wn) {
  LdsFn fn = lds_fn(wn, SNN_SYN_PLAIN8);
  if (!fn) return 0;
  int per_cu = 0, dev = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(fn), 256,
                                                   0) != hipSuccess)
    return 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
  return std::min<int>(std::min(per_cu, 1) * prop.multiProcessorCount, int(kLdsMaxGrid));
}

hipError_t launch_lds(const DeviceNet &d, uint32_t group, uint32_t n_groups, uint32_t win0,
                      uint32_t nwin, uint32_t n, hipStream_t s) {
  LdsFn fn = lds_fn(d.lds_window, d.syn_format);
  if (!fn || nwin == 0 || nwin > kLdsMaxGrid || win0 + nwin > d.n_lwin || group >= n_groups)
    return hipErrorInvalidConfiguration;
  DeviceNet dv = d;
  uint32_t steps = n, g = group, last = group + 1 == n_groups ? 1u : 0u, w0 = win0;
  uint32_t spin = 1u << 24;
  void *args[] = {&dv, &steps, &g, &last, &w0, &spin};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(fn), dim3(nwin), dim3(256), args,
                                    0, s);
}

}  // namespace snn
