// kernels.hip -- CDNA4 (gfx950) kernels of the clock-driven microcircuit
// simulation: FP64 propagators, the neuron update with Philox thalamic drive
// and wave-ballot spike compaction, and the push transfer of every spike's
// synapses into the int32 delay ring buffer.
//
// Numerics: FP32 state, every product and sum rounded on its own (the file is
// compiled with -ffp-contract=off, denormals kept), synaptic input summed as
// exact int32 in 2^-8 pA, so the order in which atomics land cannot change
// the result.
#include "engine.hpp"

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
// Neuron update of one quad (4 consecutive neurons of one instance).
// ---------------------------------------------------------------------------
struct Props {
  float p11, p22, p21;
};

__device__ __forceinline__ uint32_t population(const InstDev *__restrict__ ip, uint32_t local) {
  uint32_t p = 0;
#pragma unroll
  for (int k = 1; k < 8; ++k) p += local >= ip->pop_off[k] ? 1u : 0u;
  return p;
}

// eqn:mem / eqn:ref / eqn:psc for the quad; w holds the ring-buffer row t of
// the four neurons.  Returns a 4-bit mask of the neurons that spiked.
__device__ __forceinline__ uint32_t update_quad(const InstDev *__restrict__ ip,
                                                const uint32_t *__restrict__ thr, uint32_t lq,
                                                uint64_t t, Props k, float (&u)[4], float (&i)[4],
                                                uint32_t &r4, const int32_t (&w)[4],
                                                uint32_t &tsum, int64_t &consumed) {
  const uint64_t seed = ip->seed;
  const Philox4 x = philox4x32_10(lq, uint32_t(t), uint32_t(t >> 32), kStreamThalamic,
                                  uint32_t(seed), uint32_t(seed >> 32));
  const uint32_t n = ip->n;
  const int32_t wext = ip->w_ext_q;
  uint32_t flags = 0, rout = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    uint32_t r = (r4 >> (8 * j)) & 0xFFu;
    const uint32_t local = lq * 4u + uint32_t(j);
    if (local < n) {
      const uint32_t p = population(ip, local);
      const uint32_t off = ip->thr_off[p];
      const uint32_t len = ip->thr_len[p];
      uint32_t T = 0;
      while (T < len && x.v[j] >= thr[off + T]) ++T;
      if (r == 0) {
        const float a = k.p22 * u[j];
        const float b = k.p21 * i[j];
        float xm = a + b;
        if (xm >= kTheta) {
          flags |= 1u << j;
          xm = 0.0f;
          r = kRefSteps;
        }
        u[j] = xm;
      } else {
        u[j] = 0.0f;
        r -= 1;
      }
      const int32_t q = int32_t(T) * wext + w[j];
      const float c = k.p11 * i[j];
      const float e = __int2float_rn(q) * 0x1p-8f;
      i[j] = c + e;
      tsum += T;
      consumed += w[j];
    }
    rout |= r << (8 * j);
  }
  r4 = rout;
  return flags;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const uint32_t lane = __lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Wave-level compaction of up to 4 spikes per lane: this lane's offset in the
// wave's output and the wave's total.
__device__ __forceinline__ void wave_compact(uint32_t flags, uint32_t &lane_off, uint32_t &total) {
  const uint64_t lt = lanemask_lt();
  lane_off = 0;
  total = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint64_t b = __ballot((flags >> j) & 1u);
    lane_off += __popcll(b & lt);
    total += __popcll(b);
  }
}

__device__ __forceinline__ float4 ld4(const float *p) { return *reinterpret_cast<const float4 *>(p); }

// ---------------------------------------------------------------------------
// Stepwise engine, kernel 1 of 2: update every neuron for step t, read and
// clear ring row t, append spikes to the step's sender list and the raster.
// ---------------------------------------------------------------------------
template <int BS>
__global__ __launch_bounds__(BS) void k_update(DeviceNet d, uint32_t k_step) {
  constexpr int NW = BS / 64;
  __shared__ uint32_t s_wave[NW];
  __shared__ uint32_t s_base;
  __shared__ unsigned long long s_rbase;
  const uint64_t t = d.ctl->t_base + k_step;
  const uint32_t slot = uint32_t(t & 1u);
  const uint32_t q = blockIdx.x * BS + threadIdx.x;
  const uint32_t wave = threadIdx.x >> 6;
  if (blockIdx.x == 0 && threadIdx.x == 0) d.ctl->spk_cnt[slot ^ 1u] = 0;

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
    uint32_t r4 = d.R4[q];
    flags = update_quad(ip, d.thr, lq, t, k, u, i, r4, w, tsum, consumed);
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
// Stepwise engine, kernel 2 of 2: push transfer (lst:push2).  The senders of
// step t and their storage segments are staged in LDS with an exclusive
// prefix over segment lengths; the whole grid then strides over the
// concatenated synapse range, one synapse per thread per iteration, and adds
// each weight to W[(t + d) mod 64][target] with a device-scope int32 atomic.
// ---------------------------------------------------------------------------
constexpr int kSegCap = 1024;

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

template <int BS, bool COMP>
__global__ __launch_bounds__(BS) void k_transfer(DeviceNet d, uint32_t k_step) {
  constexpr int IPT = kSegCap / BS;
  __shared__ uint64_t s_start[kSegCap];
  __shared__ uint32_t s_excl[kSegCap];
  __shared__ uint32_t s_tbase[kSegCap];
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
    // Stage this thread's IPT consecutive segments.
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
        s_start[s] = st;
        s_tbase[s] = ip->gbase + (win << kTargetBlockBits);
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

    for (uint32_t e = blockIdx.x * BS + threadIdx.x; e < total; e += gridDim.x * BS) {
      // last segment whose exclusive prefix is <= e (empty segments skipped)
      uint32_t lo = 0, hi = nseg;
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (s_excl[mid] <= e) lo = mid; else hi = mid;
      }
      const uint64_t idx = s_start[lo] + (e - s_excl[lo]);
      uint32_t tgt, dl;
      int32_t wq;
      if (COMP) {
        tgt = s_tbase[lo] + d.tgt16[idx];
        wq = int32_t(d.w16[idx]) * 8;
        dl = d.d8[idx];
      } else {
        const uint64_t rec = d.rec8[idx];
        const uint32_t hiw = uint32_t(rec >> 32);
        wq = int32_t(uint32_t(rec));
        tgt = hiw >> 6;
        dl = hiw & 63u;
      }
      atomicAdd(d.W + size_t((t + dl) & (kRing - 1)) * d.ntot + tgt, wq);
    }
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
    hipLaunchKernelGGL(k_update<BS>, dim3(ublocks), dim3(BS), 0, s, d, k);
    if (d.syn_format == SNN_SYN_COMPRESSED5)
      hipLaunchKernelGGL((k_transfer<BS, true>), dim3(sh.scatter_blocks), dim3(BS), 0, s, d, k);
    else
      hipLaunchKernelGGL((k_transfer<BS, false>), dim3(sh.scatter_blocks), dim3(BS), 0, s, d, k);
  }
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, d.ctl, n);
  return hipGetLastError();
}

}  // namespace snn
