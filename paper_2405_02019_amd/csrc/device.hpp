// device.hpp -- device helpers shared by the step-loop kernels (kernels.hip,
// band.hip): the FP32 neuron update of eqn:mem / eqn:psc / eqn:ref,
// population codes, wave-level compaction and prefix sums, and the
// device-coherent loads and stores that carry data between blocks.
#pragma once

#include "engine.hpp"

namespace snn {

struct Props {
  float p11, p22, p21;
};

__device__ __forceinline__ uint32_t population(const InstDev *__restrict__ ip, uint32_t local) {
  uint32_t p = 0;
#pragma unroll
  for (int k = 1; k < 8; ++k) p += local >= ip->pop_off[k] ? 1u : 0u;
  return p;
}

// Population code of a quad: 3 bits per neuron, and bit 12 + m set when
// neuron m is a real neuron of the instance (not padding).
__device__ __forceinline__ uint32_t quad_code(const InstDev *__restrict__ ip, uint32_t lq) {
  uint32_t c = 0;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const uint32_t local = lq * 4u + uint32_t(m);
    if (local < ip->n) c |= (population(ip, local) << (3 * m)) | (1u << (12 + m));
  }
  return c;
}

// lif_quad for quads whose padding neurons hold u = i = 0 and r = 0: such a
// neuron stays at 0 below the threshold, so every lane updates all four
// neurons without tests or branches.  Same arithmetic as lif_quad (the
// stepwise and persistent kernels).
__device__ __forceinline__ uint32_t lif_quad_padded(Props k, float (&u)[4], const float (&i)[4],
                                                    uint32_t &r4) {
  uint32_t flags = 0, rout = 0;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const uint32_t r = (r4 >> (8 * m)) & 0xFFu;
    const float a = k.p22 * u[m];
    const float b = k.p21 * i[m];
    const float xm = a + b;
    const bool spike = r == 0 && xm >= kTheta;
    u[m] = (r == 0 && !spike) ? xm : 0.0f;
    const uint32_t rn = spike ? kRefSteps : (r ? r - 1u : 0u);
    flags |= uint32_t(spike) << m;
    rout |= rn << (8 * m);
  }
  r4 = rout;
  return flags;
}

// eqn:psc: I <- p11 I + (T w_ext + W) 2^-8, the input summed as an integer.
__device__ __forceinline__ float next_current(float i, int32_t T, int32_t wext, int32_t w,
                                              float p11) {
  const int32_t q = T * wext + w;
  const float c = p11 * i;
  const float e = __int2float_rn(q) * 0x1p-8f;
  return c + e;
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

// A 64-bit value from its two 32-bit halves.  The lane builtins return int:
// their results must reach here as uint32_t, or a low half with bit 31 set
// is sign-extended over the high half (record indices of networks with more
// than 2^31 record slots).
__device__ __forceinline__ uint64_t join64(uint32_t hi, uint32_t lo) {
  return (uint64_t(hi) << 32) | uint64_t(lo);
}

__device__ __forceinline__ uint32_t ld_ag(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_ag(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_ag(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_ag(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive prefix sum of v over the wave's lanes, and the wave's total: one
// ballot per bit of v, so the cost grows with the bit length of the largest
// value, not with the lane count (all lanes active).
__device__ __forceinline__ uint32_t wave_prefix(uint32_t v, uint32_t &total) {
  uint32_t p = 0, tot = 0;
  for (uint32_t b = 0; b < 32u && __ballot(int(v >> b)) != 0ull; ++b) {
    const uint64_t m = __ballot(int((v >> b) & 1u));
    p += __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u)) << b;
    tot += uint32_t(__popcll(m)) << b;
  }
  total = tot;
  return p;
}

}  // namespace snn
