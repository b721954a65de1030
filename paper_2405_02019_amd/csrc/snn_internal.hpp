// snn_internal.hpp -- definitions shared by the simulator library's own
// translation units (host sampler, runtime and HIP kernels).
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/snn.h"

#if defined(__HIPCC__)
#define SNN_HD __host__ __device__
#else
#define SNN_HD
#endif

namespace snn {

// Ring buffer of 64 rows: delays are 1..63 steps (Sec. 3.2).
constexpr int kRing = 64;
constexpr int kMaxDelay = kRing - 1;
// Refractory period 2 ms = 20 steps of 0.1 ms; threshold -50 mV = 15 mV above
// the resting potential (tab:params).
constexpr int kRefSteps = 20;
constexpr float kTheta = 15.0f;
// Neurons of an instance are padded to whole waves of quads (64 x 4), so a
// wavefront never mixes two instances.
constexpr uint32_t kInstAlign = 256;
constexpr uint32_t kTargetBlockBits = 16;  // compressed targets: 16-bit offsets
constexpr uint32_t kNoWindows = 1u << 26;   // window size meaning "one segment per sender"
constexpr int kMaxPoisson = 64;            // longest thalamic table
constexpr uint32_t kMaxInstances = 256;

// Philox counter word 3 names the random stream.
constexpr uint32_t kStreamSynapse = 1;   // (k, 2 * pair + half, 0)
constexpr uint32_t kStreamInitialV = 2;  // (neuron, 0, 0)
constexpr uint32_t kStreamThalamic = 3;  // (neuron / 4, step lo, step hi)

// Philox4x32-10 of Salmon et al. (SC'11): ten rounds of two 32x32->64-bit
// multiplications with the Philox constants, XOR with the round key, and a
// word permutation; the key advances by the golden-ratio Weyl increments.
struct Philox4 {
  uint32_t v[4];
};

SNN_HD inline Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                    uint32_t k0, uint32_t k1) {
#if defined(__HIPCC__)
#pragma unroll
#endif
  for (int r = 0; r < 10; ++r) {
    const uint64_t a = uint64_t(0xD2511F53u) * c0;
    const uint64_t b = uint64_t(0xCD9E8D57u) * c2;
    const uint32_t n0 = uint32_t(b >> 32) ^ c1 ^ k0;
    const uint32_t n2 = uint32_t(a >> 32) ^ c3 ^ k1;
    c1 = uint32_t(b);
    c3 = uint32_t(a);
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return Philox4{{c0, c1, c2, c3}};
}

// Delay bands of the banded LDS engine (Sec. 3.4, lst:horizon2, with the
// one-step delays split off): with H ring rows, band 0 holds the synapses of
// delay 1 and slow band j >= 1 those of delays [2 + (j-1) H, 1 + j H]
// (clipped at 63).  A spike of step s is delivered band by band: band j at
// step s + band_lo(j), when its rows all lie inside the H live rows.
SNN_HD constexpr uint32_t band_count(uint32_t H) { return 1u + (62u + H - 1u) / H; }
SNN_HD constexpr uint32_t band_lo(uint32_t j, uint32_t H) { return j == 0 ? 1u : 2u + (j - 1u) * H; }
SNN_HD constexpr uint32_t band_of(uint32_t d, uint32_t H) { return d <= 1 ? 0u : 1u + (d - 2u) / H; }
// Compressed banded records: weight (16 bits) << 16 | (delay - band_lo) << OB
// | offset in the window (OB bits), OB = 16 - log2(H).
SNN_HD constexpr uint32_t band_offset_bits(uint32_t H) {
  return H >= 64 ? 10u : H >= 32 ? 11u : H >= 16 ? 12u : H >= 8 ? 13u : 0u;
}
// Deviation-format banded locators (Sec. 5.3: the pair's mean and the band's
// first delay implicit): doubled-pair bit << 15 | (delay - band_lo) << OD |
// offset in the window (OD bits), OD = 15 - log2(H); the 8-bit deviation is a
// parallel stream, -128 marking an unused slot.
SNN_HD constexpr uint32_t band_dev_offset_bits(uint32_t H) {
  return band_offset_bits(H) ? band_offset_bits(H) - 1u : 0u;
}

// Per-instance table the kernels read (device memory, uniform per wave).
struct InstDev {
  uint64_t seed;
  uint32_t gbase;        // first global neuron id (multiple of kInstAlign)
  uint32_t n;            // neurons
  uint32_t npad;         // neurons rounded up to kInstAlign
  int32_t w_ext_q;       // thalamic weight, 2^-8 pA
  uint32_t pop_off[9];   // local population boundaries
  uint32_t thr_off[8];   // first threshold of each population in the table
  uint32_t thr_len[8];
  uint32_t seg_base;     // first segment of the instance
  uint32_t nwin;         // segments per sender: target windows the instance overlaps
  uint32_t win_first;    // global index of the first of those windows
  uint32_t win_size;     // neurons per target window
  uint32_t tbase0;       // global id of the first target of window 0 of the instance
  int32_t dev_mq[16];    // deviation format: mean weight of (sender population, doubled pair)
  int32_t dev_sq[16];    // and its step, both in 2^-8 pA; index 2 * population + doubled
};

// FP32 propagators, computed in FP64 on the device (eqn:p11p22, eqn:p21).
struct DevConsts {
  float p11, p22, p21, pad;
  double p11d, p22d, p21d, padd;
};

// Host side of one instance after sampling.
struct HostInstance {
  snn_instance_cfg cfg{};
  std::vector<double> conn;          // 64, [target][source]
  uint32_t n = 0;
  uint32_t pop_off[9] = {};
  uint64_t pair_count[64] = {};      // [target * 8 + source]
  uint64_t nsyn = 0;
  double w_f = 0.0, w_ext = 0.0;
  int32_t w_ext_q = 0;
  uint32_t thr[8][kMaxPoisson] = {};
  uint32_t thr_len[8] = {};
  std::vector<float> u0;
  // Storage: one segment per (sender, target window); windows of win_size
  // neurons are aligned at multiples of win_size in the coordinate
  // win_origin + local id; [n * nwin + 1] pointers into the record streams.
  uint32_t win_size = 0, win_origin = 0, win_first = 0;
  uint32_t nwin = 1;
  std::vector<uint64_t> seg_ptr;     // compact layout: segment pointers
  // Padded layout: segment (sender s of population c, window w) holds
  // cls_cap[w * 8 + c] record slots starting at
  // cls_base[w * 8 + c] + (s - pop_off[c]) * cls_cap[w * 8 + c]; unused
  // slots have delay 0.  outdeg[s] counts the sender's real synapses.
  bool padded = false;
  uint32_t band_h = 0;               // banded layout: ring rows of the engine, else 0
  uint32_t nband = 1;                // delay bands per (sender, window)
  std::vector<uint64_t> cls_base;
  std::vector<uint32_t> cls_cap;
  std::vector<uint32_t> outdeg;
  uint64_t nrec = 0;                 // record slots (== nsyn unless padded)
  std::vector<uint64_t> rec8;        // plain: w_q | (target << 6 | delay) << 32
  std::vector<uint32_t> rec4;        // compressed, padded layout: w16 << 16 | delay << 10 | offset
  std::vector<uint16_t> tgt16;       // compressed streams
  std::vector<int16_t> w16;
  std::vector<uint8_t> d8;
  std::vector<uint16_t> rec2;        // deviation format: doubled << 15 | delay << 9 | offset
  std::vector<int8_t> dev8;          // and the weight's deviation from its pair's mean
  int32_t dev_mq[16] = {};           // mean weight of (sender population, doubled pair), 2^-8 pA
  int32_t dev_sq[16] = {};           // deviation step of the same, 2^-8 pA
};

// Model (model.cpp).
struct ModelConstants {
  double w_f, p11, p22, p21;
};
ModelConstants model_constants();
int pair_counts(const snn_instance_cfg &cfg, const std::vector<double> &conn,
                const uint32_t n_pop[8], uint64_t out[64], std::string &err);
int poisson_thresholds(double lam, uint32_t *thr, uint32_t cap, uint32_t *len, std::string &err);
void population_sizes(double scale, uint32_t n_pop[8]);
std::vector<double> connectivity(const snn_instance_cfg &cfg);
extern const uint32_t kPopFull[8];
extern const uint32_t kKext[8];

// Sampler (builder.cpp).  Rows are split into target windows of win_size
// neurons aligned in the coordinate win_origin + local id (win_size >= 2^26:
// one segment per sender); `pad` selects the fixed-capacity layout.  Plain
// records hold instance-local targets (the runtime offsets them by the
// instance's first global id on upload); compressed records hold the
// target's offset inside its window (< 2^16).
int sample_instance(const snn_instance_cfg &cfg, uint32_t syn_format, uint32_t win_size,
                    uint32_t win_origin, bool pad, int threads, HostInstance &out,
                    std::string &err);
// Banded layout (band.hip): windows of win_size neurons from the instance's
// first neuron, segments per (sender, window, delay band) for a ring of
// band_h rows; cls_cap / cls_base are indexed [(window * nband + band) * 8 +
// class].  Plain records as above; compressed records weight << 16 | (delay -
// band_lo) << band_offset_bits | offset in the window; deviation-format
// locators as band_dev_offset_bits describes, with the deviation stream.
int sample_instance_banded(const snn_instance_cfg &cfg, uint32_t syn_format, uint32_t win_size,
                           uint32_t band_h, int threads, HostInstance &out, std::string &err);
// Population sizes of an instance (for placement before sampling).
uint32_t instance_neurons(const snn_instance_cfg &cfg);
// Longest thalamic count table of an instance's populations.
uint32_t thalamic_table_max(const snn_instance_cfg &cfg);

}  // namespace snn
