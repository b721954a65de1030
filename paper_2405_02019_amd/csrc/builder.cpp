// builder.cpp -- host sampler of one microcircuit instance (Sec. 2.2) and its
// sender-sorted synapse storage (Sec. 3.5, lst:index), written straight into
// the device record formats.
//
// Each synapse k of the population pair (target b, source a) is a pure
// function of (seed, b, a, k): two Philox4x32-10 blocks give its sender,
// receiver, weight deviate and delay deviate.  The sampler therefore runs on
// any number of threads in two passes over the generation order
// (b, a, k): pass 1 counts synapses per storage segment and thread, a prefix
// sum turns the counts into per-thread write cursors, and pass 2 regenerates
// every synapse and writes it at its cursor.  Segments keep generation order,
// so the result does not depend on the thread count.
//
// Two layouts: compact segments addressed through a pointer array (sender
// rows, optionally split by target window), or fixed-capacity segments per
// (sender, window) whose capacity is the largest segment of the sender's
// population in that window, so the address is computable from the sender.
//
// Model readings: weights Normal(mu, 0.1 |mu|) with mu = w_f * PSP,
// PSP = 0.15 mV (excitatory sender), g * 0.15 mV (inhibitory sender), 0.30 mV
// for L4e -> L23e; a weight that would change sign becomes 0.  Delays
// Normal(1.5, 0.75) ms / Normal(0.75, 0.375) ms in 0.1 ms steps, rounded half
// to even and clipped to [1, 63].  Initial potentials Normal(mean, sd) of
// tab:params2, stored relative to -65 mV.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <thread>

#include "snn_internal.hpp"

namespace snn {
namespace {

constexpr double kTwoPi = 6.283185307179586;

inline double unit_open(uint32_t w) { return (double(w) + 0.5) * 0x1p-32; }

// Box-Muller (cosine branch) from two 32-bit words.
inline double gauss(uint32_t a, uint32_t b) {
  return std::sqrt(-2.0 * std::log(unit_open(a))) * std::cos(kTwoPi * unit_open(b));
}

inline uint32_t scale_word(uint32_t w, uint32_t n) { return uint32_t((uint64_t(w) * n) >> 32); }

const double kV0Mean[8] = {-68.28, -63.16, -63.33, -63.45, -63.11, -61.66, -66.72, -61.43};
const double kV0Sd[8] = {5.36, 4.57, 4.74, 4.94, 4.94, 4.55, 5.46, 4.48};

struct Pair {
  uint64_t first;   // generation index of synapse 0 of the pair
  uint64_t count;
  uint32_t tgt, src;
  uint32_t tgt0, ntgt, src0, nsrc;
  double mu_w, sd_w, mu_d, sd_d;
};

template <class F>
void parallel_for(int threads, F &&f) {
  std::vector<std::thread> pool;
  for (int t = 1; t < threads; ++t) pool.emplace_back(f, t);
  f(0);
  for (auto &th : pool) th.join();
}

}  // namespace

uint32_t instance_neurons(const snn_instance_cfg &cfg) {
  uint32_t n_pop[8];
  population_sizes(cfg.scale, n_pop);
  uint32_t n = 0;
  for (int p = 0; p < 8; ++p) n += n_pop[p];
  return n;
}

uint32_t thalamic_table_max(const snn_instance_cfg &cfg) {
  if (cfg.bg_const_T >= 0) return uint32_t(cfg.bg_const_T);
  uint32_t m = 0, thr[kMaxPoisson], len = 0;
  std::string err;
  for (int p = 0; p < 8; ++p) {
    const double lam = (cfg.bg_rate_hz * double(kKext[p])) * 1e-4;
    if (poisson_thresholds(lam, thr, kMaxPoisson, &len, err) != SNN_OK) return kMaxPoisson + 1;
    m = std::max(m, len);
  }
  return m;
}

namespace {

// Everything of an instance but its synapses: populations, pair counts,
// weights of the thalamic drive and its count tables, initial potentials,
// and the population pairs in generation order (target-major).
int prepare_instance(const snn_instance_cfg &cfg, uint32_t syn_format, int &threads,
                     HostInstance &out, std::vector<Pair> &pairs, uint32_t n_pop[8], uint32_t &tmax,
                     std::string &err) {
  if (!(cfg.scale > 0.0 && cfg.scale <= 64.0)) {
    err = "scale must lie in (0, 64]";
    return SNN_E_INVAL;
  }
  if (!(cfg.g <= 0.0) || !(cfg.bg_rate_hz >= 0.0) || !(cfg.psp_ext_mv >= 0.0)) {
    err = "need g <= 0, bg_rate_hz >= 0 and psp_ext_mv >= 0";
    return SNN_E_INVAL;
  }
  if (syn_format != SNN_SYN_PLAIN8 && syn_format != SNN_SYN_COMPRESSED5 &&
      syn_format != SNN_SYN_DEV8) {
    err = "unknown synapse format";
    return SNN_E_INVAL;
  }
  if (threads <= 0) {
    unsigned hc = std::thread::hardware_concurrency();
    threads = int(std::min(16u, std::max(1u, hc)));
  }
  out.cfg = cfg;
  out.cfg.conn = nullptr;
  out.conn = connectivity(cfg);

  population_sizes(cfg.scale, n_pop);
  out.pop_off[0] = 0;
  for (int p = 0; p < 8; ++p) out.pop_off[p + 1] = out.pop_off[p] + n_pop[p];
  out.n = out.pop_off[8];
  if (out.n == 0) {
    err = "the scale leaves no neurons";
    return SNN_E_INVAL;
  }
  if (out.n >= (1u << 26)) {
    err = "more than 2^26 neurons per instance";
    return SNN_E_RANGE;
  }
  int rc = pair_counts(cfg, out.conn, n_pop, out.pair_count, err);
  if (rc) return rc;

  const ModelConstants mc = model_constants();
  out.w_f = mc.w_f;
  out.w_ext = mc.w_f * cfg.psp_ext_mv;
  const double wq_ext = std::nearbyint(out.w_ext * 256.0);
  if (!(std::fabs(wq_ext) < 2147483647.0)) {
    err = "thalamic weight does not fit int32 fixed point";
    return SNN_E_RANGE;
  }
  out.w_ext_q = int32_t(wq_ext);

  // Thalamic drive: Poisson with mean v_th K dt (dt = 1e-4 s), or a constant.
  tmax = 0;
  for (int p = 0; p < 8; ++p) {
    if (cfg.bg_const_T >= 0) {
      if (cfg.bg_const_T > kMaxPoisson) {
        err = "constant thalamic count above 64";
        return SNN_E_INVAL;
      }
      for (int k = 0; k < cfg.bg_const_T; ++k) out.thr[p][k] = 0;
      out.thr_len[p] = uint32_t(cfg.bg_const_T);
    } else {
      const double lam = (cfg.bg_rate_hz * double(kKext[p])) * 1e-4;
      rc = poisson_thresholds(lam, out.thr[p], kMaxPoisson, &out.thr_len[p], err);
      if (rc) return rc;
    }
    tmax = std::max(tmax, out.thr_len[p]);
  }

  // Initial membrane potentials.
  out.u0.assign(out.n, 0.0f);
  for (int p = 0; p < 8; ++p)
    for (uint32_t i = out.pop_off[p]; i < out.pop_off[p + 1]; ++i) {
      const Philox4 r = philox4x32_10(i, 0, 0, kStreamInitialV, uint32_t(cfg.seed),
                                      uint32_t(cfg.seed >> 32));
      const double v = kV0Mean[p] + kV0Sd[p] * gauss(r.v[0], r.v[1]);
      out.u0[i] = float(v - (-65.0));
    }

  // Population pairs in generation order (target-major).
  pairs.clear();
  uint64_t S = 0;
  const double w_f = mc.w_f;
  for (uint32_t b = 0; b < 8; ++b)
    for (uint32_t a = 0; a < 8; ++a) {
      const uint64_t c = out.pair_count[b * 8 + a];
      if (!c) continue;
      Pair pr{};
      pr.first = S;
      pr.count = c;
      pr.tgt = b;
      pr.src = a;
      pr.tgt0 = out.pop_off[b];
      pr.ntgt = n_pop[b];
      pr.src0 = out.pop_off[a];
      pr.nsrc = n_pop[a];
      const bool exc = (a % 2) == 0;
      double psp = exc ? 0.15 : cfg.g * 0.15;
      if (b == 0 && a == 2) psp = 2.0 * 0.15;
      pr.mu_w = psp * w_f;
      pr.sd_w = 0.1 * std::fabs(pr.mu_w);
      pr.mu_d = exc ? 15.0 : 7.5;
      pr.sd_d = exc ? 7.5 : 3.75;
      pairs.push_back(pr);
      S += c;
      // Deviation format (Sec. 5.3: weights as deviations from the mean of
      // their Gaussian): the mean of the pair and a step of 5 sd / 127, both
      // in 2^-8 pA.  Pairs of one sender population share them, except the
      // doubled L4e -> L2/3e pair.
      const int di = int(2 * a + ((b == 0 && a == 2) ? 1 : 0));
      const double st = std::nearbyint(5.0 * pr.sd_w * 256.0 / 127.0);
      out.dev_mq[di] = int32_t(std::nearbyint(pr.mu_w * 256.0));
      out.dev_sq[di] = st < 1.0 ? 1 : int32_t(st);
    }
  out.nsyn = S;

  return SNN_OK;
}

}  // namespace

int sample_instance(const snn_instance_cfg &cfg, uint32_t syn_format, uint32_t win_size,
                    uint32_t win_origin, bool pad, int threads, HostInstance &out,
                    std::string &err) {
  std::vector<Pair> pairs;
  uint32_t n_pop[8], tmax = 0;
  int rc = prepare_instance(cfg, syn_format, threads, out, pairs, n_pop, tmax, err);
  if (rc) return rc;
  const uint64_t S = out.nsyn;
  const bool comp = syn_format == SNN_SYN_COMPRESSED5;
  const bool dev = syn_format == SNN_SYN_DEV8;
  if (dev && (!pad || win_size > 512)) {
    err = "the deviation format needs the LDS engine's layout (windows of at most 512 neurons)";
    return SNN_E_INVAL;
  }
  if (win_size == 0 || (comp && win_size > (1u << kTargetBlockBits))) {
    err = "target windows must hold 1 .. 65,536 neurons for 16-bit target offsets";
    return SNN_E_RANGE;
  }
  const uint64_t wlo = uint64_t(win_origin) / win_size;
  const uint64_t whi = (uint64_t(win_origin) + out.n - 1) / win_size;
  const uint32_t nwin = uint32_t(whi - wlo + 1);
  out.win_size = win_size;
  out.win_origin = win_origin;
  out.win_first = uint32_t(wlo);
  out.nwin = nwin;
  const uint64_t nseg = uint64_t(out.n) * nwin;
  // target window of a receiver, relative to the instance's first window
  auto window = [&](uint32_t post) {
    return uint32_t((uint64_t(win_origin) + post) / win_size - wlo);
  };
  const uint32_t key0 = uint32_t(cfg.seed), key1 = uint32_t(cfg.seed >> 32);

  // Thread ranges over the generation order.
  const int P = int(std::max<uint64_t>(1, std::min<uint64_t>(uint64_t(threads), S ? S : 1)));
  std::vector<uint64_t> lo(P + 1);
  for (int t = 0; t <= P; ++t) lo[t] = S / P * t + std::min<uint64_t>(S % P, t);

  auto locate = [&](uint64_t e) {  // pair containing generation index e
    size_t i = std::upper_bound(pairs.begin(), pairs.end(), e,
                                [](uint64_t v, const Pair &p) { return v < p.first; }) -
               pairs.begin();
    return i - 1;
  };

  // Pass 1: per-thread segment counts.
  std::vector<std::vector<uint64_t>> cur(P);
  parallel_for(P, [&](int t) {
    std::vector<uint64_t> &h = cur[t];
    h.assign(nseg, 0);
    if (lo[t] == lo[t + 1]) return;
    size_t pi = locate(lo[t]);
    for (uint64_t e = lo[t]; e < lo[t + 1]; ++e) {
      while (e >= pairs[pi].first + pairs[pi].count) ++pi;
      const Pair &pr = pairs[pi];
      const uint32_t k = uint32_t(e - pr.first);
      const uint32_t code = 2u * (pr.tgt * 8u + pr.src);
      const Philox4 r = philox4x32_10(k, code, 0, kStreamSynapse, key0, key1);
      const uint32_t pre = pr.src0 + scale_word(r.v[0], pr.nsrc);
      const uint32_t post = pr.tgt0 + scale_word(r.v[1], pr.ntgt);
      h[uint64_t(pre) * nwin + window(post)] += 1;
    }
  });

  auto seg_len = [&](uint64_t s) {
    uint64_t c = 0;
    for (int t = 0; t < P; ++t) c += cur[t][s];
    return c;
  };
  out.padded = pad;
  if (!pad) {
    // Segment pointers and per-thread cursors (segment-major, thread-minor).
    out.seg_ptr.assign(nseg + 1, 0);
    uint64_t run = 0;
    for (uint64_t s = 0; s < nseg; ++s) {
      out.seg_ptr[s] = run;
      for (int t = 0; t < P; ++t) {
        const uint64_t c = cur[t][s];
        cur[t][s] = run;
        run += c;
      }
    }
    out.seg_ptr[nseg] = run;
    out.nrec = run;
  } else {
    // Fixed-capacity segments: every sender of population c owns cap[w][c]
    // record slots in window w, so a segment's address follows from the
    // sender's id alone; unused slots keep delay 0.
    out.seg_ptr.clear();
    out.cls_cap.assign(size_t(nwin) * 8, 0);
    out.cls_base.assign(size_t(nwin) * 8, 0);
    out.outdeg.assign(out.n, 0);
    for (int c = 0; c < 8; ++c)
      for (uint32_t pre = out.pop_off[c]; pre < out.pop_off[c + 1]; ++pre)
        for (uint32_t w = 0; w < nwin; ++w) {
          const uint64_t len = seg_len(uint64_t(pre) * nwin + w);
          out.outdeg[pre] += uint32_t(len);
          uint32_t &cp = out.cls_cap[size_t(w) * 8 + c];
          if (len > cp) cp = uint32_t(len);
        }
    uint64_t run = 0;
    for (uint32_t w = 0; w < nwin; ++w)
      for (int c = 0; c < 8; ++c) {
        out.cls_base[size_t(w) * 8 + c] = run;
        run += uint64_t(n_pop[c]) * out.cls_cap[size_t(w) * 8 + c];
      }
    out.nrec = run;
    for (int c = 0; c < 8; ++c)
      for (uint32_t pre = out.pop_off[c]; pre < out.pop_off[c + 1]; ++pre)
        for (uint32_t w = 0; w < nwin; ++w) {
          const uint64_t s = uint64_t(pre) * nwin + w;
          uint64_t at = out.cls_base[size_t(w) * 8 + c] +
                        uint64_t(pre - out.pop_off[c]) * out.cls_cap[size_t(w) * 8 + c];
          for (int t = 0; t < P; ++t) {
            const uint64_t cnt = cur[t][s];
            cur[t][s] = at;
            at += cnt;
          }
        }
  }

  const uint64_t R = out.nrec;
  // Compressed records of the padded layout pack into one 32-bit word: the
  // 16-bit weight, the delay (6 bits) and the offset in the window (10 bits).
  const bool pack4 = comp && pad;
  if (pack4 && win_size > 1024) {
    err = "packed compressed records need target windows of at most 1,024 neurons";
    return SNN_E_RANGE;
  }
  out.rec8.clear();
  out.rec4.clear();
  out.tgt16.clear();
  out.w16.clear();
  out.d8.clear();
  out.rec2.clear();
  out.dev8.clear();
  if (dev) {
    out.rec2.assign(R, 0);
    out.dev8.assign(R, 0);
  } else if (pack4) {
    out.rec4.assign(R, 0);
  } else if (comp) {
    out.tgt16.assign(R, 0);
    out.w16.assign(R, 0);
    out.d8.assign(R, 0);
  } else {
    out.rec8.assign(R, 0);
  }

  // Pass 2: regenerate and place; per-thread worst-case input per receiver.
  std::atomic<int> bad{0};
  std::vector<std::vector<int64_t>> insum(P);
  parallel_for(P, [&](int t) {
    std::vector<uint64_t> &c = cur[t];
    std::vector<int64_t> &in = insum[t];
    in.assign(out.n, 0);
    if (lo[t] == lo[t + 1]) return;
    size_t pi = locate(lo[t]);
    for (uint64_t e = lo[t]; e < lo[t + 1]; ++e) {
      while (e >= pairs[pi].first + pairs[pi].count) ++pi;
      const Pair &pr = pairs[pi];
      const uint32_t k = uint32_t(e - pr.first);
      const uint32_t code = 2u * (pr.tgt * 8u + pr.src);
      const Philox4 r = philox4x32_10(k, code, 0, kStreamSynapse, key0, key1);
      const Philox4 s = philox4x32_10(k, code + 1u, 0, kStreamSynapse, key0, key1);
      const uint32_t pre = pr.src0 + scale_word(r.v[0], pr.nsrc);
      const uint32_t post = pr.tgt0 + scale_word(r.v[1], pr.ntgt);
      double w = pr.mu_w + pr.sd_w * gauss(r.v[2], r.v[3]);
      if (pr.mu_w > 0.0 && w < 0.0) w = 0.0;
      if (pr.mu_w < 0.0 && w > 0.0) w = 0.0;
      const double dr = std::nearbyint(pr.mu_d + pr.sd_d * gauss(s.v[0], s.v[1]));
      const uint32_t d = dr < 1.0 ? 1u : (dr > double(kMaxDelay) ? uint32_t(kMaxDelay) : uint32_t(dr));
      const uint64_t seg = uint64_t(pre) * nwin + window(post);
      const uint64_t pos = c[seg]++;
      int32_t wq;
      if (dev) {
        // mean + deviation * step, the deviation rounded half to even and
        // clipped to 8 bits.
        const uint32_t dbl = (pr.tgt == 0 && pr.src == 2) ? 1u : 0u;
        const int di = int(2 * pr.src + dbl);
        const int32_t mq = out.dev_mq[di], sq = out.dev_sq[di];
        const double r = std::nearbyint((w * 256.0 - double(mq)) / double(sq));
        const int32_t dv = r < -127.0 ? -127 : (r > 127.0 ? 127 : int32_t(r));
        const uint32_t off = uint32_t((uint64_t(win_origin) + post) % win_size);
        out.rec2[pos] = uint16_t((dbl << 15) | (d << 9) | off);
        out.dev8[pos] = int8_t(dv);
        wq = mq + dv * sq;
      } else if (comp) {
        const double q = std::nearbyint(w * 32.0);
        if (!(q >= -32768.0 && q <= 32767.0)) {
          bad.store(2);
          continue;
        }
        const uint32_t off = uint32_t((uint64_t(win_origin) + post) % win_size);
        if (pack4) {
          out.rec4[pos] = (uint32_t(uint16_t(int16_t(q))) << 16) | (d << 10) | off;
        } else {
          out.tgt16[pos] = uint16_t(off);
          out.w16[pos] = int16_t(q);
          out.d8[pos] = uint8_t(d);
        }
        wq = int32_t(q) * 8;
      } else {
        const double q = std::nearbyint(w * 256.0);
        if (!(std::fabs(q) < 2147483647.0)) {
          bad.store(1);
          continue;
        }
        wq = int32_t(q);
        out.rec8[pos] = uint64_t(uint32_t(wq)) | (uint64_t((post << 6) | d) << 32);
      }
      in[post] += std::llabs(int64_t(wq));
    }
  });
  if (bad.load() == 2) {
    err = "a weight does not fit the 16-bit compressed encoding";
    return SNN_E_RANGE;
  }
  if (bad.load() == 1) {
    err = "a weight does not fit int32 fixed point";
    return SNN_E_RANGE;
  }
  // Worst case of one step's input: every synapse onto a neuron plus the
  // longest thalamic count must stay inside int32.
  int64_t worst = 0;
  for (uint32_t i = 0; i < out.n; ++i) {
    int64_t s = 0;
    for (int t = 0; t < P; ++t) s += insum[t][i];
    worst = std::max(worst, s);
  }
  worst += int64_t(tmax) * std::llabs(int64_t(out.w_ext_q));
  if (worst >= 2147483647LL) {
    char b[128];
    std::snprintf(b, sizeof b, "worst-case input %lld exceeds the int32 accumulator",
                  (long long)worst);
    err = b;
    return SNN_E_OVERFLOW;
  }
  return SNN_OK;
}


// Banded layout of the banded LDS engine (band.hip): segments per (sender,
// target window, delay band) of fixed capacity -- the largest such segment of
// the sender's population -- so that a segment's address follows from the
// sender's id.  Built in three passes over a sender-sorted copy of the
// network (its rows keep generation order, so the result does not depend on
// the thread count): per-thread row counts, the rows themselves, then per row
// the segment lengths (capacities) and the placement.
int sample_instance_banded(const snn_instance_cfg &cfg, uint32_t syn_format, uint32_t win_size,
                           uint32_t band_h, int threads, HostInstance &out, std::string &err) {
  std::vector<Pair> pairs;
  uint32_t n_pop[8], tmax = 0;
  int rc = prepare_instance(cfg, syn_format, threads, out, pairs, n_pop, tmax, err);
  if (rc) return rc;
  const uint64_t S = out.nsyn;
  const bool comp = syn_format == SNN_SYN_COMPRESSED5;
  const bool dev = syn_format == SNN_SYN_DEV8;
  const uint32_t OB = band_offset_bits(band_h);
  const uint32_t OD = band_dev_offset_bits(band_h);
  if (!OB || (band_h & (band_h - 1u)) || band_h > 64u) {
    err = "ring rows of the banded layout must be 8, 16, 32 or 64";
    return SNN_E_INVAL;
  }
  const uint32_t NB = band_count(band_h);
  if (win_size == 0 || (comp && win_size > (1u << OB)) || (dev && win_size > (1u << OD))) {
    err = "target windows too large for the banded compressed or deviation records";
    return SNN_E_RANGE;
  }
  const uint32_t n = out.n;
  const uint32_t nwin = (n + win_size - 1) / win_size;
  out.win_size = win_size;
  out.win_origin = 0;
  out.win_first = 0;
  out.nwin = nwin;
  out.band_h = band_h;
  out.nband = NB;
  out.padded = true;
  const uint32_t key0 = uint32_t(cfg.seed), key1 = uint32_t(cfg.seed >> 32);

  const int P = int(std::max<uint64_t>(1, std::min<uint64_t>(uint64_t(threads), S ? S : 1)));
  std::vector<uint64_t> lo(P + 1);
  for (int t = 0; t <= P; ++t) lo[t] = S / P * t + std::min<uint64_t>(S % P, t);
  auto locate = [&](uint64_t e) {
    size_t i = std::upper_bound(pairs.begin(), pairs.end(), e,
                                [](uint64_t v, const Pair &p) { return v < p.first; }) -
               pairs.begin();
    return i - 1;
  };

  // Pass 1: synapses per sender and thread.
  std::vector<std::vector<uint32_t>> cur(P);
  parallel_for(P, [&](int t) {
    std::vector<uint32_t> &c = cur[t];
    c.assign(n, 0);
    if (lo[t] == lo[t + 1]) return;
    size_t pi = locate(lo[t]);
    for (uint64_t e = lo[t]; e < lo[t + 1]; ++e) {
      while (e >= pairs[pi].first + pairs[pi].count) ++pi;
      const Pair &pr = pairs[pi];
      const uint32_t k = uint32_t(e - pr.first);
      const Philox4 r = philox4x32_10(k, 2u * (pr.tgt * 8u + pr.src), 0, kStreamSynapse, key0, key1);
      c[pr.src0 + scale_word(r.v[0], pr.nsrc)] += 1;
    }
  });
  std::vector<uint64_t> row(size_t(n) + 1, 0);
  for (uint32_t pre = 0; pre < n; ++pre) {
    uint32_t run = 0;
    for (int t = 0; t < P; ++t) {
      const uint32_t c = cur[t][pre];
      cur[t][pre] = run;
      run += c;
    }
    row[pre + 1] = row[pre] + run;
  }

  // Pass 2: the sender-sorted rows, generation order within a row:
  // low word the weight (2^-8 pA, or 2^-5 pA compressed; deviation format:
  // doubled-pair bit << 8 | the 8-bit deviation), high word receiver << 6 |
  // delay.
  std::vector<uint64_t> tmp(S);
  std::atomic<int> bad{0};
  std::vector<std::vector<int64_t>> insum(P);
  parallel_for(P, [&](int t) {
    std::vector<uint32_t> &c = cur[t];
    std::vector<int64_t> &in = insum[t];
    in.assign(n, 0);
    if (lo[t] == lo[t + 1]) return;
    size_t pi = locate(lo[t]);
    for (uint64_t e = lo[t]; e < lo[t + 1]; ++e) {
      while (e >= pairs[pi].first + pairs[pi].count) ++pi;
      const Pair &pr = pairs[pi];
      const uint32_t k = uint32_t(e - pr.first);
      const uint32_t code = 2u * (pr.tgt * 8u + pr.src);
      const Philox4 r = philox4x32_10(k, code, 0, kStreamSynapse, key0, key1);
      const Philox4 s2 = philox4x32_10(k, code + 1u, 0, kStreamSynapse, key0, key1);
      const uint32_t pre = pr.src0 + scale_word(r.v[0], pr.nsrc);
      const uint32_t post = pr.tgt0 + scale_word(r.v[1], pr.ntgt);
      double w = pr.mu_w + pr.sd_w * gauss(r.v[2], r.v[3]);
      if (pr.mu_w > 0.0 && w < 0.0) w = 0.0;
      if (pr.mu_w < 0.0 && w > 0.0) w = 0.0;
      const double dr = std::nearbyint(pr.mu_d + pr.sd_d * gauss(s2.v[0], s2.v[1]));
      const uint32_t d = dr < 1.0 ? 1u : (dr > double(kMaxDelay) ? uint32_t(kMaxDelay) : uint32_t(dr));
      int32_t wv, wq;
      if (dev) {
        // mean + deviation * step, the deviation rounded half to even and
        // clipped to 8 bits (as the LDS layout's deviation records).
        const uint32_t dbl = (pr.tgt == 0 && pr.src == 2) ? 1u : 0u;
        const int di = int(2 * pr.src + dbl);
        const int32_t mq = out.dev_mq[di], sq = out.dev_sq[di];
        const double q = std::nearbyint((w * 256.0 - double(mq)) / double(sq));
        const int32_t dv = q < -127.0 ? -127 : (q > 127.0 ? 127 : int32_t(q));
        wv = int32_t((dbl << 8) | uint32_t(uint8_t(int8_t(dv))));
        wq = mq + dv * sq;
      } else if (comp) {
        const double q = std::nearbyint(w * 32.0);
        if (!(q >= -32768.0 && q <= 32767.0)) {
          bad.store(2);
          continue;
        }
        wv = int32_t(q);
        wq = wv * 8;
      } else {
        const double q = std::nearbyint(w * 256.0);
        if (!(std::fabs(q) < 2147483647.0)) {
          bad.store(1);
          continue;
        }
        wv = wq = int32_t(q);
      }
      tmp[row[pre] + c[pre]++] = uint64_t(uint32_t(wv)) | (uint64_t((post << 6) | d) << 32);
      in[post] += std::llabs(int64_t(wq));
    }
  });
  cur.clear();
  cur.shrink_to_fit();
  if (bad.load() == 2) {
    err = "a weight does not fit the 16-bit compressed encoding";
    return SNN_E_RANGE;
  }
  if (bad.load() == 1) {
    err = "a weight does not fit int32 fixed point";
    return SNN_E_RANGE;
  }
  int64_t worst = 0;
  for (uint32_t i = 0; i < n; ++i) {
    int64_t s = 0;
    for (int t = 0; t < P; ++t) s += insum[t][i];
    worst = std::max(worst, s);
  }
  insum.clear();
  worst += int64_t(tmax) * std::llabs(int64_t(out.w_ext_q));
  if (worst >= 2147483647LL) {
    char b[128];
    std::snprintf(b, sizeof b, "worst-case input %lld exceeds the int32 accumulator", (long long)worst);
    err = b;
    return SNN_E_OVERFLOW;
  }
  out.outdeg.assign(n, 0);
  for (uint32_t pre = 0; pre < n; ++pre) out.outdeg[pre] = uint32_t(row[pre + 1] - row[pre]);

  // Senders in P contiguous ranges of about equal synapse counts.
  std::vector<uint32_t> sr(P + 1, n);
  sr[0] = 0;
  for (int t = 1; t < P; ++t)
    sr[t] = uint32_t(std::lower_bound(row.begin(), row.end(), S / P * uint64_t(t)) - row.begin());
  for (int t = 1; t <= P; ++t) sr[t] = std::max(sr[t], sr[t - 1]);
  auto cls_of = [&](uint32_t pre) {
    uint32_t c = 0;
    while (pre >= out.pop_off[c + 1]) ++c;
    return c;
  };
  const size_t nkey = size_t(nwin) * NB;   // (window, band) of one sender
  auto key_of = [&](uint64_t rec) {
    const uint32_t hiw = uint32_t(rec >> 32);
    return size_t((hiw >> 6) / win_size) * NB + band_of(hiw & 63u, band_h);
  };

  // Pass 3: capacities, the largest segment per (window, band, class).
  std::vector<std::vector<uint32_t>> capt(P);
  parallel_for(P, [&](int t) {
    std::vector<uint32_t> &cp = capt[t];
    cp.assign(nkey * 8, 0);
    std::vector<uint32_t> cnt(nkey, 0);
    for (uint32_t pre = sr[t]; pre < sr[t + 1]; ++pre) {
      const uint32_t c = cls_of(pre);
      for (uint64_t e = row[pre]; e < row[pre + 1]; ++e) ++cnt[key_of(tmp[e])];
      for (uint64_t e = row[pre]; e < row[pre + 1]; ++e) {
        const size_t kk = key_of(tmp[e]);
        uint32_t &m = cp[kk * 8 + c];
        m = std::max(m, cnt[kk]);
        cnt[kk] = 0;
      }
    }
  });
  out.cls_cap.assign(nkey * 8, 0);
  for (int t = 0; t < P; ++t)
    for (size_t i = 0; i < nkey * 8; ++i) out.cls_cap[i] = std::max(out.cls_cap[i], capt[t][i]);
  capt.clear();
  out.cls_base.assign(nkey * 8, 0);
  uint64_t run = 0;
  for (size_t kk = 0; kk < nkey; ++kk)
    for (int c = 0; c < 8; ++c) {
      out.cls_base[kk * 8 + c] = run;
      run += uint64_t(n_pop[c]) * out.cls_cap[kk * 8 + c];
    }
  out.nrec = run;
  out.rec8.clear();
  out.rec4.clear();
  out.tgt16.clear();
  out.w16.clear();
  out.d8.clear();
  out.rec2.clear();
  out.dev8.clear();
  if (comp) {
    out.rec4.assign(run, 0);
  } else if (dev) {
    out.rec2.assign(run, 0);
    out.dev8.assign(run, int8_t(-128));
  } else {
    out.rec8.assign(run, 0);
  }

  // Pass 4: placement, generation order within a segment.  Unused slots stay
  // zero (weight 0: they add nothing), or hold the deviation -128, which no
  // synapse has.
  parallel_for(P, [&](int t) {
    std::vector<uint64_t> at(nkey, 0);
    std::vector<uint32_t> stamp(nkey, ~0u);
    for (uint32_t pre = sr[t]; pre < sr[t + 1]; ++pre) {
      const uint32_t c = cls_of(pre);
      for (uint64_t e = row[pre]; e < row[pre + 1]; ++e) {
        const uint64_t r = tmp[e];
        const size_t kk = key_of(r);
        if (stamp[kk] != pre) {
          stamp[kk] = pre;
          at[kk] = out.cls_base[kk * 8 + c] + uint64_t(pre - out.pop_off[c]) * out.cls_cap[kk * 8 + c];
        }
        const uint64_t pos = at[kk]++;
        if (comp) {
          const uint32_t hiw = uint32_t(r >> 32), d = hiw & 63u, post = hiw >> 6;
          const uint32_t b = uint32_t(kk % NB);
          out.rec4[pos] = (uint32_t(uint16_t(int16_t(int32_t(uint32_t(r))))) << 16) |
                          ((d - band_lo(b, band_h)) << OB) | (post % win_size);
        } else if (dev) {
          const uint32_t hiw = uint32_t(r >> 32), d = hiw & 63u, post = hiw >> 6;
          const uint32_t b = uint32_t(kk % NB), lw = uint32_t(r);
          out.rec2[pos] = uint16_t(((lw >> 8) << 15) | ((d - band_lo(b, band_h)) << OD) |
                                   (post % win_size));
          out.dev8[pos] = int8_t(uint8_t(lw & 0xFFu));
        } else {
          out.rec8[pos] = r;
        }
      }
    }
  });
  return SNN_OK;
}

}  // namespace snn
