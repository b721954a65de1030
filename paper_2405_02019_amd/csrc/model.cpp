// model.cpp -- the Potjans-Diesmann microcircuit's parameters (Sec. 2.2,
// Tables tab:params, tab:params2, tab:params3), the PSP-to-PSC factor w_f,
// the synapse-count rule and the thalamic Poisson tables.  Host code.
#include <cmath>
#include <cstdio>

#include "snn_internal.hpp"

namespace snn {

// tab:params2: population sizes N_i and thalamic in-degrees K_i, in the order
// L23e, L23i, L4e, L4i, L5e, L5i, L6e, L6i.
const uint32_t kPopFull[8] = {20683, 5834, 21915, 5479, 4850, 1065, 14395, 2948};
const uint32_t kKext[8] = {1600, 1500, 2100, 1900, 2000, 1900, 2900, 2100};

// tab:params3 exactly as printed; rows index the target population (the
// reading under which the paper's FP64 runs can equal NEST's).
static const double kConnPrinted[64] = {
    0.1009, 0.1689, 0.0437, 0.0818, 0.0323, 0.0000, 0.0076, 0.0000,  //
    0.1346, 0.1371, 0.0316, 0.0515, 0.0755, 0.0000, 0.0042, 0.0000,  //
    0.0077, 0.0059, 0.0497, 0.1350, 0.0067, 0.0003, 0.0453, 0.0000,  //
    0.0691, 0.0029, 0.0794, 0.1597, 0.0033, 0.0000, 0.1057, 0.0000,  //
    0.1004, 0.0622, 0.0505, 0.0057, 0.0831, 0.3726, 0.0204, 0.0000,  //
    0.0548, 0.0269, 0.0257, 0.0022, 0.0600, 0.3158, 0.0086, 0.0000,  //
    0.0156, 0.0066, 0.0211, 0.0166, 0.0572, 0.0197, 0.0396, 0.2252,  //
    0.0364, 0.0010, 0.0034, 0.0005, 0.0277, 0.0080, 0.0658, 0.1443,
};

std::vector<double> connectivity(const snn_instance_cfg &cfg) {
  std::vector<double> c(64);
  for (int tgt = 0; tgt < 8; ++tgt)
    for (int src = 0; src < 8; ++src) {
      const int i = tgt * 8 + src;
      if (cfg.conn)
        c[i] = cfg.conn[i];
      else
        c[i] = cfg.rows_are_sources ? kConnPrinted[src * 8 + tgt] : kConnPrinted[i];
    }
  return c;
}

void population_sizes(double scale, uint32_t n_pop[8]) {
  for (int p = 0; p < 8; ++p) n_pop[p] = uint32_t(std::floor(scale * double(kPopFull[p]) + 0.5));
}

// tab:params: C_m = 250 pF, tau_m = 10 ms, tau_syn = 0.5 ms, dt = 0.1 ms.
// w_f (Sec. 2.2) is the current amplitude per mV of PSP peak; the
// propagators advance current and membrane by one step (eqn:p11p22,
// eqn:p21).  The kernels recompute p11, p22, p21 on the GPU in FP64; the host
// copy only serves w_f and reporting.
ModelConstants model_constants() {
  const double cm = 250.0, tm = 10.0, ts = 0.5, h = 0.1;
  ModelConstants k{};
  const double d = ts - tm, p = ts * tm, q = tm / ts;
  k.w_f = cm * d / (p * (std::pow(q, tm / d) - std::pow(q, ts / d)));
  k.p11 = std::exp(-h / ts);
  k.p22 = std::exp(-h / tm);
  const double beta = ts * tm / (tm - ts);
  k.p21 = k.p11 * (beta / cm) * (std::exp(h / beta) - 1.0);
  return k;
}

// Number of synapses from source population `src` onto target population
// `tgt`: the fixed-total-number rule n = ln(1 - p) / ln(1 - 1/(N_src N_tgt)),
// rounded half up, evaluated with log1p; in in-degree mode it is evaluated at
// full scale and scaled by the target's size ratio.
int pair_counts(const snn_instance_cfg &cfg, const std::vector<double> &conn,
                const uint32_t n_pop[8], uint64_t out[64], std::string &err) {
  for (int tgt = 0; tgt < 8; ++tgt) {
    for (int src = 0; src < 8; ++src) {
      const double p = conn[tgt * 8 + src];
      uint64_t &o = out[tgt * 8 + src];
      o = 0;
      if (!(p >= 0.0 && p < 1.0)) {
        char b[160];
        std::snprintf(b, sizeof b, "connection probability %g (target %d, source %d) not in [0,1)",
                      p, tgt, src);
        err = b;
        return SNN_E_INVAL;
      }
      if (p == 0.0 || n_pop[src] == 0 || n_pop[tgt] == 0) continue;
      const double ns = cfg.indegree_mode ? double(kPopFull[src]) : double(n_pop[src]);
      const double nt = cfg.indegree_mode ? double(kPopFull[tgt]) : double(n_pop[tgt]);
      double x = cfg.count_rule == 0 ? std::log1p(-p) / std::log1p(-1.0 / (ns * nt)) : ns * nt * p;
      double n = std::floor(x + 0.5);
      if (cfg.indegree_mode) n = std::floor(n * double(n_pop[tgt]) / double(kPopFull[tgt]) + 0.5);
      if (!(n < 4294967296.0)) {
        err = "a population pair needs 2^32 or more synapses";
        return SNN_E_RANGE;
      }
      o = uint64_t(n);
    }
  }
  return SNN_OK;
}

// Thalamic count T ~ Poisson(lam) by inverse CDF on one 32-bit word u:
// thr[k] = floor(2^32 P(T <= k)) and T = #{k : u >= thr[k]}; the table ends
// once the remaining tail is below 2^-32.
int poisson_thresholds(double lam, uint32_t *thr, uint32_t cap, uint32_t *len, std::string &err) {
  if (!(lam >= 0.0) || lam > 64.0) {
    err = "thalamic Poisson mean outside [0, 64]";
    return SNN_E_INVAL;
  }
  const double scale32 = 4294967296.0;
  double term = std::exp(-lam);
  double cum = term;
  uint32_t k = 0;
  while (cum * scale32 < scale32 - 1.0) {
    if (k == cap) {
      err = "thalamic Poisson table too long";
      return SNN_E_RANGE;
    }
    thr[k] = uint32_t(std::floor(cum * scale32));
    ++k;
    term = term * lam / double(k);
    cum = cum + term;
  }
  *len = k;
  return SNN_OK;
}

}  // namespace snn
