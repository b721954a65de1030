/*
 * model.c -- oracle: model constants, PD14 tables, Philox4x32-10 and the
 * Poisson inverse-CDF tables.  Test infrastructure only (see oracle.h).
 */
#include "oracle_internal.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

static char g_err[512];

void orc_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

const char *orc_last_error(void) { return g_err; }

/* ---- Table tab:params (general parameters) -------------------------------- */
const double ORC_DT_MS = 0.1;      /* time step, ms                       */
const double ORC_C_M = 250.0;      /* membrane capacitance, pF            */
const double ORC_TAU_M = 10.0;     /* membrane time constant, ms          */
const double ORC_TAU_SYN = 0.5;    /* postsynaptic current time const, ms */
/* Refractory period 2 ms = 20 steps of 0.1 ms; potentials are kept relative
 * to the resting potential -65 mV, so the threshold -50 mV becomes 15 mV and
 * reset/rest become 0 (the listings write "x = 0"). */
const int ORC_T_REF_STEPS = 20;
const float ORC_THETA_F = 15.0f;
const double ORC_THETA = 15.0;
const double ORC_E_L = -65.0;

/* ---- Table tab:params2 (population-specific parameters) ------------------- */
const uint32_t ORC_N_FULL[8] = {20683, 5834, 21915, 5479, 4850, 1065, 14395, 2948};
const uint32_t ORC_K_EXT[8] = {1600, 1500, 2100, 1900, 2000, 1900, 2900, 2100};
const double ORC_V0_MEAN[8] = {-68.28, -63.16, -63.33, -63.45, -63.11, -61.66, -66.72, -61.43};
const double ORC_V0_SD[8] = {5.36, 4.57, 4.74, 4.94, 4.94, 4.55, 5.46, 4.48};
/* Populations alternate excitatory / inhibitory: L23e, L23i, L4e, L4i, ... */
int orc_is_exc(int p) { return (p & 1) == 0; }

/* ---- Table tab:params3 (connection probabilities), as printed ------------- */
const double ORC_CONN[8][8] = {
    {0.1009, 0.1689, 0.0437, 0.0818, 0.0323, 0.0000, 0.0076, 0.0000},
    {0.1346, 0.1371, 0.0316, 0.0515, 0.0755, 0.0000, 0.0042, 0.0000},
    {0.0077, 0.0059, 0.0497, 0.1350, 0.0067, 0.0003, 0.0453, 0.0000},
    {0.0691, 0.0029, 0.0794, 0.1597, 0.0033, 0.0000, 0.1057, 0.0000},
    {0.1004, 0.0622, 0.0505, 0.0057, 0.0831, 0.3726, 0.0204, 0.0000},
    {0.0548, 0.0269, 0.0257, 0.0022, 0.0600, 0.3158, 0.0086, 0.0000},
    {0.0156, 0.0066, 0.0211, 0.0166, 0.0572, 0.0197, 0.0396, 0.2252},
    {0.0364, 0.0010, 0.0034, 0.0005, 0.0277, 0.0080, 0.0658, 0.1443},
};

void orc_config_default(orc_config *c) {
  memset(c, 0, sizeof *c);
  c->seed = 1;
  c->scale = 1.0;
  c->indegree_mode = 0;
  c->count_rule = 0;
  c->rows_are_sources = 0;
  c->g = -4.0;
  c->bg_rate_hz = 8.0;
  c->psp_ext_mv = 0.15;
  c->bg_const_T = -1;
  c->weight_mode = ORC_W_PLAIN;
  c->conn = NULL;
}

/*
 * Constants of Sec. 2.2.  w_f converts a PSP amplitude (mV) into the PSC
 * amplitude (pA) that produces it; p11 and p22 are the per-step decay factors
 * of the synaptic current and the membrane (eqn:p11p22); p21 is the weight of
 * the current in the membrane update (eqn:p21).  All in FP64, then rounded to
 * FP32 for the FP32 arithmetic.
 */
int orc_constants(const orc_config *c, orc_consts *out) {
  const double tau_m = ORC_TAU_M, tau_s = ORC_TAU_SYN, cm = ORC_C_M, dt = ORC_DT_MS;
  double d = tau_s - tau_m;
  double p = tau_s * tau_m;
  double q = tau_m / tau_s;
  out->w_f = cm * d / (p * (pow(q, tau_m / d) - pow(q, tau_s / d)));

  out->p11 = exp(-dt / tau_s);
  out->p22 = exp(-dt / tau_m);
  double beta = tau_s * tau_m / (tau_m - tau_s);
  double gamma = beta / cm;
  out->p21 = out->p11 * gamma * (exp(dt / beta) - 1.0);

  out->p11f = (float)out->p11;
  out->p22f = (float)out->p22;
  out->p21f = (float)out->p21;

  out->w_ext = out->w_f * c->psp_ext_mv;
  double wq = nearbyint(out->w_ext * 256.0);
  if (!(fabs(wq) < 2147483647.0)) {
    orc_error("thalamic weight %g pA does not fit int32 fixed point", out->w_ext);
    return ORC_E_RANGE;
  }
  out->w_ext_q = (int32_t)wq;
  return ORC_OK;
}

/*
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11).  Ten rounds; each round multiplies counter words
 * 0 and 2 by the two Philox constants, XORs the high halves with the other
 * two words and the round key, and permutes; the key advances by the two
 * Weyl constants between rounds.
 */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t m0 = (uint64_t)0xD2511F53u * x0;
    uint64_t m1 = (uint64_t)0xCD9E8D57u * x2;
    uint32_t hi0 = (uint32_t)(m0 >> 32), lo0 = (uint32_t)m0;
    uint32_t hi1 = (uint32_t)(m1 >> 32), lo1 = (uint32_t)m1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void orc_draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t tag,
              uint32_t out[4]) {
  uint32_t ctr[4] = {c0, c1, c2, tag};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  orc_philox4x32_10(ctr, key, out);
}

/* A 32-bit word as a uniform variate strictly inside (0, 1). */
double orc_unit(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

/* Box-Muller, cosine branch: one standard normal from two words. */
double orc_normal(uint32_t a, uint32_t b) {
  const double two_pi = 6.283185307179586;
  double r = sqrt(-2.0 * log(orc_unit(a)));
  return r * cos(two_pi * orc_unit(b));
}

/*
 * Thalamic input count T_t ~ Poisson(lam) (Sec. 2.2, lam = v_th K dt) by the
 * inverse CDF on one uniform 32-bit word: thr[k] = floor(2^32 P(T <= k)), and
 * T = #{k : u >= thr[k]}.  The table stops at the first k whose remaining
 * tail mass is below 2^-32, so P(T = k) is exact to 2^-32.
 */
int orc_poisson_table(double lam, uint32_t *thr, int cap, int *len) {
  if (!(lam >= 0.0) || lam > 64.0) {
    orc_error("Poisson mean %g out of range [0, 64]", lam);
    return ORC_E_INVAL;
  }
  const double two32 = 4294967296.0;
  double pmf = exp(-lam);
  double cdf = pmf;
  int k = 0;
  for (;;) {
    double x = cdf * two32;
    if (x >= two32 - 1.0) break;
    if (k >= cap) {
      orc_error("Poisson table for mean %g needs more than %d entries", lam, cap);
      return ORC_E_RANGE;
    }
    thr[k] = (uint32_t)floor(x);
    k += 1;
    pmf = pmf * lam / (double)k;
    cdf = cdf + pmf;
  }
  *len = k;
  return ORC_OK;
}
