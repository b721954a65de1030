/*
 * network.c -- oracle: sampling of the Potjans-Diesmann microcircuit
 * (Sec. 2.2, Tables tab:params2 and tab:params3) and its storage as an array
 * of synapses sorted by sender with a per-sender index (Sec. 3.5, lst:index).
 * Test infrastructure only (see oracle.h).
 *
 * Readings of the paper used here:
 *  - tab:params3 rows index the TARGET population (the paper's double
 *    precision runs match NEST spike for spike, and NEST's table is
 *    [target][source]); a flag swaps the orientation.
 *  - Synapse counts follow the microcircuit's fixed-total-number rule,
 *    n = ln(1-p) / ln(1 - 1/(N_pre N_post)) rounded half up, which gives the
 *    full-scale total of about 3e8 synapses stated in Sec. 2.2 (N_pre N_post p
 *    gives 2.85e8).
 *    log1p evaluates both logarithms without cancellation.
 *  - Each synapse draws its sender and receiver uniformly with replacement,
 *    so multapses and autapses occur (Sec. 2.1.1, Sec. 2.2).
 *  - Weights: Normal(mu, 0.1 |mu|) with mu = w_f * PSP, PSP = 0.15 mV for
 *    excitatory senders, g * 0.15 mV for inhibitory senders, and 0.30 mV for
 *    L4e -> L23e (the doubled pair of tab:params2, whose caption misnames it).
 *    A weight that would change sign is clipped to 0.
 *  - Delays: Normal(1.5, 0.75) ms excitatory, Normal(0.75, 0.375) ms
 *    inhibitory (tab:params2 prints 0.325; half the mean is used, as for the
 *    excitatory delays), rounded to whole 0.1 ms steps and clipped to
 *    [1, 63] steps so that a 64-row ring buffer suffices (Sec. 3.2).
 */
#include "oracle_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static int pair_count(const orc_net *n, int b, int a, uint64_t *out) {
  const orc_config *c = &n->cfg;
  double p = n->conn[b][a];
  *out = 0;
  if (!(p >= 0.0) || !(p < 1.0)) {
    orc_error("connection probability %g (target %d, source %d) outside [0,1)", p, b, a);
    return ORC_E_INVAL;
  }
  if (p == 0.0) return ORC_OK;
  double na, nb;
  if (c->indegree_mode) {
    na = (double)ORC_N_FULL[a];
    nb = (double)ORC_N_FULL[b];
  } else {
    na = (double)n->n_pop[a];
    nb = (double)n->n_pop[b];
  }
  if (n->n_pop[a] == 0 || n->n_pop[b] == 0) return ORC_OK;
  double x;
  if (c->count_rule == 0)
    x = log1p(-p) / log1p(-1.0 / (na * nb));
  else
    x = na * nb * p;
  double cnt = floor(x + 0.5);
  if (c->indegree_mode) cnt = floor(cnt * (double)n->n_pop[b] / (double)ORC_N_FULL[b] + 0.5);
  if (!(cnt < 4294967296.0)) {
    orc_error("pair (%d <- %d) needs %g synapses; at most 2^32-1 supported", b, a, cnt);
    return ORC_E_RANGE;
  }
  *out = (uint64_t)cnt;
  return ORC_OK;
}

static void net_free_arrays(orc_net *n) {
  free(n->row_ptr);
  free(n->post);
  free(n->delay);
  free(n->w);
  free(n->w_q);
  free(n->u0);
  free(n->u0d);
  free(n->pop_of);
}

void orc_net_free(orc_net *n) {
  if (!n) return;
  net_free_arrays(n);
  free(n);
}

int orc_build(const orc_config *c, orc_net **out) {
  *out = NULL;
  if (!(c->scale > 0.0) || c->scale > 64.0) {
    orc_error("scale %g outside (0, 64]", c->scale);
    return ORC_E_INVAL;
  }
  if (!(c->bg_rate_hz >= 0.0) || !(c->psp_ext_mv >= 0.0) || !(c->g <= 0.0)) {
    orc_error("bg_rate_hz, psp_ext_mv must be >= 0 and g <= 0");
    return ORC_E_INVAL;
  }
  if (c->weight_mode != ORC_W_PLAIN && c->weight_mode != ORC_W_COMPRESSED &&
      c->weight_mode != ORC_W_DEV8) {
    orc_error("unknown weight mode %d", c->weight_mode);
    return ORC_E_INVAL;
  }
  orc_net *n = (orc_net *)calloc(1, sizeof *n);
  if (!n) return ORC_E_NOMEM;
  n->cfg = *c;
  n->cfg.conn = NULL;
  for (int b = 0; b < 8; ++b)
    for (int a = 0; a < 8; ++a) {
      double v;
      if (c->conn) v = c->conn[b * 8 + a];
      else v = c->rows_are_sources ? ORC_CONN[a][b] : ORC_CONN[b][a];
      n->conn[b][a] = v;
    }
  int rc = orc_constants(c, &n->k);
  if (rc) goto fail;

  /* Population sizes: N_p = floor(scale * N_p_full + 0.5), ids contiguous per
   * population in table order. */
  n->off[0] = 0;
  for (int p = 0; p < 8; ++p) {
    n->n_pop[p] = (uint32_t)floor(c->scale * (double)ORC_N_FULL[p] + 0.5);
    n->off[p + 1] = n->off[p] + n->n_pop[p];
  }
  n->N = n->off[8];
  if (n->N == 0) {
    orc_error("scale %g leaves no neurons", c->scale);
    rc = ORC_E_INVAL;
    goto fail;
  }

  uint64_t base[8][8];
  n->S = 0;
  for (int b = 0; b < 8; ++b)
    for (int a = 0; a < 8; ++a) {
      rc = pair_count(n, b, a, &n->pair_n[b][a]);
      if (rc) goto fail;
      base[b][a] = n->S;
      n->S += n->pair_n[b][a];
    }

  const uint64_t S = n->S;
  uint32_t *g_pre = (uint32_t *)malloc((S ? S : 1) * sizeof(uint32_t));
  uint32_t *g_post = (uint32_t *)malloc((S ? S : 1) * sizeof(uint32_t));
  uint8_t *g_d = (uint8_t *)malloc(S ? S : 1);
  double *g_w = (double *)malloc((S ? S : 1) * sizeof(double));
  n->row_ptr = (uint64_t *)calloc((size_t)n->N + 1, sizeof(uint64_t));
  n->post = (uint32_t *)malloc((S ? S : 1) * sizeof(uint32_t));
  n->delay = (uint8_t *)malloc(S ? S : 1);
  n->w = (double *)malloc((S ? S : 1) * sizeof(double));
  n->w_q = (int32_t *)malloc((S ? S : 1) * sizeof(int32_t));
  n->u0 = (float *)malloc((size_t)n->N * sizeof(float));
  n->u0d = (double *)malloc((size_t)n->N * sizeof(double));
  n->pop_of = (uint8_t *)malloc(n->N);
  if (!g_pre || !g_post || !g_d || !g_w || !n->row_ptr || !n->post || !n->delay || !n->w ||
      !n->w_q || !n->u0 || !n->u0d || !n->pop_of) {
    free(g_pre); free(g_post); free(g_d); free(g_w);
    orc_error("out of host memory for %llu synapses", (unsigned long long)S);
    rc = ORC_E_NOMEM;
    goto fail;
  }
  for (int p = 0; p < 8; ++p)
    for (uint32_t i = n->off[p]; i < n->off[p + 1]; ++i) n->pop_of[i] = (uint8_t)p;

  /* Generation, in (target pop, source pop, k) order.  Every synapse uses two
   * Philox blocks keyed by the seed: block 0 gives sender, receiver and the
   * weight's normal deviate, block 1 the delay's normal deviate. */
  const double psp_e = 0.15;
  for (int b = 0; b < 8; ++b)
    for (int a = 0; a < 8; ++a) {
      uint64_t cnt = n->pair_n[b][a];
      if (!cnt) continue;
      double psp = orc_is_exc(a) ? psp_e : c->g * psp_e;
      if (b == 0 && a == 2) psp = 2.0 * psp_e;
      double mu_w = psp * n->k.w_f;
      double sd_w = 0.1 * fabs(mu_w);
      n->mu_w[b][a] = mu_w;
      n->sd_w[b][a] = sd_w;
      double mu_d = orc_is_exc(a) ? 15.0 : 7.5;
      double sd_d = orc_is_exc(a) ? 7.5 : 3.75;
      uint32_t pair = (uint32_t)(8 * b + a);
      uint64_t na = n->n_pop[a], nb = n->n_pop[b];
      uint32_t a0 = n->off[a], b0 = n->off[b];
      uint64_t o = base[b][a];
      long long cnt_ll = (long long)cnt;
#pragma omp parallel for schedule(static)
      for (long long kk = 0; kk < cnt_ll; ++kk) {
        uint32_t r[4], s[4];
        orc_draw(c->seed, (uint32_t)kk, 2 * pair, 0, ORC_TAG_SYN, r);
        orc_draw(c->seed, (uint32_t)kk, 2 * pair + 1, 0, ORC_TAG_SYN, s);
        uint32_t pre = a0 + (uint32_t)(((uint64_t)r[0] * na) >> 32);
        uint32_t post = b0 + (uint32_t)(((uint64_t)r[1] * nb) >> 32);
        double w = mu_w + sd_w * orc_normal(r[2], r[3]);
        if (mu_w > 0.0 && w < 0.0) w = 0.0;
        if (mu_w < 0.0 && w > 0.0) w = 0.0;
        double dr = nearbyint(mu_d + sd_d * orc_normal(s[0], s[1]));
        int d = dr < 1.0 ? 1 : (dr > 63.0 ? 63 : (int)dr);
        g_pre[o + kk] = pre;
        g_post[o + kk] = post;
        g_w[o + kk] = w;
        g_d[o + kk] = (uint8_t)d;
      }
    }

  /* Stable counting sort by sender: row_ptr[i] .. row_ptr[i+1] holds the
   * synapses of sender i in generation order. */
  for (uint64_t e = 0; e < S; ++e) n->row_ptr[g_pre[e] + 1] += 1;
  for (uint32_t i = 0; i < n->N; ++i) n->row_ptr[i + 1] += n->row_ptr[i];
  uint64_t *cur = (uint64_t *)malloc(((size_t)n->N + 1) * sizeof(uint64_t));
  if (!cur) {
    free(g_pre); free(g_post); free(g_d); free(g_w);
    rc = ORC_E_NOMEM;
    goto fail;
  }
  memcpy(cur, n->row_ptr, ((size_t)n->N + 1) * sizeof(uint64_t));
  for (uint64_t e = 0; e < S; ++e) {
    uint64_t pos = cur[g_pre[e]]++;
    n->post[pos] = g_post[e];
    n->delay[pos] = g_d[e];
    n->w[pos] = g_w[e];
  }
  free(cur);
  free(g_pre); free(g_post); free(g_d); free(g_w);

  /* Fixed-point weights: 2^-8 pA (plain), int16 in 2^-5 pA scaled to the
   * same 2^-8 pA accumulator (compressed, Sec. 5.3's 16-bit weights), or the
   * pair's mean plus an 8-bit deviation (dev8, Sec. 5.3's deviations from the
   * mean; below). */
  for (uint64_t e = 0; e < S; ++e) {
    double w = n->w[e];
    if (c->weight_mode == ORC_W_PLAIN) {
      double q = nearbyint(w * 256.0);
      if (!(fabs(q) < 2147483647.0)) {
        orc_error("weight %g pA does not fit int32 fixed point", w);
        rc = ORC_E_RANGE;
        goto fail;
      }
      n->w_q[e] = (int32_t)q;
    } else if (c->weight_mode == ORC_W_COMPRESSED) {
      double q = nearbyint(w * 32.0);
      if (!(q >= -32768.0 && q <= 32767.0)) {
        orc_error("weight %g pA does not fit the 16-bit encoding", w);
        rc = ORC_E_RANGE;
        goto fail;
      }
      n->w_q[e] = 8 * (int32_t)q;
    }
  }
  if (c->weight_mode == ORC_W_DEV8) {
    /* The pair of a synapse: the populations of its receiver and sender. */
    for (uint32_t i = 0; i < n->N; ++i) {
      int a = n->pop_of[i];
      for (uint64_t e = n->row_ptr[i]; e < n->row_ptr[i + 1]; ++e) {
        int b = n->pop_of[n->post[e]];
        int32_t mq, sq, dev;
        orc_dev8_params(n->mu_w[b][a], n->sd_w[b][a], &mq, &sq);
        n->w_q[e] = orc_dev8_encode(n->w[e], mq, sq, &dev);
      }
    }
  }

  /* Initial membrane potential: Normal(mean, sd) of tab:params2 (absolute
   * mV), kept relative to E_L.  I and the refractory counter start at 0. */
  for (uint32_t i = 0; i < n->N; ++i) {
    int p = n->pop_of[i];
    uint32_t r[4];
    orc_draw(c->seed, i, 0, 0, ORC_TAG_V0, r);
    double v = ORC_V0_MEAN[p] + ORC_V0_SD[p] * orc_normal(r[0], r[1]);
    n->u0d[i] = v - ORC_E_L;
    n->u0[i] = (float)n->u0d[i];
  }

  /* Thalamic drive: mean v_th K dt per step (Sec. 2.2). */
  int tmax = 0;
  for (int p = 0; p < 8; ++p) {
    if (c->bg_const_T >= 0) {
      if (c->bg_const_T > ORC_POI_CAP) {
        orc_error("constant thalamic count %d above %d", c->bg_const_T, ORC_POI_CAP);
        rc = ORC_E_INVAL;
        goto fail;
      }
      for (int k = 0; k < c->bg_const_T; ++k) n->thr[p][k] = 0;
      n->thr_len[p] = c->bg_const_T;
    } else {
      double lam = (c->bg_rate_hz * (double)ORC_K_EXT[p]) * 1e-4;
      rc = orc_poisson_table(lam, n->thr[p], ORC_POI_CAP, &n->thr_len[p]);
      if (rc) goto fail;
    }
    if (n->thr_len[p] > tmax) tmax = n->thr_len[p];
  }

  /* Guard: the worst-case input of one step must fit the int32 accumulator. */
  {
    int64_t *insum = (int64_t *)calloc(n->N, sizeof(int64_t));
    if (!insum) { rc = ORC_E_NOMEM; goto fail; }
    for (uint64_t e = 0; e < S; ++e) insum[n->post[e]] += llabs((long long)n->w_q[e]);
    int64_t worst = 0;
    for (uint32_t i = 0; i < n->N; ++i)
      if (insum[i] > worst) worst = insum[i];
    free(insum);
    worst += (int64_t)tmax * llabs((long long)n->k.w_ext_q);
    if (worst >= 2147483647LL) {
      orc_error("worst-case input %lld exceeds the int32 accumulator", (long long)worst);
      rc = ORC_E_OVERFLOW;
      goto fail;
    }
  }

  *out = n;
  return ORC_OK;
fail:
  orc_net_free(n);
  return rc;
}

/* Synapse counts [target][source] of a configuration, without sampling. */
int orc_pair_counts(const orc_config *c, uint64_t counts[64]) {
  orc_net tmp;
  memset(&tmp, 0, sizeof tmp);
  tmp.cfg = *c;
  for (int b = 0; b < 8; ++b)
    for (int a = 0; a < 8; ++a)
      tmp.conn[b][a] = c->conn ? c->conn[b * 8 + a]
                               : (c->rows_are_sources ? ORC_CONN[a][b] : ORC_CONN[b][a]);
  for (int p = 0; p < 8; ++p)
    tmp.n_pop[p] = (uint32_t)floor(c->scale * (double)ORC_N_FULL[p] + 0.5);
  for (int b = 0; b < 8; ++b)
    for (int a = 0; a < 8; ++a) {
      int rc = pair_count(&tmp, b, a, &counts[b * 8 + a]);
      if (rc) return rc;
    }
  return ORC_OK;
}

uint32_t orc_net_n(const orc_net *n) { return n->N; }
uint64_t orc_net_nsyn(const orc_net *n) { return n->S; }
void orc_net_pop_offsets(const orc_net *n, uint32_t off[9]) { memcpy(off, n->off, sizeof n->off); }
uint64_t orc_net_pair_count(const orc_net *n, int target, int source) {
  return n->pair_n[target & 7][source & 7];
}
const uint64_t *orc_net_row_ptr(const orc_net *n) { return n->row_ptr; }
const uint32_t *orc_net_post(const orc_net *n) { return n->post; }
const uint8_t *orc_net_delay(const orc_net *n) { return n->delay; }
const double *orc_net_weight(const orc_net *n) { return n->w; }
const int32_t *orc_net_weight_q(const orc_net *n) { return n->w_q; }
void orc_net_dev8_pair(const orc_net *n, int target, int source, int32_t *mq, int32_t *sq) {
  orc_dev8_params(n->mu_w[target][source], n->sd_w[target][source], mq, sq);
}

void orc_dev8_params(double mu, double sd, int32_t *mq, int32_t *sq) {
  double s = nearbyint(5.0 * sd * 256.0 / 127.0);
  *mq = (int32_t)nearbyint(mu * 256.0);
  *sq = s < 1.0 ? 1 : (int32_t)s;
}

int32_t orc_dev8_encode(double w, int32_t mq, int32_t sq, int32_t *dev) {
  double r = nearbyint((w * 256.0 - (double)mq) / (double)sq);
  int32_t d = r < -127.0 ? -127 : (r > 127.0 ? 127 : (int32_t)r);
  *dev = d;
  return mq + d * sq;
}
const float *orc_net_u0(const orc_net *n) { return n->u0; }
const double *orc_net_u0_f64(const orc_net *n) { return n->u0d; }
int orc_net_poisson(const orc_net *n, int p, const uint32_t **thr, int *len) {
  if (p < 0 || p > 7) return ORC_E_INVAL;
  *thr = n->thr[p];
  *len = n->thr_len[p];
  return ORC_OK;
}
