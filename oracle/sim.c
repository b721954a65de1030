/*
 * sim.c -- oracle: the clock-driven step loop (Sec. 3, lst:basic with the
 * push transfer of lst:push / lst:push2 and the wrap-around ring buffer of
 * Sec. 3.2).  Test infrastructure only (see oracle.h).
 *
 * One step t, for every neuron i (eqn:mem, eqn:psc, eqn:ref, lst:push):
 *   if R == 0:  x = p22 U + p21 I;  if x >= theta: spike, x = 0, R = 20;  U = x
 *   else:       U = 0;  R = R - 1
 *   I = p11 I + (T_t w_ext + W[t mod 64][i]);  W[t mod 64][i] = 0
 * then, for every neuron that spiked at t and every synapse (j, d, w) it
 * sends:  W[(t + d) mod 64][j] += w.
 *
 * Readings: potentials relative to E_L (threshold 15 mV, reset 0); the
 * membrane update uses the current of the previous step; the thalamic and
 * the ring-buffer input are added to I as ONE sum.  In the INT32 arithmetic
 * that sum is an exact integer in 2^-8 pA units, converted to FP32 once, so
 * the order in which synapses deliver cannot change the result; each FP32
 * product and sum is rounded separately (no fused multiply-add).
 */
#include "oracle_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

struct orc_sim {
  const orc_net *net;
  int arith;
  uint32_t N;
  uint64_t t;
  float *U, *I;
  double *Ud, *Id;
  int32_t *R;
  int64_t *ring;     /* [64][N], INT32 arithmetic (held in int64, range-checked) */
  double *ringd;     /* [64][N], F64 arithmetic                                 */
  orc_counters cnt;
  uint32_t *spk;     /* senders of the current step                             */
  uint64_t nr, cap_r;
  uint32_t *r_step, *r_id;
  uint32_t *probe;
  uint32_t nprobe;
  uint64_t probe_steps, probe_cap;
  float *pu, *pi;
  double *pud, *pid;
  int32_t *pr;
  int rec_on;
  uint64_t rec_steps, rec_cap;
  int32_t *rec_T;
  int64_t *rec_w;
  double *rec_wd;
};

static void *grow(void *p, uint64_t *cap, uint64_t need, size_t elem) {
  if (need <= *cap) return p;
  uint64_t nc = *cap ? *cap : 1024;
  while (nc < need) nc *= 2;
  void *q = realloc(p, (size_t)nc * elem);
  if (q) *cap = nc;
  return q;
}

/* The per-neuron rule of eqn:mem / eqn:ref; returns 1 on a spike. */
static inline int membrane_f32(float *u, int32_t *r, float i, const orc_consts *k) {
  if (*r == 0) {
    float a = k->p22f * *u;
    float b = k->p21f * i;
    float x = a + b;
    int spike = 0;
    if (x >= ORC_THETA_F) {
      spike = 1;
      x = 0.0f;
      *r = ORC_T_REF_STEPS;
    }
    *u = x;
    return spike;
  }
  *u = 0.0f;
  *r -= 1;
  return 0;
}

static inline int membrane_f64(double *u, int32_t *r, double i, const orc_consts *k) {
  if (*r == 0) {
    double x = k->p22 * *u + k->p21 * i;
    int spike = 0;
    if (x >= ORC_THETA) {
      spike = 1;
      x = 0.0;
      *r = ORC_T_REF_STEPS;
    }
    *u = x;
    return spike;
  }
  *u = 0.0;
  *r -= 1;
  return 0;
}

/* eqn:psc with the combined input q (2^-8 pA units). */
static inline float current_f32(float i, int64_t q, const orc_consts *k) {
  float a = k->p11f * i;
  float b = (float)q * 0x1p-8f;
  return a + b;
}

int orc_sim_new(const orc_net *n, int arith, orc_sim **out) {
  *out = NULL;
  if (arith != ORC_ARITH_INT32 && arith != ORC_ARITH_F64) return ORC_E_INVAL;
  orc_sim *s = (orc_sim *)calloc(1, sizeof *s);
  if (!s) return ORC_E_NOMEM;
  s->net = n;
  s->arith = arith;
  s->N = n->N;
  size_t N = n->N;
  s->R = (int32_t *)calloc(N, sizeof(int32_t));
  s->spk = (uint32_t *)malloc(N * sizeof(uint32_t));
  if (arith == ORC_ARITH_INT32) {
    s->U = (float *)malloc(N * sizeof(float));
    s->I = (float *)calloc(N, sizeof(float));
    s->ring = (int64_t *)calloc(N * ORC_D_MAX, sizeof(int64_t));
    if (s->U) memcpy(s->U, n->u0, N * sizeof(float));
  } else {
    s->Ud = (double *)malloc(N * sizeof(double));
    s->Id = (double *)calloc(N, sizeof(double));
    s->ringd = (double *)calloc(N * ORC_D_MAX, sizeof(double));
    if (s->Ud) memcpy(s->Ud, n->u0d, N * sizeof(double));
  }
  if (!s->R || !s->spk || (arith == ORC_ARITH_INT32 && (!s->U || !s->I || !s->ring)) ||
      (arith == ORC_ARITH_F64 && (!s->Ud || !s->Id || !s->ringd))) {
    orc_sim_free(s);
    return ORC_E_NOMEM;
  }
  *out = s;
  return ORC_OK;
}

void orc_sim_free(orc_sim *s) {
  if (!s) return;
  free(s->U); free(s->I); free(s->Ud); free(s->Id); free(s->R);
  free(s->ring); free(s->ringd); free(s->spk);
  free(s->r_step); free(s->r_id);
  free(s->probe); free(s->pu); free(s->pi); free(s->pud); free(s->pid); free(s->pr);
  free(s->rec_T); free(s->rec_w); free(s->rec_wd);
  free(s);
}

int orc_sim_set_probes(orc_sim *s, const uint32_t *ids, uint32_t n) {
  free(s->probe);
  s->probe = NULL;
  s->nprobe = 0;
  if (!n) return ORC_OK;
  s->probe = (uint32_t *)malloc(n * sizeof(uint32_t));
  if (!s->probe) return ORC_E_NOMEM;
  for (uint32_t k = 0; k < n; ++k) {
    if (ids[k] >= s->N) return ORC_E_INVAL;
    s->probe[k] = ids[k];
  }
  s->nprobe = n;
  return ORC_OK;
}

int orc_sim_record_inputs(orc_sim *s, int on) {
  s->rec_on = on;
  return ORC_OK;
}

/* Thalamic count of neuron i at step t: one 32-bit word of the Philox block
 * (i / 4, t) against the population's inverse-CDF table. */
static inline int thalamic(const orc_net *n, uint32_t i, const uint32_t blk[4]) {
  const int p = n->pop_of[i];
  const uint32_t u = blk[i & 3u];
  int T = 0;
  for (int k = 0; k < n->thr_len[p]; ++k) T += (u >= n->thr[p][k]);
  return T;
}

static int record_step(orc_sim *s) {
  if (s->nprobe) {
    uint64_t need = (s->probe_steps + 1) * s->nprobe;
    uint64_t c0 = s->probe_cap, c1 = c0, c2 = c0;
    if (s->arith == ORC_ARITH_INT32) {
      void *a = grow(s->pu, &c0, need, sizeof(float));
      if (!a) return ORC_E_NOMEM;
      s->pu = (float *)a;
      a = grow(s->pi, &c1, need, sizeof(float));
      if (!a) return ORC_E_NOMEM;
      s->pi = (float *)a;
    } else {
      void *a = grow(s->pud, &c0, need, sizeof(double));
      if (!a) return ORC_E_NOMEM;
      s->pud = (double *)a;
      a = grow(s->pid, &c1, need, sizeof(double));
      if (!a) return ORC_E_NOMEM;
      s->pid = (double *)a;
    }
    void *a = grow(s->pr, &c2, need, sizeof(int32_t));
    if (!a) return ORC_E_NOMEM;
    s->pr = (int32_t *)a;
    s->probe_cap = c0;
    uint64_t o = s->probe_steps * s->nprobe;
    for (uint32_t k = 0; k < s->nprobe; ++k) {
      uint32_t i = s->probe[k];
      if (s->arith == ORC_ARITH_INT32) {
        s->pu[o + k] = s->U[i];
        s->pi[o + k] = s->I[i];
      } else {
        s->pud[o + k] = s->Ud[i];
        s->pid[o + k] = s->Id[i];
      }
      s->pr[o + k] = s->R[i];
    }
    s->probe_steps += 1;
  }
  return ORC_OK;
}

int orc_sim_run(orc_sim *s, uint64_t n_steps) {
  const orc_net *n = s->net;
  const orc_consts *k = &n->k;
  const uint32_t N = s->N;
  const uint64_t seed = n->cfg.seed;
  for (uint64_t step = 0; step < n_steps; ++step) {
    const uint64_t t = s->t;
    const uint32_t row = (uint32_t)(t & (ORC_D_MAX - 1));
    uint32_t nspk = 0;
    uint32_t blk[4] = {0, 0, 0, 0};
    int32_t *recT = NULL;
    int64_t *recW = NULL;
    double *recWd = NULL;
    if (s->rec_on) {
      uint64_t need = (s->rec_steps + 1) * (uint64_t)N;
      uint64_t c0 = s->rec_cap, c1 = s->rec_cap;
      void *a = grow(s->rec_T, &c0, need, sizeof(int32_t));
      if (!a) return ORC_E_NOMEM;
      s->rec_T = (int32_t *)a;
      if (s->arith == ORC_ARITH_INT32) {
        a = grow(s->rec_w, &c1, need, sizeof(int64_t));
        if (!a) return ORC_E_NOMEM;
        s->rec_w = (int64_t *)a;
      } else {
        a = grow(s->rec_wd, &c1, need, sizeof(double));
        if (!a) return ORC_E_NOMEM;
        s->rec_wd = (double *)a;
      }
      s->rec_cap = c0 < c1 ? c0 : c1;
      recT = s->rec_T + s->rec_steps * N;
      if (s->rec_w) recW = s->rec_w + s->rec_steps * N;
      if (s->rec_wd) recWd = s->rec_wd + s->rec_steps * N;
    }

    /* Update phase (parfor over neurons in the listings; sequential here). */
    for (uint32_t i = 0; i < N; ++i) {
      if ((i & 3u) == 0)
        orc_draw(seed, i >> 2, (uint32_t)t, (uint32_t)(t >> 32), ORC_TAG_POI, blk);
      const int T = thalamic(n, i, blk);
      int spike;
      if (s->arith == ORC_ARITH_INT32) {
        spike = membrane_f32(&s->U[i], &s->R[i], s->I[i], k);
        int64_t *slot = &s->ring[(size_t)row * N + i];
        const int64_t q = (int64_t)T * k->w_ext_q + *slot;
        if (q > 2147483647LL || q < -2147483647LL - 1) {
          orc_error("input %lld of neuron %u at step %llu overflows int32", (long long)q, i,
                    (unsigned long long)t);
          return ORC_E_OVERFLOW;
        }
        s->cnt.consumed += *slot;
        if (recW) recW[i] = *slot;
        *slot = 0;
        s->I[i] = current_f32(s->I[i], q, k);
      } else {
        spike = membrane_f64(&s->Ud[i], &s->R[i], s->Id[i], k);
        double *slot = &s->ringd[(size_t)row * N + i];
        const double q = (double)T * k->w_ext + *slot;
        if (recWd) recWd[i] = *slot;
        *slot = 0.0;
        s->Id[i] = k->p11 * s->Id[i] + q;
      }
      if (recT) recT[i] = T;
      s->cnt.poisson += (uint64_t)T;
      if (spike) {
        s->spk[nspk++] = i;
        if (s->nr == s->cap_r) {
          uint64_t nc = s->cap_r ? 2 * s->cap_r : 4096;
          uint32_t *a = (uint32_t *)realloc(s->r_step, (size_t)nc * sizeof(uint32_t));
          if (!a) return ORC_E_NOMEM;
          s->r_step = a;
          a = (uint32_t *)realloc(s->r_id, (size_t)nc * sizeof(uint32_t));
          if (!a) return ORC_E_NOMEM;
          s->r_id = a;
          s->cap_r = nc;
        }
        s->r_step[s->nr] = (uint32_t)t;
        s->r_id[s->nr] = i;
        s->nr += 1;
      }
    }

    /* Transfer phase (lst:push2): every synapse of every sender of step t. */
    for (uint32_t q = 0; q < nspk; ++q) {
      const uint32_t src = s->spk[q];
      const uint64_t e0 = n->row_ptr[src], e1 = n->row_ptr[src + 1];
      s->cnt.events += e1 - e0;
      for (uint64_t e = e0; e < e1; ++e) {
        const uint32_t r2 = (uint32_t)((t + n->delay[e]) & (ORC_D_MAX - 1));
        if (s->arith == ORC_ARITH_INT32) {
          s->ring[(size_t)r2 * N + n->post[e]] += n->w_q[e];
          s->cnt.injected += n->w_q[e];
        } else {
          s->ringd[(size_t)r2 * N + n->post[e]] += n->w[e];
        }
      }
    }
    s->cnt.spikes += nspk;
    if (s->rec_on) s->rec_steps += 1;
    s->t = t + 1;
    int rc = record_step(s);
    if (rc) return rc;
  }
  return ORC_OK;
}

/* The step loop of orc_sim_run for the INT32 arithmetic on several host
 * threads (OpenMP), as a CPU baseline on all cores; orc_sim_run stays the
 * checker.  Neurons are updated in parallel (four per Philox block, as
 * above), the senders of the step are collected in id order, and their
 * synapses are delivered in parallel with atomic adds into the int64 ring.
 * Each ring entry is an exact integer sum, so the results equal
 * orc_sim_run's bit for bit whatever the thread count.  Probes and input
 * recording are not supported (ORC_E_INVAL); an int32 overflow is reported
 * after the update phase of its step. */
int orc_sim_run_threads(orc_sim *s, uint64_t n_steps, int threads) {
  if (s->arith != ORC_ARITH_INT32 || s->rec_on || s->nprobe || threads < 1) return ORC_E_INVAL;
  const orc_net *n = s->net;
  const orc_consts *k = &n->k;
  const uint32_t N = s->N;
  const uint64_t seed = n->cfg.seed;
  const long long nq = (long long)((N + 3u) / 4u);
  uint8_t *fl = (uint8_t *)calloc(N ? N : 1, 1);
  if (!fl) return ORC_E_NOMEM;
  for (uint64_t step = 0; step < n_steps; ++step) {
    const uint64_t t = s->t;
    const uint32_t row = (uint32_t)(t & (ORC_D_MAX - 1));
    int overflow = 0;
    int64_t consumed = 0;
    uint64_t poisson = 0;
#pragma omp parallel for num_threads(threads) schedule(static) reduction(+ : consumed, poisson) \
    reduction(| : overflow)
    for (long long qd = 0; qd < nq; ++qd) {
      uint32_t blk[4];
      orc_draw(seed, (uint32_t)qd, (uint32_t)t, (uint32_t)(t >> 32), ORC_TAG_POI, blk);
      const uint32_t i0 = 4u * (uint32_t)qd, i1 = i0 + 4u < N ? i0 + 4u : N;
      for (uint32_t i = i0; i < i1; ++i) {
        const int T = thalamic(n, i, blk);
        const int spike = membrane_f32(&s->U[i], &s->R[i], s->I[i], k);
        int64_t *slot = &s->ring[(size_t)row * N + i];
        const int64_t q = (int64_t)T * k->w_ext_q + *slot;
        if (q > 2147483647LL || q < -2147483647LL - 1) overflow = 1;
        consumed += *slot;
        *slot = 0;
        s->I[i] = current_f32(s->I[i], q, k);
        poisson += (uint64_t)T;
        fl[i] = (uint8_t)spike;
      }
    }
    if (overflow) {
      free(fl);
      orc_error("input of a neuron at step %llu overflows int32", (unsigned long long)t);
      return ORC_E_OVERFLOW;
    }
    s->cnt.consumed += consumed;
    s->cnt.poisson += poisson;
    uint32_t nspk = 0;
    for (uint32_t i = 0; i < N; ++i) {
      if (!fl[i]) continue;
      s->spk[nspk++] = i;
      if (s->nr == s->cap_r) {
        uint64_t nc = s->cap_r ? 2 * s->cap_r : 4096;
        uint32_t *a = (uint32_t *)realloc(s->r_step, (size_t)nc * sizeof(uint32_t));
        if (!a) { free(fl); return ORC_E_NOMEM; }
        s->r_step = a;
        a = (uint32_t *)realloc(s->r_id, (size_t)nc * sizeof(uint32_t));
        if (!a) { free(fl); return ORC_E_NOMEM; }
        s->r_id = a;
        s->cap_r = nc;
      }
      s->r_step[s->nr] = (uint32_t)t;
      s->r_id[s->nr] = i;
      s->nr += 1;
    }
    int64_t injected = 0;
    uint64_t events = 0;
#pragma omp parallel for num_threads(threads) schedule(dynamic, 1) reduction(+ : injected, events)
    for (long long qq = 0; qq < (long long)nspk; ++qq) {
      const uint32_t src = s->spk[qq];
      const uint64_t e0 = n->row_ptr[src], e1 = n->row_ptr[src + 1];
      events += e1 - e0;
      for (uint64_t e = e0; e < e1; ++e) {
        const uint32_t r2 = (uint32_t)((t + n->delay[e]) & (ORC_D_MAX - 1));
        int64_t *dst = &s->ring[(size_t)r2 * N + n->post[e]];
#pragma omp atomic
        *dst += n->w_q[e];
        injected += n->w_q[e];
      }
    }
    s->cnt.events += events;
    s->cnt.injected += injected;
    s->cnt.spikes += nspk;
    s->t = t + 1;
  }
  free(fl);
  return ORC_OK;
}

uint64_t orc_sim_t(const orc_sim *s) { return s->t; }
void orc_sim_counters(const orc_sim *s, orc_counters *c) { *c = s->cnt; }
uint64_t orc_sim_nspikes(const orc_sim *s) { return s->nr; }
const uint32_t *orc_sim_spike_steps(const orc_sim *s) { return s->r_step; }
const uint32_t *orc_sim_spike_ids(const orc_sim *s) { return s->r_id; }
const float *orc_sim_u(const orc_sim *s) { return s->U; }
const float *orc_sim_i(const orc_sim *s) { return s->I; }
const double *orc_sim_u64(const orc_sim *s) { return s->Ud; }
const double *orc_sim_i64(const orc_sim *s) { return s->Id; }
const int32_t *orc_sim_r(const orc_sim *s) { return s->R; }
const int64_t *orc_sim_ring_q(const orc_sim *s) { return s->ring; }
const double *orc_sim_ring_f64(const orc_sim *s) { return s->ringd; }
const float *orc_sim_probe_u(const orc_sim *s) { return s->pu; }
const float *orc_sim_probe_i(const orc_sim *s) { return s->pi; }
const double *orc_sim_probe_u64(const orc_sim *s) { return s->pud; }
const double *orc_sim_probe_i64(const orc_sim *s) { return s->pid; }
const int32_t *orc_sim_probe_r(const orc_sim *s) { return s->pr; }
uint64_t orc_sim_probe_steps(const orc_sim *s) { return s->probe_steps; }
const int32_t *orc_sim_rec_T(const orc_sim *s) { return s->rec_T; }
const int64_t *orc_sim_rec_w(const orc_sim *s) { return s->rec_w; }
const double *orc_sim_rec_w64(const orc_sim *s) { return s->rec_wd; }
uint64_t orc_sim_rec_steps(const orc_sim *s) { return s->rec_steps; }

/* A single neuron with no synapses, driven by the given per-step input. */
int orc_single_neuron_f32(const orc_consts *k, const int64_t *q, uint64_t n, float *u_out,
                          float *i_out, int32_t *r_out) {
  float u = 0.0f, i = 0.0f;
  int32_t r = 0;
  for (uint64_t t = 0; t < n; ++t) {
    membrane_f32(&u, &r, i, k);
    i = current_f32(i, q[t], k);
    u_out[t] = u;
    i_out[t] = i;
    r_out[t] = r;
  }
  return ORC_OK;
}

int orc_single_neuron_f64(const orc_consts *k, const double *q, uint64_t n, double *u_out,
                          double *i_out, int32_t *r_out) {
  double u = 0.0, i = 0.0;
  int32_t r = 0;
  for (uint64_t t = 0; t < n; ++t) {
    membrane_f64(&u, &r, i, k);
    i = k->p11 * i + q[t];
    u_out[t] = u;
    i_out[t] = i;
    r_out[t] = r;
  }
  return ORC_OK;
}
