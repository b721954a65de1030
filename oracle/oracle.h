/*
 * oracle.h -- plain, slow, single-threaded CPU reference for the clock-driven
 * simulation of the Potjans-Diesmann cortical microcircuit.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the simulator library links, includes
 * or calls this code; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg load it.  It shares no source with the GPU path: the
 * random-number generator, the model tables, the network sampler and the step
 * loop are all written out again here, in the order the paper states them.
 *
 * What each part follows (paper: "Fast Algorithms for Spiking Neural Network
 * Simulation with FPGAs", Lindqvist & Podobas):
 *   - model constants w_f, p11, p22, p21 ........ Sec. 2.2, equations for w_f,
 *                                                  eqn:p11p22 and eqn:p21
 *   - population / connectivity tables ........... Tables tab:params,
 *                                                  tab:params2, tab:params3
 *   - neuron recurrences ......................... eqn:mem, eqn:psc, eqn:ref
 *                                                  and listing lst:push
 *   - thalamic Poisson drive ...................... Sec. 2.2 (T_t ~ Poisson)
 *   - push delivery into a wrap-around ring ...... Sec. 3.1-3.2 (lst:push,
 *                                                  lst:push2, D_MAX = 64)
 *   - synapse storage sorted by sender ........... Sec. 3.5 (lst:index)
 *   - 16-bit weights ............................. Sec. 5.3 (Future Research)
 *
 * Readings taken where the paper is silent or ambiguous are listed in the
 * project's design notes; each is restated next to the code it affects.
 *
 * Conventions: every function returns 0 on success or a negative ORC_E_* code.
 */
#ifndef SNN_ORACLE_H
#define SNN_ORACLE_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_OK = 0,
  ORC_E_INVAL = -1,     /* bad configuration value                       */
  ORC_E_NOMEM = -2,     /* allocation failed                             */
  ORC_E_RANGE = -4,     /* a sampled value does not fit its encoding     */
  ORC_E_OVERFLOW = -5   /* an int32 accumulator would overflow           */
};

/* Arithmetic of the step loop. */
enum {
  ORC_ARITH_INT32 = 0,  /* FP32 neuron state, int32 fixed-point input (2^-8 pA) */
  ORC_ARITH_F64 = 1     /* FP64 state and propagators, FP64 unquantised weights */
};

/* Weight encoding used by ORC_ARITH_INT32. */
enum {
  ORC_W_PLAIN = 0,      /* w_q = round(w * 2^8)                  (2^-8 pA)  */
  ORC_W_COMPRESSED = 1, /* w_q = 8 * round(w * 2^5), int16 range (2^-5 pA) */
  ORC_W_DEV8 = 2        /* w_q = mq + dev * sq: the pair's mean mq and an
                           8-bit deviation dev in steps sq (Sec. 5.3's
                           deviations from the mean; orc_dev8_params)      */
};

typedef struct {
  uint64_t seed;            /* Philox key for every stream of this instance */
  double scale;             /* N_p = floor(scale * N_p_full + 0.5)           */
  int indegree_mode;        /* 0: probabilities of tab:params3 unchanged;
                               1: full-scale synapse counts scaled by the
                                  target size, so in-degrees are kept     */
  int count_rule;           /* 0: fixed total number, log formula;
                               1: expected count N_pre * N_post * p        */
  int rows_are_sources;     /* 0: tab:params3 rows index the target population */
  double g;                 /* inhibitory PSP = g * 0.15 mV (default -4)      */
  double bg_rate_hz;        /* thalamic rate v_th (default 8 Hz)              */
  double psp_ext_mv;        /* thalamic PSP amplitude omega_ext (0.15 mV)     */
  int bg_const_T;           /* -1: Poisson drive; >= 0: T_t fixed to this     */
  int weight_mode;          /* ORC_W_PLAIN, ORC_W_COMPRESSED or ORC_W_DEV8    */
  const double *conn;       /* NULL, or 64 probabilities [target][source]     */
} orc_config;

/* Fills *c with the paper's defaults (scale 1, seed 1, g -4, 8 Hz, ...). */
void orc_config_default(orc_config *c);

/* ---- model constants (FP64) ---------------------------------------------- */
typedef struct {
  double w_f;               /* PSP -> PSC factor, pA per mV                  */
  double p11, p22, p21;     /* exact-integration propagators (FP64)          */
  float p11f, p22f, p21f;   /* the same rounded to FP32                      */
  double w_ext;             /* thalamic PSC amplitude, pA                    */
  int32_t w_ext_q;          /* the same in 2^-8 pA units (round half even)   */
} orc_consts;

int orc_constants(const orc_config *c, orc_consts *out);

/* ORC_W_DEV8 (Sec. 5.3: the synaptic weights are drawn from Gaussians with
 * known means, so their deviations from the mean need fewer bits).  For a
 * population pair of mean weight mu and standard deviation sd (pA):
 *   mq  = round(mu * 2^8)                         (2^-8 pA, round half even)
 *   sq  = max(1, round(5 sd * 2^8 / 127))         (the step: 5 sd over 127)
 *   dev = clamp(round((w * 2^8 - mq) / sq), -127, 127)
 *   w_q = mq + dev * sq
 * so |w_q - w * 2^8| <= sq / 2 unless |w - mu| exceeds about 5 sd. */
void orc_dev8_params(double mu, double sd, int32_t *mq, int32_t *sq);
int32_t orc_dev8_encode(double w, int32_t mq, int32_t sq, int32_t *dev);

/* Philox4x32-10 (Salmon et al., SC'11): out = bijection(ctr) under key. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Poisson inverse-CDF thresholds for mean lam: thr[k] = floor(2^32 CDF(k)),
 * k = 0..len-1, with len the first k whose tail mass is below 2^-32.
 * T = number of k with u >= thr[k] for a uniform 32-bit word u. */
int orc_poisson_table(double lam, uint32_t *thr, int cap, int *len);

/* ---- network ---------------------------------------------------------------*/
typedef struct orc_net orc_net;

int orc_build(const orc_config *c, orc_net **out);
void orc_net_free(orc_net *n);
/* Synapse counts [target * 8 + source] of a configuration, without sampling. */
int orc_pair_counts(const orc_config *c, uint64_t counts[64]);

uint32_t orc_net_n(const orc_net *n);                 /* neurons                */
uint64_t orc_net_nsyn(const orc_net *n);              /* synapses               */
void orc_net_pop_offsets(const orc_net *n, uint32_t off[9]);
uint64_t orc_net_pair_count(const orc_net *n, int target, int source);
/* CSR by sender: row_ptr[N+1], post[S], delay[S] (ticks), w[S] (pA, FP64),
 * w_q[S] (int32, in the weight mode of the build).  Pointers stay valid until
 * orc_net_free. */
const uint64_t *orc_net_row_ptr(const orc_net *n);
const uint32_t *orc_net_post(const orc_net *n);
const uint8_t *orc_net_delay(const orc_net *n);
const double *orc_net_weight(const orc_net *n);
const int32_t *orc_net_weight_q(const orc_net *n);
/* Mean and step (2^-8 pA) of pair [target][source] under ORC_W_DEV8. */
void orc_net_dev8_pair(const orc_net *n, int target, int source, int32_t *mq, int32_t *sq);
const float *orc_net_u0(const orc_net *n);            /* initial U, mV rel. E_L */
const double *orc_net_u0_f64(const orc_net *n);
/* Poisson table of population p. */
int orc_net_poisson(const orc_net *n, int p, const uint32_t **thr, int *len);

/* ---- simulation -------------------------------------------------------------*/
typedef struct orc_sim orc_sim;

typedef struct {
  uint64_t spikes;          /* spikes emitted                                 */
  uint64_t events;          /* synapses activated = sum of sender out-degrees */
  uint64_t poisson;         /* thalamic events = sum of T                     */
  int64_t consumed;         /* sum of ring-buffer values read (2^-8 pA units) */
  int64_t injected;         /* sum of w_q over activated synapses             */
} orc_counters;

int orc_sim_new(const orc_net *n, int arith, orc_sim **out);
void orc_sim_free(orc_sim *s);
/* Record U, I, R of these neurons after every step (copied). */
int orc_sim_set_probes(orc_sim *s, const uint32_t *ids, uint32_t n);
/* Record, for every neuron and step, T and the ring-buffer value read
 * (tiny networks only: 12 bytes per neuron per step). */
int orc_sim_record_inputs(orc_sim *s, int on);
int orc_sim_run(orc_sim *s, uint64_t n_steps);
/* The same loop (INT32 arithmetic only, no probes or recording) on `threads`
 * host threads; equal to orc_sim_run bit for bit.  A CPU baseline. */
int orc_sim_run_threads(orc_sim *s, uint64_t n_steps, int threads);

uint64_t orc_sim_t(const orc_sim *s);
void orc_sim_counters(const orc_sim *s, orc_counters *c);
/* Raster, sorted by (step, id). */
uint64_t orc_sim_nspikes(const orc_sim *s);
const uint32_t *orc_sim_spike_steps(const orc_sim *s);
const uint32_t *orc_sim_spike_ids(const orc_sim *s);
/* Current state; exactly one of the FP32 / FP64 triples is non-NULL. */
const float *orc_sim_u(const orc_sim *s);
const float *orc_sim_i(const orc_sim *s);
const double *orc_sim_u64(const orc_sim *s);
const double *orc_sim_i64(const orc_sim *s);
const int32_t *orc_sim_r(const orc_sim *s);
/* Ring buffer row r of 64 (int64 sums for INT32 arithmetic, else NULL). */
const int64_t *orc_sim_ring_q(const orc_sim *s);
const double *orc_sim_ring_f64(const orc_sim *s);
/* Probe traces: [step][probe] */
const float *orc_sim_probe_u(const orc_sim *s);
const float *orc_sim_probe_i(const orc_sim *s);
const double *orc_sim_probe_u64(const orc_sim *s);
const double *orc_sim_probe_i64(const orc_sim *s);
const int32_t *orc_sim_probe_r(const orc_sim *s);
uint64_t orc_sim_probe_steps(const orc_sim *s);
/* Recorded inputs: [step][neuron] */
const int32_t *orc_sim_rec_T(const orc_sim *s);
const int64_t *orc_sim_rec_w(const orc_sim *s);
const double *orc_sim_rec_w64(const orc_sim *s);
uint64_t orc_sim_rec_steps(const orc_sim *s);

/* One neuron driven by a given per-step input (2^-8 pA units for INT32,
 * pA for F64): the step rule of eqn:mem/eqn:psc/eqn:ref in isolation.
 * u_out[k], i_out[k], r_out[k] hold the state after step k. */
int orc_single_neuron_f32(const orc_consts *k, const int64_t *q, uint64_t n,
                          float *u_out, float *i_out, int32_t *r_out);
int orc_single_neuron_f64(const orc_consts *k, const double *q, uint64_t n,
                          double *u_out, double *i_out, int32_t *r_out);

const char *orc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
