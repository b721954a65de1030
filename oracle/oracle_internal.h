/* oracle_internal.h -- definitions shared by the oracle's own .c files only. */
#ifndef SNN_ORACLE_INTERNAL_H
#define SNN_ORACLE_INTERNAL_H

#include "oracle.h"

#define ORC_D_MAX 64          /* ring-buffer rows (Sec. 3.2)                 */
#define ORC_POI_CAP 64        /* longest Poisson table accepted              */

/* Philox counter word 3 names the stream. */
#define ORC_TAG_SYN 1u        /* synapse sampling: (k, 2*(8*tgt+src)+half)   */
#define ORC_TAG_V0 2u         /* initial membrane potential: (neuron, 0)     */
#define ORC_TAG_POI 3u        /* thalamic counts: (neuron/4, step lo, hi)    */

extern const double ORC_DT_MS, ORC_C_M, ORC_TAU_M, ORC_TAU_SYN, ORC_THETA, ORC_E_L;
extern const float ORC_THETA_F;
extern const int ORC_T_REF_STEPS;
extern const uint32_t ORC_N_FULL[8], ORC_K_EXT[8];
extern const double ORC_V0_MEAN[8], ORC_V0_SD[8];
extern const double ORC_CONN[8][8];

int orc_is_exc(int p);
void orc_error(const char *fmt, ...);
void orc_draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t tag,
              uint32_t out[4]);
double orc_unit(uint32_t w);
double orc_normal(uint32_t a, uint32_t b);

struct orc_net {
  orc_config cfg;
  double conn[8][8];          /* [target][source]                            */
  orc_consts k;
  uint32_t N;
  uint32_t n_pop[8];
  uint32_t off[9];
  uint64_t pair_n[8][8];      /* [target][source]                            */
  double mu_w[8][8];          /* mean weight of each pair, pA [target][source] */
  double sd_w[8][8];          /* its standard deviation, pA                    */
  uint64_t S;
  uint64_t *row_ptr;          /* N + 1                                       */
  uint32_t *post;
  uint8_t *delay;
  double *w;
  int32_t *w_q;
  float *u0;
  double *u0d;
  uint8_t *pop_of;            /* population of each neuron                   */
  uint32_t thr[8][ORC_POI_CAP];
  int thr_len[8];
};

#endif
