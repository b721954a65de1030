/*
 * snn.h -- C ABI of the MI355X (gfx950) simulator of the Potjans-Diesmann
 * cortical microcircuit: clock-driven leaky integrate-and-fire neurons with
 * exponential current synapses, exactly integrated at dt = 0.1 ms, push
 * delivery of every spike into per-neuron delay ring buffers, and Poisson
 * thalamic drive.
 *
 * Paper: B. A. Lindqvist, A. Podobas, "Fast Algorithms for Spiking Neural
 * Network Simulation with FPGAs" (arXiv 2405.02019).
 *
 * Conventions
 *   - Every int-returning call returns SNN_OK (0) or a negative SNN_E_* code;
 *     snn_last_error() then describes the failure.  A failed snn_build leaves
 *     nothing allocated.
 *   - Host buffers are owned by the caller.  Device memory is owned by the
 *     simulator handle: it comes from the caller's allocator callbacks when
 *     given (e.g. the PyTorch caching allocator), otherwise from hipMalloc,
 *     and is released by snn_destroy.
 *   - Work is queued on one HIP stream (the caller's, or one the library
 *     creates).  snn_step_n is asynchronous; the read calls synchronise.
 *   - One handle must not be used from two host threads at once.
 *   - Membrane potentials are in mV relative to the resting potential
 *     (-65 mV): threshold 15 mV, reset 0.  Currents are in pA.  Synaptic
 *     input is accumulated in int32 fixed point of 2^-8 pA.
 */
#ifndef SNN_H
#define SNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SNN_ABI_VERSION 4u

enum snn_status {
  SNN_OK = 0,
  SNN_E_INVAL = -1,     /* invalid argument or configuration                  */
  SNN_E_NOMEM = -2,     /* host or device allocation failed                   */
  SNN_E_HIP = -3,       /* a HIP runtime call or a kernel launch failed       */
  SNN_E_RANGE = -4,     /* a value does not fit its encoding, or a caller
                           buffer is too small                                */
  SNN_E_OVERFLOW = -5,  /* an int32 accumulator or the device raster could
                           overflow                                           */
  SNN_E_DEVICE = -6     /* the device reported a failure (a persistent kernel's
                           bounded wait expired); the handle is unusable      */
};

/* Synapse storage formats. */
enum snn_syn_format {
  /* 8-byte records {int32 weight in 2^-8 pA; uint32 target << 6 | delay},
     sorted by sender (Sec. 3.5, lst:index; the paper's 8-byte synapse). */
  SNN_SYN_PLAIN8 = 0,
  /* 5 bytes in three streams: uint16 target offset inside a 65,536-neuron
     target block, int16 weight in 2^-5 pA, uint8 delay; sorted by sender,
     then target block (the 16-bit weights of Sec. 5.3).  The LDS engines
     pack the same weight, delay and window offset into one 4-byte record. */
  SNN_SYN_COMPRESSED5 = 1,
  /* 3 bytes in two streams, LDS and banded engines only: a uint16 locator
     and an int8 deviation of the weight from the mean of its population
     pair, in steps of 5 sd / 127 of that pair; the weight is mean +
     deviation * step in 2^-8 pA, both rounded to that unit (Sec. 5.3: the
     weights are drawn from Gaussians of known mean, so their deviations from
     the mean need fewer bits).  LDS engine locator: bit 15 the doubled
     L4e -> L2/3e pair, bits 9-14 the delay, bits 0-8 the target offset in a
     window of at most 512 neurons.  Banded engine locator (H ring rows):
     bit 15 the doubled pair, then the delay minus its band's first delay in
     log2(H) bits, then the target offset in 15 - log2(H) bits; deviation
     -128 marks an unused slot. */
  SNN_SYN_DEV8 = 2
};

/* Step-loop engines. */
enum snn_engine {
  SNN_ENGINE_AUTO = 0,        /* LDS when it fits, else banded, else persistent,
                                 else stepwise                                    */
  SNN_ENGINE_STEPWISE = 1,    /* two kernels per step (update, then transfer)    */
  SNN_ENGINE_PERSISTENT = 2,  /* one cooperative kernel per chunk of steps, one
                                 grid-wide barrier per step, ring in HBM          */
  SNN_ENGINE_LDS = 3,         /* persistent, each block owning up to 320 or 512
                                 neurons and their 64 ring rows in LDS; synapses
                                 stored per (sender, destination block).  The
                                 automatic choice when the whole network fits
                                 the co-resident blocks; requested explicitly,
                                 instances beyond that run as several launches
                                 per chunk (groups of whole instances)            */
  SNN_ENGINE_BAND = 4         /* persistent, each block owning up to 3,584 neurons
                                 and H = 64, 16 or 8 rows of their ring in LDS:
                                 horizon-based transfer (Sec. 3.4, lst:horizon2)
                                 with synapses stored per (sender, destination
                                 block, delay band); the slow bands are
                                 delivered while the spikes of the last step
                                 propagate between blocks, the one-step delays
                                 once they have arrived                           */
};

/* One microcircuit instance.  Defaults (snn_instance_default) are the
 * paper's: Tables tab:params, tab:params2, tab:params3. */
typedef struct {
  uint64_t seed;           /* keys every random stream of the instance          */
  double scale;            /* N_p = floor(scale * N_p(full) + 0.5), 0 < s <= 64  */
  int32_t indegree_mode;   /* 0: connection probabilities unchanged;
                              1: full-scale synapse counts scaled by the target
                                 size, so in-degrees stay at full scale          */
  int32_t count_rule;      /* 0: fixed total number n = ln(1-p)/ln(1-1/(N N'));
                              1: expected count N N' p                           */
  int32_t rows_are_sources;/* orientation of tab:params3; 0 = rows are targets */
  double g;                /* inhibitory PSP = g * 0.15 mV, g <= 0 (default -4) */
  double bg_rate_hz;       /* thalamic rate v_th (default 8 Hz)                 */
  double psp_ext_mv;       /* thalamic PSP amplitude omega_ext (0.15 mV)        */
  int32_t bg_const_T;      /* -1: Poisson thalamic counts; >= 0: fixed count    */
  const double *conn;      /* NULL, or 64 probabilities [target * 8 + source]   */
} snn_instance_cfg;

typedef struct {
  uint32_t abi_version;        /* SNN_ABI_VERSION                                */
  uint32_t n_instances;        /* >= 1; instances evolve independently           */
  const snn_instance_cfg *inst;
  uint32_t syn_format;         /* enum snn_syn_format                            */
  uint32_t engine;             /* enum snn_engine                                */
  uint32_t chunk_steps;        /* steps per captured graph / persistent launch;
                                  0 = 100                                         */
  uint32_t block_size;         /* threads per block; 0 = tuned                   */
  uint32_t grid_blocks;        /* blocks of the persistent kernel; 0 = tuned     */
  uint64_t raster_capacity;    /* device raster entries between drains; 0 = auto;
                                  two buffers of it (one for the graph-replayed
                                  stepwise engine): the step loop swaps them at
                                  a drain and reads the full one back while the
                                  next chunk runs                                */
  int32_t host_threads;        /* threads of the network sampler; 0 = auto       */
  int32_t use_graphs;          /* 1: replay chunks from a captured HIP graph     */
  uint32_t window_neurons;     /* LDS engines: neurons per window (a multiple of
                                  4); 0 = the shortest that fills one launch     */
  uint32_t reserved0;          /* 0                                              */
  const uint32_t *inst_window_neurons;
                               /* LDS engines: NULL, or one window length per
                                  instance (n_instances entries, multiples of 4,
                                  window_neurons = 0): an instance that fires
                                  more gets shorter windows, so that every block
                                  delivers about as many synaptic events a step
                                  (snn_build_tuned derives them from measured
                                  event counts); read during the call only      */
  void *hip_stream;            /* hipStream_t; NULL = a stream of the library    */
  void *(*dev_alloc)(size_t bytes, void *ctx); /* NULL = hipMalloc              */
  void (*dev_free)(void *ptr, void *ctx);
  void *alloc_ctx;
} snn_config;

typedef struct snn_net snn_net;

/* Fill with defaults: one instance is NOT attached (inst = NULL). */
void snn_config_default(snn_config *cfg);
void snn_instance_default(snn_instance_cfg *inst);

/*
 * snn_build -- sample the network(s) on the host, upload them, precompute the
 * propagators on the GPU and prepare the step loop.
 *   Model: Sec. 2.2 (tables tab:params..tab:params3; w_f, eqn:p11p22, eqn:p21);
 *   storage: Sec. 3.5 (lst:index).  Synapse counts per population pair,
 *   Gaussian weights (sd 10 % of the mean, sign kept) and delays (rounded to
 *   steps, clipped to [1, 63]) are drawn from counter-based Philox4x32-10
 *   streams keyed by the instance seed; initial potentials from tab:params2.
 * On success *out owns all device memory; on failure *out is NULL.
 * Errors: SNN_E_INVAL (bad config), SNN_E_RANGE (a delay/weight/target that
 * does not fit the chosen format), SNN_E_OVERFLOW (a neuron's worst-case
 * input could overflow int32), SNN_E_NOMEM, SNN_E_HIP.
 */
int snn_build(const snn_config *cfg, snn_net **out);

/*
 * snn_step_n -- advance every instance by n_steps steps of dt = 0.1 ms.
 *   One step (Sec. 3, lst:basic with lst:push / lst:push2):
 *     for every neuron: if R == 0: x = p22 U + p21 I; x >= 15 mV => spike,
 *     x = 0, R = 20; U = x; else U = 0, R -= 1 (eqn:mem, eqn:ref);
 *     I = p11 I + (T w_ext + W[t mod 64]) with T ~ Poisson(v_th K dt)
 *     (eqn:psc), then W[t mod 64] = 0;
 *     for every spike and every synapse (j, d, w): W[(t+d) mod 64][j] += w.
 * Asynchronous: work is queued on the handle's stream.  May synchronise to
 * drain the device raster before it could overflow.
 * Errors: SNN_E_HIP, SNN_E_DEVICE.
 */
int snn_step_n(snn_net *h, uint64_t n_steps);

/*
 * snn_step_n_noalloc -- snn_step_n for callers that cannot allocate memory
 * (tight serving loops, harnesses that forbid allocation): advances every
 * instance by n_steps steps without any device or host allocation and
 * without synchronising.  LDS and banded engines only (SNN_E_INVAL for the
 * others); the handle's device must be current.
 *   d_raster: device buffer of raster_cap uint64 entries receiving this
 *     call's spikes as (step << 32 | global neuron id), where instance k's
 *     ids start at the sum of the earlier instances' neuron counts, each
 *     rounded up to a multiple of 256; in runs of one window each in (step,
 *     id) order, the runs in no particular order.  raster_cap must hold the
 *     worst case, every neuron spiking once per 21 steps
 *     (neurons * ((n_steps + 20) / 21)), else SNN_E_RANGE.
 *   d_status: device buffer of 2 uint64 receiving, when the queued work
 *     completes, the number of raster entries written and the device error
 *     word (0 = success; nonzero: a bounded wait expired, the state is
 *     invalid).
 * The per-call state of the step loop (control words, flag words, sender
 * lists and the sender history) lives in a static 32 MiB device array per
 * GPU, cleared at the start of every call; networks needing more return
 * SNN_E_RANGE (the LDS engine fits up to about 2 million neurons; the
 * banded engine, whose sender history takes 272 bytes per neuron plus 48 KiB
 * per block below 1,024 threads, about 77,000 at 256 threads and 304-neuron
 * windows, 107,000 at 512 threads, 123,000 at 1,024).  Calls on one GPU must
 * not overlap: they
 * share that array.  State, counters and snn_read_state are as after
 * snn_step_n; the spikes of this call are not in the handle's raster.
 * Errors: SNN_E_INVAL, SNN_E_RANGE, SNN_E_HIP, SNN_E_DEVICE.
 */
int snn_step_n_noalloc(snn_net *h, uint64_t n_steps, uint64_t *d_raster, uint64_t raster_cap,
                       uint64_t *d_status);

/*
 * snn_read_spikes -- spikes of instance `inst` emitted in steps [t0, t1),
 * sorted by (step, neuron id).  A spike of step t is a neuron whose membrane
 * update of step t crossed the threshold (eqn:mem, eqn:ref): the neurons
 * lst:push2 collects in its queue Q at step t, i.e. the senders whose
 * synapses that step's transfer activates.  Ids are instance-local
 * (population p holds [pop_offset[p], pop_offset[p+1]) in table order).
 * steps[k], ids[k] receive at most `cap` entries (either pointer may be NULL
 * to skip it; both NULL only counts); *n_out is the number of spikes in the
 * range.  Spikes discarded by snn_discard_spikes are no longer returned.
 * Synchronises.
 * Errors: SNN_E_INVAL, SNN_E_RANGE (cap < *n_out; nothing written),
 * SNN_E_OVERFLOW (the device raster overflowed), SNN_E_HIP.
 */
int snn_read_spikes(snn_net *h, uint32_t inst, uint64_t t0, uint64_t t1, uint32_t *steps,
                    uint32_t *ids, uint64_t cap, uint64_t *n_out);

/*
 * snn_discard_spikes -- drop the host-side record of every spike (all
 * instances) of steps before t_before, so that long runs keep a bounded
 * raster store; later reads of those steps return nothing.  Synchronises
 * (drains the device raster first).
 * Errors: SNN_E_INVAL (NULL handle), SNN_E_HIP, SNN_E_DEVICE.
 */
int snn_discard_spikes(snn_net *h, uint64_t t_before);

/* State of one instance.  Array pointers are caller buffers (or NULL to
 * skip): U, I, R hold n_neurons entries; W holds 64 * n_neurons entries,
 * row r of the ring buffer at W[r * n_neurons + i]. */
typedef struct {
  float *U;
  float *I;
  int32_t *R;
  int32_t *W;
  uint64_t t;              /* out: steps simulated                         */
  uint32_t n_neurons;      /* out                                          */
  uint64_t n_synapses;     /* out                                          */
  uint64_t spikes;         /* out: spikes emitted                          */
  uint64_t events;         /* out: synapses activated (sum of out-degrees) */
  uint64_t poisson;        /* out: thalamic events (sum of T)              */
  int64_t consumed;        /* out: ring-buffer charge read, 2^-8 pA units  */
  float p11, p21, p22;     /* out: FP32 propagators computed on the GPU    */
  int32_t w_ext_q;         /* out: thalamic weight, 2^-8 pA                */
  double w_f;              /* out: PSP -> PSC factor, pA per mV            */
} snn_state;

/*
 * snn_read_state -- copy the state of instance `inst` (after the last queued
 * step) into the caller's buffers.  Synchronises.
 *   U, I, R are the neuron state of eqn:mem, eqn:psc and eqn:ref after step
 *   t-1: U the membrane potential, I the synaptic current that step t's
 *   membrane update reads (it already holds the thalamic and ring input of
 *   step t-1), R the refractory steps left.  W is the wrap-around ring
 *   buffer of Sec. 3.2 (64 rows, row (s mod 64) collects the input read at
 *   step s) holding every delivery of every spike emitted so far, in int32
 *   units of 2^-8 pA.  The counters are exact: spikes, synapse activations
 *   (each spike activates its sender's out-degree), thalamic events and the
 *   int64 sum of ring values read (charge conservation: consumed + sum of W
 *   equals the sum of w_q over all activations).
 * Errors: SNN_E_INVAL, SNN_E_HIP.
 */
int snn_read_state(snn_net *h, uint32_t inst, snn_state *out);

/* Free all device and host memory of the handle.  NULL-safe. */
void snn_destroy(snn_net *h);

/* Message of the last failure on this handle (h == NULL: the last failure of
 * snn_build in this thread).  Never NULL. */
const char *snn_last_error(const snn_net *h);

/* ---- launch description (for profiling and tuning reports) -------------- */
typedef struct {
  uint32_t engine;         /* engine in use                                  */
  uint32_t block_size;
  uint32_t grid_blocks;    /* persistent grid, or transfer-kernel grid      */
  uint32_t quads_per_thread;
  uint32_t chunk_steps;
  uint32_t n_neurons_total;/* all instances, each padded to a multiple of 4 */
  uint64_t n_synapses_total;
  uint64_t device_bytes;   /* device memory held                            */
  double build_seconds;    /* host sampling + upload                        */
  uint32_t launches_per_chunk; /* kernel launches one chunk of steps takes    */
  uint32_t window_neurons; /* LDS engine: neurons of the longest window      */
  uint32_t graphs;         /* 1: full chunks replay from a captured hipGraph */
  uint32_t ring_rows;      /* ring-buffer rows kept on chip (LDS engines), or
                              the 64 rows in device memory                    */
} snn_info;

int snn_get_info(const snn_net *h, snn_info *out);

/* ---- launch-shape tuning ----------------------------------------------- */
typedef struct {
  uint32_t engine;
  uint32_t candidates;        /* shapes timed (0: taken from the tuning cache) */
  uint32_t block_size;        /* shape adopted                                 */
  uint32_t grid_blocks;
  uint32_t quads_per_thread;
  uint32_t window_neurons;    /* LDS engines: window length adopted            */
  double us_per_step_first;   /* the handle's shape before tuning              */
  double us_per_step_best;    /* the adopted shape                             */
} snn_tune_report;

/*
 * snn_autotune -- time candidate launch shapes of the handle's engine on the
 * live simulation and keep the fastest.  Each candidate runs trial_steps
 * steps for real (they advance the simulation; every shape gives the same
 * results).  Persistent engine: block size x quads per thread, each at the
 * smallest co-resident grid; stepwise engine: grid of the transfer kernel
 * (the chunk graph is captured again); the LDS engine's shape is fixed by its
 * storage layout and is reported as the one candidate.  Synchronises.
 * Errors: as snn_step_n; SNN_E_INVAL for trial_steps = 0 or a NULL argument.
 */
int snn_autotune(snn_net *h, uint32_t trial_steps, snn_tune_report *out);

/*
 * snn_build_tuned -- snn_build with the storage layout chosen by timing: for
 * the LDS engines (engine AUTO, LDS or BAND) each candidate -- the engine
 * (LDS, or banded with its ring rows) and the window length (the shortest
 * that fills one launch, and longer ones up to the kernel's capacity: fewer,
 * larger destination classes of Sec. 3.6) -- is built, run for trial_steps / 4
 * warm-up and trial_steps timed steps, and the fastest is built again from
 * step 0 and returned in *out.  With several instances, the first candidate's
 * run also counts each instance's synaptic events per neuron and step, and
 * the winner's kernel is timed once more with per-instance window lengths
 * (inst_window_neurons) that give every block about the same events per step.
 * Results do not depend on the choice.
 *   cache_path: NULL, or a text file of earlier choices keyed by the GPU's
 *   architecture name and a digest of the configuration (one line each:
 *   architecture, digest, engine, window length, best and first us per step,
 *   and per-instance window lengths joined by commas when those won); a hit
 *   builds the cached choice without timing (rep->candidates = 0), a miss
 *   appends the new choice.  Configurations that fix window_neurons or
 *   inst_window_neurons, and other engines: as snn_build (no candidates).
 * Errors: as snn_build and snn_step_n; SNN_E_INVAL for trial_steps = 0.
 */
int snn_build_tuned(const snn_config *cfg, uint32_t trial_steps, const char *cache_path,
                    snn_net **out, snn_tune_report *rep);

/*
 * snn_time_steps -- queue n_steps steps (as snn_step_n) between two HIP events
 * recorded on the handle's stream and return the elapsed milliseconds.
 * Synchronises.  Errors: as snn_step_n.
 */
int snn_time_steps(snn_net *h, uint64_t n_steps, double *elapsed_ms);

/* ---- host-only network sampling (no GPU needed) --------------------------- */
/* The network exactly as snn_build samples it, for inspection and tests:
 * sender-sorted synapses of one instance with instance-local neuron ids. */
typedef struct {
  uint32_t n_neurons;
  uint64_t n_synapses;
  uint32_t pop_offset[9];  /* neuron ids of population p: [off[p], off[p+1]) */
  uint64_t *row_ptr;       /* n_neurons + 1                                  */
  uint32_t *post;          /* n_synapses: receiver                           */
  uint8_t *delay;          /* n_synapses: steps, 1..63                       */
  int32_t *w_q;            /* n_synapses: weight, 2^-8 pA                    */
  float *u0;               /* n_neurons: initial potential (mV rel. E_L)     */
} snn_host_network;

/*
 * snn_sample_network -- run the sampler of snn_build for one instance on the
 * host (syn_format selects the weight quantisation: 2^-8 pA, or 2^-5 pA
 * widened to 2^-8 pA) and return it; free with snn_free_network.
 * Errors: as snn_build, minus SNN_E_HIP.
 */
int snn_sample_network(const snn_instance_cfg *inst, uint32_t syn_format, int32_t host_threads,
                       snn_host_network **out);

/*
 * snn_sample_network_windows -- as snn_sample_network, but stored in the
 * layout of the LDS engine with `window`-neuron target windows (256 or 512):
 * per (sender, window) a segment of fixed capacity, the largest segment of
 * the sender's population in that window (Sec. 3.6's synapse classes by
 * destination), read back into rows ordered by window.  window = 0 gives
 * snn_sample_network.  Errors: SNN_E_INVAL for another window; as
 * snn_sample_network otherwise.
 */
int snn_sample_network_windows(const snn_instance_cfg *inst, uint32_t syn_format, uint32_t window,
                               int32_t host_threads, snn_host_network **out);
/*
 * snn_sample_network_bands -- as snn_sample_network_windows, but stored in
 * the layout of the banded engine: `window`-neuron target windows (4 ..
 * 4,096, a multiple of 4), and per (sender, window) one fixed-capacity
 * segment per delay band of a ring of `ring_rows` rows (64, 32, 16 or 8):
 * band 0 holds delay 1, band j >= 1 the delays [2 + (j-1) H, 1 + j H]
 * (Sec. 3.4's horizon bands, Sec. 3.5's index by sender and delay), read
 * back into rows ordered by window, then band.  A synapse of weight 0 is
 * stored like an unused slot and is not read back.
 * Errors: SNN_E_INVAL for another window or ring size; as
 * snn_sample_network otherwise.
 */
int snn_sample_network_bands(const snn_instance_cfg *inst, uint32_t syn_format, uint32_t window,
                             uint32_t ring_rows, int32_t host_threads, snn_host_network **out);
void snn_free_network(snn_host_network *net);

/*
 * snn_balanced_windows -- host only: the per-instance window lengths that
 * snn_build_tuned tries for several instances (Sec. 3.6's destination
 * classes sized by load).  Instance k (n_neurons[k] neurons, load[k]
 * synaptic events per neuron and step, >= 0) gets windows of about T /
 * load[k] neurons, a multiple of 4 in [4, max_window] (max_window for a
 * silent instance), for the smallest per-block load T whose windows -- the
 * instance's quads cut into windows of at most that many neurons -- number
 * at most max_blocks in all.  window_out (caller-owned, n_instances entries)
 * receives the lengths.
 * Errors: SNN_E_INVAL (NULL array, no instances, a negative or non-finite
 * load, max_window not a positive multiple of 4); SNN_E_RANGE when even
 * max_window-neuron windows exceed max_blocks.
 */
int snn_balanced_windows(uint32_t n_instances, const uint32_t *n_neurons, const double *load,
                         uint32_t max_window, uint32_t max_blocks, uint32_t *window_out);

#ifdef __cplusplus
}
#endif
#endif
