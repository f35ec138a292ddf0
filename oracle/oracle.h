/*
 * oracle.h -- plain, slow FP64 CPU reference of spike delivery and the
 * exact-integration neuron update around it.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links
 * or calls this code; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source with the GPU path: its RNG,
 * tables, propagators, connection generation, transposition, delivery and
 * update are all written independently here.
 *
 * Paper: Pronold et al., "Routing brain traffic through the von Neumann
 * bottleneck" (Parallel Computing 2022, arXiv 2109.12855).
 *   - simulation cycle update -> communicate -> deliver every min-delay
 *     interval: Sec. 1 and Sec. 2.1 (Simulation engine);
 *   - static synapses, ring buffers, target segments: Sec. 3.1;
 *   - the delivery result is defined by Alg. REF: Sec. 3.2;
 *   - balanced random network benchmark: Sec. 2.2.
 * The paper gives no neuron equations, RNG, or parameter tables; the
 * readings used here are listed in the design notes of the repository.
 */
#ifndef SD_ORACLE_H
#define SD_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_DELTA = 0, OR_ALPHA = 1 };
enum { OR_W_FP32 = 0, OR_W_BF16 = 1, OR_W_BF16_RESID = 2 };
/* Philox key word 1 (stream) values; key word 0 is the seed. */
enum { OR_STREAM_SYN = 1, OR_STREAM_INIT = 2, OR_STREAM_DRIVE = 3, OR_STREAM_SRC = 4 };

typedef struct {
  int32_t model;            /* OR_DELTA / OR_ALPHA                                  */
  int32_t wform;            /* weight representation the oracle decodes to         */
  int64_t n_exc, n_inh;     /* local neurons: E ids [0,n_exc), I ids [n_exc,n)     */
  int64_t n_src_exc;        /* open loop: virtual E sources; 0 = closed loop       */
  int64_t n_src_inh;        /* open loop: virtual I sources                        */
  int32_t k_exc, k_inh;     /* fixed in-degree per target                          */
  int32_t d_lo, d_hi;       /* delay draws uniform in [d_lo, d_hi] steps           */
  int32_t d_min, d_max;     /* min / max delay of the network (slice = d_min steps)*/
  int32_t ring_len;         /* ring buffer length L (>= d_min + d_max)             */
  double h;                 /* resolution (ms)                                     */
  double w_exc, w_cv, g;    /* mean E weight, coefficient of variation, I = -g*draw*/
  double tau_m, c_m, tau_syn, e_l, v_th, v_reset, t_ref, i_e;
  double v0_lo, v0_hi;      /* initial V uniform in [v0_lo, v0_hi)                 */
  double drive_rate_hz;     /* Poisson drive per neuron (Hz)                       */
  double drive_w;           /* drive event weight (mV delta, pA alpha)             */
  double src_rate_hz;       /* open loop: rate of every virtual source (Hz)        */
  uint64_t seed;
  int64_t tgt_lo, tgt_hi;   /* generate targets [tgt_lo, tgt_hi) only (sampling);  */
                            /* tgt_hi = 0 means all local neurons                  */
  /* Plastic synapses (Sec. 6: weight updates driven by presynaptic spikes,  */
  /* computed when the weight becomes visible to the target, reading the     */
  /* time of the target's last spike).  plastic = 0: static synapses.        */
  int32_t plastic;
  double stdp_tau_plus, stdp_tau_minus;  /* ms                                   */
  double stdp_a_plus, stdp_a_minus;      /* weight units (pA / mV)               */
  double stdp_w_max;                     /* excitatory weights stay in [0, w_max] */
} or_config;

typedef struct or_net or_net;

/* --- counter-based RNG, tables, propagators ------------------------------ */
void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
double or_ndtri(double p);
void or_weight_tables(const or_config* c, float* w_e, float* w_i); /* 65536 each */
int or_poisson_thresholds(double lambda, uint32_t* out, int cap);
void or_propagators(const or_config* c, double out[7]); /* P11 P21 P22 P31 P32 P33 P30 */
float or_bf16_round(float x);
float or_decode_weight(const or_config* c, int is_inh, float w32);
int32_t or_ref_steps(const or_config* c);

/* --- network -------------------------------------------------------------- */
or_net* or_net_create(const or_config* c);
void or_net_destroy(or_net* n);
const char* or_last_error(void);
int64_t or_n_local(const or_net* n);
int64_t or_n_src(const or_net* n);
int64_t or_n_syn(const or_net* n);
/* target-major draws as generated: src, delay, weight index (k order)        */
void or_export_target_major(const or_net* n, uint32_t* src, uint8_t* dly, uint16_t* widx);
/* source-major table sorted by (src, target, k): row[n_src+1], tgt, dly, w   */
void or_export_source_major(const or_net* n, int64_t* row, int32_t* tgt, uint8_t* dly, double* w);
void or_out_weight(const or_net* n, double* out_w, int64_t* out_deg);

/* --- dynamics ------------------------------------------------------------- */
int64_t or_t_now(const or_net* n);
/* advance n_steps with the slice structure of the simulation cycle; spikes are
 * written (step, local id) in emission order; returns count or -1 on overflow */
int64_t or_simulate(or_net* n, int64_t n_steps, int64_t* spk_step, uint32_t* spk_id, int64_t cap);
/* deliver an explicit spike list: RB[(t0+lag+d) mod L][j] += w, cnt += 1      */
int or_deliver(or_net* n, const uint32_t* src, const uint8_t* lag, int64_t n_spk, int64_t t0,
               double* w_sum, int64_t* n_events);
/* update only (no delivery), appending nothing to the pending slice           */
int64_t or_update(or_net* n, int64_t n_steps, int64_t* spk_step, uint32_t* spk_id, int64_t cap);
/* ring buffer rows for steps [t_now, t_now+n_slots): out[s][j]                 */
void or_read_rb(const or_net* n, double* out, int64_t n_slots);
void or_read_counts(const or_net* n, uint32_t* out, int64_t n_slots);
void or_read_state(const or_net* n, double* v, double* y1, double* y2, int32_t* r);
void or_write_state(or_net* n, const double* v, const double* y1, const double* y2, const int32_t* r);
/* pending (emitted, not yet delivered) spikes of the open slice */
int64_t or_pending(const or_net* n, uint32_t* src, uint8_t* lag, int64_t cap, int64_t* slice_t0);
/* open-loop virtual sources: spikes of steps [t0, t0+n_steps), (lag, src) order */
int64_t or_open_loop_spikes(const or_config* c, int64_t t0, int32_t n_steps,
                            uint32_t* src, uint8_t* lag, int64_t cap);
/* the same for virtual sources [s_lo, s_hi) only                              */
int64_t or_open_loop_spikes_range(const or_config* c, int64_t t0, int32_t n_steps, int64_t s_lo,
                                  int64_t s_hi, uint32_t* src, uint8_t* lag, int64_t cap);
/* membrane potential of every held neuron just before the threshold test of
 * the last updated step (before any reset)                                   */
void or_read_vpre(const or_net* n, double* out);
/* Poisson drive count of neuron j (global id) at step t                        */
int32_t or_drive_count(const or_net* n, int64_t j, int64_t t);
/* plastic synapses: the nearest-spike pair update of one excitatory weight at
 * the delivery of a presynaptic spike (t_prev, t_last: -1 for none)           */
double or_stdp_update(const or_config* c, double w, int64_t t_pre, int64_t t_prev,
                      int64_t t_last, int32_t d);
/* current weights of the source-major table (plastic nets change them)        */
void or_read_weights(const or_net* n, double* w);

#ifdef __cplusplus
}
#endif
#endif
