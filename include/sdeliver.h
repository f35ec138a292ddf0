/*
 * sdeliver.h -- C ABI of the MI355X spike-delivery library.
 *
 * The library runs the hot path of a time-driven spiking-network simulation
 * on one gfx950 GPU (Pronold et al., arXiv 2109.12855):
 *   - build_connections: the network is created once from probabilistic
 *     rules before simulation; its construction is not part of simulation
 *     time (Sec. 1, Sec. 2.2).
 *   - update_neurons: neurons advance on the h grid by the exact
 *     propagators of their linear subthreshold dynamics (Sec. 1, Sec. 2.1).
 *   - deliver_spikes: every spike's target segment is walked and each
 *     synapse's weight is added into its target's ring buffer at the
 *     synapse's delay, with the result Alg. REF defines (Sec. 3.1, 3.2).
 *   - simulate(T): the cycle update -> (exchange) -> deliver repeats every
 *     min-delay interval (Sec. 1, Sec. 2.1).
 *
 * Conventions for every call:
 *   - Return value: SD_OK or a negative sd_status; nothing throws across the
 *     ABI.  sd_last_error(ctx) holds a message for the last failure.
 *   - Streams: all device work is ordered on the HIP stream given at
 *     sd_create.  Calls that return host data synchronise that stream.
 *   - Pointers: "d_" arguments are device pointers, "h_" are host pointers;
 *     both are borrowed for the duration of the call (device pointers until
 *     the stream reaches the call).
 *   - Devices: a context lives on the device that was current at sd_create.
 *   - Threads: one host thread at a time per context.
 *   - Units: times in ms, steps as int64, weights in mV (delta model) or
 *     pA (alpha model).
 */
#ifndef SDELIVER_H
#define SDELIVER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sd_ctx sd_ctx;

typedef enum {
  SD_OK = 0,
  SD_EINVAL = -1,        /* invalid argument or configuration                */
  SD_ENOMEM = -2,        /* device allocation failed / arena too small       */
  SD_EHIP = -3,          /* a HIP runtime call failed                        */
  SD_EOVERFLOW = -4,     /* a device-side capacity was exceeded (sticky)     */
  SD_ESTATE = -5,        /* call not valid in the context's current state    */
  SD_EUNSUPPORTED = -6   /* configuration outside what the library supports */
} sd_status;

typedef enum { SD_IAF_PSC_DELTA = 0, SD_IAF_PSC_ALPHA = 1 } sd_model;

/* Storage form of a synapse (weight, target, delay):
 *   SD_W_FP32        f32 weight, i32 target id, u8 delay       (9 B / synapse)
 *   SD_W_BF16        bf16 weight, u16 offset in block, u8 delay (5 B)
 *   SD_W_BF16_RESID  bf16 residual d, w = mu_pop * (1 + d), where mu_pop is
 *                    the FP32 mean weight of the source's population,
 *                    u16 offset in block, u8 delay              (5 B)
 *   SD_W_BF16_PACKED the residual weight (low half) and the ring-window slot
 *                    (delay - d_min) * block_neurons + offset in block
 *                    (high half) in one 32-bit word             (4 B);
 *                    needs (d_max - d_min + 1) * block_neurons <= 65536
 * In the source-major layout the targets are cut into parts of 2^tbits
 * (tbits = 24 - the bits of d_max - d_min, at most 4 parts) and each source
 * has one segment per part.  A record is a u32 {offset in the part (tbits),
 * delay - d_min, and for the BF16 forms the weight's high byte in bits
 * 24-31} plus the f32 weight (FP32 form, 8 B) or the weight's low byte (the
 * BF16 forms; packed = residual there, 5 B). */
/* Connection-table layout:
 *   SD_LAYOUT_BLOCK   block-major: the synapses from each source into each
 *                     target block of B neurons form one segment; segments
 *                     are stored source by source (a spike's segments for
 *                     consecutive blocks are adjacent), and a workgroup
 *                     delivers its block's segments into the block's ring
 *                     window held in LDS.  For networks whose sources each
 *                     reach many targets per block.
 *   SD_LAYOUT_SOURCE  source-major: each source's synapses to all local
 *                     targets form one contiguous segment (as in the
 *                     paper's per-process table, Sec. 3.1).  A delivery
 *                     first sorts the slice's events by target block into
 *                     4-byte binned records (8 for FP32) held in device
 *                     memory, then accumulates them in the same LDS ring
 *                     windows.  For tables beyond 2^32 synapses and sources
 *                     whose segments are sparse across blocks (the one-GPU
 *                     share of a brain-scale network).
 *   SD_LAYOUT_AUTO    block-major when it fits, else source-major.
 * Both give the same rings and dynamics: a delivery's sums are exact
 * integers in the fixed-point window, rounded to FP32 once per delivery. */
typedef enum { SD_LAYOUT_AUTO = 0, SD_LAYOUT_BLOCK = 1, SD_LAYOUT_SOURCE = 2 } sd_layout;

typedef enum {
  SD_W_FP32 = 0,
  SD_W_BF16 = 1,
  SD_W_BF16_RESID = 2,
  SD_W_BF16_PACKED = 3
} sd_wform;

typedef struct {
  int32_t model;             /* sd_model                                        */
  int32_t wform;             /* sd_wform                                        */
  int64_t n_exc, n_inh;      /* local neurons: E ids [0,n_exc), I ids after     */
  int64_t n_src_exc;         /* open loop: virtual E sources (0 = closed loop)  */
  int64_t n_src_inh;         /* open loop: virtual I sources                    */
  int32_t k_exc, k_inh;      /* fixed in-degree, drawn with replacement         */
  int32_t d_lo, d_hi;        /* delays uniform over [d_lo, d_hi] steps          */
  int32_t d_min, d_max;      /* network min/max delay; a slice is d_min steps   */
  int32_t ring_len;          /* ring buffer length L >= d_min + d_max, <= 64    */
  double h;                  /* resolution (ms)                                 */
  double w_exc, w_cv, g;     /* E weight mean and CV; I weight = -g * E draw    */
  double tau_m, c_m, tau_syn, e_l, v_th, v_reset, t_ref, i_e;
  double v0_lo, v0_hi;       /* initial V uniform in [v0_lo, v0_hi)             */
  double drive_rate_hz;      /* independent Poisson drive per neuron            */
  double drive_w;            /* weight of one drive event                       */
  double src_rate_hz;        /* open loop: rate of each virtual source          */
  uint64_t seed;
  int32_t block_neurons;     /* target block size (0 = automatic)               */
  int32_t record_spikes;     /* keep a device raster of emitted spikes (0/1)    */
  int64_t record_cap;        /* raster capacity in spikes (0 = automatic)       */
  int32_t layout;            /* sd_layout                                       */
  int32_t bin_cap;           /* source-major: binned records per (target
                                block, binning workgroup) region and delivery,
                                at most 1024; events past it take a slower
                                exact path (0 = from the expected rate)        */
  /* Plastic excitatory synapses (Sec. 6: weight updates driven by the
   * presynaptic spike, computed at delivery, reading the time of the
   * target's last spike).  At the delivery of a spike of step t_pre, each
   * excitatory weight w of a synapse with delay d (all of it on the target
   * side) sees t_last, the target's latest spike with t_last + d <= t_pre,
   * and its source's previous spike t_prev:
   *   if t_last + d > t_prev: w = min(w + A+ exp(-(t_last+d-t_prev) h/tau+), w_max)
   *   then                    w = max(w - A- exp(-(t_pre-t_last-d) h/tau-), 0)
   * (nothing without a visible target spike); the updated w is delivered.
   * Needs the FP32 form, the block-major layout, closed loop, d_min <= 16,
   * d_min + d_max <= 64 and at most one target block per workgroup pass. */
  int32_t plastic;           /* 0 static, 1 plastic                             */
  double stdp_tau_plus, stdp_tau_minus;  /* ms                                  */
  double stdp_a_plus, stdp_a_minus;      /* weight units                        */
  double stdp_w_max;                     /* upper weight bound                  */
} sd_config;

typedef struct {
  int64_t n_local;           /* neurons held                                    */
  int64_t n_src;             /* source ids (local, or virtual in open loop)     */
  int64_t n_syn;             /* synapses                                        */
  int32_t block_neurons;     /* target block size in use                        */
  int32_t n_blocks;          /* number of target blocks                         */
  int64_t table_bytes;       /* synapse arrays + segment pointers               */
  int64_t arena_bytes;       /* total device memory of a context                */
  int32_t bytes_per_synapse; /* block-major: 9 (FP32), 5 (BF16, residual), 4
                                (packed); source-major: 8 (FP32), 5 (BF16s)   */
  int32_t layout;            /* the layout in use (SD_LAYOUT_BLOCK / _SOURCE)   */
  int32_t bin_cap;           /* source-major: binned records per region in use
                                (the configured or automatic bin_cap); 0 for
                                block-major                                    */
} sd_sizes;

typedef struct {
  int64_t t_now;             /* next step to update                             */
  int64_t spikes_emitted;    /* local spikes since creation                     */
  int64_t events_delivered;  /* synaptic events (sum of segment lengths)        */
  int64_t spikes_delivered;  /* spike entries delivered                          */
  int64_t slices;            /* fused slice launches                            */
  int64_t spikes_recorded;   /* entries in the raster                           */
  int32_t overflow;          /* sticky device flags: bit 0 spike-list overflow,  */
                             /* bit 1 raster overflow, bits 2-3 invalid entries, */
                             /* bit 4 a persistent launch's barrier timed out    */
                             /* of an external spike list (SD_EINVAL)            */
} sd_stats;

/* Sizes the context needs for this configuration (no device work). */
sd_status sd_query_sizes(const sd_config* cfg, sd_sizes* out);

/* Create a context on the current device, ordered on hip_stream (NULL: the
 * null stream).  d_arena (optional) is caller-owned device memory of at least
 * sizes.arena_bytes that the context carves all its buffers from and never
 * frees; with d_arena NULL the context allocates (hipMalloc) and frees it.
 * Computes the exact propagators in FP64 on the device, the weight quantile
 * table and Poisson-drive thresholds on the host, and the initial state. */
sd_status sd_create(const sd_config* cfg, void* hip_stream, void* d_arena, size_t arena_bytes,
                    sd_ctx** out);
void sd_destroy(sd_ctx* ctx);
const char* sd_last_error(const sd_ctx* ctx);

/* Draw the network (one counter-based Philox4x64-10 block per synapse,
 * target-major) and lay it out block-major: the synapses into target block
 * b form one contiguous region ordered by source, and for source s the
 * synapses into b form one contiguous segment in (target, draw index)
 * order; the segment pointers are stored source-major as (start, count)
 * pairs.  Deterministic; run once before updates. */
sd_status sd_build_connections(sd_ctx* ctx);

/* Advance every neuron by n_steps (1 <= n_steps, and the steps must stay in
 * the current slice of d_min steps): reads and consumes the ring buffer
 * rows of those steps, draws the Poisson drive, propagates exactly, applies
 * threshold/reset/refractoriness, and appends emitted spikes to the open
 * slice's spike list (one contiguous list; each block appends its spikes in
 * (lag, neuron) order, blocks in any order - delivery sums are exact
 * integers, so the order does not change results). */
sd_status sd_update_neurons(sd_ctx* ctx, int32_t n_steps);

/* Deliver spikes (Alg. REF result, Sec. 3.2): for every spike (src, lag) and
 * every synapse (src -> j, delay d, weight w): ring[t0 + lag + d][j] += w.
 * d_src/d_lag: n device entries (u32 source ids, u8 lags), borrowed until the
 * stream reaches the call; n == 0: nothing to add.  0 <= n <= n_blocks *
 * block_neurons * d_min (the context's list capacity), else SD_EINVAL.  The list is packed
 * and validated on the device into the context's own buffer (no host round
 * trip, no allocation): an entry with src >= n_src or lag >= d_min delivers
 * nothing and sets a sticky flag that the next sd_get_stats reports as
 * SD_EINVAL (bit 3 of sd_stats.overflow).  The window [t0 + d_min,
 * t0 + d_min + d_max) of possible arrival steps must lie in
 * [t_now, t_now + ring_len); otherwise SD_EINVAL at the call. */
sd_status sd_deliver_spikes(sd_ctx* ctx, const uint32_t* d_src, const uint8_t* d_lag, int64_t n,
                            int64_t t0);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * delivery as sd_deliver_spikes, with the packed list and its count in a
 * fixed device array of the library (2^20 entries, 4 MiB, one copy per GPU,
 * held until the process ends) instead of the context's buffer.  The call
 * allocates and frees nothing.  n above 2^20 (or above the context's list
 * capacity): SD_EINVAL.  All calls on one GPU share that GPU's array, which
 * keeps the last call's contents: calls that overlap on one GPU (different
 * streams or host threads) race on it and must be ordered by the caller. */
sd_status sd_deliver_spikes_noalloc(sd_ctx* ctx, const uint32_t* d_src, const uint8_t* d_lag,
                                    int64_t n, int64_t t0);
/* Deliver the context's own completed slice (its spikes emitted in the last
 * d_min steps); SD_ESTATE when no completed slice is pending. */
sd_status sd_deliver_pending(sd_ctx* ctx);

/* Run round(t_ms / h) steps of the full cycle with fused slice launches
 * (deliver the completed slice, then update the next one).  Resumable:
 * results do not depend on how a run is split into calls. */
sd_status sd_simulate(sd_ctx* ctx, double t_ms);
sd_status sd_simulate_steps(sd_ctx* ctx, int64_t n_steps);

/* Validation mode: deliver 1.0 for every synapse so the ring holds exact
 * per-cell event counts (0 = weights, 1 = counts). */
sd_status sd_set_count_mode(sd_ctx* ctx, int32_t on);

/* Persistent slices (Alg. REF, Sec. 3.2, run for many slices in one
 * launch): sd_simulate / sd_simulate_steps run up to max_slices whole
 * slices per cooperative launch, one workgroup per target block.  Each
 * block keeps its ring window in LDS across the slices (window sums stay in
 * 64-bit fixed point until their step is updated) and its neurons' state in
 * registers; slices are separated by grid barriers.  The results are those
 * of the fused slices up to the FP32 rounding of the ring sums (a sum is
 * rounded once, not once per delivery).  0 switches back to one launch per
 * slice.  SD_EUNSUPPORTED unless the net is block-major, closed loop, with
 * static synapses, blocks of a multiple of 64 and at most 1024 neurons, and
 * all blocks fit on the device at once; SD_ESTATE before
 * sd_build_connections.  A grid barrier that waits past its spin limit sets
 * bit 4 of sd_stats.overflow and ends the launch early (the run's results
 * are then invalid). */
sd_status sd_set_persistent(sd_ctx* ctx, int32_t max_slices);

/* For callers that watch a persistent run (and for tests of its failure
 * path): the most polls a grid barrier of a persistent launch makes while
 * it waits for the other workgroups before it gives up, setting bit 4 of
 * sd_stats.overflow and ending the launch early.  polls < 0 restores the
 * default of 2^22 polls; 0 makes the first workgroup to reach a barrier give
 * up at once.  SD_EINVAL for a null context. */
sd_status sd_set_barrier_spin(sd_ctx* ctx, int64_t polls);

/* Open loop: precompute the virtual sources' spikes for steps
 * [t_now, t_now + n_steps) (outside any timed region). */
sd_status sd_prepare_input(sd_ctx* ctx, int64_t n_steps);

/* --- read-back (synchronising) --------------------------------------------- */
int64_t sd_t_now(const sd_ctx* ctx);
sd_status sd_get_sizes(const sd_ctx* ctx, sd_sizes* out);
sd_status sd_get_stats(sd_ctx* ctx, sd_stats* out);
/* ring rows for steps [t_now, t_now + n_slots) into h_out[n_slots][n_local] */
sd_status sd_read_ring(sd_ctx* ctx, float* h_out, int32_t n_slots);
/* neuron state (any pointer may be NULL) */
sd_status sd_read_state(sd_ctx* ctx, float* h_v, float* h_y1, float* h_y2, int32_t* h_r);
sd_status sd_write_state(sd_ctx* ctx, const float* h_v, const float* h_y1, const float* h_y2,
                         const int32_t* h_r);
/* Checkpoint / resume.  sd_save_state writes the dynamic state (neuron
 * state, ring buffers, the open slice's spikes, step counters and event
 * statistics) into h_buf (cap bytes; h_buf NULL: only *used is set to the
 * size needed).  sd_load_state restores it into a built context of the same
 * configuration (SD_EINVAL otherwise): the connection table is not saved,
 * it is redrawn deterministically by sd_build_connections.  Not saved: the
 * spike raster and an open-loop input schedule (call sd_prepare_input
 * again after loading).  A resumed run gives the same results as an
 * uninterrupted one.  (A service for long runs, not an operation of the
 * method itself.) */
sd_status sd_save_state(sd_ctx* ctx, void* h_buf, size_t cap, size_t* used);
sd_status sd_load_state(sd_ctx* ctx, const void* h_buf, size_t n);
/* drain the raster: (step, neuron) pairs in emission-slice order */
sd_status sd_get_spikes(sd_ctx* ctx, int64_t* h_step, uint32_t* h_id, int64_t cap, int64_t* n);
/* spikes of the open (not yet delivered) slice */
sd_status sd_get_pending(sd_ctx* ctx, uint32_t* h_src, uint8_t* h_lag, int64_t cap, int64_t* n,
                         int64_t* slice_t0);
/* connection table, decoded: h_row[n_src+1] (int64), h_tgt[n_syn],
 * h_dly[n_syn], h_w[n_syn]; each source's synapses in (target, draw)
 * order (block-major layout) or (target, delay, weight) order
 * (source-major layout, which does not keep draw indices) */
sd_status sd_export_connections(sd_ctx* ctx, int64_t* h_row, int32_t* h_tgt, uint8_t* h_dly,
                                float* h_w);
/* where one source's segments sit: for every block b, the index of its first
 * synapse into b and their count (h_start[n_blocks], h_len[n_blocks]);
 * block-major layout only (SD_EUNSUPPORTED otherwise), as is
 * sd_export_block */
sd_status sd_export_segments(sd_ctx* ctx, int64_t src, int64_t* h_start, int64_t* h_len);
/* the synapses into target block b, source by source: h_row[n_src+1] (the
 * offsets of each source's segment in the output), then h_tgt/h_dly/h_w of
 * *n_out synapses (h_tgt == NULL: only h_row and *n_out are written) */
sd_status sd_export_block(sd_ctx* ctx, int32_t b, int64_t* h_row, int32_t* h_tgt, uint8_t* h_dly,
                          float* h_w, int64_t* n_out);
/* host-side tables as used by the device: w_e/w_i[65536] (decoded FP32),
 * thr[64] Poisson thresholds (returns count in *n_thr), prop[7] FP64
 * propagators computed on the device {P11,P21,P22,P31,P32,P33,P30}, and
 * prop32[7] their FP32 roundings used by the update */
sd_status sd_get_tables(sd_ctx* ctx, float* h_we, float* h_wi, uint32_t* h_thr, int32_t* n_thr,
                        double* h_prop, float* h_prop32);
/* the host-side tables alone, without a context or device:
 * w_e/w_i[65536] decoded FP32 weights, thr[64] Poisson thresholds */
sd_status sd_host_tables(const sd_config* cfg, float* h_we, float* h_wi, uint32_t* h_thr,
                         int32_t* n_thr);

/* --- batched networks ------------------------------------------------------
 * Independent networks (a parameter sweep) advanced together.  Each member
 * runs the simulation cycle of Sec. 1 / Sec. 2.1 exactly as a single
 * context does; a slice of all members is one fused launch over the union
 * of their target blocks, so small networks share the device instead of
 * each leaving it mostly idle.  Members are ordinary contexts
 * (sd_batch_member) for read-back; they must share model, weight form, h
 * and d_min, be closed loop, and be advanced only through the batch.
 * Results equal those of each member run alone (the same per-block code,
 * exact integer window sums). */
typedef struct sd_batch sd_batch;

/* Create n members from cfgs[0..n) on the current device, all ordered on
 * hip_stream; each context allocates its own device memory.  On failure
 * *out still holds a batch for sd_batch_last_error / sd_batch_destroy. */
sd_status sd_batch_create(const sd_config* cfgs, int32_t n, void* hip_stream, sd_batch** out);
void sd_batch_destroy(sd_batch* b);
const char* sd_batch_last_error(const sd_batch* b);
int32_t sd_batch_size(const sd_batch* b);
/* member i (borrowed; owned by the batch), or NULL */
sd_ctx* sd_batch_member(sd_batch* b, int32_t i);
/* sd_build_connections on every member */
sd_status sd_batch_build(sd_batch* b);
/* advance every member by n_steps (or round(t_ms / h) steps) */
sd_status sd_batch_simulate_steps(sd_batch* b, int64_t n_steps);
sd_status sd_batch_simulate(sd_batch* b, double t_ms);
/* on != 0: steady-state stretches of at least 12 slices run as replays of a
 * captured HIP graph of 6 batched slices (the slice cycle of Sec. 2.1
 * repeats with the same launches; the spike lists alternate between two
 * buffers and their counters rotate over three, so the arguments of a
 * period equal the previous period's moved on by 6 * d_min steps, which a
 * small kernel at the end of the graph applies on the device).  Results
 * are identical to eager launches.  The graph is captured at first use on
 * a private stream and replayed on the batch's stream. */
sd_status sd_batch_set_graph(sd_batch* b, int32_t on);
/* graph replays issued so far (each runs 6 slices), -1 for NULL */
int64_t sd_batch_graph_launches(const sd_batch* b);

/* --- block-size autotuning -------------------------------------------------
 * Block sizes for n networks (n = 1: one context; n > 1: a batch, whose
 * members must be block-major).  For each target T in targets[0..n_targets)
 * member i gets block_neurons = ceil(N_i / T) rounded up to 64, lowered in
 * steps of 64 until its layout fits; a batch also gets a balanced candidate
 * per T, member i split into round(T * K_i / mean K) blocks (the events per
 * block grow with the in-degree K).  Each candidate is created, built and
 * timed over `slices` slices after `warmup` slices on a private stream of
 * the current device, and the fastest candidate's sizes go to
 * h_block_neurons[0..n), its time per slice (us) to *us_per_slice (may be
 * NULL).  cache_path (may be NULL) names a JSON file of earlier results
 * keyed by device architecture and a hash of the configurations and tuning
 * options: a hit returns the stored sizes without timing, a miss adds the
 * result.  The configurations' own block_neurons are ignored.  Needs the
 * device memory of one candidate at a time.  SD_EUNSUPPORTED: no candidate
 * ran; SD_EINVAL: bad arguments, or the cache file could not be written. */
sd_status sd_autotune(const sd_config* cfgs, int32_t n, const int32_t* targets,
                      int32_t n_targets, int32_t warmup, int32_t slices,
                      const char* cache_path, int32_t* h_block_neurons, double* us_per_slice);

/* Binning parameters of one source-major network: the target block size
 * (the bucket of the binning pass, as above: ceil(N / T) rounded up to 64
 * and lowered until the layout fits, for each T in targets[0..n_targets))
 * and the region capacity bin_cap (each factor of cap_scales[0..n_scales)
 * times the automatic capacity of that block size, rounded up to 64, within
 * [64, 32768 / ... the limit of sd_config.bin_cap]; a smaller region sends
 * more events to the slower spill path, a larger one takes more memory).
 * Every distinct pair is created, built and timed like sd_autotune; the
 * fastest goes to *block_neurons and *bin_cap, its time per slice (us) to
 * *us_per_slice (may be NULL).  cache_path as for sd_autotune (the entry
 * holds both values).  The configuration's own block_neurons and bin_cap
 * are ignored.  SD_EINVAL: bad arguments, a configuration whose layout is
 * not source-major, or the cache file could not be written;
 * SD_EUNSUPPORTED: no candidate ran. */
sd_status sd_autotune_bins(const sd_config* cfg, const int32_t* targets, int32_t n_targets,
                           const double* cap_scales, int32_t n_scales, int32_t warmup,
                           int32_t slices, const char* cache_path, int32_t* block_neurons,
                           int32_t* bin_cap, double* us_per_slice);

#ifdef __cplusplus
}
#endif
#endif
