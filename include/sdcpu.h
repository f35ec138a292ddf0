/* sdcpu.h -- multithreaded CPU spike delivery with the paper's algorithms.
 *
 * A host comparator for the GPU path: the reference delivery algorithm
 * (Alg. REF, Sec. 3.2) and its batched form with target-segment batches of
 * B_TS spike entries, synapse/ring-buffer batches of B_RB and group prefetch
 * of the ring buffers (Alg. bwTSRB*, Sec. 4.4), run by a pool of threads
 * that each own a contiguous range of target neurons with their own
 * source-indexed synapse table (the thread-local layout of Sec. 3.1).  Ring
 * buffers are FP64, one array of ring_len cells per neuron.
 *
 * Both algorithms add every weight of a cell in the same order (spike entries
 * in list order, a segment's synapses in table order), so their rings are
 * bitwise equal, for any thread count and batch sizes.
 *
 * Errors: functions returning int give 0 on success, -1 on invalid
 * arguments (the handle is left unchanged).  Memory is owned by the handle.
 */
#ifndef SDCPU_H
#define SDCPU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sdc_net sdc_net;

enum { SDC_REF = 0, SDC_BWTSRB = 1 };
#define SDC_MAX_BATCH 256

/* Tables from a source-major CSR over all targets (Sec. 3.1): row[n_src+1]
 * (int64 offsets), tgt[e] in [0, n_tgt), dly[e] in [1, ring_len), w[e].
 * Targets are split into n_threads contiguous ranges; each thread keeps the
 * synapses of its targets in the input order.  The arrays are copied.
 * Returns NULL for offsets that do not start at 0 or decrease, targets or
 * delays out of range, or out of memory. */
sdc_net* sdc_create_from_csr(int64_t n_src, int64_t n_tgt, const int64_t* row,
                             const int32_t* tgt, const uint8_t* dly, const double* w,
                             int32_t ring_len, int32_t n_threads);

/* Tables of a random network drawn in place (a benchmark workload): every
 * target draws k_exc sources from [0, n_src_exc) and k_inh from
 * [n_src_exc, n_src), uniform with replacement, delays uniform in
 * [d_lo, d_hi], weights w_exc or -g * w_exc with a +-10% spread, from a
 * counter-based hash of (seed, target, k).  Per-thread tables are built by
 * the threads themselves. */
sdc_net* sdc_generate(int64_t n_tgt, int64_t n_src_exc, int64_t n_src_inh, int32_t k_exc,
                      int32_t k_inh, int32_t d_lo, int32_t d_hi, double w_exc, double g,
                      uint64_t seed, int32_t ring_len, int32_t n_threads);

/* Deliver n spike entries (src[i], lag[i]) at slice start t0: every synapse
 * (s -> j, d, w) of a spiking source adds w to cell (t0 + lag + d) mod
 * ring_len of j.  alg: SDC_REF or SDC_BWTSRB (b_ts, b_rb in [1,
 * SDC_MAX_BATCH]; ignored for REF).  Returns the number of synaptic events,
 * or -1. */
int64_t sdc_deliver(sdc_net* net, const uint32_t* src, const uint8_t* lag, int64_t n, int64_t t0,
                    int32_t alg, int32_t b_ts, int32_t b_rb);

/* Ring buffers out as [ring_len][n_tgt] (slot-major, like the GPU ring). */
int sdc_read_ring(const sdc_net* net, double* out);
/* Zero every ring buffer. */
void sdc_clear(sdc_net* net);
/* Place neuron j's ring buffer at cell j * stride of its thread's array
 * (stride >= ring_len; ring_len by default, the rings packed back to back).
 * A larger stride stands for ring buffers held inside larger neuron objects,
 * as in the simulator the paper studies: fewer of them share a cache line
 * or fit in the caches.  The rings are reallocated and zeroed. */
int sdc_set_ring_stride(sdc_net* net, int32_t stride);
int64_t sdc_n_synapses(const sdc_net* net);
int32_t sdc_n_threads(const sdc_net* net);
void sdc_destroy(sdc_net* net);

#ifdef __cplusplus
}
#endif
#endif
