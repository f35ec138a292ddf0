/* sd_cpu.c -- multithreaded CPU spike delivery: Alg. REF (Sec. 3.2) and
 * Alg. bwTSRB* (Sec. 4.4) over thread-local synapse tables (Sec. 3.1).
 *
 * Thread t owns targets [lo_t, hi_t) and a source-indexed table of the
 * synapses onto them: row_t[s] .. row_t[s+1] is source s's target segment on
 * this thread, entries (local target, delay, weight).  Every thread walks
 * the whole spike list; the threads touch disjoint ring buffers, so they
 * need no synchronisation besides the join.
 */
#include "../../include/sdcpu.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int64_t lo, hi;  /* targets [lo, hi) */
  int64_t* row;    /* [n_src + 1] */
  uint32_t* tgt;   /* local target index */
  uint8_t* dly;
  double* w;
  double* rb;      /* [hi - lo][stride], ring_len cells used per neuron */
} part;

struct sdc_net {
  int64_t n_src, n_tgt, n_syn;
  int32_t L, T;
  int32_t stride;  /* cells between two neurons' ring buffers (>= L) */
  part* p;
};

static void free_part(part* q) {
  free(q->row);
  free(q->tgt);
  free(q->dly);
  free(q->w);
  free(q->rb);
}

void sdc_destroy(sdc_net* n) {
  if (!n) return;
  for (int t = 0; t < n->T; ++t) free_part(&n->p[t]);
  free(n->p);
  free(n);
}

static sdc_net* new_net(int64_t n_src, int64_t n_tgt, int32_t L, int32_t T) {
  if (n_src < 1 || n_tgt < 1 || L < 2 || T < 1) return NULL;
  if ((int64_t)T > n_tgt) T = (int32_t)n_tgt;
  sdc_net* n = (sdc_net*)calloc(1, sizeof(sdc_net));
  if (!n) return NULL;
  n->n_src = n_src;
  n->n_tgt = n_tgt;
  n->L = L;
  n->T = T;
  n->stride = L;
  n->p = (part*)calloc((size_t)T, sizeof(part));
  if (!n->p) {
    free(n);
    return NULL;
  }
  for (int t = 0; t < T; ++t) {
    n->p[t].lo = n_tgt * t / T;
    n->p[t].hi = n_tgt * (t + 1) / T;
  }
  return n;
}

static int alloc_part(part* q, int64_t n_src, int64_t m, int32_t L) {
  q->row = (int64_t*)calloc((size_t)n_src + 1, sizeof(int64_t));
  q->tgt = (uint32_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(uint32_t));
  q->dly = (uint8_t*)malloc((size_t)(m > 0 ? m : 1));
  q->w = (double*)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
  q->rb = (double*)calloc((size_t)(q->hi - q->lo) * (size_t)L, sizeof(double));  /* stride L */
  return (q->row && q->tgt && q->dly && q->w && q->rb) ? 0 : -1;
}

/* ---- tables from a caller's CSR ------------------------------------- */
typedef struct {
  sdc_net* n;
  int t;
  const int64_t* row;
  const int32_t* tgt;
  const uint8_t* dly;
  const double* w;
  int rc;
} csr_job;

static void* csr_worker(void* arg) {
  csr_job* j = (csr_job*)arg;
  sdc_net* n = j->n;
  part* q = &n->p[j->t];
  int64_t m = 0;
  for (int64_t e = 0; e < j->row[n->n_src]; ++e)
    if (j->tgt[e] >= q->lo && j->tgt[e] < q->hi) ++m;
  if (alloc_part(q, n->n_src, m, n->L)) {
    j->rc = -1;
    return NULL;
  }
  int64_t at = 0;
  for (int64_t s = 0; s < n->n_src; ++s) {
    q->row[s] = at;
    for (int64_t e = j->row[s]; e < j->row[s + 1]; ++e) {
      if (j->tgt[e] < q->lo || j->tgt[e] >= q->hi) continue;
      q->tgt[at] = (uint32_t)(j->tgt[e] - q->lo);
      q->dly[at] = j->dly[e];
      q->w[at] = j->w[e];
      ++at;
    }
  }
  q->row[n->n_src] = at;
  j->rc = 0;
  return NULL;
}

static int run_jobs(int T, void* jobs, size_t job_size, void* (*fn)(void*)) {
  pthread_t* th = (pthread_t*)malloc((size_t)T * sizeof(pthread_t));
  if (!th) return -1;
  int started = 0, rc = 0;
  for (int t = 0; t < T; ++t) {
    if (pthread_create(&th[t], NULL, fn, (char*)jobs + (size_t)t * job_size) != 0) {
      rc = -1;
      break;
    }
    ++started;
  }
  for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
  free(th);
  return rc;
}

sdc_net* sdc_create_from_csr(int64_t n_src, int64_t n_tgt, const int64_t* row,
                             const int32_t* tgt, const uint8_t* dly, const double* w,
                             int32_t ring_len, int32_t n_threads) {
  if (!row || !tgt || !dly || !w) return NULL;
  if (n_src < 1 || row[0] != 0) return NULL;
  for (int64_t s = 0; s < n_src; ++s)
    if (row[s + 1] < row[s]) return NULL;  /* offsets must not decrease */
  sdc_net* n = new_net(n_src, n_tgt, ring_len, n_threads);
  if (!n) return NULL;
  for (int64_t e = 0; e < row[n_src]; ++e)
    if (tgt[e] < 0 || tgt[e] >= n_tgt || dly[e] < 1 || dly[e] >= ring_len) {
      sdc_destroy(n);
      return NULL;
    }
  csr_job* jobs = (csr_job*)calloc((size_t)n->T, sizeof(csr_job));
  if (!jobs) {
    sdc_destroy(n);
    return NULL;
  }
  for (int t = 0; t < n->T; ++t) {
    csr_job c = {n, t, row, tgt, dly, w, -1};
    jobs[t] = c;
  }
  int rc = run_jobs(n->T, jobs, sizeof(csr_job), csr_worker);
  for (int t = 0; t < n->T; ++t) rc |= jobs[t].rc;
  free(jobs);
  if (rc) {
    sdc_destroy(n);
    return NULL;
  }
  n->n_syn = row[n_src];
  return n;
}

/* ---- tables of a drawn network ---------------------------------------- */
/* splitmix64 finaliser over a combined key: a counter-based hash, so the
 * two passes below draw the same synapses without storing them */
static inline uint64_t mix(uint64_t x) {
  x += 0x9e3779b97f4a7c15ULL;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ULL;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebULL;
  return x ^ (x >> 31);
}

typedef struct {
  sdc_net* n;
  int t;
  int64_t n_exc;
  int32_t k_exc, k_inh, d_lo, d_hi;
  double w_exc, g;
  uint64_t seed;
  int rc;
} gen_job;

static inline void draw(const gen_job* j, int64_t tg, int32_t k, uint32_t* src, uint8_t* d,
                        double* w) {
  const uint64_t h = mix(j->seed ^ mix(((uint64_t)tg << 20) ^ (uint64_t)k));
  const uint64_t h2 = mix(h);
  const int64_t n_inh = j->n->n_src - j->n_exc;
  const int exc = k < j->k_exc;
  *src = exc ? (uint32_t)((h >> 11) % (uint64_t)j->n_exc)
             : (uint32_t)(j->n_exc + (int64_t)((h >> 11) % (uint64_t)n_inh));
  *d = (uint8_t)(j->d_lo + (int)(h2 % (uint64_t)(j->d_hi - j->d_lo + 1)));
  const double spread = 0.9 + 0.2 * (double)(h2 >> 11) * (1.0 / 9007199254740992.0);
  *w = (exc ? j->w_exc : -j->g * j->w_exc) * spread;
}

static void* gen_worker(void* arg) {
  gen_job* j = (gen_job*)arg;
  sdc_net* n = j->n;
  part* q = &n->p[j->t];
  const int32_t K = j->k_exc + j->k_inh;
  const int64_t m = (q->hi - q->lo) * (int64_t)K;
  if (alloc_part(q, n->n_src, m, n->L)) {
    j->rc = -1;
    return NULL;
  }
  uint32_t s;
  uint8_t d;
  double w;
  for (int64_t tg = q->lo; tg < q->hi; ++tg)
    for (int32_t k = 0; k < K; ++k) {
      draw(j, tg, k, &s, &d, &w);
      q->row[s + 1] += 1;
    }
  for (int64_t i = 0; i < n->n_src; ++i) q->row[i + 1] += q->row[i];
  int64_t* fill = (int64_t*)malloc((size_t)n->n_src * sizeof(int64_t));
  if (!fill) {
    j->rc = -1;
    return NULL;
  }
  memcpy(fill, q->row, (size_t)n->n_src * sizeof(int64_t));
  for (int64_t tg = q->lo; tg < q->hi; ++tg)
    for (int32_t k = 0; k < K; ++k) {
      draw(j, tg, k, &s, &d, &w);
      const int64_t at = fill[s]++;
      q->tgt[at] = (uint32_t)(tg - q->lo);
      q->dly[at] = d;
      q->w[at] = w;
    }
  free(fill);
  j->rc = 0;
  return NULL;
}

sdc_net* sdc_generate(int64_t n_tgt, int64_t n_src_exc, int64_t n_src_inh, int32_t k_exc,
                      int32_t k_inh, int32_t d_lo, int32_t d_hi, double w_exc, double g,
                      uint64_t seed, int32_t ring_len, int32_t n_threads) {
  if (n_src_exc < 1 || n_src_inh < 1 || k_exc < 0 || k_inh < 0 || d_lo < 1 || d_hi < d_lo ||
      d_hi >= ring_len || d_hi > 255 || n_tgt >= ((int64_t)1 << 32))
    return NULL;
  sdc_net* n = new_net(n_src_exc + n_src_inh, n_tgt, ring_len, n_threads);
  if (!n) return NULL;
  gen_job* jobs = (gen_job*)calloc((size_t)n->T, sizeof(gen_job));
  if (!jobs) {
    sdc_destroy(n);
    return NULL;
  }
  for (int t = 0; t < n->T; ++t) {
    gen_job c = {n, t, n_src_exc, k_exc, k_inh, d_lo, d_hi, w_exc, g, seed, -1};
    jobs[t] = c;
  }
  int rc = run_jobs(n->T, jobs, sizeof(gen_job), gen_worker);
  for (int t = 0; t < n->T; ++t) rc |= jobs[t].rc;
  free(jobs);
  if (rc) {
    sdc_destroy(n);
    return NULL;
  }
  n->n_syn = n_tgt * (int64_t)(k_exc + k_inh);
  return n;
}

/* ---- delivery ---------------------------------------------------------- */
typedef struct {
  sdc_net* n;
  int t;
  const uint32_t* src;
  const uint8_t* lag;
  int64_t n_spk, t0;
  int32_t alg, b_ts, b_rb;
  int64_t events;
} del_job;

/* Alg. REF: every spike entry in list order, its target segment synapse by
 * synapse, each weight added into the target's ring buffer at once. */
static int64_t deliver_ref(part* q, int32_t L, int64_t S, const del_job* j) {
  int64_t ev = 0;
  for (int64_t i = 0; i < j->n_spk; ++i) {
    const uint32_t s = j->src[i];
    const int base = (int)((j->t0 + j->lag[i]) % L);
    for (int64_t e = q->row[s]; e < q->row[s + 1]; ++e) {
      int slot = base + q->dly[e];
      if (slot >= L) slot -= L;
      q->rb[(int64_t)q->tgt[e] * S + slot] += q->w[e];
    }
    ev += q->row[s + 1] - q->row[s];
  }
  return ev;
}

/* Alg. bwTSRB* (Sec. 4.4), restated: spike entries are taken b_ts at a time,
 * and the bounds of all their target segments are read before any synapse
 * (hiding the latency of the segment lookups).  The batch's synapses are
 * then visited as one flat sequence across segment boundaries and staged as
 * (ring-buffer cell, weight) pairs; every b_rb pairs, the cells are
 * prefetched together and the weights added in staging order.  Per cell the
 * additions happen in the same order as in REF, so the sums are bitwise
 * equal. */
typedef struct {
  int64_t first[SDC_MAX_BATCH], len[SDC_MAX_BATCH];  /* segment of each entry   */
  int ring_base[SDC_MAX_BATCH];                      /* emission slot of each   */
  int n;
} spike_batch;

/* position in the flat synapse sequence of a spike batch */
typedef struct {
  const spike_batch* sb;
  int seg;
  int64_t next;
} flat_cursor;

static int flat_next(flat_cursor* fc, int64_t* syn, int* ring_base) {
  const spike_batch* sb = fc->sb;
  while (fc->seg < sb->n && fc->next >= sb->first[fc->seg] + sb->len[fc->seg]) {
    if (++fc->seg < sb->n) fc->next = sb->first[fc->seg];
  }
  if (fc->seg >= sb->n) return 0;
  *syn = fc->next++;
  *ring_base = sb->ring_base[fc->seg];
  return 1;
}

typedef struct {
  double* cell[SDC_MAX_BATCH];
  double add[SDC_MAX_BATCH];
  int used, cap;
} rb_stage;

static void stage_flush(rb_stage* st, int prefetch) {
  if (prefetch)
    for (int r = 0; r < st->used; ++r) __builtin_prefetch(st->cell[r], 1, 3);
  for (int r = 0; r < st->used; ++r) *st->cell[r] += st->add[r];
  st->used = 0;
}

static void stage_put(rb_stage* st, double* cell, double w) {
  st->cell[st->used] = cell;
  st->add[st->used] = w;
  if (++st->used == st->cap) stage_flush(st, 1);
}

static int64_t deliver_bwtsrb(part* q, int32_t L, int64_t S, const del_job* j) {
  rb_stage st;
  st.used = 0;
  st.cap = j->b_rb;
  int64_t ev = 0;
  int64_t at = 0;
  while (at < j->n_spk) {
    spike_batch sb;
    sb.n = 0;
    for (; sb.n < j->b_ts && at < j->n_spk; ++sb.n, ++at) {
      const uint32_t s = j->src[at];
      sb.first[sb.n] = q->row[s];
      sb.len[sb.n] = q->row[s + 1] - q->row[s];
      sb.ring_base[sb.n] = (int)((j->t0 + j->lag[at]) % L);
      ev += sb.len[sb.n];
    }
    flat_cursor fc = {&sb, 0, sb.n ? sb.first[0] : 0};
    int64_t e;
    int rb0;
    while (flat_next(&fc, &e, &rb0)) {
      int slot = rb0 + q->dly[e];
      if (slot >= L) slot -= L;
      stage_put(&st, &q->rb[(int64_t)q->tgt[e] * S + slot], q->w[e]);
    }
  }
  stage_flush(&st, 0);  /* pairs still staged at the end */
  return ev;
}

static void* del_worker(void* arg) {
  del_job* j = (del_job*)arg;
  part* q = &j->n->p[j->t];
  const sdc_net* n = j->n;
  j->events = j->alg == SDC_REF ? deliver_ref(q, n->L, n->stride, j)
                                 : deliver_bwtsrb(q, n->L, n->stride, j);
  return NULL;
}

int64_t sdc_deliver(sdc_net* n, const uint32_t* src, const uint8_t* lag, int64_t n_spk, int64_t t0,
                    int32_t alg, int32_t b_ts, int32_t b_rb) {
  if (!n || n_spk < 0 || (n_spk > 0 && (!src || !lag)) || t0 < 0) return -1;
  if (alg != SDC_REF && alg != SDC_BWTSRB) return -1;
  if (alg == SDC_BWTSRB && (b_ts < 1 || b_ts > SDC_MAX_BATCH || b_rb < 1 || b_rb > SDC_MAX_BATCH))
    return -1;
  for (int64_t i = 0; i < n_spk; ++i)
    if ((int64_t)src[i] >= n->n_src || (int)lag[i] >= n->L) return -1;
  del_job* jobs = (del_job*)calloc((size_t)n->T, sizeof(del_job));
  if (!jobs) return -1;
  for (int t = 0; t < n->T; ++t) {
    del_job c = {n, t, src, lag, n_spk, t0, alg, b_ts, b_rb, 0};
    jobs[t] = c;
  }
  int64_t ev = -1;
  if (run_jobs(n->T, jobs, sizeof(del_job), del_worker) == 0) {
    ev = 0;
    for (int t = 0; t < n->T; ++t) ev += jobs[t].events;
  }
  free(jobs);
  return ev;
}

int sdc_read_ring(const sdc_net* n, double* out) {
  if (!n || !out) return -1;
  for (int t = 0; t < n->T; ++t) {
    const part* q = &n->p[t];
    for (int64_t j = q->lo; j < q->hi; ++j)
      for (int32_t s = 0; s < n->L; ++s)
        out[(int64_t)s * n->n_tgt + j] = q->rb[(j - q->lo) * n->stride + s];
  }
  return 0;
}

void sdc_clear(sdc_net* n) {
  if (!n) return;
  for (int t = 0; t < n->T; ++t)
    memset(n->p[t].rb, 0, (size_t)(n->p[t].hi - n->p[t].lo) * (size_t)n->stride * sizeof(double));
}

int sdc_set_ring_stride(sdc_net* n, int32_t stride) {
  if (!n || stride < n->L) return -1;
  double** fresh = (double**)calloc((size_t)n->T, sizeof(double*));
  if (!fresh) return -1;
  for (int t = 0; t < n->T; ++t) {
    fresh[t] = (double*)calloc((size_t)(n->p[t].hi - n->p[t].lo) * (size_t)stride, sizeof(double));
    if (!fresh[t]) {
      for (int u = 0; u <= t; ++u) free(fresh[u]);
      free(fresh);
      return -1;
    }
  }
  for (int t = 0; t < n->T; ++t) {
    free(n->p[t].rb);
    n->p[t].rb = fresh[t];
  }
  free(fresh);
  n->stride = stride;
  return 0;
}

int64_t sdc_n_synapses(const sdc_net* n) { return n ? n->n_syn : -1; }
int32_t sdc_n_threads(const sdc_net* n) { return n ? n->T : -1; }
