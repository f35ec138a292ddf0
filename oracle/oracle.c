/*
 * oracle.c -- plain, slow FP64 CPU reference (test infrastructure only).
 *
 * Written for readability, not speed: every loop follows the definition it
 * implements, in the order the paper states the simulation cycle.  Nothing
 * here is shared with the GPU library.
 *
 * Paper passages followed (Pronold et al., arXiv 2109.12855):
 *   Sec. 1 / Sec. 2.1  time-driven grid of resolution h; cycle of update,
 *                      communication and delivery every min-delay interval;
 *                      linear subthreshold dynamics integrated exactly with
 *                      precomputed propagators.
 *   Sec. 2.2           balanced random network with static synapses.
 *   Sec. 3.1           synapses stored with their targets, sorted by source
 *                      into target segments; each neuron owns a spike ring
 *                      buffer that holds inputs until they are due.
 *   Sec. 3.2, Alg. REF for every spike entry, walk its target segment and add
 *                      each synapse's weight into the target's ring buffer at
 *                      the synapse's delay.
 * Readings where the paper is silent (equations, RNG, parameters, slice and
 * arrival conventions) are listed in the repository's design notes.
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static char g_err[256];
static void set_err(const char* m) { snprintf(g_err, sizeof g_err, "%s", m); }
const char* or_last_error(void) { return g_err; }

/* ------------------------------------------------------------------------- */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as    */
/* easy as 1, 2, 3", SC'11): ten rounds of two 64x64->128 multiplications    */
/* with a Weyl-sequence key schedule.                                         */
/* ------------------------------------------------------------------------- */
void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k0 += W0; k1 += W1; }
    unsigned __int128 p0 = (unsigned __int128)M0 * x0;
    unsigned __int128 p1 = (unsigned __int128)M1 * x2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t y0 = hi1 ^ x1 ^ k0;
    uint64_t y1 = lo1;
    uint64_t y2 = hi0 ^ x3 ^ k1;
    uint64_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void philox(uint64_t seed, uint64_t stream, uint64_t c0, uint64_t c1, uint64_t out[4]) {
  uint64_t ctr[4] = {c0, c1, 0, 0}, key[2] = {seed, stream};
  or_philox4x64_10(ctr, key, out);
}

/* floor(r * n / 2^64): an exact integer map of a 64-bit word onto [0, n). */
static uint64_t scale64(uint64_t r, uint64_t n) {
  return (uint64_t)(((unsigned __int128)r * n) >> 64);
}

/* 32-bit uniform for step t from one Philox call per 8 steps (the 256 output
 * bits hold eight 32-bit halves, low half first). */
static uint32_t half32(const uint64_t r[4], int64_t t) {
  uint64_t w = r[(t & 7) >> 1];
  return (t & 1) ? (uint32_t)(w >> 32) : (uint32_t)(w & 0xffffffffu);
}

/* ------------------------------------------------------------------------- */
/* Inverse standard normal CDF, Wichura's algorithm AS 241 (PPND16),          */
/* Applied Statistics 37 (1988) 477-484: rational approximations on the      */
/* central region |p-1/2| <= 0.425 and two tail regions in sqrt(-log r).     */
/* ------------------------------------------------------------------------- */
static double poly8(const double* a, double x) {
  double s = a[7];
  for (int i = 6; i >= 0; --i) s = s * x + a[i];
  return s;
}

double or_ndtri(double p) {
  static const double A[8] = {3.3871328727963666080e0, 1.3314166789178437745e+2,
                              1.9715909503065514427e+3, 1.3731693765509461125e+4,
                              4.5921953931549871457e+4, 6.7265770927008700853e+4,
                              3.3430575583588128105e+4, 2.5090809287301226727e+3};
  static const double B[8] = {1.0, 4.2313330701600911252e+1, 6.8718700749205790830e+2,
                              5.3941960214247511077e+3, 2.1213794301586595867e+4,
                              3.9307895800092710610e+4, 2.8729085735721942674e+4,
                              5.2264952788528545610e+3};
  static const double C[8] = {1.42343711074968357734e0, 4.63033784615654529590e0,
                              5.76949722146069140550e0, 3.64784832476320460504e0,
                              1.27045825245236838258e0, 2.41780725177450611770e-1,
                              2.27238449892691845833e-2, 7.74545014278341407640e-4};
  static const double D[8] = {1.0, 2.05319162663775882187e0, 1.67638483018380384940e0,
                              6.89767334985100004550e-1, 1.48103976427480074590e-1,
                              1.51986665636164571966e-2, 5.47593808499534494600e-4,
                              1.05075007164441684324e-9};
  static const double E[8] = {6.65790464350110377720e0, 5.46378491116411436990e0,
                              1.78482653991729133580e0, 2.96560571828504891230e-1,
                              2.65321895265761230930e-2, 1.24266094738807843860e-3,
                              2.71155556874348757815e-5, 2.01033439929228813265e-7};
  static const double F[8] = {1.0, 5.99832206555887937690e-1, 1.36929880922735805310e-1,
                              1.48753612908506148525e-2, 7.86869131145613259100e-4,
                              1.84631831751005468180e-5, 1.42151175831644588870e-7,
                              2.04426310338993978564e-15};
  double q = p - 0.5;
  if (fabs(q) <= 0.425) {
    double r = 0.180625 - q * q;
    return q * poly8(A, r) / poly8(B, r);
  }
  double r = (q < 0.0) ? p : 1.0 - p;
  r = sqrt(-log(r));
  double v;
  if (r <= 5.0) {
    r -= 1.6;
    v = poly8(C, r) / poly8(D, r);
  } else {
    r -= 5.0;
    v = poly8(E, r) / poly8(F, r);
  }
  return (q < 0.0) ? -v : v;
}

/* Weight of quantile cell i of N(mu, (cv*mu)^2): mu * (1 + cv * z_i) with
 * z_i = Phi^{-1}((i + 1/2) / 2^16), rounded to FP32.  The I table is -g times
 * the same draw (static synapses, Sec. 2.2; distribution from the workload). */
void or_weight_tables(const or_config* c, float* w_e, float* w_i) {
  for (int i = 0; i < 65536; ++i) {
    double z = or_ndtri(((double)i + 0.5) / 65536.0);
    double we = c->w_exc * (1.0 + c->w_cv * z);
    w_e[i] = (float)we;
    w_i[i] = (float)(-c->g * we);
  }
}

/* Thresholds T_k = floor(2^32 F(k)) of the Poisson(lambda) CDF, with
 * F(k) = sum_{i<=k} e^-lambda lambda^i / i!; the drive count of a uniform
 * 32-bit u is #{k : u >= T_k}.  The table stops at the first k whose T_k
 * reaches 2^32 - 1, so the truncated tail has probability below 2^-32. */
int or_poisson_thresholds(double lambda, uint32_t* out, int cap) {
  double p = exp(-lambda), F = p;
  int n = 0;
  for (int k = 0; n < cap; ++k) {
    if (k > 0) { p = p * lambda / (double)k; F += p; }
    double t = floor(F * 4294967296.0);
    if (t >= 4294967295.0) break;
    out[n++] = (uint32_t)t;
  }
  return n;
}

/* Exact propagators of the linear subthreshold dynamics over one step h.
 * delta:  tau_m dV/dt = -(V-E_L) + tau_m I_e / C_m
 * alpha:  dy1/dt = -y1/tau_s, dy2/dt = y1 - y2/tau_s,
 *         dV/dt = -(V-E_L)/tau_m + (y2 + I_e)/C_m
 * out = {P11, P21, P22, P31, P32, P33, P30}; the delta model uses P33, P30. */
void or_propagators(const or_config* c, double out[7]) {
  double h = c->h, tm = c->tau_m, ts = c->tau_syn, C = c->c_m;
  double P33 = exp(-h / tm);
  double P30 = (tm / C) * (-expm1(-h / tm));
  double P11 = 0, P21 = 0, P22 = 0, P31 = 0, P32 = 0;
  if (c->model == OR_ALPHA) {
    double es = exp(-h / ts);
    double a = 1.0 / ts - 1.0 / tm;
    P11 = es;
    P22 = es;
    P21 = h * es;
    /* V response to y2(0)=1: (1/C) int_0^h e^{-(h-s)/tm} e^{-s/ts} ds */
    P32 = (1.0 / C) * (P33 - es) / a;
    /* V response to y1(0)=1: y2(s) = s e^{-s/ts}, giving
     * (1/C) e^{-h/tm} (1 - e^{-x}(1+x)) / a^2 with x = a h; the bracket is
     * formed as -expm1(-x) - x e^{-x} to limit cancellation at small x. */
    double x = a * h;
    P31 = (1.0 / C) * P33 * (-expm1(-x) - x * exp(-x)) / (a * a);
  }
  out[0] = P11; out[1] = P21; out[2] = P22; out[3] = P31;
  out[4] = P32; out[5] = P33; out[6] = P30;
}

int32_t or_ref_steps(const or_config* c) { return (int32_t)llround(c->t_ref / c->h); }

/* round-to-nearest-even FP32 -> BF16, returned as the decoded FP32 value */
float or_bf16_round(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  uint32_t r = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
  float y;
  memcpy(&y, &r, 4);
  return y;
}

/* Decoded value of an FP32 weight in the chosen storage form.
 * BF16: RNE to bfloat16.  BF16 residual: w = mu * (1 + delta) with mu the
 * population's FP32 mean weight and delta = bf16(fp32(w/mu - 1)); the decode
 * is one rounding of mu + mu*delta (exact in FP64 before the rounding). */
float or_decode_weight(const or_config* c, int is_inh, float w32) {
  if (c->wform == OR_W_FP32) return w32;
  if (c->wform == OR_W_BF16) return or_bf16_round(w32);
  float mu = is_inh ? (float)(-c->g * c->w_exc) : (float)c->w_exc;
  float delta = or_bf16_round((float)((double)w32 / (double)mu - 1.0));
  return (float)((double)mu + (double)mu * (double)delta);
}

/* ------------------------------------------------------------------------- */
struct or_net {
  or_config c;
  int64_t n_local;          /* neurons held (tgt_hi - tgt_lo)                  */
  int64_t lo;               /* first held neuron id                           */
  int64_t n_src;
  int64_t n_syn;
  int32_t K;
  /* target-major draws (generation order) */
  uint32_t* tm_src;
  uint8_t* tm_dly;
  uint16_t* tm_widx;
  /* source-major table sorted by (src, target, k) */
  int64_t* row;
  int32_t* tgt;
  uint8_t* dly;
  double* w;
  /* dynamics */
  double P[7];
  uint32_t thr[64];
  int n_thr;
  int32_t ref_steps;
  double *V, *y1, *y2;
  double* vpre;             /* V before the threshold test, last step        */
  int32_t* r;
  double* rb;               /* [L][n_local]                                  */
  uint32_t* cnt;            /* [L][n_local] events per cell                  */
  int64_t t_now;
  /* plastic synapses: every spike step of each held neuron (full record),
   * and each source's latest spike delivered so far */
  int64_t** hist;
  int64_t* hist_n;
  int64_t* hist_cap;
  int64_t* prev_pre;        /* [n_src], -1: none                              */
  int64_t src_e_end;        /* sources below this id are excitatory           */
  /* pending slice: spikes emitted since slice start pend_t0, not delivered */
  int64_t pend_t0;
  int pend_open;
  uint32_t* pend_src;
  uint8_t* pend_lag;
  int64_t pend_n, pend_cap;
};

int64_t or_n_local(const or_net* n) { return n->n_local; }
int64_t or_n_src(const or_net* n) { return n->n_src; }
int64_t or_n_syn(const or_net* n) { return n->n_syn; }
int64_t or_t_now(const or_net* n) { return n->t_now; }

static int open_loop(const or_config* c) { return c->n_src_exc > 0; }

void or_net_destroy(or_net* n) {
  if (!n) return;
  free(n->tm_src); free(n->tm_dly); free(n->tm_widx);
  free(n->row); free(n->tgt); free(n->dly); free(n->w);
  free(n->V); free(n->y1); free(n->y2); free(n->r); free(n->vpre);
  free(n->rb); free(n->cnt); free(n->pend_src); free(n->pend_lag);
  if (n->hist)
    for (int64_t j = 0; j < n->n_local; ++j) free(n->hist[j]);
  free(n->hist); free(n->hist_n); free(n->hist_cap); free(n->prev_pre);
  free(n);
}

or_net* or_net_create(const or_config* cfg) {
  const or_config* c = cfg;
  int64_t N = c->n_exc + c->n_inh;
  if (N <= 0 || c->k_exc < 0 || c->k_inh < 0 || c->d_lo < 1 || c->d_hi < c->d_lo ||
      c->d_min < 1 || c->d_min > c->d_lo || c->d_max < c->d_hi ||
      c->ring_len < c->d_min + c->d_max || c->h <= 0) {
    set_err("invalid config");
    return NULL;
  }
  or_net* n = (or_net*)calloc(1, sizeof(or_net));
  n->c = *c;
  n->lo = c->tgt_lo;
  int64_t hi = c->tgt_hi > 0 ? c->tgt_hi : N;
  if (n->lo < 0 || hi > N || hi <= n->lo) { set_err("invalid target range"); free(n); return NULL; }
  n->n_local = hi - n->lo;
  n->n_src = open_loop(c) ? c->n_src_exc + c->n_src_inh : N;
  int64_t src_e_n = open_loop(c) ? c->n_src_exc : c->n_exc;
  int64_t src_i_n = open_loop(c) ? c->n_src_inh : c->n_inh;
  int64_t src_i_base = src_e_n;
  n->K = c->k_exc + c->k_inh;
  n->n_syn = n->n_local * (int64_t)n->K;

  /* Step 1: draw every connection target-major, (j, k) in order; one Philox
   * call per synapse keyed by (seed, SYN) at counter (j, k). */
  n->tm_src = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n->n_syn ? n->n_syn : 1));
  n->tm_dly = (uint8_t*)malloc((size_t)(n->n_syn ? n->n_syn : 1));
  n->tm_widx = (uint16_t*)malloc(sizeof(uint16_t) * (size_t)(n->n_syn ? n->n_syn : 1));
  uint64_t nd = (uint64_t)(c->d_hi - c->d_lo + 1);
  for (int64_t jl = 0; jl < n->n_local; ++jl) {
    int64_t j = n->lo + jl;
    for (int32_t k = 0; k < n->K; ++k) {
      uint64_t r[4];
      philox(c->seed, OR_STREAM_SYN, (uint64_t)j, (uint64_t)k, r);
      uint64_t s = (k < c->k_exc) ? scale64(r[0], (uint64_t)src_e_n)
                                  : (uint64_t)src_i_base + scale64(r[0], (uint64_t)src_i_n);
      int64_t e = jl * n->K + k;
      n->tm_src[e] = (uint32_t)s;
      n->tm_dly[e] = (uint8_t)(c->d_lo + (int32_t)scale64(r[1], nd));
      n->tm_widx[e] = (uint16_t)(r[2] >> 48);
    }
  }

  /* Step 2: weights as stored, decoded to the oracle's chosen form. */
  float* we = (float*)malloc(sizeof(float) * 65536);
  float* wi = (float*)malloc(sizeof(float) * 65536);
  if (c->w_cv != 0.0) or_weight_tables(c, we, wi);

  /* Step 3: transpose into the source-major table (Sec. 3.1: synapses sorted
   * by source into target segments).  A stable counting sort by source keeps
   * the (target, k) order inside each source's segment. */
  n->row = (int64_t*)calloc((size_t)n->n_src + 1, sizeof(int64_t));
  for (int64_t e = 0; e < n->n_syn; ++e) n->row[n->tm_src[e] + 1] += 1;
  for (int64_t s = 0; s < n->n_src; ++s) n->row[s + 1] += n->row[s];
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n->n_src + 1));
  memcpy(fill, n->row, sizeof(int64_t) * (size_t)(n->n_src + 1));
  n->tgt = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n->n_syn ? n->n_syn : 1));
  n->dly = (uint8_t*)malloc((size_t)(n->n_syn ? n->n_syn : 1));
  n->w = (double*)malloc(sizeof(double) * (size_t)(n->n_syn ? n->n_syn : 1));
  for (int64_t e = 0; e < n->n_syn; ++e) {
    int64_t jl = e / n->K;
    int32_t k = (int32_t)(e % n->K);
    int inh = k >= c->k_exc;
    float w32;
    if (c->w_cv != 0.0) w32 = inh ? wi[n->tm_widx[e]] : we[n->tm_widx[e]];
    else w32 = inh ? (float)(-c->g * c->w_exc) : (float)c->w_exc;
    int64_t pos = fill[n->tm_src[e]]++;
    n->tgt[pos] = (int32_t)(n->lo + jl);
    n->dly[pos] = n->tm_dly[e];
    n->w[pos] = (double)or_decode_weight(c, inh, w32);
  }
  free(fill); free(we); free(wi);

  /* Dynamics tables and initial state. */
  or_propagators(c, n->P);
  n->n_thr = or_poisson_thresholds(c->drive_rate_hz * c->h * 1e-3, n->thr, 64);
  n->ref_steps = or_ref_steps(c);
  size_t nl = (size_t)n->n_local;
  n->V = (double*)malloc(sizeof(double) * nl);
  n->y1 = (double*)calloc(nl, sizeof(double));
  n->y2 = (double*)calloc(nl, sizeof(double));
  n->r = (int32_t*)calloc(nl, sizeof(int32_t));
  n->vpre = (double*)calloc(nl, sizeof(double));
  for (int64_t jl = 0; jl < n->n_local; ++jl) {
    uint64_t r[4];
    philox(c->seed, OR_STREAM_INIT, (uint64_t)(n->lo + jl), 0, r);
    double u = (double)(r[0] >> 11) * 0x1.0p-53;
    n->V[jl] = (double)(float)(c->v0_lo + (c->v0_hi - c->v0_lo) * u);
  }
  n->rb = (double*)calloc((size_t)c->ring_len * nl, sizeof(double));
  n->cnt = (uint32_t*)calloc((size_t)c->ring_len * nl, sizeof(uint32_t));
  n->pend_cap = 1024;
  n->pend_src = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n->pend_cap);
  n->pend_lag = (uint8_t*)malloc((size_t)n->pend_cap);
  n->src_e_end = src_e_n;
  if (c->plastic) {
    n->hist = (int64_t**)calloc(nl, sizeof(int64_t*));
    n->hist_n = (int64_t*)calloc(nl, sizeof(int64_t));
    n->hist_cap = (int64_t*)calloc(nl, sizeof(int64_t));
    n->prev_pre = (int64_t*)malloc(sizeof(int64_t) * (size_t)n->n_src);
    for (int64_t s = 0; s < n->n_src; ++s) n->prev_pre[s] = -1;
  }
  return n;
}

void or_export_target_major(const or_net* n, uint32_t* src, uint8_t* dly, uint16_t* widx) {
  memcpy(src, n->tm_src, sizeof(uint32_t) * (size_t)n->n_syn);
  memcpy(dly, n->tm_dly, (size_t)n->n_syn);
  memcpy(widx, n->tm_widx, sizeof(uint16_t) * (size_t)n->n_syn);
}

void or_export_source_major(const or_net* n, int64_t* row, int32_t* tgt, uint8_t* dly, double* w) {
  memcpy(row, n->row, sizeof(int64_t) * (size_t)(n->n_src + 1));
  memcpy(tgt, n->tgt, sizeof(int32_t) * (size_t)n->n_syn);
  memcpy(dly, n->dly, (size_t)n->n_syn);
  memcpy(w, n->w, sizeof(double) * (size_t)n->n_syn);
}

void or_out_weight(const or_net* n, double* out_w, int64_t* out_deg) {
  for (int64_t s = 0; s < n->n_src; ++s) {
    double acc = 0.0;
    for (int64_t e = n->row[s]; e < n->row[s + 1]; ++e) acc += n->w[e];
    out_w[s] = acc;
    out_deg[s] = n->row[s + 1] - n->row[s];
  }
}

int32_t or_drive_count(const or_net* n, int64_t j, int64_t t) {
  uint64_t r[4];
  philox(n->c.seed, OR_STREAM_DRIVE, (uint64_t)j, (uint64_t)(t >> 3), r);
  uint32_t u = half32(r, t);
  int32_t c = 0;
  for (int k = 0; k < n->n_thr; ++k)
    if (u >= n->thr[k]) c += 1;
  return c;
}

/* Plastic synapses (Sec. 6): the update of an excitatory weight is driven by
 * the presynaptic spike and computed when the spike is delivered, so that the
 * weight the target sees is the updated one.  The whole delay d is taken to
 * lie on the target side: the presynaptic spike of step t_pre meets the
 * synapse at t_pre, a target spike of step t meets it at t + d.  The only
 * target information read is the time of its last spike visible at the
 * synapse, t_last (the latest target spike with t_last + d <= t_pre).  Pairs
 * interact nearest-neighbour style with exponential windows:
 *   potentiation: if that target spike came after the source's previous spike
 *     t_prev (t_last + d > t_prev), it pairs with t_prev:
 *       w += A+ exp(-(t_last + d - t_prev) h / tau+), then w = min(w, w_max);
 *   depression: the current spike pairs with that target spike:
 *       w -= A- exp(-(t_pre - t_last - d) h / tau-), then w = max(w, 0).
 * No visible target spike: no change.  Steps are integers, times t h. */
double or_stdp_update(const or_config* c, double w, int64_t t_pre, int64_t t_prev,
                      int64_t t_last, int32_t d) {
  if (t_last < 0) return w;
  if (t_prev >= 0 && t_last + d > t_prev) {
    w += c->stdp_a_plus * exp(-(double)(t_last + d - t_prev) * c->h / c->stdp_tau_plus);
    if (w > c->stdp_w_max) w = c->stdp_w_max;
  }
  w -= c->stdp_a_minus * exp(-(double)(t_pre - t_last - d) * c->h / c->stdp_tau_minus);
  if (w < 0.0) w = 0.0;
  return w;
}

/* latest recorded spike of held neuron jl at or before step t, or -1 */
static int64_t last_spike_upto(const or_net* n, int64_t jl, int64_t t) {
  for (int64_t i = n->hist_n[jl] - 1; i >= 0; --i)
    if (n->hist[jl][i] <= t) return n->hist[jl][i];
  return -1;
}

void or_read_weights(const or_net* n, double* w) {
  memcpy(w, n->w, sizeof(double) * (size_t)n->n_syn);
}

/* Alg. REF (Sec. 3.2): for each spike entry in the given order, walk the
 * source's target segment and add each weight into the target's ring buffer
 * at arrival step t0 + lag + delay.  Plastic nets first update each
 * excitatory weight (or_stdp_update) and add the updated weight. */
int or_deliver(or_net* n, const uint32_t* src, const uint8_t* lag, int64_t n_spk, int64_t t0,
               double* w_sum, int64_t* n_events) {
  const int64_t L = n->c.ring_len;
  double ws = 0.0;
  int64_t ne = 0;
  for (int64_t i = 0; i < n_spk; ++i) {
    if ((int64_t)src[i] >= n->n_src) { set_err("spike source out of range"); return -1; }
    const int64_t t_pre = t0 + (int64_t)lag[i];
    const int plastic_src = n->c.plastic && (int64_t)src[i] < n->src_e_end;
    for (int64_t e = n->row[src[i]]; e < n->row[src[i] + 1]; ++e) {
      int64_t t_arr = t0 + (int64_t)lag[i] + (int64_t)n->dly[e];
      if (t_arr < n->t_now || t_arr >= n->t_now + L) { set_err("arrival outside ring"); return -1; }
      int64_t cell = (t_arr % L) * n->n_local + ((int64_t)n->tgt[e] - n->lo);
      if (plastic_src) {
        const int64_t jl = (int64_t)n->tgt[e] - n->lo;
        const int64_t t_last = last_spike_upto(n, jl, t_pre - (int64_t)n->dly[e]);
        n->w[e] = or_stdp_update(&n->c, n->w[e], t_pre, n->prev_pre[src[i]], t_last,
                                 (int32_t)n->dly[e]);
      }
      n->rb[cell] += n->w[e];
      n->cnt[cell] += 1;
      ws += n->w[e];
      ne += 1;
    }
    if (n->c.plastic) n->prev_pre[src[i]] = t_pre;
  }
  if (w_sum) *w_sum = ws;
  if (n_events) *n_events = ne;
  return 0;
}

static void pend_push(or_net* n, uint32_t s, uint8_t lag) {
  if (n->pend_n == n->pend_cap) {
    n->pend_cap *= 2;
    n->pend_src = (uint32_t*)realloc(n->pend_src, sizeof(uint32_t) * (size_t)n->pend_cap);
    n->pend_lag = (uint8_t*)realloc(n->pend_lag, (size_t)n->pend_cap);
  }
  n->pend_src[n->pend_n] = s;
  n->pend_lag[n->pend_n] = lag;
  n->pend_n += 1;
}

/* One grid step t for every held neuron (Sec. 2.1: exact propagation on the
 * h grid).  Input arriving at step t is read from the ring and cleared. */
static int64_t update_steps(or_net* n, int64_t m, int to_pending, int64_t* spk_step,
                            uint32_t* spk_id, int64_t cap, int64_t n_out) {
  const or_config* c = &n->c;
  const int64_t L = c->ring_len;
  const double P11 = n->P[0], P21 = n->P[1], P22 = n->P[2], P31 = n->P[3];
  const double P32 = n->P[4], P33 = n->P[5], P30 = n->P[6];
  const double in_scale = (c->model == OR_ALPHA) ? exp(1.0) / c->tau_syn : 1.0;
  for (int64_t s = 0; s < m; ++s) {
    int64_t t = n->t_now;
    for (int64_t jl = 0; jl < n->n_local; ++jl) {
      int64_t cell = (t % L) * n->n_local + jl;
      double in = n->rb[cell];
      n->rb[cell] = 0.0;
      n->cnt[cell] = 0;
      double drive = (double)or_drive_count(n, n->lo + jl, t) * c->drive_w;
      double V = n->V[jl];
      if (c->model == OR_DELTA) {
        /* inputs during refractoriness are discarded */
        if (n->r[jl] > 0) n->r[jl] -= 1;
        else V = c->e_l + P33 * (V - c->e_l) + P30 * c->i_e + in + drive;
      } else {
        double y1 = n->y1[jl], y2 = n->y2[jl];
        if (n->r[jl] == 0) V = c->e_l + P31 * y1 + P32 * y2 + P33 * (V - c->e_l) + P30 * c->i_e;
        else n->r[jl] -= 1;
        n->y2[jl] = P21 * y1 + P22 * y2;
        n->y1[jl] = P11 * y1 + in_scale * (in + drive);
      }
      n->vpre[jl] = V;
      if (V >= c->v_th) {
        V = c->v_reset;
        n->r[jl] = n->ref_steps;
        if (c->plastic) {
          if (n->hist_n[jl] == n->hist_cap[jl]) {
            n->hist_cap[jl] = n->hist_cap[jl] ? 2 * n->hist_cap[jl] : 16;
            n->hist[jl] = (int64_t*)realloc(n->hist[jl], sizeof(int64_t) * (size_t)n->hist_cap[jl]);
          }
          n->hist[jl][n->hist_n[jl]++] = t;
        }
        if (n_out >= 0) {
          if (n_out < cap) {
            if (spk_step) spk_step[n_out] = t;
            if (spk_id) spk_id[n_out] = (uint32_t)(n->lo + jl);
            n_out += 1;
          } else {
            n_out = -1;
          }
        }
        if (to_pending) pend_push(n, (uint32_t)(n->lo + jl), (uint8_t)(t - n->pend_t0));
      }
      n->V[jl] = V;
    }
    n->t_now += 1;
  }
  return n_out;
}

int64_t or_update(or_net* n, int64_t n_steps, int64_t* spk_step, uint32_t* spk_id, int64_t cap) {
  return update_steps(n, n_steps, 0, spk_step, spk_id, cap, 0);
}

/* Open-loop virtual sources [s_lo, s_hi): source s fires at step t when the
 * 32-bit uniform of step t from Philox (seed, SRC) at counter (s, t / 8) lies
 * below floor(2^32 p), p = 1 - exp(-rate h) the probability of a spike in one
 * step.  Spikes of steps [t0, t0 + n_steps) in (lag, src) order. */
int64_t or_open_loop_spikes_range(const or_config* c, int64_t t0, int32_t n_steps, int64_t s_lo,
                                  int64_t s_hi, uint32_t* src, uint8_t* lag, int64_t cap) {
  double p = -expm1(-c->src_rate_hz * c->h * 1e-3);
  uint64_t thr = (uint64_t)floor(p * 4294967296.0);
  int64_t n = 0;
  for (int32_t l = 0; l < n_steps; ++l) {
    int64_t t = t0 + l;
    for (int64_t s = s_lo; s < s_hi; ++s) {
      uint64_t r[4];
      philox(c->seed, OR_STREAM_SRC, (uint64_t)s, (uint64_t)(t >> 3), r);
      if ((uint64_t)half32(r, t) < thr) {
        if (n >= cap) return -1;
        src[n] = (uint32_t)s;
        lag[n] = (uint8_t)l;
        n += 1;
      }
    }
  }
  return n;
}

int64_t or_open_loop_spikes(const or_config* c, int64_t t0, int32_t n_steps, uint32_t* src,
                            uint8_t* lag, int64_t cap) {
  return or_open_loop_spikes_range(c, t0, n_steps, 0, c->n_src_exc + c->n_src_inh, src, lag, cap);
}

/* The simulation cycle (Sec. 1, Sec. 2.1): slices of d_min steps aligned on
 * multiples of d_min.  The spikes of a slice are delivered once the slice is
 * complete, before the next slice is updated; an incomplete slice stays
 * pending across calls, so results do not depend on call boundaries. */
int64_t or_simulate(or_net* n, int64_t n_steps, int64_t* spk_step, uint32_t* spk_id, int64_t cap) {
  const int32_t Dmin = n->c.d_min;
  int64_t n_out = 0;
  int64_t left = n_steps;
  while (left > 0) {
    if (n->pend_open && n->t_now % Dmin == 0) {
      if (open_loop(&n->c)) {
        int64_t ns = n->c.n_src_exc + n->c.n_src_inh;
        int64_t capo = ns * Dmin / 64 + 4096;
        uint32_t* s = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)capo);
        uint8_t* l = (uint8_t*)malloc((size_t)capo);
        int64_t m = or_open_loop_spikes(&n->c, n->pend_t0, Dmin, s, l, capo);
        int rc = (m < 0) ? -1 : or_deliver(n, s, l, m, n->pend_t0, NULL, NULL);
        free(s); free(l);
        if (rc) return -1;
      } else {
        if (or_deliver(n, n->pend_src, n->pend_lag, n->pend_n, n->pend_t0, NULL, NULL)) return -1;
      }
      n->pend_n = 0;
      n->pend_open = 0;
    }
    int64_t in_slice = n->t_now % Dmin;
    if (in_slice == 0) {
      n->pend_t0 = n->t_now;
      n->pend_open = 1;
      n->pend_n = 0;
    }
    int64_t m = Dmin - in_slice;
    if (m > left) m = left;
    n_out = update_steps(n, m, !open_loop(&n->c), spk_step, spk_id, cap, n_out);
    left -= m;
  }
  return n_out;
}

void or_read_rb(const or_net* n, double* out, int64_t n_slots) {
  const int64_t L = n->c.ring_len;
  for (int64_t s = 0; s < n_slots; ++s)
    for (int64_t jl = 0; jl < n->n_local; ++jl)
      out[s * n->n_local + jl] = n->rb[((n->t_now + s) % L) * n->n_local + jl];
}

void or_read_vpre(const or_net* n, double* out) {
  memcpy(out, n->vpre, sizeof(double) * (size_t)n->n_local);
}

void or_read_counts(const or_net* n, uint32_t* out, int64_t n_slots) {
  const int64_t L = n->c.ring_len;
  for (int64_t s = 0; s < n_slots; ++s)
    for (int64_t jl = 0; jl < n->n_local; ++jl)
      out[s * n->n_local + jl] = n->cnt[((n->t_now + s) % L) * n->n_local + jl];
}

void or_read_state(const or_net* n, double* v, double* y1, double* y2, int32_t* r) {
  size_t nl = (size_t)n->n_local;
  if (v) memcpy(v, n->V, nl * sizeof(double));
  if (y1) memcpy(y1, n->y1, nl * sizeof(double));
  if (y2) memcpy(y2, n->y2, nl * sizeof(double));
  if (r) memcpy(r, n->r, nl * sizeof(int32_t));
}

void or_write_state(or_net* n, const double* v, const double* y1, const double* y2,
                    const int32_t* r) {
  size_t nl = (size_t)n->n_local;
  if (v) memcpy(n->V, v, nl * sizeof(double));
  if (y1) memcpy(n->y1, y1, nl * sizeof(double));
  if (y2) memcpy(n->y2, y2, nl * sizeof(double));
  if (r) memcpy(n->r, r, nl * sizeof(int32_t));
}

int64_t or_pending(const or_net* n, uint32_t* src, uint8_t* lag, int64_t cap, int64_t* slice_t0) {
  if (slice_t0) *slice_t0 = n->pend_open ? n->pend_t0 : -1;
  int64_t m = n->pend_n < cap ? n->pend_n : cap;
  if (src) memcpy(src, n->pend_src, sizeof(uint32_t) * (size_t)m);
  if (lag) memcpy(lag, n->pend_lag, (size_t)m);
  return n->pend_n;
}
