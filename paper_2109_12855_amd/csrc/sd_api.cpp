// sd_api.cpp -- host side of the spike-delivery library (C ABI in
// include/sdeliver.h): configuration checks, device arena, host tables,
// the slice state machine and read-back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "sd_internal.h"

using namespace sd;

// ---------------------------------------------------------------------------
// host tables
// ---------------------------------------------------------------------------
namespace {

// Inverse normal CDF by Wichura's AS 241 (PPND16, Appl. Statist. 37, 1988):
// a degree-7/7 rational function in r = 0.180625 - q^2 for |q| <= 0.425
// and in s = sqrt(-log(min(p, 1-p))) shifted by 1.6 (s <= 5) or 5 beyond.
struct Rational77 {
  double num[8];
  double den[8];  // den[0] == 1
  double eval(double x) const {
    double n = 0.0, d = 0.0;
    for (int i = 7; i >= 0; --i) {
      n = n * x + num[i];
      d = d * x + den[i];
    }
    return n / d;
  }
};

constexpr Rational77 kCentral = {
    {3.3871328727963666080e0, 1.3314166789178437745e+2, 1.9715909503065514427e+3,
     1.3731693765509461125e+4, 4.5921953931549871457e+4, 6.7265770927008700853e+4,
     3.3430575583588128105e+4, 2.5090809287301226727e+3},
    {1.0, 4.2313330701600911252e+1, 6.8718700749205790830e+2, 5.3941960214247511077e+3,
     2.1213794301586595867e+4, 3.9307895800092710610e+4, 2.8729085735721942674e+4,
     5.2264952788528545610e+3}};
constexpr Rational77 kNear = {
    {1.42343711074968357734e0, 4.63033784615654529590e0, 5.76949722146069140550e0,
     3.64784832476320460504e0, 1.27045825245236838258e0, 2.41780725177450611770e-1,
     2.27238449892691845833e-2, 7.74545014278341407640e-4},
    {1.0, 2.05319162663775882187e0, 1.67638483018380384940e0, 6.89767334985100004550e-1,
     1.48103976427480074590e-1, 1.51986665636164571966e-2, 5.47593808499534494600e-4,
     1.05075007164441684324e-9}};
constexpr Rational77 kFar = {
    {6.65790464350110377720e0, 5.46378491116411436990e0, 1.78482653991729133580e0,
     2.96560571828504891230e-1, 2.65321895265761230930e-2, 1.24266094738807843860e-3,
     2.71155556874348757815e-5, 2.01033439929228813265e-7},
    {1.0, 5.99832206555887937690e-1, 1.36929880922735805310e-1, 1.48753612908506148525e-2,
     7.86869131145613259100e-4, 1.84631831751005468180e-5, 1.42151175831644588870e-7,
     2.04426310338993978564e-15}};

double inv_normal_cdf(double p) {
  const double q = p - 0.5;
  if (std::fabs(q) <= 0.425) return q * kCentral.eval(0.180625 - q * q);
  const double tail = q < 0.0 ? p : 1.0 - p;
  const double s = std::sqrt(-std::log(tail));
  const double v = s <= 5.0 ? kNear.eval(s - 1.6) : kFar.eval(s - 5.0);
  return q < 0.0 ? -v : v;
}

uint16_t bf16_bits_rne(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  const uint32_t rounded = u + 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(rounded >> 16);
}

// residual BF16 code of an FP32 weight: d = bf16(fp32(w / mu - 1))
uint16_t resid_bits(float w, float mu) {
  return bf16_bits_rne((float)((double)w / (double)mu - 1.0));
}

// Poisson(lambda) CDF thresholds scaled to 2^32 (floor), truncated where the
// scaled CDF reaches 2^32 - 1.
int poisson_table(double lambda, uint32_t* out, int cap) {
  int n = 0;
  double term = std::exp(-lambda);
  double cdf = term;
  for (int k = 0; n < cap; ++k) {
    if (k > 0) {
      term *= lambda / k;
      cdf += term;
    }
    const double scaled = std::floor(cdf * 4294967296.0);
    if (scaled >= 4294967295.0) break;
    out[n++] = (uint32_t)scaled;
  }
  return n;
}

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// FP32 weight of quantile cell i: mu (1 + cv z_i), z_i = Phi^-1((i + 1/2) / 2^16);
// the inhibitory table is -g times the same draw.
void quantile_weights(const sd_config& g, float* we, float* wi) {
  for (int i = 0; i < 65536; ++i) {
    const double z = inv_normal_cdf((i + 0.5) / 65536.0);
    const double w = g.w_exc * (1.0 + g.w_cv * z);
    we[i] = (float)w;
    wi[i] = (float)(-g.g * w);
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
namespace {

// Per-slice kernel arguments live in device memory (the kernel then loads
// fields where it uses them instead of holding the whole struct in scalar
// registers).  They are uploaded in chunks through a pinned double buffer:
// a chunk's copy and then its launches go onto the stream; the host reuses
// a half of the staging buffer only after that half's copy has completed.
struct SliceLauncher {
  int per = 1;                  // argument structs per slice (member networks)
  int cap = 0;                  // slices per chunk
  sd::SliceArgs* d_args = nullptr;  // [2][cap][per]
  sd::SliceArgs* h_args = nullptr;  // pinned staging, same shape
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool pend[2] = {false, false};
  int half = 0;
  int2* d_map = nullptr;        // workgroup -> (network, block)
  int32_t n_blocks = 0;
  int32_t single_nb = 0;        // one network: launched by value (map unused)
  size_t lds = 0;
  int wform = 0;
};

// XCD-aware workgroup map: entry list[i] goes to workgroup
// (i % per_xcd) * 8 + i / per_xcd, so consecutive entries share an XCD.
std::vector<int2> xcd_map(const std::vector<int2>& list) {
  const int64_t T = (int64_t)list.size();
  const int64_t per_xcd = (T + 7) / 8;
  std::vector<int2> map((size_t)(8 * per_xcd), make_int2(-1, 0));
  for (int64_t gx = 0; gx < 8 * per_xcd; ++gx) {
    const int64_t i = (gx & 7) * per_xcd + (gx >> 3);
    if (i < T) map[(size_t)gx] = list[(size_t)i];
  }
  return map;
}

hipError_t launcher_init(SliceLauncher& L, int per, int cap, const std::vector<int2>& map,
                         size_t lds, int wform) {
  L.per = per;
  L.cap = cap;
  L.lds = lds;
  L.wform = wform;
  L.n_blocks = (int32_t)map.size();
  const size_t nb = (size_t)2 * cap * per * sizeof(sd::SliceArgs);
  hipError_t e = hipMalloc((void**)&L.d_args, nb);
  if (e == hipSuccess) e = hipHostMalloc((void**)&L.h_args, nb, hipHostMallocDefault);
  if (e == hipSuccess) e = hipMalloc((void**)&L.d_map, map.size() * sizeof(int2));
  if (e == hipSuccess)
    e = hipMemcpy(L.d_map, map.data(), map.size() * sizeof(int2), hipMemcpyHostToDevice);
  for (int h = 0; h < 2 && e == hipSuccess; ++h) e = hipEventCreateWithFlags(&L.ev[h], hipEventDisableTiming);
  return e;
}

void launcher_free(SliceLauncher& L) {
  for (int h = 0; h < 2; ++h)
    if (L.ev[h]) (void)hipEventDestroy(L.ev[h]);
  if (L.d_args) (void)hipFree(L.d_args);
  if (L.h_args) (void)hipHostFree(L.h_args);
  if (L.d_map) (void)hipFree(L.d_map);
  L = SliceLauncher();
}

// Launch n_slices fused slices whose arguments are list[k * per + i].
hipError_t launcher_run(SliceLauncher& L, hipStream_t s, const sd::SliceArgs* list,
                        int64_t n_slices) {
  if (L.single_nb > 0) {  // one network: arguments by value, nothing to upload
    for (int64_t k = 0; k < n_slices; ++k) {
      const hipError_t e = sd::launch_slice1(s, list[k], L.lds, L.wform);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  for (int64_t k0 = 0; k0 < n_slices; k0 += L.cap) {
    const int64_t k = std::min<int64_t>(L.cap, n_slices - k0);
    const int h = L.half;
    if (L.pend[h]) {
      hipError_t e = hipEventSynchronize(L.ev[h]);
      if (e != hipSuccess) return e;
    }
    sd::SliceArgs* hs = L.h_args + (size_t)h * L.cap * L.per;
    sd::SliceArgs* ds = L.d_args + (size_t)h * L.cap * L.per;
    std::memcpy(hs, list + k0 * L.per, (size_t)k * L.per * sizeof(sd::SliceArgs));
    hipError_t e = hipMemcpyAsync(ds, hs, (size_t)k * L.per * sizeof(sd::SliceArgs),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(L.ev[h], s);
    if (e != hipSuccess) return e;
    L.pend[h] = true;
    for (int64_t i = 0; i < k; ++i) {
      e = sd::launch_slice(s, ds + i * L.per, L.d_map, L.n_blocks, L.lds, L.wform);
      if (e != hipSuccess) return e;
    }
    L.half ^= 1;
  }
  return hipSuccess;
}

}  // namespace

struct sd_ctx {
  sd_config cfg;
  sd_sizes sz;
  hipStream_t stream = nullptr;
  int device = 0;
  bool own_arena = false;
  char* arena = nullptr;
  std::string err;
  // geometry
  int64_t N = 0, n_src = 0, n_syn = 0, src_e_end = 0;
  int32_t B = 0, NB = 0, K = 0, grid_per_xcd = 0;
  int64_t list_cap = 0;  // entries of a slice's spike list
  int64_t M = 0;  // entries of the segment-pointer table
  // device buffers
  uint32_t* row = nullptr;      // block-major segment starts
  uint32_t* cursor = nullptr;
  uint2* seg = nullptr;         // source-major (start, count) pairs
  // source-major layout
  bool sm = false;
  unsigned long long* row64 = nullptr;   // segment starts per source
  unsigned long long* cursor64 = nullptr;
  unsigned long long* tiles64 = nullptr;
  uint32_t* tw = nullptr;                // record words (offset | delay | weight high byte)
  void* wbits = nullptr;                 // weights (u8 low bytes or f32)
  int32_t tbits = 0, H = 1;              // target parts of 2^tbits, H of them
  void* bins = nullptr;                  // binned records [NB][bin_P][bin_cap]
  uint32_t* bin_cnt = nullptr;           // records per region [NB][bin_P]
  long long* spill = nullptr;            // full regions' events [d_max][N]
  int32_t* spill_flag = nullptr;         // [NB]
  int32_t bin_P = 0, bin_cap = 0, bin_U = 0;
  size_t bin_lds = 0;
  uint32_t* tile_sums = nullptr;
  int64_t n_tiles = 0;
  void* syn = nullptr;          // synapse records
  uint8_t* syn_dly = nullptr;   // delays (not used by the packed form)
  float *V = nullptr, *y1 = nullptr, *y2 = nullptr;
  int32_t* r = nullptr;
  float* rb = nullptr;
  uint32_t* list[2] = {nullptr, nullptr};
  // plastic synapses: spike history per neuron, lag mask and previous spike
  // per list entry (both lists)
  uint64_t* pmask = nullptr;
  int32_t* pbefore = nullptr;
  uint32_t* aux[2] = {nullptr, nullptr};
  int32_t* prev[2] = {nullptr, nullptr};
  uint32_t* ext_list = nullptr;  // packed external spike list (list_cap entries)
  int32_t* ext_cnt = nullptr;    // its entry count (device)
  // list counters rotate over three words: the open slice's (ci), the next
  // one (always zero between calls) and the one before (cleared by the next
  // fused launch)
  int32_t* cnt3 = nullptr;
  int ci = 0;
  uint2* rec = nullptr;
  int64_t rec_cap = 0;
  void* wtab_e = nullptr;
  void* wtab_i = nullptr;
  uint32_t* thr = nullptr;
  double* prop64 = nullptr;
  float* prop32 = nullptr;
  float prop_h[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // host copy, passed by value to the slices
  unsigned long long* counters = nullptr;  // ev, spk_in, spk, rec_n
  int32_t* overflow = nullptr;
  // open-loop input schedule
  uint32_t* in_list = nullptr;
  int64_t* in_off = nullptr;     // device, per slice
  int32_t* in_cnt = nullptr;     // device, per slice
  std::vector<int64_t> in_off_h;
  int64_t in_t0 = 0, in_slices = 0;
  // host copies of tables
  std::vector<float> we_h, wi_h;
  uint32_t thr_h[kMaxThr];
  int32_t n_thr = 0;
  float mu_e = 0.f, mu_i = 0.f;
  int32_t ref_steps = 0;
  int32_t fx_shift = 0;     // ring window quantum is 2^-fx_shift
  // state machine
  bool built = false;
  int64_t t_now = 0;
  int64_t rb_hi = 0;
  bool pend_open = false;   // a slice has spikes not yet delivered
  int64_t pend_t0 = 0;      // start step of that slice
  int cur = 0;              // list buffer holding the open slice
  int32_t count_mode = 0;
  int64_t slices = 0;
  int64_t rec_read = 0;     // raster entries already drained
  SliceLauncher lau;        // this network alone
  int32_t persist = 0;      // slices per persistent launch (0: one launch per slice)
  unsigned* pbar = nullptr; // grid-barrier arrivals of a persistent launch
  int64_t bar_spin = -1;    // polls before a grid barrier gives up (< 0: default)
};

// Independent networks advanced together: every slice of all members is
// one fused launch over the union of their target blocks.
// Captured batch slices: in the steady state (every member has a pending
// delivery, t_now on a slice boundary, and its ring valid up to t_now -
// d_min + d_max), slice k + kGraphSlices launches with the arguments of
// slice k moved on by kGraphSlices * d_min steps: the spike lists alternate
// between two buffers and the list counters rotate over three words.
constexpr int kGraphSlices = 6;

struct sd_batch {
  std::vector<sd_ctx*> nets;
  hipStream_t stream = nullptr;
  std::string err;
  SliceLauncher lau;
  // graph of kGraphSlices batched launches + the argument shift, replayed
  bool graph_on = false;
  hipGraphExec_t gexec = nullptr;
  hipStream_t cap_stream = nullptr;        // capture stream (private)
  sd::SliceArgs* g_args = nullptr;         // [kGraphSlices][n] (device)
  sd::SliceArgs* g_host = nullptr;         // pinned staging of g_args
  hipEvent_t g_ev = nullptr;               // staging copy done
  bool g_pend = false;
  int64_t g_launches = 0;                  // graph replays so far
};

namespace {

sd_status fail(sd_ctx* c, sd_status s, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return s;
}

#define HIP_TRY(ctx, call)                                                         \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(ctx, SD_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));    \
  } while (0)

bool open_loop(const sd_config& c) { return c.n_src_exc > 0; }

int32_t auto_block(const sd_config& c, int64_t N) {
  if (c.block_neurons > 0) return c.block_neurons;
  // one block per compute unit, 64-aligned, at least one wave of neurons
  int64_t b = (N + 255) / 256;
  b = (b + 63) / 64 * 64;
  if (b < 64) b = 64;
  return (int32_t)b;
}

sd_status check_config(const sd_config* c, std::string* why) {
  auto bad = [&](const char* m) {
    *why = m;
    return SD_EINVAL;
  };
  if (!c) return bad("null config");
  if (c->model != SD_IAF_PSC_DELTA && c->model != SD_IAF_PSC_ALPHA) return bad("unknown model");
  if (c->wform < SD_W_FP32 || c->wform > SD_W_BF16_PACKED) return bad("unknown weight form");
  if (c->n_exc < 0 || c->n_inh < 0 || c->n_exc + c->n_inh <= 0) return bad("empty network");
  if (c->k_exc < 0 || c->k_inh < 0) return bad("negative in-degree");
  if (c->k_exc > 0 && (open_loop(*c) ? c->n_src_exc : c->n_exc) <= 0) return bad("no E sources");
  if (c->k_inh > 0 && (open_loop(*c) ? c->n_src_inh : c->n_inh) <= 0) return bad("no I sources");
  if (c->d_min < 1 || c->d_min > 31) return bad("d_min must be in [1, 31]");
  if (c->d_lo < c->d_min || c->d_hi < c->d_lo || c->d_hi > c->d_max || c->d_max > 255)
    return bad("delays must satisfy d_min <= d_lo <= d_hi <= d_max <= 255");
  if (c->ring_len < c->d_min + c->d_max || c->ring_len > 512) return bad("ring_len out of range");
  if (!(c->h > 0.0) || !(c->tau_m > 0.0) || !(c->c_m > 0.0)) return bad("non-positive h/tau/C");
  if (c->model == SD_IAF_PSC_ALPHA && (!(c->tau_syn > 0.0) || c->tau_syn == c->tau_m))
    return bad("alpha model needs tau_syn > 0 and tau_syn != tau_m");
  if (c->t_ref < 0.0 || c->drive_rate_hz < 0.0 || c->src_rate_hz < 0.0) return bad("negative rate");
  if (c->block_neurons < 0 || (c->block_neurons % 64) != 0) return bad("block_neurons % 64 != 0");
  if (c->w_cv < 0.0) return bad("negative weight CV");
  if (c->layout < SD_LAYOUT_AUTO || c->layout > SD_LAYOUT_SOURCE) return bad("unknown layout");
  if (c->plastic) {
    if (c->plastic != 1) return bad("plastic must be 0 or 1");
    if (c->wform != SD_W_FP32) return bad("plastic synapses need the FP32 form");
    if (open_loop(*c)) return bad("plastic synapses need a closed-loop network");
    if (c->layout == SD_LAYOUT_SOURCE) return bad("plastic synapses need the block-major layout");
    if (c->d_min > 16 || c->d_min + c->d_max > 64)
      return bad("plastic synapses need d_min <= 16 and d_min + d_max <= 64");
    if (!(c->stdp_tau_plus > 0.0) || !(c->stdp_tau_minus > 0.0) || c->stdp_a_plus < 0.0 ||
        c->stdp_a_minus < 0.0 || !(c->stdp_w_max >= 0.0))
      return bad("plastic synapses need tau+ , tau- > 0, A+, A- >= 0 and w_max >= 0");
  }
  return SD_OK;
}

// Everything sizes-related in one place, shared by query and create.
struct Layout {
  sd_sizes sz;
  int64_t N, n_src, n_syn, M, n_tiles, rec_cap;
  int32_t B, NB, rec_bytes, dly_bytes;
  int64_t list_cap;
  bool sm = false;  // source-major layout
  int32_t bin_P = 0, bin_cap = 0, bin_U = 0;  // binning (source-major)
  int32_t tbits = 0, H = 1;                   // source-major target parts
  size_t off_row, off_cursor, off_seg, off_tiles, off_syn, off_dly, off_V, off_y1, off_y2, off_r,
      off_rb, off_list0, off_list1, off_cnt, off_rec, off_wte, off_wti, off_thr, off_p64, off_p32,
      off_counters, off_overflow, off_bins, off_bcnt, off_spill, off_sflag, off_ext, off_extcnt,
      off_pmask, off_pbefore, off_aux0, off_aux1, off_prev0, off_prev1, off_pbar, total;
};

constexpr size_t kLdsBudget = 160 * 1024;  // LDS of one gfx950 workgroup

// Records per (block, binning workgroup) region: the expected count at the
// configured source rate (open loop) or a nominal 20 Hz (closed loop), with
// room for 6 standard deviations and a floor; fuller regions spill.
int32_t auto_bin_cap(const sd_config& c, const Layout& L) {
  const double rate = c.n_src_exc > 0 ? c.src_rate_hz : 20.0;
  const double spikes = (double)L.n_src * rate * c.d_min * c.h * 1e-3;
  const double per_src = L.n_src > 0 ? (double)L.n_syn / (double)L.n_src : 0.0;
  const double e = spikes / kBinProducers * per_src / std::max<int32_t>(L.NB, 1);
  double cap = 1.25 * e + 6.0 * std::sqrt(e) + 64.0;
  int64_t k = ((int64_t)std::ceil(cap) + 63) / 64 * 64;
  return (int32_t)std::min<int64_t>(kBinMaxCap, std::max<int64_t>(64, k));
}

// Block-major geometry and its limits (LDS window, u16/packed offsets,
// buffer-resource range, 32-bit segment pointers).
sd_status block_major_fits(const sd_config* c, Layout* L, std::string* why) {
  L->B = auto_block(*c, L->N);
  L->NB = (int32_t)((L->N + L->B - 1) / L->B);
  if (L->B > 65536 && c->wform != SD_W_FP32) {
    *why = "u16 offsets need blocks of at most 65536 neurons";
    return SD_EINVAL;
  }
  if (c->wform == SD_W_BF16_PACKED && (int64_t)(c->d_max - c->d_min + 1) * L->B > 65536) {
    *why = "packed form needs (d_max - d_min + 1) * block_neurons <= 65536";
    return SD_EUNSUPPORTED;
  }
  if (slice_lds_bytes(L->B, c->d_min, c->d_max, c->plastic != 0) > 160 * 1024) {
    *why = "ring window of a block does not fit the 160 KiB LDS; lower block_neurons";
    return SD_EUNSUPPORTED;
  }
  if (L->n_syn >= (int64_t)UINT32_MAX || L->N >= (1LL << 27) || L->n_src >= (1LL << 27)) {
    *why = "block-major layout holds at most 2^32 synapses and 2^27 neurons";
    return SD_EUNSUPPORTED;
  }
  // (start, count) pairs of every (source, block): keep them below 8 GiB
  if ((double)L->n_src * L->NB * 8.0 > 8.0 * (1LL << 30)) {
    *why = "segment-pointer table of the block-major layout exceeds 8 GiB";
    return SD_EUNSUPPORTED;
  }
  return SD_OK;
}

sd_status make_layout(const sd_config* c, Layout* L, std::string* why) {
  sd_status s = check_config(c, why);
  if (s != SD_OK) return s;
  L->N = c->n_exc + c->n_inh;
  L->n_src = open_loop(*c) ? c->n_src_exc + c->n_src_inh : L->N;
  L->n_syn = L->N * ((int64_t)c->k_exc + c->k_inh);
  if (c->layout == SD_LAYOUT_SOURCE) {
    L->sm = true;
  } else {
    s = block_major_fits(c, L, why);
    if (s != SD_OK && (c->layout == SD_LAYOUT_BLOCK || c->plastic)) return s;
    L->sm = s != SD_OK;
  }
  if (L->sm) {
    // record word: offset in a part of 2^tbits targets, then the delay
    // offset in dbits (tbits + dbits <= 24); H parts cover the targets.
    // Parts of at most 2^18 targets: the binning pass takes a part's
    // segments together, so that a sorting chunk's events fall into that
    // part's few hundred blocks and each block's run is long
    int dbits = 1;
    while ((1 << dbits) < c->d_max - c->d_min + 1) ++dbits;
    L->tbits = std::min(kRecWordBits - dbits, kPartBits);
    L->H = (int32_t)((L->N + (1LL << L->tbits) - 1) >> L->tbits);
    if (dbits > 8 || L->H > kMaxParts || L->n_src >= (1LL << 27)) {
      *why = "source-major layout holds at most 2^27 sources, d_max - d_min < 256 and "
             "64 target parts of 2^18 targets";
      return SD_EUNSUPPORTED;
    }
    // The events are binned by target block and accumulated in the same LDS
    // ring windows as the block-major layout: the largest block whose window
    // fits the LDS and whose slots fit the binned record's 15 bits.
    auto fits = [&](int64_t b) {
      return slice_lds_bytes((int)b, c->d_min, c->d_max, false, true) + 64 <= kLdsBudget &&
             (int64_t)c->d_max * b <= (1 << kBinSlotBits);
    };
    int64_t b = c->block_neurons;
    if (b <= 0) {
      b = std::min<int64_t>(kSliceThreads, (L->N + 63) / 64 * 64);
      while (b > 64 && !fits(b)) b -= 64;
    }
    if (b > kSliceThreads) {
      *why = "source-major layout needs block_neurons <= 1024";
      return SD_EINVAL;
    }
    if (!fits(b)) {
      *why = "source-major layout needs a ring window that fits the LDS and "
             "d_max * block_neurons <= 32768";
      return SD_EUNSUPPORTED;
    }
    L->B = (int32_t)b;
    L->NB = (int32_t)((L->N + L->B - 1) / L->B);
    L->bin_P = kBinProducers;
    L->bin_cap = c->bin_cap > 0 ? c->bin_cap : auto_bin_cap(*c, *L);
    if (L->bin_cap > kBinMaxCap) {
      *why = "bin_cap must be at most 1024";
      return SD_EINVAL;
    }
    if ((int64_t)L->NB * L->bin_P * L->bin_cap >= (1LL << 31)) {
      *why = "binned records of all target blocks exceed 2^31; lower bin_cap";
      return SD_EUNSUPPORTED;
    }
    const bool w8 = c->wform == SD_W_FP32;
    L->bin_U = 0;
    for (int u = w8 ? kBinMaxU8 : kBinMaxU; u >= 4; u -= 4)
      if (bin_lds_bytes(L->NB, u, w8) + 64 <= kLdsBudget) {
        L->bin_U = u;
        break;
      }
    if (L->bin_U == 0 || L->NB > 65535) {
      *why = "too many target blocks for the binning pass's LDS counters";
      return SD_EUNSUPPORTED;
    }
    L->M = L->n_src * L->H + 1;
    L->rec_bytes = 4;                                  // offset | delay | weight high byte
    L->dly_bytes = c->wform == SD_W_FP32 ? 4 : 1;      // f32 weight, or the low byte
  } else {
    L->M = L->n_src * L->NB + 1;
    L->rec_bytes = c->wform == SD_W_FP32 ? 8 : 4;
    L->dly_bytes = c->wform == SD_W_BF16_PACKED ? 0 : 1;
    if (c->plastic && L->B > kSliceThreads) {
      *why = "plastic synapses need block_neurons <= 1024";
      return SD_EUNSUPPORTED;
    }
  }
  L->n_tiles = (L->M + 4095) / 4096;
  L->list_cap = (int64_t)L->NB * L->B * c->d_min;
  L->rec_cap = c->record_spikes ? (c->record_cap > 0 ? c->record_cap
                                                     : std::max<int64_t>(1 << 20, L->N * 64))
                                : 0;
  const size_t ptr = L->sm ? 8 : 4;  // segment pointer width
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L->off_row = take((size_t)L->M * ptr);
  L->off_cursor = take((size_t)L->M * ptr);
  L->off_seg = take(L->sm ? 0 : (size_t)L->n_src * L->NB * 8);
  L->off_tiles = take((size_t)L->n_tiles * ptr);
  L->off_syn = take(std::max<size_t>((size_t)L->n_syn * L->rec_bytes, 16));  // record 0 always readable
  L->off_dly = take(std::max<size_t>((size_t)L->n_syn * L->dly_bytes, 16));
  L->off_V = take((size_t)L->N * 4);
  L->off_y1 = take((size_t)L->N * 4);
  L->off_y2 = take((size_t)L->N * 4);
  L->off_r = take((size_t)L->N * 4);
  L->off_rb = take((size_t)c->ring_len * L->N * 4);
  L->off_list0 = take((size_t)L->list_cap * 4);
  L->off_list1 = take((size_t)L->list_cap * 4);
  L->off_cnt = take(3 * 4);
  L->off_rec = take((size_t)std::max<int64_t>(L->rec_cap, 1) * 8);
  L->off_wte = take(65536 * 4);
  L->off_wti = take(65536 * 4);
  L->off_thr = take(kMaxThr * 4);
  L->off_p64 = take(8 * 8);
  L->off_p32 = take(8 * 4);
  L->off_counters = take(8 * 8);
  L->off_overflow = take(4);
  L->off_pbar = take(4);
  const size_t brec = c->wform == SD_W_FP32 ? 8 : 4;
  L->off_bins = take(L->sm ? (size_t)L->NB * L->bin_P * L->bin_cap * brec : 0);
  L->off_bcnt = take(L->sm ? (size_t)L->NB * L->bin_P * 4 : 0);
  L->off_spill = take(L->sm ? (size_t)c->d_max * L->N * 8 : 0);
  L->off_sflag = take(L->sm ? (size_t)L->NB * 4 : 0);
  // external spike lists (sd_deliver_spikes): packed entries and their count
  L->off_ext = take((size_t)L->list_cap * 4);
  L->off_extcnt = take(4);
  // plastic synapses: per-neuron spike history, per-entry lag mask and
  // previous spike of both lists
  const size_t pl = c->plastic ? 1 : 0;
  L->off_pmask = take(pl * (size_t)L->N * 8);
  L->off_pbefore = take(pl * (size_t)L->N * 4);
  L->off_aux0 = take(pl * (size_t)L->list_cap * 4);
  L->off_aux1 = take(pl * (size_t)L->list_cap * 4);
  L->off_prev0 = take(pl * (size_t)L->list_cap * 4);
  L->off_prev1 = take(pl * (size_t)L->list_cap * 4);
  L->total = o;
  sd_sizes& z = L->sz;
  z.n_local = L->N;
  z.n_src = L->n_src;
  z.n_syn = L->n_syn;
  z.block_neurons = L->B;
  z.n_blocks = L->NB;
  z.bytes_per_synapse = L->rec_bytes + L->dly_bytes;
  z.table_bytes = (int64_t)L->n_syn * z.bytes_per_synapse + L->M * (int64_t)ptr +
                  (L->sm ? 0 : L->n_src * L->NB * 8);
  z.arena_bytes = (int64_t)L->total;
  z.layout = L->sm ? SD_LAYOUT_SOURCE : SD_LAYOUT_BLOCK;
  z.bin_cap = L->sm ? L->bin_cap : 0;
  return SD_OK;
}

sd_status launch_slice_checked(sd_ctx* c, const SliceArgs& a) {
  HIP_TRY(c, launcher_run(c->lau, c->stream, &a, 1));
  return SD_OK;
}

SliceArgs base_args(sd_ctx* c) {
  SliceArgs a;
  std::memset(&a, 0, sizeof a);
  const sd_config& g = c->cfg;
  a.seg = c->seg;
  a.n_src = c->n_src;
  a.syn = c->syn;
  a.syn_dly = c->syn_dly;
  a.K = c->K;
  a.N = c->N;
  a.NB = c->NB;
  a.B = c->B;
  a.Dmin = g.d_min;
  a.Dmax = g.d_max;
  a.L = g.ring_len;
  a.win_rows = g.d_max;
  if (c->sm) {
    a.bins = c->bins;
    a.bin_cnt = c->bin_cnt;
    a.bin_cap = c->bin_cap;
    a.bin_P = c->bin_P;
    a.spill = c->spill;
    a.spill_flag = c->spill_flag;
  }
  a.src_e_end = c->src_e_end;
  {
    // fixed-point weight trunc(m1 * x + m0): x is the weight (FP32, BF16) or
    // the BF16 residual (w = mu (1 + x)); count mode adds 1.0 per synapse
    const float sc = std::ldexp(1.0f, c->fx_shift);
    const bool resid = g.wform == SD_W_BF16_RESID || g.wform == SD_W_BF16_PACKED;
    if (c->count_mode) {
      a.wm0_e = a.wm0_i = sc;
      a.wm1_e = a.wm1_i = 0.f;
    } else if (resid) {
      a.wm0_e = a.wm1_e = c->mu_e * sc;
      a.wm0_i = a.wm1_i = c->mu_i * sc;
    } else {
      a.wm0_e = a.wm0_i = 0.f;
      a.wm1_e = a.wm1_i = sc;
    }
  }
  a.fx_inv = std::ldexp(1.0f, -c->fx_shift);
  a.grid_per_xcd = c->grid_per_xcd;
  a.V = c->V;
  a.y1 = c->y1;
  a.y2 = c->y2;
  a.r = c->r;
  std::memcpy(a.prop, c->prop_h, sizeof a.prop);
  a.thr = c->thr;
  a.n_thr = c->n_thr;
  a.seed = g.seed;
  a.e_l = (float)g.e_l;
  a.v_th = (float)g.v_th;
  a.v_reset = (float)g.v_reset;
  a.drive_w = (float)g.drive_w;
  a.ref_steps = c->ref_steps;
  a.model = g.model;
  a.rb = c->rb;
  a.rb_hi = c->rb_hi;
  a.write_list = open_loop(g) ? 0 : 1;
  a.out_cap = c->list_cap;
  a.rec = c->rec_cap > 0 ? c->rec : nullptr;
  a.rec_n = c->counters + 3;
  a.rec_cap = c->rec_cap;
  a.ev_count = c->counters + 0;
  a.spk_in_count = c->counters + 1;
  a.spk_count = c->counters + 2;
  a.overflow = c->overflow;
  if (g.plastic) {
    const double ln2 = std::log(2.0);
    a.plastic = 1;
    a.pmask = c->pmask;
    a.pbefore = c->pbefore;
    a.stdp_ap = (float)g.stdp_a_plus;
    a.stdp_am = (float)g.stdp_a_minus;
    a.stdp_kp = (float)(g.h / (g.stdp_tau_plus * ln2));
    a.stdp_km = (float)(g.h / (g.stdp_tau_minus * ln2));
    a.stdp_wmax = (float)g.stdp_w_max;
  }
  return a;
}

// Rows of steps in [max(t_now, rb_hi), w_lo) would be claimed valid by a
// delivery window starting at w_lo without having been written: zero them.
sd_status fill_gap(sd_ctx* c, int64_t w_lo) {
  const int64_t lo = std::max(c->t_now, c->rb_hi);
  if (w_lo > lo) {
    HIP_TRY(c, launch_zero_rows(c->stream, c->rb, c->N, c->cfg.ring_len, lo, w_lo));
    c->rb_hi = w_lo;
  }
  return SD_OK;
}

// Source-major layout, first pass of a delivery: the events of the entries
// of in_list (count on the device) are binned by target block; the slice
// launch that follows accumulates them.
sd_status bin_events(sd_ctx* c, const uint32_t* in_list, const int32_t* in_cnt, int64_t in_cap) {
  const sd_config& g = c->cfg;
  const SliceArgs b = base_args(c);
  BinArgs a;
  std::memset(&a, 0, sizeof a);
  a.row = c->row64;
  a.tw = c->tw;
  a.wbits = c->wbits;
  a.tbits = c->tbits;
  a.H = c->H;
  a.in_list = in_list;
  a.in_cnt = in_cnt;
  a.in_cap = in_cap;
  a.n_src = c->n_src;
  a.N = c->N;
  a.B = c->B;
  a.NB = c->NB;
  a.Dmin = g.d_min;
  a.U = c->bin_U;
  a.cap = c->bin_cap;
  a.inv_B = 1.0f / (float)c->B;
  a.src_e_end = c->src_e_end;
  a.wm0_e = b.wm0_e;
  a.wm1_e = b.wm1_e;
  a.wm0_i = b.wm0_i;
  a.wm1_i = b.wm1_i;
  a.bins = c->bins;
  a.bin_cnt = c->bin_cnt;
  a.spill = c->spill;
  a.spill_flag = c->spill_flag;
  a.ev_count = c->counters + 0;
  a.spk_in_count = c->counters + 1;
  a.overflow = c->overflow;
  HIP_TRY(c, launch_bin(c->stream, a, c->bin_P, c->bin_lds, g.wform == SD_W_FP32));
  return SD_OK;
}

// Decode record e of a host copy of the synapse arrays (b: its block).
void decode_record(const sd_config& g, const uint8_t* rec, const uint8_t* dl, uint32_t e,
                   int32_t b, int32_t B, float mu, int32_t* tgt, float* w, uint8_t* dly) {
  if (g.wform == SD_W_FP32) {
    uint64_t r;
    std::memcpy(&r, rec + (size_t)e * 8, 8);
    const uint32_t wb = (uint32_t)r;
    std::memcpy(w, &wb, 4);
    *tgt = (int32_t)(r >> 32);
    *dly = dl[e];
    return;
  }
  uint32_t r;
  std::memcpy(&r, rec + (size_t)e * 4, 4);
  const uint32_t u = r << 16;
  float d;
  std::memcpy(&d, &u, 4);
  *w = g.wform == SD_W_BF16 ? d : std::fma(mu, d, mu);
  if (g.wform == SD_W_BF16_PACKED) {
    const uint32_t slot = r >> 16;  // (delay - d_min) * B + offset
    *tgt = (int32_t)((int64_t)b * B + (int32_t)(slot % (uint32_t)B));
    *dly = (uint8_t)(g.d_min + (int)(slot / (uint32_t)B));
  } else {
    *tgt = (int32_t)((int64_t)b * B + (r >> 16));
    *dly = dl[e];
  }
}

// Point the delivery arguments at the completed slice's spikes: the
// context's own block lists (closed loop) or the prepared input (open loop).
sd_status set_pending_input(sd_ctx* c, SliceArgs& a) {
  if (open_loop(c->cfg)) {
    const int64_t k = (c->pend_t0 - c->in_t0) / c->cfg.d_min;
    if (!c->in_list || c->pend_t0 < c->in_t0 || k >= c->in_slices)
      return fail(c, SD_ESTATE, "open-loop input not prepared for step %lld",
                  (long long)c->pend_t0);
    a.in_list = c->in_list + c->in_off_h[k];
    a.in_cnt = c->in_cnt + k;
    a.in_cap = c->in_off_h[k + 1] - c->in_off_h[k];
  } else {
    a.in_list = c->list[c->cur];
    a.in_cnt = c->cnt3 + c->ci;
    a.in_cap = c->list_cap;
    a.in_aux = c->aux[c->cur];
    a.in_prev = c->prev[c->cur];
  }
  return SD_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

sd_status sd_query_sizes(const sd_config* cfg, sd_sizes* out) {
  Layout L;
  std::string why;
  sd_status s = make_layout(cfg, &L, &why);
  if (s != SD_OK) return s;
  if (out) *out = L.sz;
  return SD_OK;
}

sd_status sd_create(const sd_config* cfg, void* hip_stream, void* d_arena, size_t arena_bytes,
                    sd_ctx** out) {
  if (!out) return SD_EINVAL;
  *out = nullptr;
  sd_ctx* c = new sd_ctx();
  Layout L;
  sd_status s = make_layout(cfg, &L, &c->err);
  if (s != SD_OK) {
    *out = c;  // keep the message readable; caller destroys
    return s;
  }
  c->cfg = *cfg;
  c->sz = L.sz;
  c->stream = (hipStream_t)hip_stream;
  HIP_TRY(c, hipGetDevice(&c->device));
  c->N = L.N;
  c->n_src = L.n_src;
  c->n_syn = L.n_syn;
  c->B = L.B;
  c->NB = L.NB;
  c->K = cfg->k_exc + cfg->k_inh;
  c->M = L.M;
  c->n_tiles = L.n_tiles;
  c->list_cap = L.list_cap;
  c->rec_cap = L.rec_cap;
  c->grid_per_xcd = (L.NB + 7) / 8;
  c->src_e_end = open_loop(*cfg) ? cfg->n_src_exc : cfg->n_exc;
  c->sm = L.sm;
  *out = c;
  if (d_arena) {
    if (arena_bytes < L.total) return fail(c, SD_ENOMEM, "arena of %zu bytes < %zu needed",
                                           arena_bytes, L.total);
    c->arena = (char*)d_arena;
  } else {
    if (hipMalloc((void**)&c->arena, L.total) != hipSuccess) {
      (void)hipGetLastError();
      c->arena = nullptr;
      return fail(c, SD_ENOMEM, "hipMalloc of %zu bytes failed", L.total);
    }
    c->own_arena = true;
  }
  char* A = c->arena;
  c->row = (uint32_t*)(A + L.off_row);
  c->cursor = (uint32_t*)(A + L.off_cursor);
  c->seg = (uint2*)(A + L.off_seg);
  c->tile_sums = (uint32_t*)(A + L.off_tiles);
  c->syn = A + L.off_syn;
  c->syn_dly = (uint8_t*)(A + L.off_dly);
  c->V = (float*)(A + L.off_V);
  c->y1 = (float*)(A + L.off_y1);
  c->y2 = (float*)(A + L.off_y2);
  c->r = (int32_t*)(A + L.off_r);
  if (c->sm) {
    c->row64 = (unsigned long long*)(A + L.off_row);
    c->cursor64 = (unsigned long long*)(A + L.off_cursor);
    c->tiles64 = (unsigned long long*)(A + L.off_tiles);
    c->tw = (uint32_t*)(A + L.off_syn);
    c->tbits = L.tbits;
    c->H = L.H;
    c->wbits = A + L.off_dly;
    c->bins = A + L.off_bins;
    c->bin_cnt = (uint32_t*)(A + L.off_bcnt);
    c->spill = (long long*)(A + L.off_spill);
    c->spill_flag = (int32_t*)(A + L.off_sflag);
    c->bin_P = L.bin_P;
    c->bin_cap = L.bin_cap;
    c->bin_U = L.bin_U;
    c->bin_lds = bin_lds_bytes(L.NB, L.bin_U, cfg->wform == SD_W_FP32);
    c->row = nullptr;
    c->cursor = nullptr;
    c->seg = nullptr;
    c->syn = nullptr;
    c->syn_dly = nullptr;
  }
  c->rb = (float*)(A + L.off_rb);
  c->list[0] = (uint32_t*)(A + L.off_list0);
  c->list[1] = (uint32_t*)(A + L.off_list1);
  c->ext_list = (uint32_t*)(A + L.off_ext);
  c->ext_cnt = (int32_t*)(A + L.off_extcnt);
  if (cfg->plastic) {
    c->pmask = (uint64_t*)(A + L.off_pmask);
    c->pbefore = (int32_t*)(A + L.off_pbefore);
    c->aux[0] = (uint32_t*)(A + L.off_aux0);
    c->aux[1] = (uint32_t*)(A + L.off_aux1);
    c->prev[0] = (int32_t*)(A + L.off_prev0);
    c->prev[1] = (int32_t*)(A + L.off_prev1);
  }
  c->cnt3 = (int32_t*)(A + L.off_cnt);
  c->rec = (uint2*)(A + L.off_rec);
  c->wtab_e = A + L.off_wte;
  c->wtab_i = A + L.off_wti;
  c->thr = (uint32_t*)(A + L.off_thr);
  c->prop64 = (double*)(A + L.off_p64);
  c->prop32 = (float*)(A + L.off_p32);
  c->counters = (unsigned long long*)(A + L.off_counters);
  c->overflow = (int32_t*)(A + L.off_overflow);
  c->pbar = (unsigned*)(A + L.off_pbar);

  // tables (host, FP64 -> FP32 / BF16 codes)
  const sd_config& g = *cfg;
  c->we_h.assign(65536, 0.f);
  c->wi_h.assign(65536, 0.f);
  quantile_weights(g, c->we_h.data(), c->wi_h.data());
  c->mu_e = (float)g.w_exc;
  c->mu_i = (float)(-g.g * g.w_exc);
  c->n_thr = poisson_table(g.drive_rate_hz * g.h * 1e-3, c->thr_h, kMaxThr);
  c->ref_steps = (int32_t)std::llround(g.t_ref / g.h);
  // Fixed-point quantum of the LDS window: the largest 2^-s with
  // max|w| * 2^s <= 2^30, so one synapse's code fits int32 with margin and
  // 64-bit cell sums cannot overflow for fewer than 2^32 events per cell.
  {
    double wmax = 1.0;  // count mode delivers 1.0
    if (g.w_cv == 0.0) {
      wmax = std::max({wmax, std::fabs(g.w_exc), std::fabs(g.g * g.w_exc)});
    } else {
      for (int i = 0; i < 65536; ++i)
        wmax = std::max({wmax, (double)std::fabs(c->we_h[i]), (double)std::fabs(c->wi_h[i])});
      wmax *= 1.01;  // BF16 decoding may round up by < 2^-8
    }
    int s = (int)std::floor(std::log2(1073741824.0 / wmax));
    c->fx_shift = std::max(0, std::min(s, 40));
  }
  std::vector<uint32_t> enc_e(65536), enc_i(65536);
  for (int i = 0; i < 65536; ++i) {
    if (g.wform == SD_W_FP32) {
      std::memcpy(&enc_e[i], &c->we_h[i], 4);
      std::memcpy(&enc_i[i], &c->wi_h[i], 4);
    } else if (g.wform == SD_W_BF16) {
      enc_e[i] = bf16_bits_rne(c->we_h[i]);
      enc_i[i] = bf16_bits_rne(c->wi_h[i]);
    } else {  // residual forms (plain and packed)
      enc_e[i] = resid_bits(c->we_h[i], c->mu_e);
      enc_i[i] = resid_bits(c->wi_h[i], c->mu_i);
    }
  }
  if (g.wform == SD_W_FP32) {
    HIP_TRY(c, hipMemcpyAsync(c->wtab_e, enc_e.data(), 65536 * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->wtab_i, enc_i.data(), 65536 * 4, hipMemcpyHostToDevice, c->stream));
  } else {
    std::vector<uint16_t> h_e(65536), h_i(65536);
    for (int i = 0; i < 65536; ++i) {
      h_e[i] = (uint16_t)enc_e[i];
      h_i[i] = (uint16_t)enc_i[i];
    }
    HIP_TRY(c, hipMemcpyAsync(c->wtab_e, h_e.data(), 65536 * 2, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->wtab_i, h_i.data(), 65536 * 2, hipMemcpyHostToDevice, c->stream));
  }
  HIP_TRY(c, hipMemcpyAsync(c->thr, c->thr_h, sizeof(uint32_t) * kMaxThr, hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, hipMemsetAsync(c->counters, 0, 8 * 8, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->overflow, 0, 4, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->cnt3, 0, 3 * 4, c->stream));
  if (g.plastic) {  // no spikes yet: empty histories, no earlier spike (-1)
    HIP_TRY(c, hipMemsetAsync(c->pmask, 0, (size_t)c->N * 8, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->pbefore, 0xff, (size_t)c->N * 4, c->stream));
  }
  HIP_TRY(c, launch_propagators(c->stream, g.model, g.h, g.tau_m, g.tau_syn, g.c_m, g.i_e,
                                c->prop64, c->prop32));
  HIP_TRY(c, launch_init_state(c->stream, c->N, g.seed, g.v0_lo, g.v0_hi, c->V, c->y1, c->y2,
                               c->r));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  HIP_TRY(c, hipMemcpy(c->prop_h, c->prop32, sizeof c->prop_h, hipMemcpyDeviceToHost));
  int lds_max = 0;
  HIP_TRY(c, hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));
  const size_t lds = slice_lds_bytes(c->B, g.d_min, g.d_max, g.plastic != 0, c->sm);
  if ((size_t)lds_max < lds + 64)
    return fail(c, SD_EUNSUPPORTED, "slice window needs %zu B of LDS, device allows %d", lds,
                lds_max);
  if (c->sm && (size_t)lds_max < c->bin_lds + 64)
    return fail(c, SD_EUNSUPPORTED, "binning pass needs %zu B of LDS, device allows %d",
                c->bin_lds, lds_max);
  c->lau.per = 1;
  c->lau.lds = lds;
  c->lau.wform = g.wform;
  c->lau.single_nb = c->NB;
  return SD_OK;
}

void sd_destroy(sd_ctx* c) {
  if (!c) return;
  if (c->stream || c->arena) (void)hipStreamSynchronize(c->stream);
  if (c->own_arena && c->arena) (void)hipFree(c->arena);
  if (c->in_list) (void)hipFree(c->in_list);
  if (c->in_off) (void)hipFree(c->in_off);
  if (c->in_cnt) (void)hipFree(c->in_cnt);
  launcher_free(c->lau);
  delete c;
}

const char* sd_last_error(const sd_ctx* c) { return c ? c->err.c_str() : "null context"; }

sd_status sd_build_connections(sd_ctx* c) {
  if (!c || !c->arena) return SD_EINVAL;
  const sd_config& g = c->cfg;
  BuildArgs a;
  std::memset(&a, 0, sizeof a);
  a.N = c->N;
  a.n_src = c->n_src;
  a.NB = c->NB;
  a.B = c->B;
  a.K = c->K;
  a.k_exc = g.k_exc;
  if (open_loop(g)) {
    a.src_e_n = g.n_src_exc;
    a.src_i_n = g.n_src_inh;
    a.src_i_base = g.n_src_exc;
  } else {
    a.src_e_n = g.n_exc;
    a.src_i_n = g.n_inh;
    a.src_i_base = g.n_exc;
  }
  a.d_lo = g.d_lo;
  a.n_dly = g.d_hi - g.d_lo + 1;
  a.seed = g.seed;
  a.row = c->row;
  a.cursor = c->cursor;
  a.seg = c->seg;
  a.syn = c->syn;
  a.syn_dly = c->syn_dly;
  a.wform = g.wform;
  a.d_min = g.d_min;
  a.wtab_e = c->wtab_e;
  a.wtab_i = c->wtab_i;
  a.fixed = g.w_cv == 0.0;
  const float fe = (float)g.w_exc, fi = (float)(-g.g * g.w_exc);
  a.w_fix_e = fe;
  a.w_fix_i = fi;
  if (g.wform == SD_W_BF16) {
    a.fix_bits_e = bf16_bits_rne(fe);
    a.fix_bits_i = bf16_bits_rne(fi);
  } else if (g.wform == SD_W_BF16_RESID || g.wform == SD_W_BF16_PACKED) {
    a.fix_bits_e = resid_bits(fe, c->mu_e);
    a.fix_bits_i = resid_bits(fi, c->mu_i);
  }
  if (c->sm) {
    a.row64 = c->row64;
    a.cursor64 = c->cursor64;
    a.tw = c->tw;
    a.wbits = c->wbits;
    a.tbits = c->tbits;
    a.H = c->H;
    HIP_TRY(c, hipMemsetAsync(c->row64, 0, (size_t)c->M * 8, c->stream));
    if (c->K > 0) HIP_TRY(c, launch_count_sm(c->stream, a));
    HIP_TRY(c, launch_scan64(c->stream, c->row64, c->M, c->tiles64, c->n_tiles));
    HIP_TRY(c, hipMemcpyAsync(c->cursor64, c->row64, (size_t)c->M * 8, hipMemcpyDeviceToDevice,
                              c->stream));
    if (c->K > 0) HIP_TRY(c, launch_fill_sm(c->stream, a));
    HIP_TRY(c, hipMemsetAsync(c->spill, 0, (size_t)g.d_max * c->N * 8, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->spill_flag, 0, (size_t)c->NB * 4, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    unsigned long long total = 0;
    HIP_TRY(c, hipMemcpy(&total, c->row64 + c->M - 1, 8, hipMemcpyDeviceToHost));
    if ((int64_t)total != c->n_syn)
      return fail(c, SD_EHIP, "segment table holds %llu synapses, expected %lld", total,
                  (long long)c->n_syn);
    c->built = true;
    return SD_OK;
  }
  HIP_TRY(c, hipMemsetAsync(c->row, 0, (size_t)c->M * 4, c->stream));
  if (c->K > 0) HIP_TRY(c, launch_count(c->stream, a));
  HIP_TRY(c, launch_scan(c->stream, c->row, c->M, c->tile_sums, c->n_tiles));
  HIP_TRY(c, hipMemcpyAsync(c->cursor, c->row, (size_t)c->M * 4, hipMemcpyDeviceToDevice,
                            c->stream));
  if (c->K > 0) HIP_TRY(c, launch_fill(c->stream, a));
  HIP_TRY(c, launch_seg_pairs(c->stream, a));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  uint32_t total = 0;
  HIP_TRY(c, hipMemcpy(&total, c->row + c->M - 1, 4, hipMemcpyDeviceToHost));
  if ((int64_t)total != c->n_syn)
    return fail(c, SD_EHIP, "segment table holds %u synapses, expected %lld", total,
                (long long)c->n_syn);
  c->built = true;
  return SD_OK;
}

sd_status sd_set_count_mode(sd_ctx* c, int32_t on) {
  if (!c) return SD_EINVAL;
  if (on && c->cfg.plastic) return fail(c, SD_EUNSUPPORTED, "count mode of a plastic net");
  c->count_mode = on ? 1 : 0;
  return SD_OK;
}

int64_t sd_t_now(const sd_ctx* c) { return c ? c->t_now : -1; }

sd_status sd_get_sizes(const sd_ctx* c, sd_sizes* out) {
  if (!c || !out) return SD_EINVAL;
  *out = c->sz;
  return SD_OK;
}

sd_status sd_update_neurons(sd_ctx* c, int32_t n_steps) {
  if (!c || n_steps < 1) return fail(c, SD_EINVAL, "n_steps must be >= 1");
  if (!c->built) return fail(c, SD_ESTATE, "build_connections first");
  const int32_t Dmin = c->cfg.d_min;
  const int64_t in_slice = c->t_now % Dmin;
  if (in_slice + n_steps > Dmin)
    return fail(c, SD_EINVAL, "steps [%lld, %lld) cross a slice boundary", (long long)c->t_now,
                (long long)(c->t_now + n_steps));
  const bool fresh = in_slice == 0;
  if (fresh && c->pend_open)
    return fail(c, SD_ESTATE, "the completed slice at step %lld has not been delivered",
                (long long)c->pend_t0);
  SliceArgs a = base_args(c);
  if (fresh) {
    // a new list: its counter (the one after the last) is zero; the one
    // before it is cleared for the slice after this one
    c->cur ^= 1;
    c->ci = (c->ci + 1) % 3;
    c->pend_t0 = c->t_now;
    a.zero_cnt = c->cnt3 + (c->ci + 1) % 3;
  }
  a.do_deliver = 0;
  a.n_upd = n_steps;
  a.t_upd = c->t_now;
  a.t_slice0 = c->pend_t0;
  a.out_list = c->list[c->cur];
  a.out_cnt = c->cnt3 + c->ci;
  a.out_aux = c->aux[c->cur];
  a.out_prev = c->prev[c->cur];
  sd_status s = launch_slice_checked(c, a);
  if (s != SD_OK) return s;
  c->pend_open = true;
  c->t_now += n_steps;
  return SD_OK;
}

namespace {
sd_status deliver_impl(sd_ctx* c, bool own, const uint32_t* d_src, const uint8_t* d_lag,
                       int64_t n, int64_t t0, uint32_t* list, int32_t* list_cnt, int64_t cap);
}

sd_status sd_deliver_spikes(sd_ctx* c, const uint32_t* d_src, const uint8_t* d_lag, int64_t n,
                            int64_t t0) {
  if (!c) return SD_EINVAL;
  if (n < 0 || (n > 0 && (!d_src || !d_lag))) return fail(c, SD_EINVAL, "bad spike list");
  return deliver_impl(c, false, d_src, d_lag, n, t0, c->ext_list, c->ext_cnt, c->list_cap);
}

sd_status sd_deliver_pending(sd_ctx* c) {
  if (!c) return SD_EINVAL;
  return deliver_impl(c, true, nullptr, nullptr, 0, 0, nullptr, nullptr, 0);
}

}  // extern "C"

namespace sd {
// sd_deliver_spikes with the packed list and its count in caller-chosen
// device memory of cap entries (the no-allocation entry point's scratch).
sd_status deliver_external(sd_ctx* c, const uint32_t* d_src, const uint8_t* d_lag, int64_t n,
                           int64_t t0, uint32_t* list, int32_t* list_cnt, int64_t cap) {
  if (!c) return SD_EINVAL;
  if (n < 0 || (n > 0 && (!d_src || !d_lag))) return fail(c, SD_EINVAL, "bad spike list");
  return deliver_impl(c, false, d_src, d_lag, n, t0, list, list_cnt, std::min(cap, c->list_cap));
}
sd_status set_error(sd_ctx* c, sd_status st, const char* msg) { return fail(c, st, "%s", msg); }
int ctx_device(const sd_ctx* c) { return c->device; }
}  // namespace sd

extern "C" {

namespace {
sd_status deliver_impl(sd_ctx* c, bool own, const uint32_t* d_src, const uint8_t* d_lag,
                       int64_t n, int64_t t0, uint32_t* list, int32_t* list_cnt, int64_t cap) {
  if (!c->built) return fail(c, SD_ESTATE, "build_connections first");
  const sd_config& g = c->cfg;
  SliceArgs a = base_args(c);
  a.do_deliver = 1;
  a.n_upd = 0;
  a.t_upd = c->t_now;
  if (own) {
    if (!c->pend_open || c->t_now % g.d_min != 0 || c->t_now != c->pend_t0 + g.d_min)
      return fail(c, SD_ESTATE, "no completed slice to deliver");
    t0 = c->pend_t0;
    sd_status s = set_pending_input(c, a);
    if (s != SD_OK) return s;
  } else {
    if (g.plastic)
      return fail(c, SD_EUNSUPPORTED, "plastic nets deliver their own spike lists only");
    if (t0 + g.d_min < c->t_now)
      return fail(c, SD_EINVAL, "arrivals at step %lld precede t_now %lld",
                  (long long)(t0 + g.d_min), (long long)c->t_now);
    if (t0 + g.d_min + g.d_max > c->t_now + g.ring_len)
      return fail(c, SD_EINVAL, "arrivals beyond the ring (t0 %lld)", (long long)t0);
    // pack (src << 5 | lag) into the context's external list on the device;
    // invalid entries deliver nothing and raise a sticky flag
    if (n > cap)
      return fail(c, SD_EINVAL, "%lld entries exceed the list capacity %lld", (long long)n,
                  (long long)cap);
    if (n > 0)
      HIP_TRY(c, launch_pack_list(c->stream, d_src, d_lag, n, c->n_src, g.d_min, list, list_cnt,
                                  c->overflow));
    a.in_list = list;
    a.in_cnt = list_cnt;
    a.in_cap = n;
    if (n == 0) a.do_deliver = 0;
  }
  const int64_t w_lo = t0 + g.d_min;
  sd_status s = fill_gap(c, w_lo);
  if (s != SD_OK) return s;
  a.rb_hi = c->rb_hi;
  a.w_lo = w_lo;
  if (a.do_deliver) {
    if (c->sm) s = bin_events(c, a.in_list, a.in_cnt, a.in_cap);
    if (s == SD_OK) s = launch_slice_checked(c, a);
    if (s != SD_OK) return s;
  } else {
    // an empty list still defines the window rows as zero
    HIP_TRY(c, launch_zero_rows(c->stream, c->rb, c->N, g.ring_len,
                                std::max(c->rb_hi, w_lo), w_lo + g.d_max));
  }
  c->rb_hi = std::max(c->rb_hi, w_lo + g.d_max);
  if (own) c->pend_open = false;
  return SD_OK;
}
}  // namespace

}  // extern "C"

namespace {
// Arguments of the next fused launch from an aligned t_now: deliver the
// pending slice (if any), update m <= d_min steps, and start a new list;
// advances the host state as if the launch had run.
sd_status next_fused_slice(sd_ctx* c, int32_t m, SliceArgs* out) {
  const sd_config& g = c->cfg;
  const int32_t Dmin = g.d_min;
  SliceArgs a = base_args(c);
  const bool deliver = c->pend_open;
  if (deliver) {
    sd_status s = set_pending_input(c, a);
    if (s != SD_OK) return s;
    a.do_deliver = 1;
    a.w_lo = c->pend_t0 + Dmin;  // == t_now
  }
  a.rb_hi = c->rb_hi;
  a.n_upd = m;
  a.t_upd = c->t_now;
  a.t_slice0 = c->t_now;
  const int nxt = c->cur ^ 1;
  const int cn = (c->ci + 1) % 3;
  a.out_list = c->list[nxt];
  a.out_cnt = c->cnt3 + cn;
  a.out_aux = c->aux[nxt];
  a.out_prev = c->prev[nxt];
  a.zero_cnt = c->cnt3 + (cn + 1) % 3;
  if (deliver && c->sm) {
    // source-major: the binning pass is its own launch (issued now), the
    // fused launch accumulates its records
    sd_status s = bin_events(c, a.in_list, a.in_cnt, a.in_cap);
    if (s != SD_OK) return s;
  }
  if (deliver) c->rb_hi = std::max(c->rb_hi, a.w_lo + g.d_max);
  c->cur = nxt;
  c->ci = cn;
  c->pend_open = true;
  c->pend_t0 = c->t_now;
  c->t_now += m;
  c->slices += 1;
  *out = a;
  return SD_OK;
}
// S whole slices from an aligned t_now in one persistent launch; the host
// state advances exactly as S fused slices would advance it.
sd_status run_persistent(sd_ctx* c, int32_t S) {
  const sd_config& g = c->cfg;
  const int32_t Dmin = g.d_min;
  SliceArgs a = base_args(c);
  a.in_cap = c->list_cap;
  a.zero_cnt = nullptr;
  const int32_t pend0 = c->pend_open ? 1 : 0;
  HIP_TRY(c, launch_set_word(c->stream, c->pbar, 0u));  // the grid barrier's arrival counter
  HIP_TRY(c, launch_persist(c->stream, a, c->list, c->cnt3, c->cur, c->ci, pend0, S, c->t_now,
                            c->rb_hi, c->pbar, c->bar_spin, c->lau.lds, g.wform));
  for (int32_t k = 0; k < S; ++k) {
    if (k > 0 || pend0) c->rb_hi = std::max(c->rb_hi, c->t_now + g.d_max);
    c->cur ^= 1;
    c->ci = (c->ci + 1) % 3;
    c->pend_open = true;
    c->pend_t0 = c->t_now;
    c->t_now += Dmin;
    c->slices += 1;
  }
  return SD_OK;
}
}  // namespace

extern "C" {

sd_status sd_set_persistent(sd_ctx* c, int32_t max_slices) {
  if (!c) return SD_EINVAL;
  if (max_slices < 0) return fail(c, SD_EINVAL, "max_slices must be >= 0");
  if (max_slices == 0) {
    c->persist = 0;
    return SD_OK;
  }
  if (!c->built) return fail(c, SD_ESTATE, "build_connections first");
  const sd_config& g = c->cfg;
  if (c->sm || g.plastic || open_loop(g))
    return fail(c, SD_EUNSUPPORTED,
                "persistent slices need a block-major, closed-loop net with static synapses");
  if (c->B > kSliceThreads || c->B % 64 != 0)
    return fail(c, SD_EUNSUPPORTED, "persistent slices need blocks of a multiple of 64 and at "
                "most %d neurons", kSliceThreads);
  int coop = 0, n_cu = 0;
  HIP_TRY(c, hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, c->device));
  HIP_TRY(c, hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, c->device));
  const int64_t grid = 8 * (int64_t)((c->NB + 7) / 8);
  const int occ = persist_occupancy(g.wform, c->lau.lds);
  if (!coop || (int64_t)occ * n_cu < grid)
    return fail(c, SD_EUNSUPPORTED, "persistent slices need all %lld blocks resident at once "
                "(%d per CU on %d CUs)", (long long)grid, occ, n_cu);
  c->persist = max_slices;
  return SD_OK;
}

sd_status sd_set_barrier_spin(sd_ctx* c, int64_t polls) {
  if (!c) return SD_EINVAL;
  c->bar_spin = polls < 0 ? -1 : polls;
  return SD_OK;
}

sd_status sd_simulate_steps(sd_ctx* c, int64_t n_steps) {
  if (!c || n_steps < 0) return fail(c, SD_EINVAL, "bad step count");
  if (!c->built) return fail(c, SD_ESTATE, "build_connections first");
  const int32_t Dmin = c->cfg.d_min;
  std::vector<SliceArgs> queue;  // fused launches not yet issued
  auto flush = [&]() -> sd_status {
    if (!queue.empty()) {
      HIP_TRY(c, launcher_run(c->lau, c->stream, queue.data(), (int64_t)queue.size()));
      queue.clear();
    }
    return SD_OK;
  };
  int64_t left = n_steps;
  while (left > 0) {
    const int64_t in_slice = c->t_now % Dmin;
    if (in_slice != 0) {
      // finish the open slice without delivering (its spikes are not due)
      const int32_t m = (int32_t)std::min<int64_t>(left, Dmin - in_slice);
      sd_status s = flush();
      if (s == SD_OK) s = sd_update_neurons(c, m);
      if (s != SD_OK) return s;
      left -= m;
      continue;
    }
    if (c->persist > 0 && left >= Dmin && (!c->pend_open || c->pend_t0 + Dmin == c->t_now)) {
      const int32_t S = (int32_t)std::min<int64_t>(left / Dmin, c->persist);
      sd_status s = flush();
      if (s == SD_OK) s = run_persistent(c, S);
      if (s != SD_OK) return s;
      left -= (int64_t)S * Dmin;
      continue;
    }
    const int32_t m = (int32_t)std::min<int64_t>(left, Dmin);
    SliceArgs a;
    // source-major: the binning launch is issued inside next_fused_slice,
    // so queued slices go first and this slice right after it
    sd_status s = c->sm ? flush() : SD_OK;
    if (s == SD_OK) s = next_fused_slice(c, m, &a);
    if (s != SD_OK) {
      flush();
      return s;
    }
    queue.push_back(a);
    if (c->sm) {
      s = flush();
      if (s != SD_OK) return s;
    }
    left -= m;
  }
  return flush();
}

sd_status sd_simulate(sd_ctx* c, double t_ms) {
  if (!c || !(t_ms >= 0.0)) return fail(c, SD_EINVAL, "bad duration");
  return sd_simulate_steps(c, (int64_t)std::llround(t_ms / c->cfg.h));
}

sd_status sd_prepare_input(sd_ctx* c, int64_t n_steps) {
  if (!c || n_steps < 0) return SD_EINVAL;
  const sd_config& g = c->cfg;
  if (!open_loop(g)) return fail(c, SD_ESTATE, "closed-loop network has no external input");
  const int32_t Dmin = g.d_min;
  // the schedule starts at the slice whose spikes are delivered next
  const int64_t t_start = c->pend_open ? c->pend_t0 : (c->t_now / Dmin) * Dmin;
  const int64_t t_end = c->t_now + n_steps;
  const int64_t n_sl = (t_end - t_start + Dmin - 1) / Dmin;
  const int64_t steps = n_sl * Dmin;
  if (c->in_list) (void)hipFree(c->in_list);
  if (c->in_off) (void)hipFree(c->in_off);
  if (c->in_cnt) (void)hipFree(c->in_cnt);
  c->in_list = nullptr;
  c->in_off = nullptr;
  c->in_cnt = nullptr;
  const double p = -std::expm1(-g.src_rate_hz * g.h * 1e-3);
  const uint32_t thr = (uint32_t)std::floor(p * 4294967296.0);
  HIP_TRY(c, hipMalloc((void**)&c->in_cnt, (size_t)(n_sl + 1) * 4));
  HIP_TRY(c, hipMalloc((void**)&c->in_off, (size_t)(n_sl + 1) * 8));
  HIP_TRY(c, hipMemsetAsync(c->in_cnt, 0, (size_t)(n_sl + 1) * 4, c->stream));
  HIP_TRY(c, launch_input_count(c->stream, g.seed, c->n_src, t_start, (int32_t)steps, Dmin, thr,
                                c->in_cnt));
  std::vector<int32_t> cnt((size_t)n_sl + 1);
  HIP_TRY(c, hipMemcpyAsync(cnt.data(), c->in_cnt, (size_t)(n_sl + 1) * 4, hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->in_off_h.assign((size_t)n_sl + 1, 0);
  for (int64_t k = 0; k < n_sl; ++k) c->in_off_h[k + 1] = c->in_off_h[k] + cnt[k];
  const int64_t total = c->in_off_h[n_sl];
  HIP_TRY(c, hipMalloc((void**)&c->in_list, (size_t)std::max<int64_t>(total, 1) * 4));
  HIP_TRY(c, hipMemcpyAsync(c->in_off, c->in_off_h.data(), (size_t)(n_sl + 1) * 8,
                            hipMemcpyHostToDevice, c->stream));
  int32_t* cursor = nullptr;
  HIP_TRY(c, hipMalloc((void**)&cursor, (size_t)(n_sl + 1) * 4));
  HIP_TRY(c, hipMemsetAsync(cursor, 0, (size_t)(n_sl + 1) * 4, c->stream));
  HIP_TRY(c, launch_input_fill(c->stream, g.seed, c->n_src, t_start, (int32_t)steps, Dmin, thr,
                               c->in_off, cursor, c->in_list));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  HIP_TRY(c, hipFree(cursor));
  c->in_t0 = t_start;
  c->in_slices = n_sl;
  return SD_OK;
}

sd_status sd_get_stats(sd_ctx* c, sd_stats* out) {
  if (!c || !out) return SD_EINVAL;
  unsigned long long cnt[4];
  int32_t ov = 0;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  HIP_TRY(c, hipMemcpy(cnt, c->counters, sizeof cnt, hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(&ov, c->overflow, 4, hipMemcpyDeviceToHost));
  out->t_now = c->t_now;
  out->events_delivered = (int64_t)cnt[0];
  out->spikes_delivered = (int64_t)cnt[1];
  out->spikes_emitted = (int64_t)cnt[2];
  out->spikes_recorded = (int64_t)std::min<unsigned long long>(cnt[3], (unsigned long long)c->rec_cap);
  out->slices = c->slices;
  out->overflow = ov;
  if (ov & 12) return fail(c, SD_EINVAL, "an external spike list held invalid entries (flags %d)", ov);
  return ov ? SD_EOVERFLOW : SD_OK;
}

sd_status sd_read_ring(sd_ctx* c, float* h_out, int32_t n_slots) {
  if (!c || !h_out || n_slots < 0 || n_slots > c->cfg.ring_len) return SD_EINVAL;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int32_t L = c->cfg.ring_len;
  for (int32_t s = 0; s < n_slots; ++s) {
    const int64_t t = c->t_now + s;
    float* dst = h_out + (size_t)s * c->N;
    if (t < c->rb_hi) {
      HIP_TRY(c, hipMemcpy(dst, c->rb + (t % L) * c->N, (size_t)c->N * 4, hipMemcpyDeviceToHost));
    } else {
      std::memset(dst, 0, (size_t)c->N * 4);
    }
  }
  return SD_OK;
}

sd_status sd_read_state(sd_ctx* c, float* h_v, float* h_y1, float* h_y2, int32_t* h_r) {
  if (!c) return SD_EINVAL;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const size_t n = (size_t)c->N * 4;
  if (h_v) HIP_TRY(c, hipMemcpy(h_v, c->V, n, hipMemcpyDeviceToHost));
  if (h_y1) HIP_TRY(c, hipMemcpy(h_y1, c->y1, n, hipMemcpyDeviceToHost));
  if (h_y2) HIP_TRY(c, hipMemcpy(h_y2, c->y2, n, hipMemcpyDeviceToHost));
  if (h_r) HIP_TRY(c, hipMemcpy(h_r, c->r, n, hipMemcpyDeviceToHost));
  return SD_OK;
}

sd_status sd_write_state(sd_ctx* c, const float* h_v, const float* h_y1, const float* h_y2,
                         const int32_t* h_r) {
  if (!c) return SD_EINVAL;
  const size_t n = (size_t)c->N * 4;
  if (h_v) HIP_TRY(c, hipMemcpyAsync(c->V, h_v, n, hipMemcpyHostToDevice, c->stream));
  if (h_y1) HIP_TRY(c, hipMemcpyAsync(c->y1, h_y1, n, hipMemcpyHostToDevice, c->stream));
  if (h_y2) HIP_TRY(c, hipMemcpyAsync(c->y2, h_y2, n, hipMemcpyHostToDevice, c->stream));
  if (h_r) HIP_TRY(c, hipMemcpyAsync(c->r, h_r, n, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return SD_OK;
}

}  // extern "C"

namespace {
// Checkpoint layout (host byte buffer): StateHeader, then V, y1, y2, r
// (N x 4 B each), the ring rows [L][N] (FP32), and the open slice's spike
// entries (n_pending x 4 B).  The connection table is not part of it: it is
// redrawn from the configuration by sd_build_connections.
struct StateHeader {
  char magic[8];
  uint64_t cfg_hash;
  int64_t N, t_now, rb_hi, pend_t0, slices, n_pending, rec_read;
  int32_t L, pend_open, count_mode, overflow;
  uint64_t counters[4];
};
constexpr char kStateMagic[8] = {'S', 'D', 'S', 'T', 'A', 'T', 'E', '1'};

uint64_t config_hash(const sd_config& g) {
  uint64_t h = 1469598103934665603ULL;  // FNV-1a over the fields, one by one
  auto mix = [&](const void* p, size_t n) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ULL;
  };
#define SD_MIX(f) mix(&g.f, sizeof g.f)
  SD_MIX(model); SD_MIX(wform); SD_MIX(n_exc); SD_MIX(n_inh); SD_MIX(n_src_exc);
  SD_MIX(n_src_inh); SD_MIX(k_exc); SD_MIX(k_inh); SD_MIX(d_lo); SD_MIX(d_hi); SD_MIX(d_min);
  SD_MIX(d_max); SD_MIX(ring_len); SD_MIX(h); SD_MIX(w_exc); SD_MIX(w_cv); SD_MIX(g);
  SD_MIX(tau_m); SD_MIX(c_m); SD_MIX(tau_syn); SD_MIX(e_l); SD_MIX(v_th); SD_MIX(v_reset);
  SD_MIX(t_ref); SD_MIX(i_e); SD_MIX(v0_lo); SD_MIX(v0_hi); SD_MIX(drive_rate_hz);
  SD_MIX(drive_w); SD_MIX(src_rate_hz); SD_MIX(seed); SD_MIX(block_neurons);
#undef SD_MIX
  return h;
}
}  // namespace

extern "C" {

sd_status sd_save_state(sd_ctx* c, void* h_buf, size_t cap, size_t* used) {
  if (!c || !used) return SD_EINVAL;
  if (c->cfg.plastic)
    return fail(c, SD_EUNSUPPORTED, "checkpoints of plastic nets (their weights are state)");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int32_t L = c->cfg.ring_len;
  int64_t n_pend = 0;
  if (c->pend_open && !open_loop(c->cfg)) {
    int32_t cnt = 0;
    HIP_TRY(c, hipMemcpy(&cnt, c->cnt3 + c->ci, 4, hipMemcpyDeviceToHost));
    n_pend = std::min<int64_t>(cnt, c->list_cap);
  }
  const size_t cell = 4;  // FP32 ring cells
  const size_t need = sizeof(StateHeader) + (size_t)c->N * 16 + (size_t)L * c->N * cell +
                      (size_t)n_pend * 4;
  *used = need;
  if (!h_buf) return SD_OK;
  if (cap < need) return fail(c, SD_EINVAL, "buffer of %zu B < %zu needed", cap, need);
  StateHeader hd;
  std::memset(&hd, 0, sizeof hd);
  std::memcpy(hd.magic, kStateMagic, 8);
  hd.cfg_hash = config_hash(c->cfg);
  hd.N = c->N;
  hd.t_now = c->t_now;
  hd.rb_hi = c->rb_hi;
  hd.pend_t0 = c->pend_t0;
  hd.slices = c->slices;
  hd.n_pending = n_pend;
  hd.rec_read = c->rec_read;
  hd.L = L;
  hd.pend_open = c->pend_open ? 1 : 0;
  hd.count_mode = c->count_mode;
  HIP_TRY(c, hipMemcpy(hd.counters, c->counters, 32, hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(&hd.overflow, c->overflow, 4, hipMemcpyDeviceToHost));
  char* p = (char*)h_buf;
  std::memcpy(p, &hd, sizeof hd);
  p += sizeof hd;
  const size_t n4 = (size_t)c->N * 4;
  HIP_TRY(c, hipMemcpy(p, c->V, n4, hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(p + n4, c->y1, n4, hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(p + 2 * n4, c->y2, n4, hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(p + 3 * n4, c->r, n4, hipMemcpyDeviceToHost));
  p += 4 * n4;
  HIP_TRY(c, hipMemcpy(p, c->rb, (size_t)L * n4, hipMemcpyDeviceToHost));
  p += (size_t)L * c->N * cell;
  if (n_pend > 0) HIP_TRY(c, hipMemcpy(p, c->list[c->cur], (size_t)n_pend * 4, hipMemcpyDeviceToHost));
  return SD_OK;
}

sd_status sd_load_state(sd_ctx* c, const void* h_buf, size_t n) {
  if (!c || !h_buf) return SD_EINVAL;
  if (c->cfg.plastic)
    return fail(c, SD_EUNSUPPORTED, "checkpoints of plastic nets (their weights are state)");
  if (!c->built) return fail(c, SD_ESTATE, "build_connections first");
  if (n < sizeof(StateHeader)) return fail(c, SD_EINVAL, "state buffer too short");
  StateHeader hd;
  std::memcpy(&hd, h_buf, sizeof hd);
  if (std::memcmp(hd.magic, kStateMagic, 8) != 0) return fail(c, SD_EINVAL, "not a state buffer");
  if (hd.cfg_hash != config_hash(c->cfg) || hd.N != c->N || hd.L != c->cfg.ring_len)
    return fail(c, SD_EINVAL, "state was saved from a different configuration");
  const size_t n4 = (size_t)c->N * 4;
  const size_t cell = 4;
  const size_t need =
      sizeof hd + 4 * n4 + (size_t)hd.L * c->N * cell + (size_t)hd.n_pending * 4;
  if (n < need || hd.n_pending < 0 || hd.n_pending > c->list_cap)
    return fail(c, SD_EINVAL, "state buffer holds %zu B, %zu needed", n, need);
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const char* p = (const char*)h_buf + sizeof hd;
  HIP_TRY(c, hipMemcpy(c->V, p, n4, hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(c->y1, p + n4, n4, hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(c->y2, p + 2 * n4, n4, hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(c->r, p + 3 * n4, n4, hipMemcpyHostToDevice));
  p += 4 * n4;
  HIP_TRY(c, hipMemcpy(c->rb, p, (size_t)hd.L * n4, hipMemcpyHostToDevice));
  p += (size_t)hd.L * c->N * cell;
  // the open slice's list goes to list 0 with counter 0; counter 1 (the
  // next list's) must be zero
  c->cur = 0;
  c->ci = 0;
  const int32_t cnt[3] = {(int32_t)hd.n_pending, 0, 0};
  HIP_TRY(c, hipMemcpy(c->cnt3, cnt, 12, hipMemcpyHostToDevice));
  if (hd.n_pending > 0)
    HIP_TRY(c, hipMemcpy(c->list[0], p, (size_t)hd.n_pending * 4, hipMemcpyHostToDevice));
  // the raster is not saved: it restarts empty
  hd.counters[3] = 0;
  HIP_TRY(c, hipMemcpy(c->counters, hd.counters, 32, hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(c->overflow, &hd.overflow, 4, hipMemcpyHostToDevice));
  c->t_now = hd.t_now;
  c->rb_hi = hd.rb_hi;
  c->pend_t0 = hd.pend_t0;
  c->pend_open = hd.pend_open != 0;
  c->slices = hd.slices;
  c->count_mode = hd.count_mode;
  c->rec_read = 0;
  return SD_OK;
}

sd_status sd_get_spikes(sd_ctx* c, int64_t* h_step, uint32_t* h_id, int64_t cap, int64_t* n) {
  if (!c || !n) return SD_EINVAL;
  *n = 0;
  if (c->rec_cap == 0) return fail(c, SD_ESTATE, "spike recording is off");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  unsigned long long total = 0;
  HIP_TRY(c, hipMemcpy(&total, c->counters + 3, 8, hipMemcpyDeviceToHost));
  const int64_t avail = std::min<int64_t>((int64_t)total, c->rec_cap) - c->rec_read;
  const int64_t m = std::min<int64_t>(avail, cap);
  if (m > 0) {
    std::vector<uint2> buf((size_t)m);
    HIP_TRY(c, hipMemcpy(buf.data(), c->rec + c->rec_read, (size_t)m * 8, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < m; ++i) {
      if (h_step) h_step[i] = buf[i].x;
      if (h_id) h_id[i] = buf[i].y;
    }
    c->rec_read += m;
  }
  *n = std::max<int64_t>(m, 0);
  return (int64_t)total > c->rec_cap ? SD_EOVERFLOW : SD_OK;
}

sd_status sd_get_pending(sd_ctx* c, uint32_t* h_src, uint8_t* h_lag, int64_t cap, int64_t* n,
                         int64_t* slice_t0) {
  if (!c || !n) return SD_EINVAL;
  *n = 0;
  if (slice_t0) *slice_t0 = c->pend_open ? c->pend_t0 : -1;
  if (!c->pend_open || open_loop(c->cfg)) return SD_OK;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  int32_t cnt = 0;
  HIP_TRY(c, hipMemcpy(&cnt, c->cnt3 + c->ci, 4, hipMemcpyDeviceToHost));
  const int64_t nl = std::min<int64_t>(cnt, c->list_cap);
  std::vector<uint32_t> all((size_t)nl);
  if (nl > 0)
    HIP_TRY(c, hipMemcpy(all.data(), c->list[c->cur], (size_t)nl * 4, hipMemcpyDeviceToHost));
  if (c->cfg.plastic) {  // one entry per neuron with its lags as a mask
    std::vector<uint32_t> lm((size_t)nl);
    if (nl > 0)
      HIP_TRY(c, hipMemcpy(lm.data(), c->aux[c->cur], (size_t)nl * 4, hipMemcpyDeviceToHost));
    std::vector<uint32_t> ex;
    for (int64_t i = 0; i < nl; ++i)
      for (int l = 0; l < 32; ++l)
        if ((lm[(size_t)i] >> l) & 1u) ex.push_back((all[(size_t)i] & ~31u) | (uint32_t)l);
    all.swap(ex);
  }
  // blocks append in any order: sort by (lag, src)
  std::sort(all.begin(), all.end(), [](uint32_t x, uint32_t y) {
    const uint32_t lx = x & 31u, ly = y & 31u;
    return lx != ly ? lx < ly : (x >> 5) < (y >> 5);
  });
  const int64_t m = std::min<int64_t>((int64_t)all.size(), cap);
  for (int64_t i = 0; i < m; ++i) {
    if (h_src) h_src[i] = all[i] >> 5;
    if (h_lag) h_lag[i] = (uint8_t)(all[i] & 31u);
  }
  *n = (int64_t)all.size();
  return SD_OK;
}

// Host-side gather of the whole table into canonical (source, target, draw)
// order: meant for small networks (tests); large ones use sd_export_block.
sd_status sd_export_connections(sd_ctx* c, int64_t* h_row, int32_t* h_tgt, uint8_t* h_dly,
                                float* h_w) {
  if (!c || !h_row) return SD_EINVAL;
  if (!c->built) return fail(c, SD_ESTATE, "build_connections first");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (c->sm) {
    // source-major: segments are contiguous; their order is the fill's, so
    // sort each by (target, delay, weight) for a canonical export
    // a source's part segments are adjacent: its row starts at part 0
    std::vector<unsigned long long> rp((size_t)c->M);
    HIP_TRY(c, hipMemcpy(rp.data(), c->row64, (size_t)c->M * 8, hipMemcpyDeviceToHost));
    for (int64_t s = 0; s <= c->n_src; ++s) h_row[s] = (int64_t)rp[(size_t)(s * c->H)];
    if (!h_tgt && !h_dly && !h_w) return SD_OK;
    const sd_config& g = c->cfg;
    const bool f32 = g.wform == SD_W_FP32;
    std::vector<uint32_t> td((size_t)c->n_syn);
    std::vector<uint8_t> wb((size_t)c->n_syn * (f32 ? 4 : 1));
    if (c->n_syn) {
      HIP_TRY(c, hipMemcpy(td.data(), c->tw, td.size() * 4, hipMemcpyDeviceToHost));
      HIP_TRY(c, hipMemcpy(wb.data(), c->wbits, wb.size(), hipMemcpyDeviceToHost));
    }
    const uint32_t tmask = (1u << c->tbits) - 1u;
    const uint32_t dmask = (1u << (kRecWordBits - c->tbits)) - 1u;
    struct Ent { int32_t t; uint8_t d; float w; };
    std::vector<Ent> seg;
    for (int64_t s = 0; s < c->n_src; ++s) {
      const float mu = s < c->src_e_end ? c->mu_e : c->mu_i;
      seg.clear();
      for (int32_t part = 0; part < c->H; ++part)
      for (int64_t e = (int64_t)rp[(size_t)(s * c->H + part)];
           e < (int64_t)rp[(size_t)(s * c->H + part + 1)]; ++e) {
        Ent x;
        const uint32_t w0 = td[(size_t)e];
        x.t = (int32_t)(((int64_t)part << c->tbits) | (w0 & tmask));
        x.d = (uint8_t)(g.d_min + (int)((w0 >> c->tbits) & dmask));
        if (f32) {
          std::memcpy(&x.w, wb.data() + (size_t)e * 4, 4);
        } else {
          const uint32_t h = ((w0 >> kRecWordBits) << 8) | wb[(size_t)e];
          const uint32_t u = h << 16;
          float d;
          std::memcpy(&d, &u, 4);
          x.w = g.wform == SD_W_BF16 ? d : std::fma(mu, d, mu);
        }
        seg.push_back(x);
      }
      std::sort(seg.begin(), seg.end(), [](const Ent& a, const Ent& b) {
        if (a.t != b.t) return a.t < b.t;
        if (a.d != b.d) return a.d < b.d;
        return a.w < b.w;
      });
      for (size_t i = 0; i < seg.size(); ++i) {
        const int64_t at = h_row[s] + (int64_t)i;
        if (h_tgt) h_tgt[at] = seg[i].t;
        if (h_dly) h_dly[at] = seg[i].d;
        if (h_w) h_w[at] = seg[i].w;
      }
    }
    return SD_OK;
  }
  std::vector<uint32_t> rp((size_t)c->M);
  HIP_TRY(c, hipMemcpy(rp.data(), c->row, (size_t)c->M * 4, hipMemcpyDeviceToHost));
  const int64_t S = c->n_src;
  h_row[0] = 0;
  for (int64_t s = 0; s < S; ++s) {
    int64_t deg = 0;
    for (int32_t b = 0; b < c->NB; ++b)
      deg += rp[(size_t)(s * c->NB + b + 1)] - rp[(size_t)(s * c->NB + b)];
    h_row[s + 1] = h_row[s] + deg;
  }
  if (!h_tgt && !h_dly && !h_w) return SD_OK;
  const sd_config& g = c->cfg;
  const int rb = g.wform == SD_W_FP32 ? 8 : 4;
  std::vector<uint8_t> rec((size_t)c->n_syn * rb), dl((size_t)c->n_syn);
  if (c->n_syn) {
    HIP_TRY(c, hipMemcpy(rec.data(), c->syn, rec.size(), hipMemcpyDeviceToHost));
    if (g.wform != SD_W_BF16_PACKED)
      HIP_TRY(c, hipMemcpy(dl.data(), c->syn_dly, dl.size(), hipMemcpyDeviceToHost));
  }
  for (int64_t s = 0; s < S; ++s) {
    int64_t at = h_row[s];
    const float mu = s < c->src_e_end ? c->mu_e : c->mu_i;
    for (int32_t b = 0; b < c->NB; ++b) {
      for (uint32_t e = rp[(size_t)(s * c->NB + b)]; e < rp[(size_t)(s * c->NB + b + 1)]; ++e, ++at) {
        int32_t t;
        float w;
        uint8_t d;
        decode_record(g, rec.data(), dl.data(), e, b, c->B, mu, &t, &w, &d);
        if (h_tgt) h_tgt[at] = t;
        if (h_w) h_w[at] = w;
        if (h_dly) h_dly[at] = d;
      }
    }
  }
  return SD_OK;
}

sd_status sd_export_segments(sd_ctx* c, int64_t src, int64_t* h_start, int64_t* h_len) {
  if (!c || !h_start || !h_len || src < 0 || src >= c->n_src) return SD_EINVAL;
  if (!c->built) return fail(c, SD_ESTATE, "build_connections first");
  if (c->sm) return fail(c, SD_EUNSUPPORTED, "source-major layout has no per-block segments");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int32_t b = 0; b < c->NB; ++b) {
    uint32_t p[2];
    HIP_TRY(c, hipMemcpy(p, c->row + (size_t)src * c->NB + b, 8, hipMemcpyDeviceToHost));
    h_start[b] = p[0];
    h_len[b] = (int64_t)p[1] - p[0];
  }
  return SD_OK;
}

sd_status sd_host_tables(const sd_config* cfg, float* h_we, float* h_wi, uint32_t* h_thr,
                         int32_t* n_thr) {
  std::string why;
  if (check_config(cfg, &why) != SD_OK) return SD_EINVAL;
  std::vector<float> we(65536), wi(65536);
  quantile_weights(*cfg, we.data(), wi.data());
  if (cfg->w_cv == 0.0) {
    std::fill(we.begin(), we.end(), (float)cfg->w_exc);
    std::fill(wi.begin(), wi.end(), (float)(-cfg->g * cfg->w_exc));
  }
  // decode to the storage form
  const float mu_e = (float)cfg->w_exc, mu_i = (float)(-cfg->g * cfg->w_exc);
  for (int i = 0; i < 65536; ++i) {
    if (cfg->wform == SD_W_BF16) {
      const uint32_t be = (uint32_t)bf16_bits_rne(we[i]) << 16, bi = (uint32_t)bf16_bits_rne(wi[i]) << 16;
      std::memcpy(&we[i], &be, 4);
      std::memcpy(&wi[i], &bi, 4);
    } else if (cfg->wform == SD_W_BF16_RESID || cfg->wform == SD_W_BF16_PACKED) {
      const uint32_t de = (uint32_t)resid_bits(we[i], mu_e) << 16, di = (uint32_t)resid_bits(wi[i], mu_i) << 16;
      float fe, fi;
      std::memcpy(&fe, &de, 4);
      std::memcpy(&fi, &di, 4);
      we[i] = (float)((double)mu_e + (double)mu_e * (double)fe);
      wi[i] = (float)((double)mu_i + (double)mu_i * (double)fi);
    }
  }
  if (h_we) std::memcpy(h_we, we.data(), 65536 * 4);
  if (h_wi) std::memcpy(h_wi, wi.data(), 65536 * 4);
  uint32_t thr[kMaxThr];
  const int n = poisson_table(cfg->drive_rate_hz * cfg->h * 1e-3, thr, kMaxThr);
  if (h_thr) std::memcpy(h_thr, thr, sizeof thr);
  if (n_thr) *n_thr = n;
  return SD_OK;
}

sd_status sd_export_block(sd_ctx* c, int32_t b, int64_t* h_row, int32_t* h_tgt, uint8_t* h_dly,
                          float* h_w, int64_t* n_out) {
  if (!c || !h_row || b < 0 || b >= c->NB) return SD_EINVAL;
  if (!c->built) return fail(c, SD_ESTATE, "build_connections first");
  if (c->sm) return fail(c, SD_EUNSUPPORTED, "source-major layout has no block regions");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int64_t S = c->n_src;
  // the block's (start, count) column of the segment pointers
  std::vector<uint2> col((size_t)S);
  HIP_TRY(c, hipMemcpy2D(col.data(), sizeof(uint2), c->seg + b, (size_t)c->NB * sizeof(uint2),
                         sizeof(uint2), (size_t)S, hipMemcpyDeviceToHost));
  h_row[0] = 0;
  for (int64_t s = 0; s < S; ++s) h_row[s + 1] = h_row[s] + col[(size_t)s].y;
  const int64_t tot = h_row[S];
  if (n_out) *n_out = tot;
  if (!h_tgt || tot == 0) return SD_OK;
  const sd_config& g = c->cfg;
  const int rb = g.wform == SD_W_FP32 ? 8 : 4;
  const bool has_dly = g.wform != SD_W_BF16_PACKED;
  // gather the block's segments source by source on the device
  int64_t* d_off = nullptr;
  char* d_out = nullptr;
  hipError_t e = hipMalloc((void**)&d_off, (size_t)S * 8);
  if (e == hipSuccess) e = hipMalloc((void**)&d_out, (size_t)tot * (rb + 1));
  if (e == hipSuccess) e = hipMemcpy(d_off, h_row, (size_t)S * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = launch_gather_block(c->stream, c->seg, S, c->NB, b, d_off, c->syn,
                            has_dly ? c->syn_dly : nullptr, rb, d_out,
                            has_dly ? (uint8_t*)(d_out + (size_t)tot * rb) : nullptr);
  std::vector<uint8_t> rec((size_t)tot * rb), dl((size_t)tot);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = hipMemcpy(rec.data(), d_out, rec.size(), hipMemcpyDeviceToHost);
  if (e == hipSuccess && has_dly)
    e = hipMemcpy(dl.data(), d_out + (size_t)tot * rb, dl.size(), hipMemcpyDeviceToHost);
  if (d_off) (void)hipFree(d_off);
  if (d_out) (void)hipFree(d_out);
  if (e != hipSuccess) return fail(c, SD_EHIP, "block export failed: %s", hipGetErrorString(e));
  for (int64_t s = 0; s < S; ++s) {
    const float mu = s < c->src_e_end ? c->mu_e : c->mu_i;
    for (int64_t k = h_row[s]; k < h_row[s + 1]; ++k)
      decode_record(g, rec.data(), dl.data(), (uint32_t)k, b, c->B, mu, &h_tgt[k], &h_w[k],
                    &h_dly[k]);
  }
  return SD_OK;
}

sd_status sd_get_tables(sd_ctx* c, float* h_we, float* h_wi, uint32_t* h_thr, int32_t* n_thr,
                        double* h_prop, float* h_prop32) {
  if (!c) return SD_EINVAL;
  if (h_we) std::memcpy(h_we, c->we_h.data(), 65536 * 4);
  if (h_wi) std::memcpy(h_wi, c->wi_h.data(), 65536 * 4);
  if (h_thr) std::memcpy(h_thr, c->thr_h, sizeof(uint32_t) * kMaxThr);
  if (n_thr) *n_thr = c->n_thr;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (h_prop) HIP_TRY(c, hipMemcpy(h_prop, c->prop64, 7 * 8, hipMemcpyDeviceToHost));
  if (h_prop32) HIP_TRY(c, hipMemcpy(h_prop32, c->prop32, 8 * 4, hipMemcpyDeviceToHost));
  return SD_OK;
}

// ---------------------------------------------------------------------------
// batched networks
// ---------------------------------------------------------------------------
namespace {
sd_status bfail(sd_batch* bt, sd_status st, const std::string& msg) {
  if (bt) bt->err = msg;
  return st;
}
}  // namespace

sd_status sd_batch_create(const sd_config* cfgs, int32_t n, void* hip_stream, sd_batch** out) {
  if (!out) return SD_EINVAL;
  *out = nullptr;
  auto* bt = new sd_batch;
  *out = bt;
  bt->stream = (hipStream_t)hip_stream;
  if (!cfgs || n < 1) return bfail(bt, SD_EINVAL, "empty batch");
  const sd_config& c0 = cfgs[0];
  for (int32_t i = 0; i < n; ++i) {
    const sd_config& ci = cfgs[i];
    if (ci.model != c0.model || ci.wform != c0.wform || ci.h != c0.h || ci.d_min != c0.d_min)
      return bfail(bt, SD_EINVAL,
                   "member " + std::to_string(i) + ": model, weight form, h and d_min must match");
    if (open_loop(ci))
      return bfail(bt, SD_EUNSUPPORTED, "member " + std::to_string(i) + ": open loop");
    if (ci.plastic)
      return bfail(bt, SD_EUNSUPPORTED, "member " + std::to_string(i) + ": plastic synapses");
  }
  std::vector<int2> blocks;
  size_t lds = 0;
  for (int32_t i = 0; i < n; ++i) {
    sd_ctx* c = nullptr;
    const sd_status st = sd_create(&cfgs[i], hip_stream, nullptr, 0, &c);
    if (st != SD_OK) {
      const std::string m = "member " + std::to_string(i) + ": " + sd_last_error(c);
      sd_destroy(c);
      return bfail(bt, st, m);
    }
    bt->nets.push_back(c);
    if (c->sm)
      return bfail(bt, SD_EUNSUPPORTED, "member " + std::to_string(i) +
                                            ": batches hold block-major networks only");
    for (int32_t b = 0; b < c->NB; ++b) blocks.push_back(make_int2(i, b));
    lds = std::max(lds, slice_lds_bytes(c->B, cfgs[i].d_min, cfgs[i].d_max));
  }
  const hipError_t e = launcher_init(bt->lau, n, 256, xcd_map(blocks), lds, c0.wform);
  if (e != hipSuccess)
    return bfail(bt, SD_EHIP, std::string("launcher set-up failed: ") + hipGetErrorString(e));
  return SD_OK;
}

void sd_batch_destroy(sd_batch* bt) {
  if (!bt) return;
  if (bt->stream || !bt->nets.empty()) (void)hipStreamSynchronize(bt->stream);
  for (sd_ctx* c : bt->nets) sd_destroy(c);
  launcher_free(bt->lau);
  if (bt->gexec) (void)hipGraphExecDestroy(bt->gexec);
  if (bt->cap_stream) (void)hipStreamDestroy(bt->cap_stream);
  if (bt->g_args) (void)hipFree(bt->g_args);
  if (bt->g_host) (void)hipHostFree(bt->g_host);
  if (bt->g_ev) (void)hipEventDestroy(bt->g_ev);
  delete bt;
}

sd_status sd_batch_set_graph(sd_batch* bt, int32_t on) {
  if (!bt) return SD_EINVAL;
  bt->graph_on = on != 0;
  return SD_OK;
}

int64_t sd_batch_graph_launches(const sd_batch* bt) { return bt ? bt->g_launches : -1; }

const char* sd_batch_last_error(const sd_batch* bt) { return bt ? bt->err.c_str() : "null batch"; }

int32_t sd_batch_size(const sd_batch* bt) { return bt ? (int32_t)bt->nets.size() : 0; }

sd_ctx* sd_batch_member(sd_batch* bt, int32_t i) {
  if (!bt || i < 0 || i >= (int32_t)bt->nets.size()) return nullptr;
  return bt->nets[(size_t)i];
}

sd_status sd_batch_build(sd_batch* bt) {
  if (!bt) return SD_EINVAL;
  for (size_t i = 0; i < bt->nets.size(); ++i) {
    const sd_status st = sd_build_connections(bt->nets[i]);
    if (st != SD_OK)
      return bfail(bt, st, "member " + std::to_string(i) + ": " + sd_last_error(bt->nets[i]));
  }
  return SD_OK;
}

namespace {
// Capture, once: kGraphSlices batched launches reading their arguments from
// g_args, then the shift of those arguments to the next period.
sd_status batch_graph(sd_batch* bt) {
  if (bt->gexec) return SD_OK;
  const size_t n = bt->nets.size();
  const size_t bytes = (size_t)kGraphSlices * n * sizeof(sd::SliceArgs);
  hipError_t e = hipMalloc((void**)&bt->g_args, bytes);
  if (e == hipSuccess) e = hipHostMalloc((void**)&bt->g_host, bytes, hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&bt->g_ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&bt->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) return bfail(bt, SD_EHIP, std::string("graph set-up: ") + hipGetErrorString(e));
  const int64_t shift = (int64_t)kGraphSlices * bt->nets[0]->cfg.d_min;
  hipGraph_t g = nullptr;
  e = hipStreamBeginCapture(bt->cap_stream, hipStreamCaptureModeThreadLocal);
  for (int j = 0; j < kGraphSlices && e == hipSuccess; ++j)
    e = sd::launch_slice(bt->cap_stream, bt->g_args + (size_t)j * n, bt->lau.d_map,
                         bt->lau.n_blocks, bt->lau.lds, bt->lau.wform);
  if (e == hipSuccess)
    e = sd::launch_shift_args(bt->cap_stream, bt->g_args, (int32_t)(kGraphSlices * n), shift);
  const hipError_t e2 = hipStreamEndCapture(bt->cap_stream, &g);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipGraphInstantiate(&bt->gexec, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    bt->gexec = nullptr;
    return bfail(bt, SD_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
  }
  return SD_OK;
}

bool batch_steady(const sd_batch* bt) {
  for (const sd_ctx* c : bt->nets) {
    const sd_config& g = c->cfg;
    if (!c->pend_open || c->t_now % g.d_min != 0 || c->pend_t0 != c->t_now - g.d_min ||
        c->rb_hi != c->t_now - g.d_min + g.d_max)
      return false;
  }
  return true;
}

// Run reps * kGraphSlices steady-state slices through the captured graph.
sd_status batch_replay(sd_batch* bt, int64_t reps) {
  sd_status st = batch_graph(bt);
  if (st != SD_OK) return st;
  const size_t n = bt->nets.size();
  if (bt->g_pend) {
    const hipError_t e = hipEventSynchronize(bt->g_ev);  // staging free again
    if (e != hipSuccess) return bfail(bt, SD_EHIP, hipGetErrorString(e));
    bt->g_pend = false;
  }
  // arguments of the next period (advances every member by kGraphSlices)
  for (int j = 0; j < kGraphSlices; ++j)
    for (size_t i = 0; i < n; ++i) {
      const int32_t m = bt->nets[i]->cfg.d_min;
      st = next_fused_slice(bt->nets[i], m, &bt->g_host[(size_t)j * n + i]);
      if (st != SD_OK) return bfail(bt, st, sd_last_error(bt->nets[i]));
    }
  hipError_t e = hipMemcpyAsync(bt->g_args, bt->g_host, (size_t)kGraphSlices * n * sizeof(sd::SliceArgs),
                                hipMemcpyHostToDevice, bt->stream);
  if (e == hipSuccess) e = hipEventRecord(bt->g_ev, bt->stream);
  if (e != hipSuccess) return bfail(bt, SD_EHIP, hipGetErrorString(e));
  bt->g_pend = true;
  for (int64_t r = 0; r < reps; ++r) {
    e = hipGraphLaunch(bt->gexec, bt->stream);
    if (e != hipSuccess) return bfail(bt, SD_EHIP, std::string("graph launch: ") + hipGetErrorString(e));
    ++bt->g_launches;
  }
  // the host state after the further periods
  const int64_t k = (reps - 1) * kGraphSlices;
  for (sd_ctx* c : bt->nets) {
    const int64_t d = k * c->cfg.d_min;
    c->t_now += d;
    c->pend_t0 += d;
    c->rb_hi += d;
    c->slices += k;
  }
  return SD_OK;
}
}  // namespace

sd_status sd_batch_simulate_steps(sd_batch* bt, int64_t n_steps) {
  if (!bt || n_steps < 0) return SD_EINVAL;
  const size_t n = bt->nets.size();
  if (n == 0) return SD_OK;
  const int64_t t0 = bt->nets[0]->t_now;
  for (size_t i = 0; i < n; ++i) {
    if (!bt->nets[i]->built) return bfail(bt, SD_ESTATE, "build the batch first");
    if (bt->nets[i]->t_now != t0)
      return bfail(bt, SD_ESTATE, "members were advanced separately (t_now differs)");
  }
  const int32_t Dmin = bt->nets[0]->cfg.d_min;
  std::vector<SliceArgs> queue;  // n argument structs per fused launch
  auto flush = [&]() -> sd_status {
    if (!queue.empty()) {
      const hipError_t e =
          launcher_run(bt->lau, bt->stream, queue.data(), (int64_t)(queue.size() / n));
      if (e != hipSuccess) return bfail(bt, SD_EHIP, hipGetErrorString(e));
      queue.clear();
    }
    return SD_OK;
  };
  int64_t left = n_steps;
  while (left > 0) {
    const int64_t in_slice = bt->nets[0]->t_now % Dmin;
    if (in_slice != 0) {
      const int32_t m = (int32_t)std::min<int64_t>(left, Dmin - in_slice);
      sd_status st = flush();
      for (size_t i = 0; i < n && st == SD_OK; ++i) {
        st = sd_update_neurons(bt->nets[i], m);
        if (st != SD_OK) bfail(bt, st, sd_last_error(bt->nets[i]));
      }
      if (st != SD_OK) return st;
      left -= m;
      continue;
    }
    const int64_t period = (int64_t)kGraphSlices * Dmin;
    if (bt->graph_on && left >= 2 * period && batch_steady(bt)) {
      sd_status st = flush();
      if (st == SD_OK) st = batch_replay(bt, left / period);
      if (st != SD_OK) return st;
      left -= (left / period) * period;
      continue;
    }
    const int32_t m = (int32_t)std::min<int64_t>(left, Dmin);
    for (size_t i = 0; i < n; ++i) {
      SliceArgs a;
      const sd_status st = next_fused_slice(bt->nets[i], m, &a);
      if (st != SD_OK) return bfail(bt, st, sd_last_error(bt->nets[i]));
      queue.push_back(a);
    }
    left -= m;
  }
  return flush();
}

sd_status sd_batch_simulate(sd_batch* bt, double t_ms) {
  if (!bt || bt->nets.empty() || !(t_ms >= 0.0)) return SD_EINVAL;
  return sd_batch_simulate_steps(bt, (int64_t)std::llround(t_ms / bt->nets[0]->cfg.h));
}

}  // extern "C"
