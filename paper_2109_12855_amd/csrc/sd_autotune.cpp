// sd_autotune.cpp -- block-size autotuner for single networks and batches,
// and the binning parameters of source-major networks.
//
// A client of the C ABI: every candidate is an ordinary context (or batch),
// created, built and timed with HIP events on a private stream, then
// destroyed.  The block size sets how many synapses of a spike a target
// block receives per segment (K * B / N): small blocks fill the device with
// workgroups but walk short segments, large blocks walk long segments with
// fewer workgroups and fewer resident per compute unit.  Which side wins
// depends on the network sizes and rates, so it is measured.
//
// For a batch two rules give a candidate per target T: every member split
// into T blocks (uniform), or member i into T * K_i / mean(K) blocks
// (balanced: the events per block of a slice grow with the in-degree, and
// one launch waits for its slowest blocks).
//
// A source-major network's binning pass sorts each slice's events into one
// bucket per target block, in regions of bin_cap records per (block,
// binning workgroup): sd_autotune_bins times block sizes (the buckets) and
// region capacities together.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "../../include/sdeliver.h"

namespace {

uint64_t fnv(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ULL;
  return h;
}

// Key of a tuning problem: the networks (field by field, without the block
// size and the recording options), the candidates and the timing length.
uint64_t problem_hash(const sd_config* cfgs, int32_t n, const int32_t* targets, int32_t nt,
                      int32_t warmup, int32_t slices) {
  uint64_t h = 1469598103934665603ULL;
  for (int32_t i = 0; i < n; ++i) {
    const sd_config& g = cfgs[i];
#define SD_MIX(f) h = fnv(h, &g.f, sizeof g.f)
    SD_MIX(model); SD_MIX(wform); SD_MIX(n_exc); SD_MIX(n_inh); SD_MIX(n_src_exc);
    SD_MIX(n_src_inh); SD_MIX(k_exc); SD_MIX(k_inh); SD_MIX(d_lo); SD_MIX(d_hi); SD_MIX(d_min);
    SD_MIX(d_max); SD_MIX(ring_len); SD_MIX(h); SD_MIX(w_exc); SD_MIX(w_cv); SD_MIX(g);
    SD_MIX(tau_m); SD_MIX(c_m); SD_MIX(tau_syn); SD_MIX(e_l); SD_MIX(v_th); SD_MIX(v_reset);
    SD_MIX(t_ref); SD_MIX(i_e); SD_MIX(v0_lo); SD_MIX(v0_hi); SD_MIX(drive_rate_hz);
    SD_MIX(drive_w); SD_MIX(src_rate_hz); SD_MIX(seed); SD_MIX(layout);
#undef SD_MIX
  }
  h = fnv(h, targets, sizeof(int32_t) * (size_t)nt);
  const uint32_t rules = 2;  // uniform and balanced candidates
  h = fnv(h, &rules, sizeof rules);
  const uint32_t graph = n > 1 ? 1u : 0u;  // batches are timed through the captured graph
  h = fnv(h, &graph, sizeof graph);
  h = fnv(h, &warmup, sizeof warmup);
  h = fnv(h, &slices, sizeof slices);
  return h;
}

std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t p;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) {
    (void)hipGetLastError();
    return "unknown";
  }
  std::string a = p.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

// --- cache: a JSON object {"<arch>:<n>:<hash>": {"target": T,
// "us_per_slice": x, "block_neurons": [..]}, ...}, read and appended with
// plain string handling (this file writes every entry it reads back).
std::string read_file(const char* path) {
  std::string s;
  FILE* f = std::fopen(path, "rb");
  if (!f) return s;
  char buf[4096];
  size_t k;
  while ((k = std::fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, k);
  std::fclose(f);
  return s;
}

bool cache_lookup(const std::string& text, const std::string& key, int32_t n,
                  std::vector<int32_t>* bn, double* us, int32_t* bin_cap = nullptr) {
  const size_t at = text.find("\"" + key + "\"");
  if (at == std::string::npos) return false;
  const size_t end = text.find('}', at);
  const size_t pu = text.find("\"us_per_slice\":", at);
  const size_t pb = text.find("\"block_neurons\": [", at);
  if (end == std::string::npos || pu == std::string::npos || pb == std::string::npos || pu > end ||
      pb > end)
    return false;
  if (bin_cap) {
    const size_t pc = text.find("\"bin_cap\":", at);
    if (pc == std::string::npos || pc > end) return false;
    *bin_cap = (int32_t)std::strtol(text.c_str() + pc + 10, nullptr, 10);
  }
  *us = std::strtod(text.c_str() + pu + 15, nullptr);
  bn->clear();
  const char* c = text.c_str() + pb + 18;
  while (*c && *c != ']') {
    char* next = nullptr;
    const long v = std::strtol(c, &next, 10);
    if (next == c) break;
    bn->push_back((int32_t)v);
    c = next;
    while (*c == ',' || *c == ' ') ++c;
  }
  return (int32_t)bn->size() == n;
}

bool cache_store(const char* path, const std::string& key, int32_t target, const char* rule,
                 double us, const std::vector<int32_t>& bn, int32_t bin_cap = -1) {
  std::string text = read_file(path);
  const size_t close = text.rfind('}');
  if (text.find('{') == std::string::npos || close == std::string::npos) text = "{\n}\n";
  const size_t last = text.rfind('}');
  const bool empty = text.find('"') == std::string::npos;
  char head[256];
  std::snprintf(head, sizeof head,
                "  \"%s\": {\"target\": %d, \"rule\": \"%s\", \"us_per_slice\": %.3f, ",
                key.c_str(), target, rule, us);
  std::string entry = std::string(empty ? "" : ",\n") + head;
  if (bin_cap >= 0) entry += "\"bin_cap\": " + std::to_string(bin_cap) + ", ";
  entry += "\"block_neurons\": [";
  for (size_t i = 0; i < bn.size(); ++i) entry += (i ? ", " : "") + std::to_string(bn[i]);
  entry += "]}\n";
  // drop the whitespace before the closing brace, then append the entry
  size_t cut = last;
  while (cut > 0 && (text[cut - 1] == '\n' || text[cut - 1] == ' ')) --cut;
  text = text.substr(0, cut) + (empty ? "\n" : "") + entry + "}\n";
  FILE* f = std::fopen(path, "wb");
  if (!f) return false;
  const bool ok = std::fwrite(text.data(), 1, text.size(), f) == text.size();
  return std::fclose(f) == 0 && ok;
}

// Block size of a network for a target of T blocks scaled by s (rounded, at
// least one block): ceil(N / blocks) rounded up to 64, lowered in steps of
// 64 until the layout fits (block-major for a batch member).
int32_t block_for(const sd_config& c, int32_t T, double s, bool batch) {
  const int64_t N = c.n_exc + c.n_inh;
  const int64_t nb = std::max<int64_t>(1, std::llround((double)T * s));
  int64_t b = (N + nb - 1) / nb;
  b = std::max<int64_t>(64, (b + 63) / 64 * 64);
  b = std::min<int64_t>(b, 1 << 16);
  for (; b >= 64; b -= 64) {
    sd_config t = c;
    t.block_neurons = (int32_t)b;
    if (batch) t.layout = SD_LAYOUT_BLOCK;
    sd_sizes z;
    if (sd_query_sizes(&t, &z) == SD_OK) return (int32_t)b;
  }
  return 0;
}

// Mean time of one slice over `slices` slices after `warmup`, or < 0.
double time_candidate(const std::vector<sd_config>& cfgs, int32_t warmup, int32_t slices) {
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return -1.0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const int32_t d_min = cfgs[0].d_min;
  double us = -1.0;
  if (cfgs.size() == 1) {
    sd_ctx* c = nullptr;
    bool ok = sd_create(&cfgs[0], s, nullptr, 0, &c) == SD_OK && sd_build_connections(c) == SD_OK;
    if (ok && cfgs[0].n_src_exc > 0)
      ok = sd_prepare_input(c, (int64_t)(warmup + slices + 2) * d_min) == SD_OK;
    ok = ok && sd_simulate_steps(c, (int64_t)warmup * d_min) == SD_OK;
    ok = ok && hipEventRecord(e0, s) == hipSuccess;
    ok = ok && sd_simulate_steps(c, (int64_t)slices * d_min) == SD_OK;
    ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
    float ms = 0.f;
    if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) us = ms * 1e3 / slices;
    sd_destroy(c);
  } else {
    sd_batch* b = nullptr;
    // batches run their steady-state slices from the captured graph, as the
    // tuned configuration will (the timed stretch spans several replays)
    bool ok = sd_batch_create(cfgs.data(), (int32_t)cfgs.size(), s, &b) == SD_OK &&
              sd_batch_build(b) == SD_OK && sd_batch_set_graph(b, 1) == SD_OK;
    ok = ok && sd_batch_simulate_steps(b, (int64_t)warmup * d_min) == SD_OK;
    ok = ok && hipEventRecord(e0, s) == hipSuccess;
    ok = ok && sd_batch_simulate_steps(b, (int64_t)slices * d_min) == SD_OK;
    ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
    float ms = 0.f;
    if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) us = ms * 1e3 / slices;
    sd_batch_destroy(b);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  (void)hipGetLastError();
  return us;
}

}  // namespace

extern "C" {

sd_status sd_autotune(const sd_config* cfgs, int32_t n, const int32_t* targets, int32_t n_targets,
                      int32_t warmup, int32_t slices, const char* cache_path,
                      int32_t* h_block_neurons, double* us_per_slice) {
  if (!cfgs || n < 1 || !targets || n_targets < 1 || warmup < 0 || slices < 1 || !h_block_neurons)
    return SD_EINVAL;
  for (int32_t k = 0; k < n_targets; ++k)
    if (targets[k] < 1) return SD_EINVAL;
  char hx[17];
  std::snprintf(hx, sizeof hx, "%016llx",
                (unsigned long long)problem_hash(cfgs, n, targets, n_targets, warmup, slices));
  const std::string key = device_arch() + ":" + std::to_string(n) + ":" + hx;
  std::vector<int32_t> best;
  double best_us = -1.0;
  if (cache_path && cache_lookup(read_file(cache_path), key, n, &best, &best_us)) {
    std::copy(best.begin(), best.end(), h_block_neurons);
    if (us_per_slice) *us_per_slice = best_us;
    return SD_OK;
  }
  const bool batch = n > 1;
  double k_mean = 0.0;
  for (int32_t i = 0; i < n; ++i) k_mean += (double)(cfgs[i].k_exc + cfgs[i].k_inh);
  k_mean = std::max(k_mean / n, 1.0);
  int32_t best_t = 0;
  const char* best_rule = "uniform";
  for (int32_t k = 0; k < n_targets; ++k) {
    for (int rule = 0; rule < (batch ? 2 : 1); ++rule) {
      std::vector<sd_config> cand(cfgs, cfgs + n);
      std::vector<int32_t> bn((size_t)n);
      bool ok = true;
      for (int32_t i = 0; i < n && ok; ++i) {
        const double s = rule ? (double)(cfgs[i].k_exc + cfgs[i].k_inh) / k_mean : 1.0;
        bn[(size_t)i] = block_for(cfgs[i], targets[k], s, batch);
        ok = bn[(size_t)i] > 0;
        cand[(size_t)i].block_neurons = bn[(size_t)i];
        cand[(size_t)i].record_spikes = 0;
      }
      if (!ok) continue;
      const double us = time_candidate(cand, warmup, slices);
      if (us > 0.0 && (best_us < 0.0 || us < best_us)) {
        best_us = us;
        best = bn;
        best_t = targets[k];
        best_rule = rule ? "balanced" : "uniform";
      }
    }
  }
  if (best_us < 0.0) return SD_EUNSUPPORTED;
  std::copy(best.begin(), best.end(), h_block_neurons);
  if (us_per_slice) *us_per_slice = best_us;
  if (cache_path && !cache_store(cache_path, key, best_t, best_rule, best_us, best))
    return SD_EINVAL;
  return SD_OK;
}

sd_status sd_autotune_bins(const sd_config* cfg, const int32_t* targets, int32_t n_targets,
                           const double* cap_scales, int32_t n_scales, int32_t warmup,
                           int32_t slices, const char* cache_path, int32_t* block_neurons,
                           int32_t* bin_cap, double* us_per_slice) {
  if (!cfg || !targets || n_targets < 1 || !cap_scales || n_scales < 1 || warmup < 0 ||
      slices < 1 || !block_neurons || !bin_cap)
    return SD_EINVAL;
  for (int32_t k = 0; k < n_targets; ++k)
    if (targets[k] < 1) return SD_EINVAL;
  for (int32_t k = 0; k < n_scales; ++k)
    if (!(cap_scales[k] > 0.0) || !(cap_scales[k] < 1e6)) return SD_EINVAL;
  {
    sd_config t = *cfg;
    t.block_neurons = 0;
    t.bin_cap = 0;
    sd_sizes z;
    if (sd_query_sizes(&t, &z) != SD_OK || z.layout != SD_LAYOUT_SOURCE) return SD_EINVAL;
  }
  uint64_t h = problem_hash(cfg, 1, targets, n_targets, warmup, slices);
  h = fnv(h, cap_scales, sizeof(double) * (size_t)n_scales);
  char hx[17];
  std::snprintf(hx, sizeof hx, "%016llx", (unsigned long long)h);
  const std::string key = device_arch() + ":bins:" + hx;
  std::vector<int32_t> best;
  double best_us = -1.0;
  int32_t best_cap = 0;
  if (cache_path && cache_lookup(read_file(cache_path), key, 1, &best, &best_us, &best_cap)) {
    *block_neurons = best[0];
    *bin_cap = best_cap;
    if (us_per_slice) *us_per_slice = best_us;
    return SD_OK;
  }
  int32_t best_t = 0;
  std::vector<std::pair<int32_t, int32_t>> tried;
  for (int32_t k = 0; k < n_targets; ++k) {
    const int32_t b = block_for(*cfg, targets[k], 1.0, false);
    if (b <= 0) continue;
    sd_config cand = *cfg;
    cand.block_neurons = b;
    cand.bin_cap = 0;
    cand.record_spikes = 0;
    sd_sizes z;
    if (sd_query_sizes(&cand, &z) != SD_OK || z.layout != SD_LAYOUT_SOURCE) continue;
    for (int32_t q = 0; q < n_scales; ++q) {
      int64_t cap = (int64_t)std::ceil(cap_scales[q] * z.bin_cap);
      cap = std::min<int64_t>(1024, std::max<int64_t>(64, (cap + 63) / 64 * 64));
      const std::pair<int32_t, int32_t> pr(b, (int32_t)cap);
      if (std::find(tried.begin(), tried.end(), pr) != tried.end()) continue;
      tried.push_back(pr);
      cand.bin_cap = (int32_t)cap;
      sd_sizes zc;
      if (sd_query_sizes(&cand, &zc) != SD_OK) continue;
      const double us = time_candidate(std::vector<sd_config>(1, cand), warmup, slices);
      if (us > 0.0 && (best_us < 0.0 || us < best_us)) {
        best_us = us;
        best.assign(1, b);
        best_cap = (int32_t)cap;
        best_t = targets[k];
      }
    }
  }
  if (best_us < 0.0) return SD_EUNSUPPORTED;
  *block_neurons = best[0];
  *bin_cap = best_cap;
  if (us_per_slice) *us_per_slice = best_us;
  if (cache_path && !cache_store(cache_path, key, best_t, "bins", best_us, best, best_cap))
    return SD_EINVAL;
  return SD_OK;
}

}  // extern "C"
