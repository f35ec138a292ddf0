// sd_kernels.hip -- gfx950 kernels of the spike-delivery library.
//
// Hot path (one fused launch per slice of d_min steps):
//   k_slice1 (one network, arguments by value) / k_slice (a batch, arguments
//   in device memory): a workgroup owns one block of B target neurons.  It
//   first walks the target segments of every spike of the completed slice
//   (Alg. REF, Sec. 3.2) and adds each weight into an LDS copy of its
//   block's ring window (d_max rows x B neurons, 64-bit fixed point), then
//   advances its neurons through the next slice with the exact propagators
//   (Sec. 2.1), reading inputs straight from the LDS window, and finally
//   compacts the new spikes (each wave's ballot of a step kept as two mask
//   words, then a block scan of their bit counts) and appends them, ordered
//   (lag, neuron) within the block, to the slice's contiguous spike list.
//   Rows of the window that are due in later slices are written to the ring
//   in HBM by the threads without a neuron, during the update.
//   Source-major layout: k_bin first sorts the slice's events by target
//   block into binned records, walking its spikes' rows one target part at
//   a time; the slice kernel then accumulates those instead of walking
//   segments (k_slice1<form, true, dyn>).
//   k_shift_args moves the device-resident arguments of a captured batch
//   graph on by one period.  k_persist (opt-in) runs several slices in one
//   cooperative launch, each block's ring window kept in LDS across them,
//   with grid barriers between slices.
//
// Build (once, untimed, Sec. 2.2):
//   k_count / scan / k_fill lay out the block-major table: segment (src, b)
//   holds the synapses from src into target block b in (target, draw) order,
//   and the segments are stored source by source, so one spike's segments
//   for blocks 0, 1, 2, ... lie next to each other.  The blocks walking a
//   spike then read neighbouring pieces of one row of the table (shared
//   lines, open DRAM pages) rather than a piece of each block's own region.
//   k_fill ranks equal sources inside each chunk of draws with an LDS
//   bitonic sort, so the layout is deterministic.  k_seg_pairs stores the
//   segment pointers as (start, count) pairs in the same order: the blocks
//   resolving one spike read neighbouring words.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sd_internal.h"

namespace sd {

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11); counter (c0, c1, 0, 0), key (seed,
// stream).  Device-only implementation.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox(uint64_t seed, uint64_t stream, uint64_t c0, uint64_t c1,
                                       uint64_t out[4]) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t x0 = c0, x1 = c1, x2 = 0, x3 = 0, k0 = seed, k1 = stream;
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const uint64_t hi0 = __umul64hi(M0, x0), lo0 = M0 * x0;
    const uint64_t hi1 = __umul64hi(M1, x2), lo1 = M1 * x2;
    const uint64_t n0 = hi1 ^ x1 ^ k0, n2 = hi0 ^ x3 ^ k1;
    x0 = n0;
    x1 = lo1;
    x2 = n2;
    x3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

// floor(r * n / 2^64)
__device__ __forceinline__ uint64_t mul_range(uint64_t r, uint64_t n) { return __umul64hi(r, n); }

// ---------------------------------------------------------------------------
// setup kernels
// ---------------------------------------------------------------------------
// The once-per-run FP64 work: exact propagators of the linear subthreshold
// dynamics over one step, then their FP32 roundings for the update.
__global__ void k_propagators(int model, double h, double tau_m, double tau_syn, double c_m,
                              double i_e, double* p64, float* p32) {
  const double em = exp(-h / tau_m);
  double P11 = 0.0, P21 = 0.0, P22 = 0.0, P31 = 0.0, P32 = 0.0;
  const double P33 = em;
  const double P30 = -(tau_m / c_m) * expm1(-h / tau_m);
  double in_scale = 1.0;
  if (model == MODEL_ALPHA) {
    const double es = exp(-h / tau_syn);
    const double a = 1.0 / tau_syn - 1.0 / tau_m;  // rate difference
    const double x = a * h;
    P11 = es;
    P22 = es;
    P21 = h * es;
    P32 = (em - es) / (a * c_m);
    P31 = em * (-expm1(-x) - x * exp(-x)) / (a * a * c_m);
    in_scale = exp(1.0) / tau_syn;
  }
  const double v[7] = {P11, P21, P22, P31, P32, P33, P30};
  for (int i = 0; i < 7; ++i) p64[i] = v[i];
  for (int i = 0; i < 6; ++i) p32[i] = (float)v[i];
  p32[6] = (float)(P30 * i_e);
  p32[7] = (float)in_scale;
}

__global__ void k_init_state(int64_t N, uint64_t seed, double v0_lo, double v0_hi, float* V,
                             float* y1, float* y2, int32_t* r) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  uint64_t w[4];
  philox(seed, STREAM_INIT, (uint64_t)j, 0, w);
  const double u = (double)(w[0] >> 11) * 0x1.0p-53;
  V[j] = (float)__dadd_rn(v0_lo, __dmul_rn(v0_hi - v0_lo, u));
  y1[j] = 0.f;
  y2[j] = 0.f;
  r[j] = 0;
}

// ---------------------------------------------------------------------------
// connection build
// ---------------------------------------------------------------------------
struct Draw {
  uint32_t src;
  uint32_t dly;
  uint32_t widx;
  uint32_t inh;
};

__device__ __forceinline__ Draw draw_synapse(const BuildArgs& a, int64_t j, int32_t k) {
  uint64_t w[4];
  philox(a.seed, STREAM_SYN, (uint64_t)j, (uint64_t)k, w);
  Draw d;
  d.inh = k >= a.k_exc;
  d.src = d.inh ? (uint32_t)(a.src_i_base + (int64_t)mul_range(w[0], (uint64_t)a.src_i_n))
                : (uint32_t)mul_range(w[0], (uint64_t)a.src_e_n);
  d.dly = (uint32_t)(a.d_lo + (int32_t)mul_range(w[1], (uint64_t)a.n_dly));
  d.widx = (uint32_t)(w[2] >> 48);
  return d;
}

// histogram of (source, block) pairs; one workgroup per target
__global__ void __launch_bounds__(256) k_count(BuildArgs a) {
  const int64_t j = blockIdx.x;
  const int32_t b = (int32_t)(j / a.B);
  for (int32_t k = threadIdx.x; k < a.K; k += blockDim.x) {
    const Draw d = draw_synapse(a, j, k);
    atomicAdd(&a.row[(int64_t)d.src * a.NB + b], 1u);
  }
}

// three-phase exclusive scan of a u32 array (tiles of 4096)
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 4;
constexpr int kScanTile = kScanThreads * kScanPer;

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

// exclusive block scan of one value per thread; sh holds nthreads/64 + 1 words
template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* sh, T& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  T inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T t = __shfl_up(inc, d, 64);
    if (lane >= d) inc += t;
  }
  if (lane == 63) sh[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T acc = 0;
    for (int i = 0; i < nw; ++i) {
      const T x = sh[i];
      sh[i] = acc;
      acc += x;
    }
    sh[nw] = acc;
  }
  __syncthreads();
  const T res = inc - v + sh[w];
  total = sh[nw];
  __syncthreads();
  return res;
}

// The same scan with one barrier: every thread adds up the wave totals
// before its own wave.  sh must not be reused before the caller's next
// barrier.
template <typename T>
__device__ __forceinline__ T block_excl_scan1(T v, T* sh, T& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  T inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T t = __shfl_up(inc, d, 64);
    if (lane >= d) inc += t;
  }
  if (lane == 63) sh[w] = inc;
  __syncthreads();
  T before = 0, all = 0;
  for (int i = 0; i < nw; ++i) {
    const T x = sh[i];
    before += i < w ? x : (T)0;
    all += x;
  }
  total = all;
  return inc - v + before;
}

template <typename T>
__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(const T* data, int64_t n,
                                                            T* tile_sums) {
  __shared__ T sh[kScanThreads / 64 + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  T s = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i)
    if (base + i < n) s += data[base + i];
  T tot;
  block_excl_scan<T>(s, sh, tot);
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

template <typename T>
__global__ void __launch_bounds__(kScanThreads) k_scan_sums(T* tile_sums, int64_t n_tiles) {
  __shared__ T sh[kScanThreads / 64 + 1];
  T carry = 0;
  for (int64_t c0 = 0; c0 < n_tiles; c0 += kScanThreads) {
    const int64_t i = c0 + threadIdx.x;
    const T v = i < n_tiles ? tile_sums[i] : (T)0;
    T tot;
    const T ex = block_excl_scan<T>(v, sh, tot);
    if (i < n_tiles) tile_sums[i] = carry + ex;
    carry += tot;
  }
}

template <typename T>
__global__ void __launch_bounds__(kScanThreads) k_scan_apply(T* data, int64_t n,
                                                            const T* tile_sums) {
  __shared__ T sh[kScanThreads / 64 + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  T v[kScanPer];
  T s = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    v[i] = (base + i < n) ? data[base + i] : (T)0;
    s += v[i];
  }
  T tot;
  T run = block_excl_scan<T>(s, sh, tot) + tile_sums[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    if (base + i < n) data[base + i] = run;
    run += v[i];
  }
}

// Deterministic fill: workgroup b walks the draws of its block in
// (target, k) order, kFillChunk at a time; equal sources inside a chunk are
// ranked by an LDS bitonic sort of (src, position) keys, so each segment
// receives its synapses in draw order.  Only workgroup b touches the cursors
// (src, b) of its block.
__global__ void __launch_bounds__(kFillThreads) k_fill(BuildArgs a) {
  __shared__ uint64_t keys[kFillChunk];
  __shared__ uint32_t meta[kFillChunk];  // widx | inh << 16 | dly << 24
  const int32_t b = blockIdx.x;
  const int64_t j0 = (int64_t)b * a.B;
  const int64_t nb = (a.N - j0) < a.B ? (a.N - j0) : a.B;
  const int64_t n_el = nb * a.K;
  const int tid = threadIdx.x;
  for (int64_t c0 = 0; c0 < n_el; c0 += kFillChunk) {
    const int n_in = (int)((n_el - c0) < kFillChunk ? (n_el - c0) : kFillChunk);
    for (int i = tid; i < kFillChunk; i += kFillThreads) {
      if (i < n_in) {
        const int64_t e = c0 + i;
        const int64_t jl = e / a.K;
        const int32_t k = (int32_t)(e - jl * a.K);
        const Draw d = draw_synapse(a, j0 + jl, k);
        keys[i] = ((uint64_t)d.src << 11) | (uint64_t)i;
        meta[i] = d.widx | (d.inh << 16) | (d.dly << 24);
      } else {
        keys[i] = ~0ULL;
      }
    }
    __syncthreads();
    for (int kk = 2; kk <= kFillChunk; kk <<= 1) {
      for (int jj = kk >> 1; jj > 0; jj >>= 1) {
        for (int i = tid; i < kFillChunk; i += kFillThreads) {
          const int ixj = i ^ jj;
          if (ixj > i) {
            const uint64_t x = keys[i], y = keys[ixj];
            const bool up = (i & kk) == 0;
            if ((x > y) == up) {
              keys[i] = y;
              keys[ixj] = x;
            }
          }
        }
        __syncthreads();
      }
    }
    for (int p = tid; p < n_in; p += kFillThreads) {
      const uint64_t key = keys[p];
      const uint32_t src = (uint32_t)(key >> 11);
      const int idx = (int)(key & 2047);
      int rank = 0;
      while (p - rank - 1 >= 0 && (uint32_t)(keys[p - rank - 1] >> 11) == src) ++rank;
      const int64_t cell = (int64_t)src * a.NB + b;
      const int64_t pos = (int64_t)a.cursor[cell] + rank;
      const uint32_t m = meta[idx];
      const uint32_t widx = m & 0xffffu, inh = (m >> 16) & 1u, dly = m >> 24;
      const int64_t jl = (c0 + idx) / a.K;
      if (a.wform == WF_FP32) {
        float w;
        if (a.fixed) w = inh ? a.w_fix_i : a.w_fix_e;
        else w = inh ? ((const float*)a.wtab_i)[widx] : ((const float*)a.wtab_e)[widx];
        ((uint64_t*)a.syn)[pos] =
            ((uint64_t)(uint32_t)(j0 + jl) << 32) | (uint64_t)__float_as_uint(w);
      } else {
        uint32_t wb;
        if (a.fixed) wb = inh ? a.fix_bits_i : a.fix_bits_e;
        else wb = inh ? ((const uint16_t*)a.wtab_i)[widx] : ((const uint16_t*)a.wtab_e)[widx];
        uint32_t rec = (wb & 0xffffu) | ((uint32_t)jl << 16);
        if (a.wform == WF_PACKED)
          rec = (wb & 0xffffu) | ((uint32_t)((int64_t)(dly - a.d_min) * a.B + jl) << 16);
        ((uint32_t*)a.syn)[pos] = rec;
      }
      if (a.wform != WF_PACKED) a.syn_dly[pos] = (uint8_t)dly;
    }
    __syncthreads();
    for (int p = tid; p < n_in; p += kFillThreads) {
      const uint32_t src = (uint32_t)(keys[p] >> 11);
      const bool last = (p == n_in - 1) || ((uint32_t)(keys[p + 1] >> 11) != src);
      if (last) {
        int run = 1;
        while (p - run >= 0 && (uint32_t)(keys[p - run] >> 11) == src) ++run;
        a.cursor[(int64_t)src * a.NB + b] += (uint32_t)run;
      }
    }
    __syncthreads();
  }
}

// Segment pointers: seg[s * NB + b] = (start, count) of the synapses from s
// into block b, from the scan of the (s, b) counts.
__global__ void k_seg_pairs(const uint32_t* row, int64_t n_src, int32_t NB, uint2* seg) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_src * NB) return;
  const uint32_t lo = row[i];
  seg[i] = make_uint2(lo, row[i + 1] - lo);
}

// Block b's segments gathered source by source (export): dst_off[s] is the
// first output record of source s.
__global__ void k_gather_block(const uint2* seg, int64_t n_src, int32_t NB, int32_t b,
                               const int64_t* dst_off, const void* syn, const uint8_t* dly,
                               int32_t rec_bytes, void* out, uint8_t* out_dly) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_src) return;
  const uint2 sg = seg[s * NB + b];
  const int64_t o = dst_off[s];
  for (uint32_t k = 0; k < sg.y; ++k) {
    const uint64_t e = (uint64_t)sg.x + k;
    if (rec_bytes == 8) ((uint64_t*)out)[o + k] = ((const uint64_t*)syn)[e];
    else ((uint32_t*)out)[o + k] = ((const uint32_t*)syn)[e];
    if (dly) out_dly[o + k] = dly[e];
  }
}

// Source-major layout: per-source histogram, then a fill that appends each
// synapse to its source's segment through a per-source cursor.  The order
// inside a segment depends on atomic timing; delivery sums are exact
// integers, so results do not, and exports sort segments canonically.
__global__ void __launch_bounds__(256) k_count_sm(BuildArgs a) {
  const int64_t j = blockIdx.x;
  const int64_t part = j >> a.tbits;
  for (int32_t k = threadIdx.x; k < a.K; k += blockDim.x) {
    const Draw d = draw_synapse(a, j, k);
    atomicAdd(&a.row64[(int64_t)d.src * a.H + part], 1ull);
  }
}

__global__ void __launch_bounds__(256) k_fill_sm(BuildArgs a) {
  const int64_t j = blockIdx.x;
  const int64_t part = j >> a.tbits;
  const uint32_t off = (uint32_t)(j - (part << a.tbits));
  for (int32_t k = threadIdx.x; k < a.K; k += blockDim.x) {
    const Draw d = draw_synapse(a, j, k);
    const unsigned long long pos = atomicAdd(&a.cursor64[(int64_t)d.src * a.H + part], 1ull);
    const uint32_t word = off | ((uint32_t)(d.dly - a.d_min) << a.tbits);
    if (a.wform == WF_FP32) {
      float w;
      if (a.fixed) w = d.inh ? a.w_fix_i : a.w_fix_e;
      else w = d.inh ? ((const float*)a.wtab_i)[d.widx] : ((const float*)a.wtab_e)[d.widx];
      a.tw[pos] = word;
      ((float*)a.wbits)[pos] = w;
    } else {
      uint32_t wb;
      if (a.fixed) wb = d.inh ? a.fix_bits_i : a.fix_bits_e;
      else wb = d.inh ? ((const uint16_t*)a.wtab_i)[d.widx] : ((const uint16_t*)a.wtab_e)[d.widx];
      a.tw[pos] = word | ((wb >> 8) << kRecWordBits);
      ((uint8_t*)a.wbits)[pos] = (uint8_t)wb;
    }
  }
}

// ---------------------------------------------------------------------------
// source-major delivery, pass 1: binning by target block
// ---------------------------------------------------------------------------
// In the one-GPU share of a brain-scale network a source reaches ~1 target
// per block of B neurons, so per-(source, block) segments degenerate
// (Sec. 3.2: segments shrink as the network is spread over more processes).
// The slice's events are instead sorted by target block on the fly: each of
// P workgroups takes a contiguous share of the spike list, walks the spikes'
// (spike, target part) segments part by part (coalesced), and sorts chunks
// of U * 1024 events by block in LDS (a returning LDS atomic on the block's
// counter gives an event's rank, a block scan over the chunk's part's blocks
// the bin starts).  Taking a part's segments together keeps a chunk's events
// in a few hundred blocks, so each block's run of a chunk is tens of records
// rather than a handful.  Each bin's run is then appended to the
// workgroup's own region of that block with coalesced stores, so no global
// atomics are involved.  A region that fills up sends further events to the
// fixed-point spill rows with global atomics and flags the block.
struct BinLds {
  size_t stage, dst, cc, pre, lo, mt, seg, scr, total;
};
__host__ __device__ inline BinLds bin_lds_layout(int NB, int U, bool w8) {
  auto up = [](size_t x) { return (x + 15) / 16 * 16; };
  BinLds L;
  size_t o = 0;
  // sorted chunk: {record, destination} (4-byte records) or {record, FP32
  // weight} with the destinations apart (8-byte records)
  L.stage = o; o = up(o + (size_t)U * kBinThreads * 8);
  L.dst = o;   o = up(o + (w8 ? (size_t)U * kBinThreads * 4 : 0));
  // per block {count in the chunk, then the bin's start; records in this
  // workgroup's region before the chunk}, and the chunk's run lengths
  L.cc = o;    o = up(o + (size_t)(NB + 1) * 8 + (size_t)NB * 4);
  L.pre = o;   o = up(o + (size_t)(kBinSpikes + 1) * 8);  // event prefix per segment entry
  L.lo = o;    o = up(o + (size_t)kBinSpikes * 8);  // table index of the batch's event 0, per entry
  L.mt = o;    o = up(o + (size_t)kBinSpikes * 4);  // lag | inhibitory << 15 | part << 16
  L.seg = o;   o = up(o + (size_t)kBinSegTab * 2);  // entry holding event k << sh of the batch
  L.scr = o;   o = up(o + (size_t)(kBinThreads / 64 + 2) * 8);
  L.total = o;
  return L;
}

size_t bin_lds_bytes(int NB, int U, bool w8) { return bin_lds_layout(NB, U, w8).total; }

template <bool W8>
__global__ void __launch_bounds__(kBinThreads) k_bin(BinArgs args) {
  // fields are read where used, through a pointer to the kernel-argument
  // segment (the whole struct in scalar registers would spill)
  const BinArgs& a = *(const BinArgs*)__builtin_amdgcn_kernarg_segment_ptr();
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int tid = threadIdx.x;
  const int p = blockIdx.x, P = gridDim.x;
  const int NB = a.NB, B = a.B, U = a.U, cap = a.cap;
  const BinLds Lo = bin_lds_layout(NB, U, W8);
  uint2* stage2 = (uint2*)(lds_raw + Lo.stage);
  uint32_t* dst = (uint32_t*)(lds_raw + Lo.dst);
  uint2* const cc = (uint2*)(lds_raw + Lo.cc);              // [NB + 1]
  uint32_t* const runs = (uint32_t*)(lds_raw + Lo.cc + (size_t)(NB + 1) * 8);  // [NB]
  __shared__ int s_bl, s_bh;       // block range of the chunk
  __shared__ uint32_t s_nchunk;    // events of the chunk
  unsigned long long* pre = (unsigned long long*)(lds_raw + Lo.pre);
  unsigned long long* lo = (unsigned long long*)(lds_raw + Lo.lo);
  uint32_t* mt = (uint32_t*)(lds_raw + Lo.mt);
  uint16_t* seg = (uint16_t*)(lds_raw + Lo.seg);
  unsigned long long* scr64 = (unsigned long long*)(lds_raw + Lo.scr);
  uint32_t* scr32 = (uint32_t*)(lds_raw + Lo.scr);

  int64_t total = (int64_t)*a.in_cnt;
  if (total > a.in_cap) total = a.in_cap;  // overflow is flagged by the writer
  if (total < 0) total = 0;
  const int64_t s_lo = total * p / P, s_hi = total * (p + 1) / P;
  for (int i = tid; i < NB + 1; i += kBinThreads) cc[i] = make_uint2(0u, 0u);
  unsigned long long ev = 0;
  const int tbits = a.tbits, H = a.H;
  const uint32_t tmask = (1u << tbits) - 1u;
  const uint32_t dmask = (1u << (kRecWordBits - tbits)) - 1u;
  const uint32_t region0 = (uint32_t)p * (uint32_t)cap;  // this workgroup's region in a block's area
  const uint32_t area = (uint32_t)P * (uint32_t)cap;     // records per block

  // every spike has H segments, one per target part: the share walks its
  // spikes' (spike, part) segment entries part by part, so that a chunk's
  // events fall into the few blocks of one part and each block's run is
  // long
  const int64_t nsp = s_hi - s_lo;
  for (int64_t sb = 0; sb < nsp * H; sb += kBinSpikes) {
    const int ns = (int)((nsp * H - sb) < kBinSpikes ? (nsp * H - sb) : kBinSpikes);
    // (1) every thread resolves one segment entry
    unsigned long long len = 0, l0 = 0;
    if (tid < ns) {
      const int64_t se = sb + tid;
      const int64_t pe = se / nsp;
      const int64_t i = s_lo + (se - pe * nsp);
      const uint32_t part = (uint32_t)pe;
      const uint32_t ent = a.in_list[i];
      const uint32_t src = ent >> 5;
      const uint32_t lag = ent & 31u;
      if ((int)lag < a.Dmin && (int64_t)src < a.n_src) {
        l0 = a.row[(int64_t)src * H + part];
        len = a.row[(int64_t)src * H + part + 1] - l0;
      } else if (part == 0) {
        atomicOr(a.overflow, 4);
      }
      mt[tid] = lag | (((int64_t)src >= a.src_e_end) ? 0x8000u : 0u) | (part << 16);
    }
    unsigned long long n_batch;
    const unsigned long long ex = block_excl_scan1<unsigned long long>(len, scr64, n_batch);
    // event f of the batch is table entry lo[s] + f of the segment entry s
    // holding it; seg[k] names the entry holding event k << sh, with sh >= 6
    // the smallest that keeps the table within kBinSegTab entries (the 64
    // events of one wave's slot share a table entry)
    int sh = 6;
    while (((n_batch + (1ull << sh) - 1) >> sh) > (unsigned long long)kBinSegTab) ++sh;
    if (tid < ns) {
      pre[tid] = ex;
      lo[tid] = l0 - ex;
      const unsigned long long g = (1ull << sh) - 1;
      for (unsigned long long k = (ex + g) >> sh; k < ((ex + len + g) >> sh); ++k)
        seg[k] = (uint16_t)tid;
    }
    if (tid == 0) pre[ns] = n_batch;
    ev += n_batch;  // the same value in every thread; thread 0 reports it
    __syncthreads();

    // (2) chunks of U * 1024 events of the batch, event f of the batch at
    // thread f % 1024, slot f / 1024 (consecutive lanes read consecutive
    // records of a segment).  Each thread's events of a chunk sit in
    // registers: target|delay word, weight bits, and lag / population packed
    // four to a register.  A chunk's loads are issued right after the
    // previous chunk's write-out.
    const unsigned long long E_c = (unsigned long long)U * kBinThreads;
    constexpr int UM = W8 ? kBinMaxU8 : kBinMaxU;  // register budget
    uint32_t tdk[UM], wbr[UM], rec8[W8 ? UM : 1], m4[UM / 2];
    auto issue = [&](unsigned long long f0) {
      const unsigned long long left = n_batch - f0;
      const uint32_t n_ev = left < E_c ? (uint32_t)left : (uint32_t)E_c;
#pragma unroll
      for (int u = 0; u < UM / 2; ++u) m4[u] = 0u;
      // kBinGrp events at a time: their segment entries from the lookup
      // table, then the entries' table offsets, ends and meta words (two LDS
      // round trips for the group); a lane whose event lies past its table
      // entry's segment moves on (a wave slot crosses a segment's end with
      // probability ~64 / segment length)
#pragma unroll
      for (int h = 0; h < UM; h += kBinGrp) {
        int sp[kBinGrp];
#pragma unroll
        for (int u = h; u < h + kBinGrp; ++u) {
          const uint32_t fr = (uint32_t)(u * kBinThreads + tid);
          sp[u - h] = (u < U && fr < n_ev) ? (int)seg[(f0 + fr) >> sh] : 0;
        }
        unsigned long long l0[kBinGrp], p1[kBinGrp];
        uint32_t m[kBinGrp];
#pragma unroll
        for (int u = h; u < h + kBinGrp; ++u) {
          l0[u - h] = lo[sp[u - h]];
          p1[u - h] = pre[sp[u - h] + 1];
          m[u - h] = mt[sp[u - h]];
        }
#pragma unroll
        for (int u = h; u < h + kBinGrp; ++u) {
          const uint32_t fr = (uint32_t)(u * kBinThreads + tid);
          tdk[u] = 0u;
          wbr[u] = 0u;
          if (u < U && fr < n_ev) {
            const unsigned long long f = f0 + fr;
            int s = sp[u - h];
            unsigned long long b0 = l0[u - h], e1 = p1[u - h];
            uint32_t mm = m[u - h];
            while (e1 <= f) {  // pre[ns] = n_batch lies past every event
              ++s;
              b0 = lo[s];
              e1 = pre[s + 1];
              mm = mt[s];
            }
            const unsigned long long e = b0 + f;
            tdk[u] = a.tw[e];
            if constexpr (W8) wbr[u] = ((const uint32_t*)a.wbits)[e];
            else wbr[u] = ((const uint8_t*)a.wbits)[e];
            // lag | inh << 5 | part << 6 (16 bits per event)
            m4[u >> 1] |= ((mm & 31u) | ((mm >> 10) & 32u) | (((mm >> 16) & 63u) << 6))
                          << ((u & 1) * 16);
          }
        }
      }
    };
    if (n_batch > 0) issue(0);
    for (unsigned long long f0 = 0; f0 < n_batch; f0 += E_c) {
      const unsigned long long left = n_batch - f0;
      const uint32_t n_ev = left < E_c ? (uint32_t)left : (uint32_t)E_c;
      // the chunk's blocks: those of the parts of its first and last events
      // (segments are ordered by part, so every event lies in between)
      if (tid == 0) {
        int pr[2];
        for (int k = 0; k < 2; ++k) {
          const unsigned long long f = f0 + (k ? n_ev - 1 : 0);
          int sq = (int)seg[f >> sh];
          while (pre[sq + 1] <= f) ++sq;
          pr[k] = (int)((mt[sq] >> 16) & 63u);
        }
        const int64_t bl = ((int64_t)pr[0] << tbits) / B;
        const int64_t bh = ((((int64_t)pr[1] + 1) << tbits) - 1) / B;
        s_bl = (int)bl;
        s_bh = (int)(bh < NB - 1 ? bh : NB - 1);
      }
      // classify: tdk[u] becomes the event's key (block << 16 | rank in the
      // block's bin), wbr[u] (4-byte form) or rec8[u] (FP32) its record
      // Eight events at a time: their rank atomics are all issued before
      // the first rank is used, so one wait covers them.  The block size
      // and its inverse are copied to vector registers first: read from the
      // scalar registers a scalar load filled, each event would wait on the
      // counter that the previous event's LDS atomic also counts against.
      float inv_B = a.inv_B;
      int Bv = B;
      asm volatile("" : "+v"(inv_B), "+v"(Bv));
#pragma unroll
      for (int h = 0; h < UM; h += 8) {
        uint32_t rk[8];
#pragma unroll
        for (int u = h; u < h + 8 && u < UM; ++u) {
          const uint32_t fr = (uint32_t)(u * kBinThreads + tid);
          const uint32_t td = tdk[u];
          tdk[u] = 0xffffffffu;  // no event
          rk[u - h] = 0u;
          if constexpr (W8) rec8[u] = 0u;
          if (u < U && fr < n_ev) {
            const uint32_t m = (m4[u >> 1] >> ((u & 1) * 16)) & 0xffffu;
            const int tgt = (int)(((m >> 6) << tbits) | (td & tmask));
            // block = tgt / B from an FP32 estimate, corrected by one step
            int blk = (int)((float)tgt * inv_B);
            int off = tgt - blk * Bv;
            if (off < 0) { --blk; off += Bv; }
            if (off >= Bv) { ++blk; off -= Bv; }
            const int q = (int)(m & 31u) + (int)((td >> tbits) & dmask);
            const uint32_t r = (uint32_t)(q * Bv + off) | ((m & 32u) << 10);
            if constexpr (W8) rec8[u] = r;
            else wbr[u] = r | ((((td >> kRecWordBits) << 8) | wbr[u]) << 16);
            rk[u - h] = __hip_atomic_fetch_add(&cc[blk].x, 1u, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
            tdk[u] = (uint32_t)blk << 16;
          }
        }
#pragma unroll
        for (int u = h; u < h + 8 && u < UM; ++u)
          if (tdk[u] != 0xffffffffu) tdk[u] |= rk[u - h];
      }
      __syncthreads();
      // (3) bin starts: exclusive scan of the counts of the chunk's blocks,
      // in place; the runs are kept for the fills
      const int bl = s_bl, bh = s_bh;
      {
        const int nr = bh - bl + 1;
        const int per = (nr + kBinThreads - 1) / kBinThreads;
        const int i0 = bl + tid * per, i1 = (i0 + per) < bh + 1 ? i0 + per : bh + 1;
        uint32_t sum = 0;
        for (int i = i0; i < i1; ++i) sum += cc[i].x;
        uint32_t n_chunk;
        uint32_t run = block_excl_scan1<uint32_t>(sum, scr32, n_chunk);
        for (int i = i0; i < i1; ++i) {
          const uint32_t c = cc[i].x;
          runs[i] = c;
          cc[i].x = run;
          run += c;
        }
        if (tid == 0) s_nchunk = n_chunk;
      }
      __syncthreads();
      // (4) scatter into bin order, with each record's destination: its
      // index in the bin area (block * P * cap + this region's start +
      // fill + rank), or kNoDst | block when the region is full.  The bins'
      // (start, fill) words of kBinGrp events are read before the first is
      // used (one LDS wait per group, not one per event).
      constexpr uint32_t kNoDst = 0x80000000u;
#pragma unroll
      for (int h = 0; h < UM; h += kBinGrp) {
        uint2 cw[kBinGrp];
#pragma unroll
        for (int u = h; u < h + kBinGrp; ++u)
          cw[u - h] = cc[tdk[u] != 0xffffffffu ? tdk[u] >> 16 : 0u];
#pragma unroll
        for (int u = h; u < h + kBinGrp; ++u) {
          if (tdk[u] != 0xffffffffu) {
            const uint32_t blk = tdk[u] >> 16;
            const uint32_t at = cw[u - h].x + (tdk[u] & 0xffffu);
            const uint32_t pos = cw[u - h].y + (tdk[u] & 0xffffu);
            const uint32_t d = pos < (uint32_t)cap ? blk * area + region0 + pos : kNoDst | blk;
            if constexpr (W8) {
              stage2[at] = make_uint2(rec8[u], wbr[u]);
              dst[at] = d;
            } else {
              stage2[at] = make_uint2(wbr[u], d);
            }
          }
        }
      }
      __syncthreads();
      // (5) every thread stores sorted records f, f + 1024, ...: a bin's run
      // goes to consecutive addresses (coalesced stores of ~U * 1024 / NB
      // records), then the fills advance.  Sorted entries are read kBinGrp
      // at a time (one LDS wait per group); the bin area's address is held
      // in registers (read through the argument pointer inside the loop it
      // would be reloaded, and waited for, before every store, since the
      // stores might alias it); events of full regions are added in a
      // separate, rarely taken pass.
      const uint32_t n_chunk = s_nchunk;
      // the regions' fills advance by this chunk's runs; counts clear for
      // the next chunk (the scatter, which read the fills, is behind the
      // barrier above)
      {
        const int nr = bh - bl + 1;
        for (int i = bl + tid; i < bl + nr; i += kBinThreads) {
          cc[i].y += runs[i];
          cc[i].x = 0u;
        }
      }
      {
        void* const bins = a.bins;
        bool spill = false;
#pragma unroll
        for (int h = 0; h < UM; h += kBinGrp) {
          uint32_t rv[kBinGrp], dv[kBinGrp], xv[kBinGrp];
#pragma unroll
          for (int u = h; u < h + kBinGrp; ++u) {
            const uint32_t ic = (u < U) ? (uint32_t)(u * kBinThreads + tid) : 0u;
            const uint2 x = stage2[ic];  // entries past U * 1024 do not exist
            rv[u - h] = x.x;
            if constexpr (W8) {
              xv[u - h] = x.y;
              dv[u - h] = dst[ic];
            } else {
              dv[u - h] = x.y;
            }
          }
#pragma unroll
          for (int u = h; u < h + kBinGrp; ++u) {
            const uint32_t i = (uint32_t)(u * kBinThreads + tid);
            if (i < n_chunk) {
              if (!(dv[u - h] & kNoDst)) {
                if constexpr (W8) ((uint2*)bins)[dv[u - h]] = make_uint2(rv[u - h], xv[u - h]);
                else ((uint32_t*)bins)[dv[u - h]] = rv[u - h];
              } else {
                spill = true;
              }
            }
          }
        }
        if (spill) {
          // region full: add the event's fixed-point weight into the spill
          // rows with a global atomic
          for (int u = 0; u < UM; ++u) {
            const uint32_t i = (uint32_t)(u * kBinThreads + tid);
            if (i >= n_chunk) continue;
            const uint2 x = stage2[i];
            const uint32_t d = W8 ? dst[i] : x.y;
            if (!(d & kNoDst)) continue;
            const int bk = (int)(d & ~kNoDst);
            const uint32_t r = x.x;
            const float w = W8 ? __uint_as_float(x.y) : __uint_as_float(r & 0xffff0000u);
            const int slot = (int)(r & ((1u << kBinSlotBits) - 1u));
            const int q = slot / B, off = slot - q * B;
            const bool inh = (r & 0x8000u) != 0u;
            const long long v =
                (long long)(int)fmaf(inh ? a.wm1_i : a.wm1_e, w, inh ? a.wm0_i : a.wm0_e);
            atomicAdd((unsigned long long*)&a.spill[(int64_t)q * a.N + (int64_t)bk * B + off],
                      (unsigned long long)v);
            a.spill_flag[bk] = 1;
          }
        }
      }
      // The next chunk's loads (the registers are free after the scatter),
      // issued after this chunk's stores: the classify's first wait for a
      // load also waits for every store issued before it.
      if (f0 + E_c < n_batch) issue(f0 + E_c);
      // the next chunk's counts start from the zeros written above
      __syncthreads();
    }
  }
  // record counts of this workgroup's regions: the last chunk's fills plus
  // its runs (all zero if there was no chunk)
  {
    for (int b = tid; b < NB; b += kBinThreads) {
      const uint32_t f = cc[b].y;
      a.bin_cnt[(size_t)b * P + p] = f < (uint32_t)cap ? f : (uint32_t)cap;
    }
  }
  if (tid == 0) {
    if (ev) atomicAdd(a.ev_count, ev);
    if (p == 0) atomicAdd(a.spk_in_count, (unsigned long long)total);
  }
}

// ---------------------------------------------------------------------------
// the fused slice kernel
// ---------------------------------------------------------------------------
// Raw synapse record as loaded (decoded only when its add is issued, so a
// wave keeps one to three registers per segment in flight).
template <int WF> struct SynRaw;
template <> struct SynRaw<WF_FP32> { uint64_t r; uint32_t d; };
template <> struct SynRaw<WF_BF16> { uint32_t r; uint32_t d; };
template <> struct SynRaw<WF_BF16_RESID> { uint32_t r; uint32_t d; };
template <> struct SynRaw<WF_PACKED> { uint32_t r; };

// Segments a wave takes from the chunk at a time (all loads in flight
// before the adds).  Measured on the 112,500-neuron network (~44-synapse
// segments): smaller groups spread a chunk's ~900 spikes more evenly over
// the 16 waves and keep the blocks of an XCD on nearby spikes; below these
// sizes the loads in flight no longer cover the latency.
template <int WF> struct SynGroup { static constexpr int n = 12; };
template <> struct SynGroup<WF_FP32> { static constexpr int n = 8; };
template <> struct SynGroup<WF_PACKED> { static constexpr int n = 12; };
constexpr int kMaxGroup = 32;

// Binned records (source-major layout) are read through a buffer resource
// over one block's bin area: element index i, or kOobIndex for a lane or
// slot with nothing to load (that offset lies past the area, checked at
// creation, so the load returns zero without reading memory).
constexpr uint32_t kOobIndex = 1u << 28;
constexpr int kBufWord3 = 0x00020000;  // gfx9 buffer resource: 32-bit dword format

// Record i of the block-major table (index 0 for a lane or slot with
// nothing to load: the table always holds a record there, the value is
// not used).
template <int WF>
__device__ __forceinline__ SynRaw<WF> syn_fetch(const void* syn, const uint8_t* dly, uint32_t i) {
  SynRaw<WF> x;
  if constexpr (WF == WF_FP32) {
    const uint2 v = ((const uint2*)syn)[i];
    x.r = ((uint64_t)v.y << 32) | v.x;
    x.d = dly[i];
  } else if constexpr (WF == WF_PACKED) {
    x.r = ((const uint32_t*)syn)[i];
  } else {
    x.r = ((const uint32_t*)syn)[i];
    x.d = dly[i];
  }
  return x;
}

// Window slot ((delay - d_min) * B + offset in block) and fixed-point weight
// trunc(m1 * x + m0) of a record, x its BF16 residual or its weight.  With
// the window quantum chosen so that max|w| * 2^s <= 2^30, w * 2^s is exact
// in FP32 for |w| * 2^s >= 2^23, so the truncation only rounds weights
// below 2^-7 of the largest.
template <int WF>
__device__ __forceinline__ void syn_decode(const SynRaw<WF>& x, int32_t j0, int Dmin, int B,
                                           float m0, float m1, int& slot, int& v) {
  float w;
  if constexpr (WF == WF_FP32) {
    w = __uint_as_float((uint32_t)x.r);
    slot = ((int)x.d - Dmin) * B + ((int)(x.r >> 32) - j0);
  } else if constexpr (WF == WF_PACKED) {
    w = __uint_as_float(x.r << 16);
    slot = (int)(x.r >> 16);
  } else {
    w = __uint_as_float(x.r << 16);
    slot = ((int)x.d - Dmin) * B + (int)(x.r >> 16);
  }
  v = (int)fmaf(m1, w, m0);  // conversion truncates toward zero
}

// Window cell (64-bit fixed point, quantum inv = 2^-s) to FP32: the
// integer is rounded once to the nearest FP32 (ties to even; the int64 ->
// FP32 conversion is correctly rounded), and the power-of-two scale is
// exact.  Same value as an FP64 product rounded to FP32, with no FP64.
__device__ __forceinline__ float from_fixed(long long q, float inv) {
  return (float)q * inv;
}

template <bool V> struct BoolC { static constexpr bool value = V; };

// A thread keeps the staged HBM ring rows of its own neuron in registers
// when every neuron has its own thread and a slice has at most this many
// steps; otherwise they are staged in LDS.
constexpr int kRegRows = 16;
__host__ __device__ inline bool staged_in_regs(int B, int Dmin) {
  return B <= kSliceThreads && Dmin <= kRegRows;
}

// LDS layout of a slice workgroup (byte offsets, 16-byte aligned pieces)
struct SliceLds {
  size_t win, carry, dcnt, mask, thr, scr, desc, meta, pm, pb, lagm, tpv, total;
};
__host__ __device__ inline SliceLds slice_lds_layout(int B, int Dmin, int win_rows,
                                                     bool plastic = false, bool bin = false) {
  auto up = [](size_t x) { return (x + 15) / 16 * 16; };
  SliceLds L;
  size_t o = 0;
  L.win = o;   o = up(o + (size_t)win_rows * B * 8);    // int64 ring window
  L.carry = o; o = up(o + (staged_in_regs(B, Dmin) ? 0 : (size_t)Dmin * B * 4));  // staged HBM rows
  L.dcnt = o;  o = up(o + (size_t)Dmin * B);            // Poisson-drive counts (u8)
  L.mask = o;  o = up(o + (size_t)Dmin * (B / 32) * 4); // spike bitmask
  L.thr = o;   o = up(o + (size_t)kMaxThr * 4);         // drive thresholds
  L.scr = o;   o = up(o + (size_t)(kSliceThreads / 64 + 2) * 4);
  // one descriptor per spike of a chunk, plus one group of padding so a
  // wave's last group reads in bounds without clamping its index; binned
  // records use the same array for their work items (at most P * cap /
  // kBinSlice <= 1024) and need no meta words, which lets the source-major
  // layout fit 896-neuron blocks
  L.desc = o;  o = up(o + (size_t)(kSliceThreads + kMaxGroup) * 8);  // (start in block, count)
  L.meta = o;  o = up(o + (bin ? 0 : (size_t)(kSliceThreads + kMaxGroup) * 4));  // lag row, count, pop.
  // plastic synapses: the block's post-spike masks and earlier spikes, and
  // per spike of a chunk its lag mask and its source's previous spike
  const size_t np = plastic ? 1 : 0;
  L.pm = o;    o = up(o + np * (size_t)B * 8);
  L.pb = o;    o = up(o + np * (size_t)B * 4);
  L.lagm = o;  o = up(o + np * (size_t)(kSliceThreads + kMaxGroup) * 4);
  L.tpv = o;   o = up(o + np * (size_t)(kSliceThreads + kMaxGroup) * 4);
  L.total = o;
  return L;
}

size_t slice_lds_bytes(int B, int Dmin, int win_rows, bool plastic, bool bin) {
  return slice_lds_layout(B, Dmin, win_rows, plastic, bin).total;
}

// Plastic synapses: one excitatory weight w (delay d, target row of the
// block's post-spike mask pm / earlier spike pb) takes the source's spikes
// of one slice in lag order (bits of lm; t0 the slice start, tprev the
// source's spike before it), each updated by the nearest-spike pair rule and
// then added into the window row of its arrival step.  T is the first step
// after the masks (the window's first step): bit k of pm is step T - 1 - k.
// The arrival row of lag l is l + d - Dmin.
__device__ __forceinline__ float plastic_walk(const SliceArgs& a, float w, int d, uint64_t pm,
                                              int32_t pb, uint32_t lm, int32_t tprev, int32_t t0,
                                              int32_t T, int Dmin, int B, int jl, long long* win,
                                              float m1) {
  while (lm) {
    const int l = __ffs(lm) - 1;
    lm &= lm - 1;
    const int32_t t_pre = t0 + l;
    const int32_t c = t_pre - d;          // latest step whose target spike the synapse sees
    const int k = T - 1 - c;              // in [Dmin, Dmin + Dmax - 1] <= 63
    const uint64_t mk = pm >> k;
    const int32_t t_last = mk ? c - (int32_t)__builtin_ctzll(mk) : pb;
    if (t_last >= 0) {
      if (tprev >= 0 && t_last + d > tprev) {
        w += a.stdp_ap * exp2f(-(float)(t_last + d - tprev) * a.stdp_kp);
        w = fminf(w, a.stdp_wmax);
      }
      w -= a.stdp_am * exp2f(-(float)(t_pre - t_last - d) * a.stdp_km);
      w = fmaxf(w, 0.f);
    }
    const int v = (int)(m1 * w);          // conversion truncates toward zero
    __hip_atomic_fetch_add((unsigned long long*)&win[(l + d - Dmin) * B + jl],
                           (unsigned long long)(long long)v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
    tprev = t_pre;
  }
  return w;
}

// One workgroup's slice for target block b of the network described by a.
// BIN: the slice's events arrive binned by target block (source-major
// layout, k_bin; WF_FP32 for 8-byte records, any other form for 4-byte
// ones); otherwise they are read from the block-major segments.
// DYN: how the window rows due later are flushed (see the flush below).
template <int WF, bool BIN, bool DYN, bool PL = false>
__device__ __forceinline__ void slice_block(const SliceArgs& a, const int b) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  constexpr int nwv = kSliceThreads / 64;
  const int B = a.B;
  const int64_t j0 = (int64_t)b * B;
  const int nb = (int)((a.N - j0) < B ? (a.N - j0) : B);
  const int Wd = B >> 5;
  const int Dmin = a.Dmin;

  const SliceLds Lo = slice_lds_layout(B, Dmin, a.win_rows, PL, BIN);
  long long* win = (long long*)(lds_raw + Lo.win);
  float* carry = (float*)(lds_raw + Lo.carry);
  uint8_t* dcnt = lds_raw + Lo.dcnt;
  uint32_t* mask = (uint32_t*)(lds_raw + Lo.mask);
  uint32_t* thr = (uint32_t*)(lds_raw + Lo.thr);
  int32_t* scr = (int32_t*)(lds_raw + Lo.scr);
  // spike c0 + i of the current chunk: its segment in this block (start
  // relative to the block's first synapse, count) and its meta word
  // lag * B << 7 | min(count, 65) | excitatory 0 / inhibitory 1 << 31, read
  // back by whole waves as LDS broadcasts
  uint2* desc = (uint2*)(lds_raw + Lo.desc);
  uint32_t* meta = (uint32_t*)(lds_raw + Lo.meta);
  uint64_t* pm = (uint64_t*)(lds_raw + Lo.pm);
  int32_t* pb = (int32_t*)(lds_raw + Lo.pb);
  uint32_t* lagm = (uint32_t*)(lds_raw + Lo.lagm);
  int32_t* tpv = (int32_t*)(lds_raw + Lo.tpv);
  if constexpr (PL) {
    // the block's post-spike history, read by the delivery (visible after
    // the first chunk's barrier) and advanced by the update
    for (int i = tid; i < nb; i += kSliceThreads) {
      pm[i] = a.pmask[j0 + i];
      pb[i] = a.pbefore[j0 + i];
    }
  }

  // Loads consumed only after the first wait of the delivery below, so
  // their latency overlaps the ring-row and state loads.  The list count
  // is a vector load: a scalar one would make every later scalar load of an
  // argument wait for it.
  const uint32_t thr_v = (tid < kMaxThr && tid < a.n_thr) ? a.thr[tid] : 0xffffffffu;
  const int32_t total_raw =
      (!BIN && a.do_deliver)
          ? __hip_atomic_load(a.in_cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
          : 0;
  // this thread's list entry of the first chunk, read within the list's
  // capacity before its length is known
  const uint32_t ent0 = (!BIN && a.do_deliver && tid < a.in_cap) ? a.in_list[tid] : 0u;
  uint32_t bin_len = 0;
  int spill_on = 0;
  if constexpr (BIN) {
    if (a.do_deliver) {
      if (tid < a.bin_P) bin_len = a.bin_cnt[(size_t)b * a.bin_P + tid];
      spill_on = __hip_atomic_load(a.spill_flag + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }

  // window rows cover steps [w_lo, w_lo + Dmax)
  const int64_t w_lo = a.w_lo;
  if (a.do_deliver)
    for (int i = tid; i < a.Dmax * B; i += kSliceThreads) win[i] = 0;
  for (int i = tid; i < Dmin * Wd; i += kSliceThreads) mask[i] = 0u;
  // events of this block, summed in LDS: one global atomic per workgroup
  // (thousands of same-address global atomics per launch back up the
  // memory queues of every compute unit)
  __shared__ unsigned long long s_ev;
  __shared__ long long s_zero;  // read by the update for steps outside the window
  __shared__ int s_fl;          // DYN: next neuron whose window rows go to the ring
  if (tid == 0) {
    s_ev = 0;
    s_zero = 0;
    s_fl = 0;
  }
  // the list counter of a later slice starts at zero
  if (b == 0 && tid == 0 && a.zero_cnt) *a.zero_cnt = 0;

  // ---- prologue: issue the loads the update will need -------------------
  // Carried ring rows (deliveries of earlier slices) and this thread's
  // neuron state are loaded into registers now; they arrive while the
  // spikes are delivered.
  constexpr int kRows = kRegRows;
  int rows = 0;
  if (a.n_upd > 0) {
    int64_t t_hi = a.t_upd + a.n_upd;
    if (t_hi > a.rb_hi) t_hi = a.rb_hi;
    rows = (int)(t_hi > a.t_upd ? t_hi - a.t_upd : 0);
  }
  const int r0 = (int)(a.t_upd % a.L);
  const bool regs = staged_in_regs(B, Dmin);  // rows <= n_upd <= Dmin <= kRows
  const bool fast = regs && rows > 0;
  const int n_own = tid < nb ? tid : nb - 1;  // in-bounds neuron of this thread
  // Raw values: rows at or past rb_hi hold no earlier input and are masked
  // where the update reads them, so nothing here waits for these loads.
  float stage[kRows];
#pragma unroll
  for (int q = 0; q < kRows; ++q) stage[q] = 0.f;
  if (fast) {
#pragma unroll
    for (int q = 0; q < kRows; ++q) {
      int rr = r0 + (q < rows ? q : 0);
      if (rr >= a.L) rr -= a.L;
      stage[q] = a.rb[(int64_t)rr * a.N + j0 + n_own];
    }
  }
  float sV = 0.f, sy1 = 0.f, sy2 = 0.f;
  int sr = 0;
  if (a.n_upd > 0) {
    sV = a.V[j0 + n_own];
    sr = a.r[j0 + n_own];
    if (a.model == MODEL_ALPHA) {
      sy1 = a.y1[j0 + n_own];
      sy2 = a.y2[j0 + n_own];
    }
  }

  // Poisson drive of the steps to update: one Philox4x64-10 block per
  // (neuron, 8-step chunk) gives eight 32-bit uniforms; the count is the
  // number of CDF thresholds at or below each uniform.  Round k covers tasks
  // k*1024 + tid; rounds are interleaved with the delivery loads below.
  int64_t c0 = 0;
  int n_tasks = 0;
  if (a.n_upd > 0) {
    c0 = a.t_upd >> 3;
    const int64_t c1 = (a.t_upd + a.n_upd - 1) >> 3;
    n_tasks = (int)(c1 - c0 + 1) * nb;
  }
  const int n_rounds = (n_tasks + kSliceThreads - 1) / kSliceThreads;
  auto drive_round = [&](int k) {
    const int task = k * kSliceThreads + tid;
    if (task >= n_tasks) return;
    const int n = task % nb;
    const int64_t c = c0 + task / nb;
    uint64_t rr[4];
    philox(a.seed, STREAM_DRIVE, (uint64_t)(j0 + n), (uint64_t)c, rr);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t t = c * 8 + q;
      if (t < a.t_upd || t >= a.t_upd + a.n_upd) continue;
      const uint64_t word = rr[q >> 1];
      const uint32_t u = (q & 1) ? (uint32_t)(word >> 32) : (uint32_t)word;
      int cnt = 0;
      while (cnt < a.n_thr && u >= thr[cnt]) ++cnt;  // thresholds ascend
      dcnt[(int)(t - a.t_upd) * B + n] = (uint8_t)cnt;
    }
  };
  int rounds_done = 0;

  // ---- deliver the completed slice into the LDS window (Alg. REF) -------
  // The drive thresholds go to LDS right before the first barrier, behind
  // a wait for loads issued after theirs.
  if (BIN && a.do_deliver) {
    if (tid < kMaxThr) thr[tid] = thr_v;
    __syncthreads();  // thr / zeroing visible
    // Work items of up to kBinSlice records of one region of this block's
    // bin area; waves take GB items at a time from a shared counter, RB
    // records per lane each, all loads in flight before the adds (slots
    // past a region's count load nothing: their buffer offset is out of
    // range).  The record holds the window slot, so the adds need no
    // per-item state.
    constexpr bool W8 = WF == WF_FP32;
    constexpr int GB = 8, RB = kBinSlice / 64;
    int n_items;
    const int n_it = (int)((bin_len + kBinSlice - 1) / kBinSlice);
    const int it0 = block_excl_scan<int>(n_it, scr, n_items);
    for (int i = 0; i < n_it; ++i) {
      const uint32_t r0 = (uint32_t)(i * kBinSlice);
      const uint32_t ln = (bin_len - r0) < (uint32_t)kBinSlice ? bin_len - r0 : (uint32_t)kBinSlice;
      desc[it0 + i] = make_uint2((uint32_t)tid * (uint32_t)a.bin_cap + r0, ln);
    }
    __shared__ int s_nb;
    if (tid == 0) s_nb = 0;
    __syncthreads();
    const size_t area = (size_t)a.bin_P * a.bin_cap;
    constexpr size_t rbytes = W8 ? 8 : 4;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)((const unsigned char*)a.bins + (size_t)b * area * rbytes), 0,
        (int)(area * rbytes), kBufWord3);
    for (;;) {
      int g0 = 0;
      if (lane == 0)
        g0 = __hip_atomic_fetch_add(&s_nb, GB, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      g0 = __builtin_amdgcn_readfirstlane(g0);
      if (g0 >= n_items) break;
      uint2 d[GB];
      uint32_t r[GB][RB], x[GB][W8 ? RB : 1];
#pragma unroll
      for (int u = 0; u < GB; ++u) {
        d[u] = desc[g0 + u];  // past n_items: stale or padding, masked
        if (g0 + u >= n_items) d[u].y = 0u;
#pragma unroll
        for (int k = 0; k < RB; ++k) {
          const uint32_t idx = (uint32_t)(k * 64 + lane);
          const uint32_t e = idx < d[u].y ? d[u].x + idx : kOobIndex;
          if constexpr (W8) {
            const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)(e * 8u), 0, 0);
            r[u][k] = v[0];
            x[u][k] = v[1];
          } else {
            r[u][k] = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)(e * 4u), 0, 0);
          }
        }
      }
      // ALU work while the loads are in flight
      if (rounds_done < n_rounds) drive_round(rounds_done++);
#pragma unroll
      for (int u = 0; u < GB; ++u) {
#pragma unroll
        for (int k = 0; k < RB; ++k) {
          const uint32_t idx = (uint32_t)(k * 64 + lane);
          if (idx < d[u].y) {
            const uint32_t rr = r[u][k];
            const uint32_t sel = 0u - ((rr >> 15) & 1u);  // all ones: inhibitory
            const float m0 = __uint_as_float((__float_as_uint(a.wm0_e) & ~sel) |
                                             (__float_as_uint(a.wm0_i) & sel));
            const float m1 = __uint_as_float((__float_as_uint(a.wm1_e) & ~sel) |
                                             (__float_as_uint(a.wm1_i) & sel));
            float w;
            if constexpr (W8) w = __uint_as_float(x[u][k]);
            else w = __uint_as_float(rr & 0xffff0000u);
            const int v = (int)fmaf(m1, w, m0);  // conversion truncates toward zero
            __hip_atomic_fetch_add((unsigned long long*)&win[rr & ((1u << kBinSlotBits) - 1u)],
                                   (unsigned long long)(long long)v, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
          }
        }
      }
    }
    // events that found their region full: fixed-point spill rows
    if (__builtin_amdgcn_readfirstlane(spill_on)) {
      for (int i = tid; i < a.Dmax * nb; i += kSliceThreads) {
        const int q = i / nb, n = i - q * nb;
        long long* cell = a.spill + (int64_t)q * a.N + j0 + n;
        const long long v = *cell;
        if (v != 0) {
          __hip_atomic_fetch_add((unsigned long long*)&win[q * B + n], (unsigned long long)v,
                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          *cell = 0;
        }
      }
      if (tid == 0) a.spill_flag[b] = 0;
    }
  } else if (!BIN && a.do_deliver) {
    // Spikes are taken in chunks of one per thread, in list order in every
    // block: the blocks then read neighbouring segments of the same spikes
    // at about the same time.  The barrier after a chunk's descriptors also
    // makes the window zeroing visible to the walk.
    constexpr int G = SynGroup<WF>::n;
    __shared__ int s_next;  // next unclaimed spike of the chunk
    uint64_t ev = 0;
    int64_t total = 0;
    int n_in_spk = 0;  // plastic: input spikes (entries carry several)
    for (int64_t c0 = 0;; c0 += kSliceThreads) {
      // (1) every thread resolves one spike into its segment of this block:
      // the list entry (the first chunk's was loaded with the ring rows),
      // then the segment's (start, count) pair
      const int64_t i = c0 + tid;
      uint32_t ent = ent0;
      if (c0 > 0) ent = i < a.in_cap ? a.in_list[i] : 0u;
      if (c0 == 0) {
        // overflow beyond the list's capacity is flagged by its writer
        const int64_t t = (int64_t)__builtin_amdgcn_readfirstlane(total_raw);
        total = t < a.in_cap ? t : a.in_cap;
      }
      if (c0 >= total) break;
      const int n_c = (int)((total - c0) < kSliceThreads ? (total - c0) : kSliceThreads);
      if (tid < n_c) {
        const uint32_t src = ent >> 5;
        const int lag = (int)(ent & 31u);
        uint2 sg = make_uint2(0u, 0u);
        if (lag < Dmin && (int64_t)src < a.n_src) sg = a.seg[(int64_t)src * a.NB + b];
        else atomicOr(a.overflow, 4);
        const uint32_t len = sg.y;
        desc[tid] = sg;
        meta[tid] = ((uint32_t)(lag * B) << 7) | (len < 65u ? len : 65u) |
                    (((int64_t)src >= a.src_e_end) ? 0x80000000u : 0u);
        if constexpr (PL) {
          // one entry per spiking source and slice: its lags as a mask
          const uint32_t lm = a.in_aux[i];
          lagm[tid] = lm;
          tpv[tid] = a.in_prev[i];
          ev += (uint64_t)len * (uint64_t)__popc(lm);
          n_in_spk += __popc(lm);
        } else {
          ev += (uint64_t)len;
        }
      }
      if (c0 == 0 && tid < kMaxThr) thr[tid] = thr_v;
      if (tid == 0) s_next = 0;
      __syncthreads();
      // (2) waves take groups of G spikes from a shared counter until the
      // chunk is done (a wave slowed by issue priority or memory latency
      // simply takes fewer groups).  G loads issue back to back (lanes past
      // a segment's end and slots past the chunk read record 0, unused),
      // then the adds; the group bound is uniform.
      for (;;) {
        int g0 = 0;
        if (lane == 0)
          g0 = __hip_atomic_fetch_add(&s_next, G, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        g0 = __builtin_amdgcn_readfirstlane(g0);
        if (g0 >= n_c) break;
        const int n_here = (n_c - g0) < G ? (n_c - g0) : G;
        SynRaw<WF> raw[G];
#pragma unroll
        for (int u = 0; u < G; ++u) {
          const uint2 d = desc[g0 + u];  // past the share: stale or padding, masked
          // the start also enters the predicate, so both halves are read
          // unconditionally (no per-slot branch around the LDS read)
          const bool on = (u < n_here) & (lane < (int)d.y) & (d.x != 0xffffffffu);
          raw[u] = syn_fetch<WF>(a.syn, a.syn_dly, on ? d.x + (uint32_t)lane : 0u);
        }
        // ALU work while the loads are in flight
        if (rounds_done < n_rounds) drive_round(rounds_done++);
        uint32_t mt[G];
        bool any_long = false;
#pragma unroll
        for (int u = 0; u < G; ++u) {
          mt[u] = meta[g0 + u];
          any_long |= (mt[u] & 127u) > 64u;  // unconditional use: no sinking
        }
        if constexpr (PL) {
          // plastic: each lane's synapse takes the entry's spikes in lag
          // order, its weight updated before each add and stored back
          const int32_t T = (int32_t)w_lo;
          const int32_t t0s = (int32_t)(w_lo - Dmin);
#pragma unroll
          for (int u = 0; u < G; ++u) {
            const uint32_t m = __builtin_amdgcn_readfirstlane(mt[u]);
            const uint32_t lm = __builtin_amdgcn_readfirstlane(lagm[g0 + u]);
            const int32_t tp0 = __builtin_amdgcn_readfirstlane(tpv[g0 + u]);
            const uint32_t sx = __builtin_amdgcn_readfirstlane(desc[g0 + u].x);
            const bool inh = (int32_t)m < 0;
            const float m1 = inh ? a.wm1_i : a.wm1_e;
            if ((u < n_here) & (lane < (int)(m & 127u)) & (lane < 64)) {
              if constexpr (WF == WF_FP32) {
                float w = __uint_as_float((uint32_t)raw[u].r);
                const int jl = (int)(raw[u].r >> 32) - (int)j0;
                const int dd = (int)raw[u].d;
                if (inh) {
                  const int v = (int)(m1 * w);
                  uint32_t lmi = lm;
                  while (lmi) {
                    const int l = __ffs(lmi) - 1;
                    lmi &= lmi - 1;
                    __hip_atomic_fetch_add((unsigned long long*)&win[(l + dd - Dmin) * B + jl],
                                           (unsigned long long)(long long)v, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                  }
                } else {
                  w = plastic_walk(a, w, dd, pm[jl], pb[jl], lm, tp0, t0s, T, Dmin, B, jl, win,
                                   m1);
                  ((uint32_t*)a.syn)[2 * (size_t)(sx + (uint32_t)lane)] = __float_as_uint(w);
                }
              }
            }
          }
        } else {
#pragma unroll
        for (int u = 0; u < G; ++u) {
          // the meta word is uniform: population constants and the lag row
          // come out of scalar registers
          const uint32_t m = __builtin_amdgcn_readfirstlane(mt[u]);
          const uint32_t sel = (uint32_t)((int32_t)m >> 31);  // all ones: inhibitory
          const float m0 = __uint_as_float((__float_as_uint(a.wm0_e) & ~sel) |
                                           (__float_as_uint(a.wm0_i) & sel));
          const float m1 = __uint_as_float((__float_as_uint(a.wm1_e) & ~sel) |
                                           (__float_as_uint(a.wm1_i) & sel));
          long long* row = win + ((m >> 7) & 0xffffffu);
          if ((u < n_here) & (lane < (int)(m & 127u))) {
            int slot, v;
            syn_decode<WF>(raw[u], (int32_t)j0, Dmin, B, m0, m1, slot, v);
            __hip_atomic_fetch_add((unsigned long long*)&row[slot], (unsigned long long)(long long)v,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          }
        }
        }  // static synapses
        // segments longer than one wave (rare: a block's share of a source's
        // targets is ~K/NB)
        if (__builtin_amdgcn_readfirstlane((int)any_long)) {
          for (int u = 0; u < n_here; ++u) {
            const uint2 d = desc[g0 + u];
            const uint32_t m = meta[g0 + u];
            const int sl = __builtin_amdgcn_readfirstlane((int)d.y);
            const bool inh = (int)m < 0;
            for (int e0 = 64; e0 < sl; e0 += 64) {
              const bool on = lane + e0 < sl;
              const SynRaw<WF> x =
                  syn_fetch<WF>(a.syn, a.syn_dly, on ? d.x + (uint32_t)(e0 + lane) : 0u);
              if constexpr (PL && WF == WF_FP32) {
                if (on) {
                  const uint32_t lm = lagm[g0 + u];
                  float w = __uint_as_float((uint32_t)x.r);
                  const int jl = (int)(x.r >> 32) - (int)j0;
                  const int dd = (int)x.d;
                  const float m1 = inh ? a.wm1_i : a.wm1_e;
                  if (inh) {
                    const int v = (int)(m1 * w);
                    uint32_t lmi = lm;
                    while (lmi) {
                      const int l = __ffs(lmi) - 1;
                      lmi &= lmi - 1;
                      __hip_atomic_fetch_add((unsigned long long*)&win[(l + dd - Dmin) * B + jl],
                                             (unsigned long long)(long long)v, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                  } else {
                    w = plastic_walk(a, w, dd, pm[jl], pb[jl], lm, tpv[g0 + u],
                                     (int32_t)(w_lo - Dmin), (int32_t)w_lo, Dmin, B, jl, win, m1);
                    ((uint32_t*)a.syn)[2 * (size_t)(d.x + (uint32_t)(e0 + lane))] =
                        __float_as_uint(w);
                  }
                }
                continue;
              }
              if (on) {
                int slot, v;
                syn_decode<WF>(x, (int32_t)j0, Dmin, B, inh ? a.wm0_i : a.wm0_e,
                               inh ? a.wm1_i : a.wm1_e, slot, v);
                __hip_atomic_fetch_add(
                    (unsigned long long*)&win[(int)((m >> 7) & 0xffffffu) + slot],
                    (unsigned long long)(long long)v, __ATOMIC_RELAXED,
                    __HIP_MEMORY_SCOPE_WORKGROUP);
              }
            }
          }
        }
      }
      __syncthreads();  // the next chunk overwrites the descriptors
    }
    if (total == 0) {  // no chunk stored the thresholds or made the zeroing visible
      if (tid < kMaxThr) thr[tid] = thr_v;
      __syncthreads();
    }
    // events of this wave
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) ev += __shfl_xor(ev, d, 64);
    if (lane == 0 && ev)
      __hip_atomic_fetch_add(&s_ev, (unsigned long long)ev, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
    if constexpr (PL) {
      // input spikes of the slice (entries carry several): block 0 counts
      if (b == 0) {
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) n_in_spk += __shfl_xor(n_in_spk, d, 64);
        if (lane == 0 && n_in_spk) atomicAdd(a.spk_in_count, (unsigned long long)n_in_spk);
      }
    } else {
      if (tid == 0 && b == 0) atomicAdd(a.spk_in_count, (unsigned long long)total);
    }
  } else {
    if (tid < kMaxThr) thr[tid] = thr_v;
    __syncthreads();  // thr / zeroing visible
  }
  while (rounds_done < n_rounds) drive_round(rounds_done++);

  // staged rows into LDS (when they are not kept in registers)
  if (a.n_upd > 0 && !regs) {
    for (int i = tid; i < rows * nb; i += kSliceThreads) {
      const int q = i / nb, n = i - q * nb;
      int rr = r0 + q;
      while (rr >= a.L) rr -= a.L;
      const int64_t at = (int64_t)rr * a.N + j0 + n;
      carry[q * B + n] = a.rb[at];
    }
    // rows at or past rb_hi hold no earlier input
    for (int i = tid; i < (a.n_upd - rows) * nb; i += kSliceThreads) {
      const int q = rows + i / nb, n = i - (i / nb) * nb;
      carry[q * B + n] = 0.f;
    }
  }
  __syncthreads();
  if (tid == 0 && a.do_deliver && s_ev) atomicAdd(a.ev_count, s_ev);

  // ---- rows of the window due in later slices go to the HBM ring -------
  // Rows [t_first, w_lo + Dmax): all window reads first, then the stores
  // (adds into rows that already hold earlier deliveries).  Threads without
  // a neuron to update write them while the others update; when every
  // thread updates, all write them afterwards.  With fewer free threads
  // than neurons (DYN, blocks of more than half a workgroup), neurons are
  // handed out one at a time from an LDS counter and the updating threads
  // join when their update is done; a fixed share per free thread would
  // keep the flush running long after the update.
  auto flush_rows = [&](int t0, int stride) {
    constexpr int kFl = 8;
    const float inv = a.fx_inv;
    int64_t t_first = a.t_upd + a.n_upd;
    if (t_first < w_lo) t_first = w_lo;
    const int nrows = (int)(w_lo + a.Dmax - t_first);
    const int q0 = (int)(t_first - w_lo);
    const int row0 = (int)(t_first % a.L);
    int64_t add_rows = a.rb_hi - t_first;  // leading rows that are added into
    if (add_rows < 0) add_rows = 0;
    if (add_rows > nrows) add_rows = nrows;
    const int n_add = (int)add_rows;
    for (int n = t0;; n += stride) {
      if constexpr (DYN)
        n = __hip_atomic_fetch_add(&s_fl, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (n >= nb) break;
      for (int k0 = 0; k0 < nrows; k0 += kFl) {
        // Rows past nrows are clamped to the last one, so every read is in
        // range and none sits behind a branch: the ring loads of the rows
        // added into issue together, and one wait covers them.
        float v[kFl], old[kFl];
        float* p[kFl];
#pragma unroll
        for (int k = 0; k < kFl; ++k) {
          const int kk = (k0 + k < nrows) ? k0 + k : nrows - 1;
          int row = row0 + kk;
          if (row >= a.L) row -= a.L;  // row0 < L and nrows <= Dmax < L
          p[k] = a.rb + (int64_t)row * a.N + j0 + n;
          old[k] = k0 + k < n_add ? *p[k] : 0.f;
          v[k] = from_fixed(win[(q0 + kk) * B + n], inv);
        }
#pragma unroll
        for (int k = 0; k < kFl; ++k)
          if (k0 + k < nrows) *p[k] = old[k] + v[k];
      }
    }
  };
  const bool split = a.n_upd > 0 && nb < kSliceThreads;
  if (a.do_deliver && split && tid >= nb) flush_rows(tid - nb, kSliceThreads - nb);

  // ---- update the next slice's steps (exact propagation, Sec. 2.1) -------
  // Two compiled forms, staged rows in registers (kRegs) or in LDS: with
  // one run-time form the compiler puts each step's read behind a branch
  // on the (uniform) choice and waits for it there.
  auto update = [&](auto regs_tag) {
    constexpr bool kRegs = decltype(regs_tag)::value;
    const float P11 = a.prop[0], P21 = a.prop[1], P22 = a.prop[2], P31 = a.prop[3];
    const float P32 = a.prop[4], P33 = a.prop[5], P30Ie = a.prop[6], insc = a.prop[7];
    const float inv = a.fx_inv;
    for (int n = tid; n < nb; n += kSliceThreads) {
      const int64_t gn = j0 + n;
      float V, y1 = 0.f, y2 = 0.f;
      int r;
      uint64_t hm = 0;
      int32_t hb = -1;
      if constexpr (PL) {
        hm = pm[n];
        hb = pb[n];
      }
      if (n == tid) {
        V = sV;
        r = sr;
        y1 = sy1;
        y2 = sy2;
      } else {
        V = a.V[gn];
        r = a.r[gn];
        if (a.model == MODEL_ALPHA) {
          y1 = a.y1[gn];
          y2 = a.y2[gn];
        }
      }
      // inputs of up to 16 steps are read from LDS up front (independent
      // reads), then the steps run on registers
      constexpr int kSteps = 16;
      const int qw = (int)(a.t_upd - w_lo);  // window row of the first step
      // fields used per step, read once (a read inside a step would wait
      // for the LDS reads issued before it: both share one counter)
      const int n_upd = a.n_upd, Dmax = a.Dmax;
      const bool deliv = a.do_deliver != 0;
      const float drive_w = a.drive_w;
      const float e_l = a.e_l, v_th = a.v_th, v_reset = a.v_reset;
      const int ref_steps = a.ref_steps, lag_upd = (int)(a.t_upd - a.t_slice0);
      const bool delta = a.model == MODEL_DELTA;
      for (int s0 = 0; s0 < n_upd; s0 += kSteps) {
        // All reads at in-range rows (clamped), results masked afterwards.
        // The scheduling barrier keeps the scheduler from pairing each read
        // with its use, so the reads issue back to back and one wait covers
        // them.
        long long wq[kSteps];
        uint32_t dc[kSteps];
        float cv[kSteps];
#pragma unroll
        for (int q = 0; q < kSteps; ++q) {
          const int s = s0 + q;
          const bool on = s < n_upd;
          const int sc = on ? s : 0;
          const bool w_on = deliv & on & (qw + s >= 0) & (qw + s < Dmax);
          // the address is chosen, not the value: a read whose value is
          // selected by a uniform condition ends up behind a branch
          wq[q] = *(w_on ? &win[(qw + s) * B + n] : &s_zero);
          dc[q] = dcnt[sc * B + n];
          if constexpr (!kRegs) cv[q] = carry[sc * B + n];
        }
        __builtin_amdgcn_sched_barrier(0);
        float in_s[kSteps], dr_s[kSteps];
#pragma unroll
        for (int q = 0; q < kSteps; ++q) {
          const int s = s0 + q;
          const bool on = s < n_upd;
          float in;
          if constexpr (kRegs) in = s < rows ? stage[q] : 0.f;  // one pass (s == q), n == tid
          else in = cv[q];
          in += from_fixed(wq[q], inv);
          in_s[q] = on ? in : 0.f;
          dr_s[q] = on ? (float)dc[q] * drive_w : 0.f;
        }
        for (int q = 0; q < kSteps; ++q) {
        const int s = s0 + q;
        if (s >= n_upd) break;
        const float in = in_s[q];
        const float drive = dr_s[q];
        if (delta) {
          if (r > 0) --r;
          else V = e_l + P33 * (V - e_l) + P30Ie + in + drive;
        } else {
          if (r == 0) V = e_l + P31 * y1 + P32 * y2 + P33 * (V - e_l) + P30Ie;
          else --r;
          const float y2n = P21 * y1 + P22 * y2;
          y1 = P11 * y1 + insc * (in + drive);
          y2 = y2n;
        }
        const bool spk = V >= v_th;
        if (spk) {
          V = v_reset;
          r = ref_steps;
        }
        if constexpr (PL) {
          // the step leaving the 64-step history becomes the earlier spike
          if (hm >> 63) hb = (int32_t)(a.t_upd + s) - 64;
          hm = (hm << 1) | (uint64_t)spk;
        }
        {
          // the step's spikes of this wave's 64 neurons (consecutive, first
          // lane active whenever any is): one ballot, two mask words
          const uint64_t bal = __ballot(spk);
          if (lane == 0) {
            const int w0 = (n - lane) >> 5;
            mask[(lag_upd + s) * Wd + w0] = (uint32_t)bal;
            mask[(lag_upd + s) * Wd + w0 + 1] = (uint32_t)(bal >> 32);
          }
        }
        }
      }
      if constexpr (PL) {
        pm[n] = hm;
        pb[n] = hb;
        a.pmask[gn] = hm;
        a.pbefore[gn] = hb;
      }
      a.V[gn] = V;
      a.r[gn] = r;
      if (a.model == MODEL_ALPHA) {
        a.y1[gn] = y1;
        a.y2[gn] = y2;
      }
    }
  };
  if (a.n_upd > 0) {
    if (regs) update(BoolC<true>{});
    else update(BoolC<false>{});
  }

  if (a.do_deliver && (!split || (DYN && tid < nb))) flush_rows(tid, kSliceThreads);
  __syncthreads();

  // ---- plastic nets: one entry per spiking neuron, when its slice is complete
  if constexpr (PL) {
    if (a.n_upd > 0 && a.t_upd + a.n_upd == a.t_slice0 + Dmin) {
      uint32_t lm = 0;
      int32_t tprev = -1;
      if (tid < nb) {
        // bit k of the history is step t_slice0 + Dmin - 1 - k: lag l is bit
        // Dmin - 1 - l; older bits give the spike before the slice
        const uint64_t hm = pm[tid];
        for (int l = 0; l < Dmin; ++l) lm |= (uint32_t)((hm >> (Dmin - 1 - l)) & 1u) << l;
        const uint64_t older = hm >> Dmin;
        tprev = older ? (int32_t)(a.t_slice0 - 1) - (int32_t)__builtin_ctzll(older) : pb[tid];
      }
      // entry positions: wave ballot + mbcnt, wave counts scanned in LDS;
      // neuron order within the block
      const bool has = lm != 0u;
      const uint64_t bal = __ballot(has);
      const int in_wave =
          (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                         __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
      __shared__ int s_wc[kSliceThreads / 64 + 1];
      __shared__ int s_ebase;
      if (lane == 0) s_wc[wv] = __popcll(bal);
      __syncthreads();
      if (tid == 0) {
        int acc = 0;
        for (int i = 0; i < nwv; ++i) {
          const int c = s_wc[i];
          s_wc[i] = acc;
          acc += c;
        }
        s_ebase = acc ? atomicAdd(a.out_cnt, acc) : 0;
      }
      __syncthreads();
      if (has) {
        const int64_t pos = (int64_t)s_ebase + s_wc[wv] + in_wave;
        const int64_t gn = j0 + tid;
        if (pos < a.out_cap) {
          a.out_list[pos] = (uint32_t)gn << 5;
          a.out_aux[pos] = lm;
          a.out_prev[pos] = tprev;
        } else {
          atomicOr(a.overflow, 1);
        }
      }
      __syncthreads();  // s_wc is reused below
    }
  }

  // ---- compaction: this block's new spikes, (lag, neuron) ordered --------
  // (plastic nets: their list entries are built above; here the raster and
  // the spike count only)
  if (a.n_upd > 0) {
    const int write_list = PL ? 0 : a.write_list;
    const int lag0 = (int)(a.t_upd - a.t_slice0);
    const int nq = a.n_upd * Wd;
    __shared__ int s_base;
    __shared__ unsigned long long s_rbase;
    int running = 0;
    for (int q0 = 0; q0 < nq; q0 += kSliceThreads) {
      const int q = q0 + tid;
      uint32_t m = (q < nq) ? mask[lag0 * Wd + q] : 0u;
      int tot;
      const int ex = block_excl_scan<int>(__popc(m), scr, tot);
      if (tot == 0) continue;
      // one reservation per block in the slice's list (and the raster)
      if (tid == 0) {
        s_base = write_list ? atomicAdd(a.out_cnt, tot) : 0;
        s_rbase = a.rec ? atomicAdd(a.rec_n, (unsigned long long)tot) : 0ull;
      }
      __syncthreads();
      const int64_t base = s_base;
      const unsigned long long rbase = s_rbase;
      __syncthreads();
      int pos = ex;
      const int lg = lag0 + q / Wd;
      const int nbase = (q % Wd) * 32;
      while (m) {
        const int bit = __ffs(m) - 1;
        m &= m - 1;
        const int64_t gn = j0 + nbase + bit;
        if (write_list) {
          if (base + pos < a.out_cap)
            a.out_list[base + pos] = ((uint32_t)gn << 5) | (uint32_t)lg;
          else
            atomicOr(a.overflow, 1);
        }
        if (a.rec) {
          const unsigned long long rp = rbase + (unsigned long long)pos;
          if ((int64_t)rp < a.rec_cap) a.rec[rp] = make_uint2((uint32_t)(a.t_slice0 + lg), (uint32_t)gn);
          else atomicOr(a.overflow, 2);
        }
        ++pos;
      }
      running += tot;
    }
    if (tid == 0 && running) atomicAdd(a.spk_count, (unsigned long long)running);
  }
}

// The slice kernels read their argument fields where they are used (kept
// in registers for the whole kernel they would crowd out the walk's).  Each
// first read of a 64-byte line of the argument block would then be a
// scalar-cache miss of its own, one after another; one load per line at
// entry, all waited for together, brings the block in with one round trip.
template <typename T>
__device__ __forceinline__ void touch_lines(const T* p) {
  constexpr int kWords = (int)(sizeof(T) / 4);
  constexpr int kLines = (kWords + 15) / 16;
  const uint32_t* w = (const uint32_t*)p;
  uint32_t v[kLines];
#pragma unroll
  for (int i = 0; i < kLines; ++i) v[i] = w[i * 16 < kWords ? i * 16 : kWords - 1];
  // keep the loads (their values are otherwise unused)
#pragma unroll
  for (int i = 0; i < kLines; ++i) asm volatile("" ::"s"(v[i]));
}

// Workgroup gx serves target block map[gx].y of network map[gx].x (one
// network, or the members of a batch), whose arguments for this slice are
// args[map[gx].x]; map[gx].x < 0 marks a padding workgroup.  The map is
// XCD-aware: workgroups gx and gx + 8 run on the same XCD, and consecutive
// blocks of a network are placed on one XCD so they share segment-pointer
// lines in its L2.  Arguments live in device memory, so the compiler loads
// fields where they are used instead of holding the whole struct in
// scalar registers.
template <int WF>
__global__ void __launch_bounds__(kSliceThreads)
    k_slice(const SliceArgs* __restrict__ args, const int2* __restrict__ map) {
  const int2 m = map[blockIdx.x];
  if (m.x < 0) return;
  touch_lines(args + m.x);
  slice_block<WF, false, false>(args[m.x], m.y);
}

// One network: the arguments travel by value in the kernel-argument segment
// (read where used, through a pointer to that segment), and the block is
// (gx & 7) * per_xcd + (gx >> 3).  This saves the dependent loads of the
// batched form at the start of every wave.
struct SingleArgs {
  SliceArgs a;
  int32_t per_xcd;
};
template <int WF, bool BIN, bool DYN, bool PL = false>
__global__ void __launch_bounds__(kSliceThreads) k_slice1(SingleArgs s) {
  const SingleArgs* p = (const SingleArgs*)__builtin_amdgcn_kernarg_segment_ptr();
  touch_lines(p);
  const int gx = blockIdx.x;
  const int b = (gx & 7) * p->per_xcd + (gx >> 3);
  if (b >= p->a.NB) return;
  slice_block<WF, BIN, DYN, PL>(p->a, b);
}

// ---------------------------------------------------------------------------
// persistent multi-slice kernel (block-major, static synapses, closed loop)
// ---------------------------------------------------------------------------
// One cooperative launch runs S consecutive fused slices of a network whose
// blocks are all resident at once (one workgroup per block).  A workgroup
// keeps its block's delivery window in LDS for the whole launch, as a ring
// of Dmax rows indexed by step modulo Dmax: a delivery adds into the rows of
// steps [w_lo, w_lo + Dmax) (Alg. REF, Sec. 3.2), the update reads the rows
// of its steps and clears them for reuse, and only at the end do the rows
// due after the last slice go to the HBM ring.  Window sums therefore stay
// in fixed point until their step is updated.  Neuron state stays in
// registers.  Slices are separated by a grid barrier, since the spike list
// one slice writes is read by every block in the next; the lists and their
// three rotating counters are those of the one-launch-per-slice path.
constexpr int64_t kBarSpin = 1LL << 22;  // default polls before a grid barrier gives up

// All workgroups of the launch wait here; the release fence publishes this
// workgroup's global writes (spike list, counters) and the acquire fence
// drops stale lines of other workgroups' writes.  A wait past spin_limit polls
// sets bit 4 of the overflow flags, and every workgroup then leaves.
__device__ bool grid_barrier(unsigned* bar, unsigned target, int32_t* overflow,
                             int64_t spin_limit) {
  __shared__ int s_ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int64_t spins = 0;
    int ok = 1;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if ((++spins & 255) == 0 &&
          (__hip_atomic_load(overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 16)) {
        ok = 0;
        break;
      }
      if (spins > spin_limit) {
        atomicOr(overflow, 16);
        ok = 0;
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

struct PersistArgs {
  SliceArgs a;         // network constants; time and list fields of slice 0
  uint32_t* lists[2];  // the two spike-list buffers
  int32_t* cnt3;       // the three rotating list counters
  int32_t cur0, ci0;   // slice 0 reads lists[cur0] with count cnt3[ci0]
  int32_t pend0;       // slice 0 delivers that list (else no delivery)
  int32_t S;           // slices
  int32_t per_xcd;     // blocks per XCD (grid = 8 * per_xcd)
  int64_t t0;          // first step of slice 0
  int64_t rb_hi0;      // HBM ring rows of steps below this hold earlier sums
  unsigned* bar;       // grid-barrier arrivals (zero at launch)
  int64_t spin_limit;  // polls before a grid barrier gives up
};

template <int WF>
__global__ void __launch_bounds__(kSliceThreads) k_persist(PersistArgs p) {
  const PersistArgs* pp = (const PersistArgs*)__builtin_amdgcn_kernarg_segment_ptr();
  const SliceArgs& a = pp->a;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int tid = threadIdx.x, lane = tid & 63;
  const int gx = blockIdx.x;
  const int b = (gx & 7) * pp->per_xcd + (gx >> 3);
  const bool live = b < a.NB;  // padding workgroups only take part in the barriers
  const int B = a.B, Dmin = a.Dmin, R = a.Dmax, NB = a.NB;
  const int RB = R * B;
  const int64_t j0 = (int64_t)(live ? b : 0) * B;
  const int nb = live ? (int)((a.N - j0) < B ? (a.N - j0) : B) : 0;
  const int Wd = B >> 5;
  const SliceLds Lo = slice_lds_layout(B, Dmin, R);
  long long* win = (long long*)(lds_raw + Lo.win);
  uint8_t* dcnt = lds_raw + Lo.dcnt;
  uint32_t* mask = (uint32_t*)(lds_raw + Lo.mask);
  uint32_t* thr = (uint32_t*)(lds_raw + Lo.thr);
  int32_t* scr = (int32_t*)(lds_raw + Lo.scr);
  uint2* desc = (uint2*)(lds_raw + Lo.desc);
  uint32_t* meta = (uint32_t*)(lds_raw + Lo.meta);
  __shared__ int s_next, s_base;
  __shared__ unsigned long long s_rbase, s_ev;

  for (int i = tid; i < RB; i += kSliceThreads) win[i] = 0;
  if (tid < kMaxThr) thr[tid] = (tid < a.n_thr) ? a.thr[tid] : 0xffffffffu;
  if (tid == 0) s_ev = 0;
  // neuron state of this thread's neuron, in registers for the launch
  const bool own = tid < nb;
  const int64_t gn = j0 + (own ? tid : 0);
  float V = 0.f, y1 = 0.f, y2 = 0.f;
  int rf = 0;
  if (own) {
    V = a.V[gn];
    rf = a.r[gn];
    if (a.model == MODEL_ALPHA) {
      y1 = a.y1[gn];
      y2 = a.y2[gn];
    }
  }
  const float P11 = a.prop[0], P21 = a.prop[1], P22 = a.prop[2], P31 = a.prop[3];
  const float P32 = a.prop[4], P33 = a.prop[5], P30Ie = a.prop[6], insc = a.prop[7];
  const float inv = a.fx_inv, drive_w = a.drive_w;
  const float e_l = a.e_l, v_th = a.v_th, v_reset = a.v_reset;
  const int ref_steps = a.ref_steps;
  const bool delta = a.model == MODEL_DELTA;
  float m0e = a.wm0_e, m0i = a.wm0_i, m1e = a.wm1_e, m1i = a.wm1_i;
  asm volatile("" : "+s"(m0e), "+s"(m0i), "+s"(m1e), "+s"(m1i));
  unsigned long long spk_all = 0, in_all = 0;
  const int64_t t0 = pp->t0, rb_hi0 = pp->rb_hi0;
  const int S = pp->S;
  int cur = pp->cur0, ci = pp->ci0;
  bool ok = true;
  __syncthreads();  // window, thresholds

  for (int k = 0; k < S && ok; ++k) {
    const int64_t w_lo = t0 + (int64_t)k * Dmin;  // first step of slice k
    const bool deliver = k > 0 || pp->pend0;
    const uint32_t* in_list = pp->lists[cur];
    int32_t* in_cnt = pp->cnt3 + ci;
    uint32_t* out_list = pp->lists[cur ^ 1];
    int32_t* out_cnt = pp->cnt3 + (ci + 1) % 3;
    // the counter of slice k + 1's list starts at zero; its last reader was
    // slice k - 1's delivery, before the barrier
    if (gx == 0 && tid == 0) __hip_atomic_store(pp->cnt3 + (ci + 2) % 3, 0, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    for (int i = tid; i < Dmin * Wd; i += kSliceThreads) mask[i] = 0u;
    // ---- drive counts of the slice's steps (Philox, as in the fused slice)
    {
      const int64_t c0 = w_lo >> 3, c1 = (w_lo + Dmin - 1) >> 3;
      const int n_tasks = live ? (int)(c1 - c0 + 1) * nb : 0;
      for (int task = tid; task < n_tasks; task += kSliceThreads) {
        const int n = task % nb;
        const int64_t c = c0 + task / nb;
        uint64_t rr[4];
        philox(a.seed, STREAM_DRIVE, (uint64_t)(j0 + n), (uint64_t)c, rr);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int64_t t = c * 8 + q;
          if (t < w_lo || t >= w_lo + Dmin) continue;
          const uint64_t word = rr[q >> 1];
          const uint32_t u = (q & 1) ? (uint32_t)(word >> 32) : (uint32_t)word;
          int cnt = 0;
          while (cnt < a.n_thr && u >= thr[cnt]) ++cnt;
          dcnt[(int)(t - w_lo) * B + n] = (uint8_t)cnt;
        }
      }
    }
    // ---- delivery of the previous slice's spikes into the window ring ----
    if (deliver && live) {
      constexpr int G = SynGroup<WF>::n;
      const int base = (int)(w_lo % R);  // ring row of step w_lo
      int64_t total = __hip_atomic_load(in_cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (total > a.in_cap) total = a.in_cap;  // overflow is flagged by the writer
      uint64_t ev = 0;
      for (int64_t c0 = 0; c0 < total; c0 += kSliceThreads) {
        const int n_c = (int)((total - c0) < kSliceThreads ? (total - c0) : kSliceThreads);
        __syncthreads();  // the previous chunk's descriptors are no longer read
        if (tid < n_c) {
          const uint32_t ent = in_list[c0 + tid];
          const uint32_t src = ent >> 5;
          const int lag = (int)(ent & 31u);
          uint2 sg = make_uint2(0u, 0u);
          if (lag < Dmin && (int64_t)src < a.n_src) sg = a.seg[(int64_t)src * NB + b];
          else atomicOr(a.overflow, 4);
          desc[tid] = sg;
          // ring offset of the spike's arrival rows: row (base + lag + delay
          // - Dmin) mod R, the modulo taken per synapse
          meta[tid] = ((uint32_t)((lag + base) * B) << 7) | (sg.y < 65u ? sg.y : 65u) |
                      (((int64_t)src >= a.src_e_end) ? 0x80000000u : 0u);
          ev += sg.y;
        }
        if (tid == 0) s_next = 0;
        __syncthreads();
        for (;;) {
          int g0 = 0;
          if (lane == 0)
            g0 = __hip_atomic_fetch_add(&s_next, G, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          g0 = __builtin_amdgcn_readfirstlane(g0);
          if (g0 >= n_c) break;
          const int n_here = (n_c - g0) < G ? (n_c - g0) : G;
          SynRaw<WF> raw[G];
#pragma unroll
          for (int u = 0; u < G; ++u) {
            const uint2 d = desc[g0 + u];  // past the chunk: stale or padding, masked
            const bool on = (u < n_here) & (lane < (int)d.y);
            raw[u] = syn_fetch<WF>(a.syn, a.syn_dly, on ? d.x + (uint32_t)lane : 0u);
          }
          bool any_long = false;
#pragma unroll
          for (int u = 0; u < G; ++u) {
            const uint32_t m = __builtin_amdgcn_readfirstlane(meta[g0 + u]);
            any_long |= (u < n_here) & ((m & 127u) > 64u);
            const bool inh = (int32_t)m < 0;
            if ((u < n_here) & (lane < (int)(m & 127u)) & (lane < 64)) {
              int slot, v;
              syn_decode<WF>(raw[u], (int32_t)j0, Dmin, B, inh ? m0i : m0e, inh ? m1i : m1e,
                             slot, v);
              uint32_t x = ((m >> 7) & 0xffffffu) + (uint32_t)slot;
              x = min(x, x - (uint32_t)RB);  // below 2 R B: one wrap at most
              __hip_atomic_fetch_add((unsigned long long*)&win[x], (unsigned long long)(long long)v,
                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
          }
          // segments longer than one wave
          if (any_long) {
            for (int u = 0; u < n_here; ++u) {
              const uint2 d = desc[g0 + u];
              const uint32_t m = meta[g0 + u];
              const int sl = __builtin_amdgcn_readfirstlane((int)d.y);
              const bool inh = (int32_t)m < 0;
              for (int e0 = 64; e0 < sl; e0 += 64) {
                const bool on = lane + e0 < sl;
                const SynRaw<WF> xr =
                    syn_fetch<WF>(a.syn, a.syn_dly, on ? d.x + (uint32_t)(e0 + lane) : 0u);
                if (on) {
                  int slot, v;
                  syn_decode<WF>(xr, (int32_t)j0, Dmin, B, inh ? m0i : m0e, inh ? m1i : m1e,
                                 slot, v);
                  uint32_t x = ((m >> 7) & 0xffffffu) + (uint32_t)slot;
                  x = min(x, x - (uint32_t)RB);
                  __hip_atomic_fetch_add((unsigned long long*)&win[x],
                                         (unsigned long long)(long long)v, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_WORKGROUP);
                }
              }
            }
          }
        }
      }
#pragma unroll
      for (int d = 32; d > 0; d >>= 1) ev += __shfl_xor(ev, d, 64);
      if (lane == 0 && ev)
        __hip_atomic_fetch_add(&s_ev, (unsigned long long)ev, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
      if (b == 0 && tid == 0) in_all += (unsigned long long)total;
    }
    __syncthreads();  // window adds and drive counts complete
    // ---- update of the slice's Dmin steps, reading (and clearing) the ring
    if (own) {
      for (int s = 0; s < Dmin; ++s) {
        const int64_t t = w_lo + s;
        long long* cell = &win[(int)(t % R) * B + tid];
        float in = from_fixed(*cell, inv);
        *cell = 0;
        if (t < rb_hi0) in += a.rb[(t % a.L) * a.N + gn];  // sums from before the launch
        const float drive = (float)dcnt[s * B + tid] * drive_w;
        if (delta) {
          if (rf > 0) --rf;
          else V = e_l + P33 * (V - e_l) + P30Ie + in + drive;
        } else {
          if (rf == 0) V = e_l + P31 * y1 + P32 * y2 + P33 * (V - e_l) + P30Ie;
          else --rf;
          const float y2n = P21 * y1 + P22 * y2;
          y1 = P11 * y1 + insc * (in + drive);
          y2 = y2n;
        }
        const bool spk = V >= v_th;
        if (spk) {
          V = v_reset;
          rf = ref_steps;
        }
        const uint64_t bal = __ballot(spk);
        if (lane == 0) {
          const int w0 = (tid - lane) >> 5;
          mask[s * Wd + w0] = (uint32_t)bal;
          mask[s * Wd + w0 + 1] = (uint32_t)(bal >> 32);
        }
      }
    }
    __syncthreads();
    // ---- compaction into slice k + 1's list, (lag, neuron) ordered -------
    if (live) {
      const int nq = Dmin * Wd;
      for (int q0 = 0; q0 < nq; q0 += kSliceThreads) {
        const int q = q0 + tid;
        uint32_t m = (q < nq) ? mask[q] : 0u;
        int tot;
        const int ex = block_excl_scan<int>(__popc(m), scr, tot);
        if (tot == 0) continue;
        if (tid == 0) {
          s_base = atomicAdd(out_cnt, tot);
          s_rbase = a.rec ? atomicAdd(a.rec_n, (unsigned long long)tot) : 0ull;
        }
        __syncthreads();
        const int64_t lbase = s_base;
        const unsigned long long rbase = s_rbase;
        __syncthreads();
        int pos = ex;
        const int lg = q / Wd;
        const int nbase = (q % Wd) * 32;
        while (m) {
          const int bit = __ffs(m) - 1;
          m &= m - 1;
          const int64_t g = j0 + nbase + bit;
          if (lbase + pos < a.out_cap) out_list[lbase + pos] = ((uint32_t)g << 5) | (uint32_t)lg;
          else atomicOr(a.overflow, 1);
          if (a.rec) {
            const unsigned long long rp = rbase + (unsigned long long)pos;
            if ((int64_t)rp < a.rec_cap) a.rec[rp] = make_uint2((uint32_t)(w_lo + lg), (uint32_t)g);
            else atomicOr(a.overflow, 2);
          }
          ++pos;
        }
        if (tid == 0) spk_all += (unsigned long long)tot;
      }
    }
    cur ^= 1;
    ci = (ci + 1) % 3;
    if (k + 1 < S)
      ok = grid_barrier(pp->bar, (unsigned)gridDim.x * (unsigned)(k + 1), a.overflow,
                        pp->spin_limit);
  }
  if (!live) return;
  // ---- rows due after the last slice go to the HBM ring ---------------------
  const int64_t t_end = t0 + (int64_t)S * Dmin;
  const bool delivered = S > 1 || pp->pend0;
  if (ok && delivered && own) {
    const int64_t hi = t_end - Dmin + R;  // end of the last delivery window
    for (int64_t t = t_end; t < hi; ++t) {
      const float v = from_fixed(win[(int)(t % R) * B + tid], inv);
      float* cell = a.rb + (t % a.L) * a.N + gn;
      *cell = (t < rb_hi0) ? *cell + v : v;
    }
  }
  if (own) {
    a.V[gn] = V;
    a.r[gn] = rf;
    if (a.model == MODEL_ALPHA) {
      a.y1[gn] = y1;
      a.y2[gn] = y2;
    }
  }
  __syncthreads();  // s_ev complete
  if (tid == 0) {
    if (s_ev) atomicAdd(a.ev_count, s_ev);
    if (in_all) atomicAdd(a.spk_in_count, in_all);
    if (spk_all) atomicAdd(a.spk_count, spk_all);
  }
}

// ---------------------------------------------------------------------------
// helpers: ring gap zeroing, open-loop input schedule, decoded export
// ---------------------------------------------------------------------------
__global__ void k_zero_rows(float* rb, int64_t N, int32_t L, int64_t t_lo, int64_t t_hi) {
  const int64_t rows = t_hi - t_lo;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows * N;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = t_lo + i / N;
    rb[(t % L) * N + (i % N)] = 0.f;
  }
}

// One word set by a one-thread kernel: a clear issued on a stream that a
// caller may be capturing becomes a kernel node rather than a memset node.
__global__ void k_set_word(unsigned* p, unsigned v) { *p = v; }

// An external spike list (separate source and lag arrays) packed into the
// delivery's entry format (src << 5 | lag), validated on the device: an
// entry with src >= n_src or lag >= d_min becomes kBadEntry (delivers
// nothing) and sets bit 3 of the sticky flag word.  Workgroup 0's first
// thread stores the entry count, so the list needs no host round trip and
// no memset (the count is in place before any later kernel on the stream
// reads it).
constexpr uint32_t kBadEntry = 0xffffffffu;  // src 2^27 - 1 >= n_src, lag 31
__global__ void k_pack_list(const uint32_t* src, const uint8_t* lag, int64_t n, int64_t n_src,
                            int32_t Dmin, uint32_t* out, int32_t* cnt, int32_t* flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint32_t s = src[i];
    const uint32_t l = lag[i];
    const bool ok = (int64_t)s < n_src && (int32_t)l < Dmin;
    out[i] = ok ? (s << 5) | l : kBadEntry;
    bad |= !ok;
  }
  if (bad) atomicOr(flag, 8);
  if (blockIdx.x == 0 && threadIdx.x == 0) *cnt = (int32_t)n;
}

__device__ __forceinline__ uint32_t half32(const uint64_t w[4], int64_t t) {
  const uint64_t x = w[(t & 7) >> 1];
  return (t & 1) ? (uint32_t)(x >> 32) : (uint32_t)x;
}

// spikes of every virtual source over [t0, t0 + n_steps), counted per slice
// (source, 8-step chunk) items, grid-stride: a schedule of many slices of
// a brain-scale population has more items than one dispatch's 2^32
// work-items.
__global__ void k_input_count(uint64_t seed, int64_t n_src, int64_t t0, int32_t n_steps,
                              int32_t Dmin, uint32_t thr, int32_t* cnt) {
  const int64_t n_chunks = ((t0 + n_steps - 1) >> 3) - (t0 >> 3) + 1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_src * n_chunks;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = i % n_src;
    const int64_t c = (t0 >> 3) + i / n_src;
    uint64_t w[4];
    philox(seed, STREAM_SRC, (uint64_t)s, (uint64_t)c, w);
    for (int q = 0; q < 8; ++q) {
      const int64_t t = c * 8 + q;
      if (t < t0 || t >= t0 + n_steps) continue;
      if (half32(w, t) < thr) atomicAdd(&cnt[(t - t0) / Dmin], 1);
    }
  }
}

__global__ void k_input_fill(uint64_t seed, int64_t n_src, int64_t t0, int32_t n_steps,
                             int32_t Dmin, uint32_t thr, const int64_t* off, int32_t* cursor,
                             uint32_t* list) {
  const int64_t n_chunks = ((t0 + n_steps - 1) >> 3) - (t0 >> 3) + 1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_src * n_chunks;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = i % n_src;
    const int64_t c = (t0 >> 3) + i / n_src;
    uint64_t w[4];
    philox(seed, STREAM_SRC, (uint64_t)s, (uint64_t)c, w);
    for (int q = 0; q < 8; ++q) {
      const int64_t t = c * 8 + q;
      if (t < t0 || t >= t0 + n_steps) continue;
      if (half32(w, t) < thr) {
        const int64_t sl = (t - t0) / Dmin;
        const int lag = (int)((t - t0) - sl * Dmin);
        const int p = atomicAdd(&cursor[sl], 1);
        list[off[sl] + p] = ((uint32_t)s << 5) | (uint32_t)lag;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
// Workgroups of a grid-stride launch over n items: enough to fill the
// device, and far below a dispatch's 2^32 work-items.
unsigned stride_grid(int64_t n, int threads) {
  const int64_t want = (n + threads - 1) / threads;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)1 << 20));
}

hipError_t launch_propagators(hipStream_t s, int model, double h, double tau_m, double tau_syn,
                              double c_m, double i_e, double* p64, float* p32) {
  hipLaunchKernelGGL(k_propagators, dim3(1), dim3(1), 0, s, model, h, tau_m, tau_syn, c_m, i_e,
                     p64, p32);
  return hipGetLastError();
}

hipError_t launch_init_state(hipStream_t s, int64_t N, uint64_t seed, double v0_lo, double v0_hi,
                             float* V, float* y1, float* y2, int32_t* r) {
  const int nt = 256;
  const int64_t nbk = (N + nt - 1) / nt;
  hipLaunchKernelGGL(k_init_state, dim3((unsigned)nbk), dim3(nt), 0, s, N, seed, v0_lo, v0_hi, V,
                     y1, y2, r);
  return hipGetLastError();
}

hipError_t launch_count(hipStream_t s, const BuildArgs& a) {
  hipLaunchKernelGGL(k_count, dim3((unsigned)a.N), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t scan_impl(hipStream_t s, T* data, int64_t n, T* tile_sums, int64_t n_tiles_cap) {
  const int64_t n_tiles = (n + kScanTile - 1) / kScanTile;
  if (n_tiles > n_tiles_cap) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_scan_tiles<T>, dim3((unsigned)n_tiles), dim3(kScanThreads), 0, s, data, n,
                     tile_sums);
  hipLaunchKernelGGL(k_scan_sums<T>, dim3(1), dim3(kScanThreads), 0, s, tile_sums, n_tiles);
  hipLaunchKernelGGL(k_scan_apply<T>, dim3((unsigned)n_tiles), dim3(kScanThreads), 0, s, data, n,
                     tile_sums);
  return hipGetLastError();
}

hipError_t launch_scan(hipStream_t s, uint32_t* data, int64_t n, uint32_t* tile_sums,
                       int64_t n_tiles_cap) {
  return scan_impl<uint32_t>(s, data, n, tile_sums, n_tiles_cap);
}

hipError_t launch_scan64(hipStream_t s, unsigned long long* data, int64_t n,
                         unsigned long long* tile_sums, int64_t n_tiles_cap) {
  return scan_impl<unsigned long long>(s, data, n, tile_sums, n_tiles_cap);
}

hipError_t launch_count_sm(hipStream_t s, const BuildArgs& a) {
  hipLaunchKernelGGL(k_count_sm, dim3((unsigned)a.N), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fill_sm(hipStream_t s, const BuildArgs& a) {
  hipLaunchKernelGGL(k_fill_sm, dim3((unsigned)a.N), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_bin(hipStream_t s, const BinArgs& a, int32_t P, size_t lds, bool w8) {
  if (w8) hipLaunchKernelGGL(k_bin<true>, dim3((unsigned)P), dim3(kBinThreads), lds, s, a);
  else hipLaunchKernelGGL(k_bin<false>, dim3((unsigned)P), dim3(kBinThreads), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_fill(hipStream_t s, const BuildArgs& a) {
  hipLaunchKernelGGL(k_fill, dim3((unsigned)a.NB), dim3(kFillThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gather_block(hipStream_t s, const uint2* seg, int64_t n_src, int32_t NB,
                               int32_t b, const int64_t* dst_off, const void* syn,
                               const uint8_t* dly, int32_t rec_bytes, void* out, uint8_t* out_dly) {
  hipLaunchKernelGGL(k_gather_block, dim3((unsigned)((n_src + 255) / 256)), dim3(256), 0, s, seg,
                     n_src, NB, b, dst_off, syn, dly, rec_bytes, out, out_dly);
  return hipGetLastError();
}

hipError_t launch_seg_pairs(hipStream_t s, const BuildArgs& a) {
  const int64_t n = a.n_src * a.NB;
  hipLaunchKernelGGL(k_seg_pairs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a.row, a.n_src,
                     a.NB, a.seg);
  return hipGetLastError();
}

hipError_t launch_slice(hipStream_t s, const SliceArgs* d_args, const int2* d_map,
                        int32_t n_blocks, size_t lds, int wform) {
  if (n_blocks <= 0) return hipSuccess;
  const dim3 grid((unsigned)n_blocks), block(kSliceThreads);
  switch (wform) {
    case WF_FP32:
      hipLaunchKernelGGL(k_slice<WF_FP32>, grid, block, lds, s, d_args, d_map);
      break;
    case WF_BF16:
      hipLaunchKernelGGL(k_slice<WF_BF16>, grid, block, lds, s, d_args, d_map);
      break;
    case WF_PACKED:
      hipLaunchKernelGGL(k_slice<WF_PACKED>, grid, block, lds, s, d_args, d_map);
      break;
    default:
      hipLaunchKernelGGL(k_slice<WF_BF16_RESID>, grid, block, lds, s, d_args, d_map);
      break;
  }
  return hipGetLastError();
}

template <bool DYN>
void launch_slice1_as(hipStream_t s, const SingleArgs& sa, size_t lds, int wform) {
  const dim3 grid((unsigned)(8 * sa.per_xcd)), block(kSliceThreads);
  if (sa.a.plastic) {  // plastic synapses: FP32 block-major only
    hipLaunchKernelGGL((k_slice1<WF_FP32, false, DYN, true>), grid, block, lds, s, sa);
    return;
  }
  if (sa.a.bins) {
    // binned records: 8 bytes (FP32 weight) or 4 (BF16 bits)
    if (wform == WF_FP32) hipLaunchKernelGGL((k_slice1<WF_FP32, true, DYN>), grid, block, lds, s, sa);
    else hipLaunchKernelGGL((k_slice1<WF_BF16, true, DYN>), grid, block, lds, s, sa);
    return;
  }
  switch (wform) {
    case WF_FP32:
      hipLaunchKernelGGL((k_slice1<WF_FP32, false, DYN>), grid, block, lds, s, sa);
      break;
    case WF_BF16:
      hipLaunchKernelGGL((k_slice1<WF_BF16, false, DYN>), grid, block, lds, s, sa);
      break;
    case WF_PACKED:
      hipLaunchKernelGGL((k_slice1<WF_PACKED, false, DYN>), grid, block, lds, s, sa);
      break;
    default:
      hipLaunchKernelGGL((k_slice1<WF_BF16_RESID, false, DYN>), grid, block, lds, s, sa);
      break;
  }
}

hipError_t launch_slice1(hipStream_t s, const SliceArgs& a, size_t lds, int wform) {
  SingleArgs sa;
  sa.a = a;
  sa.per_xcd = (a.NB + 7) / 8;
  // blocks of more than half a workgroup: fewer free threads than neurons
  if (kSliceThreads - a.B < a.B) launch_slice1_as<true>(s, sa, lds, wform);
  else launch_slice1_as<false>(s, sa, lds, wform);
  return hipGetLastError();
}

// Workgroups per CU that a persistent launch of this weight form can hold.
int persist_occupancy(int wform, size_t lds) {
  int occ = 0;
  hipError_t e;
  switch (wform) {
    case WF_FP32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_persist<WF_FP32>, kSliceThreads, lds); break;
    case WF_BF16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_persist<WF_BF16>, kSliceThreads, lds); break;
    case WF_PACKED: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_persist<WF_PACKED>, kSliceThreads, lds); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_persist<WF_BF16_RESID>, kSliceThreads, lds); break;
  }
  return e == hipSuccess ? occ : 0;
}

// Cooperative launch: the runtime refuses a grid that cannot be resident at
// once, so the grid barriers cannot wait on a workgroup that never starts.
hipError_t launch_persist(hipStream_t s, const SliceArgs& a, uint32_t* const lists[2],
                          int32_t* cnt3, int32_t cur0, int32_t ci0, int32_t pend0, int32_t S,
                          int64_t t0, int64_t rb_hi0, unsigned* bar, int64_t spin_limit,
                          size_t lds, int wform) {
  PersistArgs p;
  p.a = a;
  p.lists[0] = lists[0];
  p.lists[1] = lists[1];
  p.cnt3 = cnt3;
  p.cur0 = cur0;
  p.ci0 = ci0;
  p.pend0 = pend0;
  p.S = S;
  p.per_xcd = (a.NB + 7) / 8;
  p.t0 = t0;
  p.rb_hi0 = rb_hi0;
  p.bar = bar;
  p.spin_limit = spin_limit < 0 ? kBarSpin : spin_limit;
  void* args[] = {&p};
  const dim3 grid((unsigned)(8 * p.per_xcd)), block(kSliceThreads);
  switch (wform) {
    case WF_FP32: return hipLaunchCooperativeKernel((const void*)k_persist<WF_FP32>, grid, block, args, lds, s);
    case WF_BF16: return hipLaunchCooperativeKernel((const void*)k_persist<WF_BF16>, grid, block, args, lds, s);
    case WF_PACKED: return hipLaunchCooperativeKernel((const void*)k_persist<WF_PACKED>, grid, block, args, lds, s);
    default: return hipLaunchCooperativeKernel((const void*)k_persist<WF_BF16_RESID>, grid, block, args, lds, s);
  }
}

// Captured batches: the argument sets of a period of slices move on by
// shift steps (the time fields of a steady-state fused slice).
__global__ void k_shift_args(SliceArgs* args, int32_t n, int64_t shift) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= n) return;
  args[i].t_upd += shift;
  args[i].t_slice0 += shift;
  args[i].w_lo += shift;
  args[i].rb_hi += shift;
}

hipError_t launch_shift_args(hipStream_t s, SliceArgs* args, int32_t n, int64_t shift) {
  hipLaunchKernelGGL(k_shift_args, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, args, n, shift);
  return hipGetLastError();
}

hipError_t launch_set_word(hipStream_t s, unsigned* p, unsigned v) {
  hipLaunchKernelGGL(k_set_word, dim3(1), dim3(1), 0, s, p, v);
  return hipGetLastError();
}

hipError_t launch_zero_rows(hipStream_t s, float* rb, int64_t N, int32_t L, int64_t t_lo,
                            int64_t t_hi) {
  if (t_hi <= t_lo) return hipSuccess;
  const int64_t n = (t_hi - t_lo) * N;
  hipLaunchKernelGGL(k_zero_rows, dim3(stride_grid(n, 256)), dim3(256), 0, s, rb, N, L, t_lo,
                     t_hi);
  return hipGetLastError();
}

hipError_t launch_pack_list(hipStream_t s, const uint32_t* src, const uint8_t* lag, int64_t n,
                            int64_t n_src, int32_t Dmin, uint32_t* out, int32_t* cnt,
                            int32_t* flag) {
  const int64_t want = (n + 255) / 256;
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, 4096));
  hipLaunchKernelGGL(k_pack_list, dim3(grid), dim3(256), 0, s, src, lag, n, n_src, Dmin, out,
                     cnt, flag);
  return hipGetLastError();
}

hipError_t launch_input_count(hipStream_t s, uint64_t seed, int64_t n_src, int64_t t0,
                              int32_t n_steps, int32_t Dmin, uint32_t thr, int32_t* cnt) {
  const int64_t n_chunks = ((t0 + n_steps - 1) >> 3) - (t0 >> 3) + 1;
  const int64_t n = n_src * n_chunks;
  hipLaunchKernelGGL(k_input_count, dim3(stride_grid(n, 256)), dim3(256), 0, s, seed,
                     n_src, t0, n_steps, Dmin, thr, cnt);
  return hipGetLastError();
}

hipError_t launch_input_fill(hipStream_t s, uint64_t seed, int64_t n_src, int64_t t0,
                             int32_t n_steps, int32_t Dmin, uint32_t thr, const int64_t* off,
                             int32_t* cursor, uint32_t* list) {
  const int64_t n_chunks = ((t0 + n_steps - 1) >> 3) - (t0 >> 3) + 1;
  const int64_t n = n_src * n_chunks;
  hipLaunchKernelGGL(k_input_fill, dim3(stride_grid(n, 256)), dim3(256), 0, s, seed,
                     n_src, t0, n_steps, Dmin, thr, off, cursor, list);
  return hipGetLastError();
}


}  // namespace sd
