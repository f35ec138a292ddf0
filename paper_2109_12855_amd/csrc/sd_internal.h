// sd_internal.h -- shared declarations between the host library and the
// gfx950 kernels (internal; not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/sdeliver.h"

namespace sd {

enum { STREAM_SYN = 1, STREAM_INIT = 2, STREAM_DRIVE = 3, STREAM_SRC = 4 };
enum { MODEL_DELTA = 0, MODEL_ALPHA = 1 };
enum { WF_FP32 = 0, WF_BF16 = 1, WF_BF16_RESID = 2, WF_PACKED = 3 };

constexpr int kMaxThr = 64;        // Poisson-drive threshold table entries
constexpr int kSliceThreads = 1024;  // threads of a slice workgroup
constexpr int kFillThreads = 512;    // threads of a build workgroup
constexpr int kFillChunk = 2048;     // draws ranked per build iteration

// Synapse record layouts (one record per synapse, plus a u8 delay array for
// the first three forms):
//   WF_FP32        u64: low word FP32 weight bits, high word i32 target id
//   WF_BF16        u32: low half BF16 weight, high half u16 offset in block
//   WF_BF16_RESID  u32: low half BF16 residual d (w = mu (1 + d)), high half
//                  u16 offset in block
//   WF_PACKED      u32: low half BF16 residual, high half the ring-window
//                  slot (delay - d_min) * B + offset in block (no delay array)

// Everything a slice launch needs (passed by value).
struct SliceArgs {
  // network layout
  const uint2* seg;        // [n_src][NB]: (first synapse, count) of source s in block b
  int64_t n_src;           // source ids
  const void* syn;         // synapse records (layout per weight form)
  const uint8_t* syn_dly;  // u8 delay in steps (not used by the packed form)
  int64_t N;               // local neurons
  int32_t NB, B;           // blocks, neurons per block
  int32_t K;               // in-degree: block b's synapses start at b * B * K
  int32_t Dmin, Dmax, L;
  int32_t win_rows;        // rows of the LDS window (Dmax; 0: no LDS delivery)
  int64_t src_e_end;       // source ids below this are excitatory
  // fixed-point weight of a synapse: trunc(m1 * x + m0) with x the decoded
  // BF16 residual (residual forms) or the weight itself (FP32, BF16); the
  // pairs hold the scale 2^s of the LDS window (count mode: m1 = 0, m0 = 2^s)
  float wm0_e, wm1_e, wm0_i, wm1_i;
  float fx_inv;            // 2^-s
  int32_t grid_per_xcd;    // blocks handled by one XCD (ceil(NB / 8))
  // delivery
  int32_t do_deliver;
  const uint32_t* in_list; // spike entries (src << 5 | lag), contiguous
  const int32_t* in_cnt;   // number of entries (device)
  int64_t in_cap;          // entries the list can hold
  int64_t w_lo;            // first step of the delivery window
  // update
  int32_t n_upd;           // steps to update (0: none)
  int64_t t_upd;           // first step to update
  int64_t t_slice0;        // start step of the slice the new spikes belong to
  float* V;
  float* y1;
  float* y2;
  int32_t* r;
  float prop[8];           // P11 P21 P22 P31 P32 P33 P30*I_e in_scale (FP32, by value)
  const uint32_t* thr;     // Poisson-drive thresholds
  int32_t n_thr;
  uint64_t seed;
  float e_l, v_th, v_reset, drive_w;
  int32_t ref_steps;
  int32_t model;
  // source-major layout: the slice's events binned by target block (k_bin).
  // Block b reads the bin_P regions [b * bin_P + p] of bin_cap records each,
  // holding bin_cnt[b * bin_P + p] records; events past a full region were
  // added into spill (64-bit fixed point, [Dmax][N] window rows), which block
  // b consumes and clears when spill_flag[b] is set.  bins null: block-major.
  const void* bins;
  const uint32_t* bin_cnt;
  int32_t bin_P, bin_cap;
  long long* spill;
  int32_t* spill_flag;
  // plastic synapses (block-major FP32 form, closed loop): per neuron the
  // spikes of the last 64 updated steps (bit k: step T - 1 - k, T the first
  // step not yet updated) and its latest spike before them (-1: none); per
  // list entry (one per spiking neuron and slice, src << 5) the slice's lag
  // mask (bit l: a spike at lag l) and the source's spike before the slice
  int32_t plastic;
  uint64_t* pmask;
  int32_t* pbefore;
  const uint32_t* in_aux;
  const int32_t* in_prev;
  uint32_t* out_aux;
  int32_t* out_prev;
  float stdp_ap, stdp_am;   // amplitudes A+, A-
  float stdp_kp, stdp_km;   // h / (tau ln 2): exp(-x h / tau) = exp2(-x k)
  float stdp_wmax;
  // ring buffer [L][N] (FP32)
  float* rb;
  int64_t rb_hi;           // rows of steps in [., rb_hi) hold valid sums
  // new spikes
  int32_t write_list;      // closed loop: feed spikes back
  uint32_t* out_list;      // contiguous list of out_cap entries
  int32_t* out_cnt;        // entries reserved so far (atomic; zero at a new slice)
  int64_t out_cap;
  int32_t* zero_cnt;       // list counter to clear for a later slice (may be null)
  uint2* rec;              // raster (step, id); null: off
  unsigned long long* rec_n;
  int64_t rec_cap;
  // counters
  unsigned long long* ev_count;    // synaptic events delivered
  unsigned long long* spk_in_count;// spike entries delivered
  unsigned long long* spk_count;   // spikes emitted
  int32_t* overflow;               // bit 0: list, bit 1: raster, bit 2: bad entry,
                                   // bit 3: bad entry in an external list
};

struct BuildArgs {
  int64_t N, n_src;
  int32_t NB, B, K, k_exc;
  int64_t src_e_n, src_i_n, src_i_base;
  int32_t d_lo, n_dly;
  uint64_t seed;
  uint32_t* row;           // (src, block) counts, then exclusive scan (block-major)
  uint32_t* cursor;        // fill cursors (copy of row)
  uint2* seg;              // source-major (start, count) pairs
  // source-major layout: one segment per (source, target part), parts of
  // 2^tbits targets; record word = offset in part | (delay - d_min) << tbits
  // | weight bits 8-15 << 24 (BF16 forms), plus the weight's low byte (u8) or
  // the f32 weight
  unsigned long long* row64;     // counts, then exclusive scan, per (source, part)
  unsigned long long* cursor64;  // fill cursors
  uint32_t* tw;                  // record words
  void* wbits;                   // u8 low weight bytes, or f32 weights
  int32_t tbits, H;
  void* syn;
  uint8_t* syn_dly;
  int32_t wform;
  int32_t d_min;
  const void* wtab_e;      // encoded weight per quantile index (f32 or bf16 bits)
  const void* wtab_i;
  float w_fix_e, w_fix_i;  // fixed weights (cv == 0), encoded at use
  uint32_t fix_bits_e, fix_bits_i;
  int32_t fixed;
};

// Source-major delivery, pass 1: the events of a slice's spikes are sorted by
// target block and written as binned records into per-(block, workgroup)
// regions (record layout at kBinSlotBits).
struct BinArgs {
  const unsigned long long* row;  // [n_src * H + 1] segment starts per (source, part)
  const uint32_t* tw;             // offset | (delay - d_min) << tbits | weight bits 8-15 << 24
  const void* wbits;              // u8 weight bits 0-7, or f32 weight
  int32_t tbits, H;               // target part = 2^tbits targets, H parts (<= 4)
  const uint32_t* in_list;        // (src << 5 | lag)
  const int32_t* in_cnt;
  int64_t in_cap;
  int64_t n_src, N;
  int32_t B, NB, Dmin, U;         // U: events per thread per sorting chunk
  int32_t cap;                    // records per region
  float inv_B;                    // 1 / B (estimate of target / B)
  int64_t src_e_end;
  float wm0_e, wm1_e, wm0_i, wm1_i;  // fixed-point weights of spilled events
  void* bins;                     // [NB][P][cap] records
  uint32_t* bin_cnt;              // [NB][P] records per region
  long long* spill;               // [Dmax][N]
  int32_t* spill_flag;            // [NB]
  unsigned long long* ev_count;
  unsigned long long* spk_in_count;
  int32_t* overflow;
};
// Binned record: bits [0, 15) the window slot q * B + offset in block, where
// q = lag + delay - d_min is the arrival step's row of the delivery window,
// bit 15 the inhibitory flag, bits [16, 32) the BF16 weight or residual; the
// FP32 form adds the f32 weight as a second word.
constexpr int kBinSlotBits = 15;
constexpr int kBinThreads = 1024;
constexpr int kBinSpikes = 1024;  // segment entries resolved per descriptor batch
constexpr int kBinMaxU = 12;      // events per thread per sorting chunk (4-byte records; 16 spills)
constexpr int kBinMaxU8 = 8;      // the same for 8-byte records (12 spill)
constexpr int kBinProducers = 256;
constexpr int kBinMaxCap = 1024;  // records per region (consumer work items <= 1024)
constexpr int kBinSlice = 256;    // records per consumer work item
constexpr int kBinSegTab = 8192;  // binning: event -> segment-entry lookup entries per batch
constexpr int kBinGrp = 4;        // binning: LDS reads issued before one wait (divides kBinMaxU)
size_t bin_lds_bytes(int NB, int U, bool w8);
// source-major record word: offset in part (tbits) | delay - d_min (dbits),
// tbits + dbits <= 24, the top byte holds the BF16 weight's high byte
constexpr int kRecWordBits = 24;
constexpr int kMaxParts = 64;
constexpr int kPartBits = 18;  // source-major target parts of at most 2^18 targets

// launch wrappers (sd_kernels.hip)
hipError_t launch_propagators(hipStream_t s, int model, double h, double tau_m, double tau_syn,
                              double c_m, double i_e, double* prop64, float* prop32);
hipError_t launch_init_state(hipStream_t s, int64_t N, uint64_t seed, double v0_lo, double v0_hi,
                             float* V, float* y1, float* y2, int32_t* r);
hipError_t launch_count(hipStream_t s, const BuildArgs& a);
hipError_t launch_scan(hipStream_t s, uint32_t* data, int64_t n, uint32_t* tile_sums,
                       int64_t n_tiles_cap);
hipError_t launch_fill(hipStream_t s, const BuildArgs& a);
hipError_t launch_seg_pairs(hipStream_t s, const BuildArgs& a);
hipError_t launch_gather_block(hipStream_t s, const uint2* seg, int64_t n_src, int32_t NB,
                               int32_t b, const int64_t* dst_off, const void* syn,
                               const uint8_t* dly, int32_t rec_bytes, void* out, uint8_t* out_dly);
// one fused slice of a batch: workgroup gx serves block map[gx].y of
// network map[gx].x, arguments in device memory
hipError_t launch_slice(hipStream_t s, const SliceArgs* d_args, const int2* d_map,
                        int32_t n_blocks, size_t lds, int wform);
// one fused slice of a single network, arguments by value
hipError_t launch_slice1(hipStream_t s, const SliceArgs& a, size_t lds, int wform);
int persist_occupancy(int wform, size_t lds);
hipError_t launch_persist(hipStream_t s, const SliceArgs& a, uint32_t* const lists[2],
                          int32_t* cnt3, int32_t cur0, int32_t ci0, int32_t pend0, int32_t S,
                          int64_t t0, int64_t rb_hi0, unsigned* bar, int64_t spin_limit,
                          size_t lds, int wform);
size_t slice_lds_bytes(int B, int Dmin, int win_rows, bool plastic = false, bool bin = false);
// add shift to the time fields (t_upd, t_slice0, w_lo, rb_hi) of args[0..n)
hipError_t launch_shift_args(hipStream_t s, SliceArgs* args, int32_t n, int64_t shift);
hipError_t launch_count_sm(hipStream_t s, const BuildArgs& a);
hipError_t launch_scan64(hipStream_t s, unsigned long long* data, int64_t n,
                         unsigned long long* tile_sums, int64_t n_tiles_cap);
hipError_t launch_fill_sm(hipStream_t s, const BuildArgs& a);
hipError_t launch_bin(hipStream_t s, const BinArgs& a, int32_t P, size_t lds, bool w8);
hipError_t launch_zero_rows(hipStream_t s, float* rb, int64_t N, int32_t L, int64_t t_lo,
                            int64_t t_hi);
hipError_t launch_set_word(hipStream_t s, unsigned* p, unsigned v);
// pack and validate an external spike list (see k_pack_list); cnt receives n
hipError_t launch_pack_list(hipStream_t s, const uint32_t* src, const uint8_t* lag, int64_t n,
                            int64_t n_src, int32_t Dmin, uint32_t* out, int32_t* cnt,
                            int32_t* flag);
hipError_t launch_input_count(hipStream_t s, uint64_t seed, int64_t n_src, int64_t t0,
                              int32_t n_steps, int32_t Dmin, uint32_t thr, int32_t* cnt);
hipError_t launch_input_fill(hipStream_t s, uint64_t seed, int64_t n_src, int64_t t0,
                             int32_t n_steps, int32_t Dmin, uint32_t thr, const int64_t* off,
                             int32_t* cursor, uint32_t* list);

// host library internals used by other translation units (sd_api.cpp)
// sd_deliver_spikes with the packed list (cap entries) and its count in
// caller-chosen device memory
sd_status deliver_external(sd_ctx* c, const uint32_t* d_src, const uint8_t* d_lag, int64_t n,
                           int64_t t0, uint32_t* list, int32_t* list_cnt, int64_t cap);
// record an error message on the context and return st
sd_status set_error(sd_ctx* c, sd_status st, const char* msg);
// device the context was created on
int ctx_device(const sd_ctx* c);

}  // namespace sd
