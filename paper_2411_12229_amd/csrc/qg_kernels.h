// qg_kernels.h -- launch interface between the libqg host code and its kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qgk {

struct SearchArgs {
  const uint8_t* blocks;
  int64_t block_bytes;
  int64_t N;
  const float* queries;  // [nq][D] raw queries
  const float* qrot;     // [nq][D] rotated queries
  int64_t nq;
  int k, ef, k_cap, ef_cap;
  int hash_bits;  // LDS visited hash holds 2^hash_bits ids
  int lut_pad;    // LUT layout: 1 = a padding row between lane groups, 0 = packed rows
  int flags;
  int entry;
  const int32_t* k_q;     // nullable: per-query k (then k is the bound)
  const int32_t* ef_q;    // nullable: per-query ef (then ef is the bound)
  int k_out;              // output row stride (k, or the bound of a mixed batch)
  int32_t* out_ids;
  float* out_dists;
  int32_t* out_stats;     // nullable, [nq][4]
  int* counters;          // [0] main queue, [1] overflow count, [2] overflow queue
  int32_t* overflow_list; // [nq]
  uint32_t* fb_bits;      // overflow pass: one N-bit set per wavefront
  int64_t fb_words;       // 32-bit words per set
  // learned stop (ls_mode 1 and 2)
  const uint16_t* ls_w;   // MLP parameters (bf16 bits) or null: evaluate and trace only
  float ls_theta;
  int ls_t_min, ls_t_every;
  int tr_max;             // evaluation points traced per query (0 = no trace)
  float* tr_feat;         // [nq][tr_max][16]
  int32_t* tr_nn;         // [nq][tr_max][k]
  float* tr_out;          // [nq][tr_max]
  int32_t* tr_count;      // [nq]
};

struct EstimateArgs {
  const uint8_t* blocks;
  int64_t block_bytes;
  const float* queries;
  const float* qrot;
  const int32_t* vertex;
  int32_t* out_S;
  float* out_est;
  float* out_dist;
  int lut_pad;  // LUT layout, as in SearchArgs
};

// Allocation-free search: size of the fixed per-device scratch array and its
// device address on `device` (which must be current); the address is looked
// up once per device.
constexpr size_t kNoAllocScratchBytes = (size_t)16 << 20;
constexpr int kMaxDevices = 64;
hipError_t noalloc_scratch(int device, uint8_t** out);

bool shape_supported(int D, int R);
hipError_t launch_rotate(const float* in, int64_t n, int D, const float* M, float* out, int* zero, int nzero,
                         hipStream_t st);
hipError_t launch_encode(const float* X, const float* ROT, int64_t N, int D, const int32_t* G, int R,
                         uint8_t* blocks, int64_t B, hipStream_t st);
// ls_mode: 0 plain search, 1 learned stop (MLP staged in LDS, mlp_lds_bytes()
// after the wavefront areas), 2 learned stop with trace (MLP read from global),
// 3 per-query k and ef (k_q, ef_q set), 4 per-query k and ef with the learned
// stop (MLP staged in LDS, as for 1), 5 "w/o ME" (the hash holds estimated
// vertices, not visited ones)
// nb: beam registers per lane (0: beam in LDS; 1, 2: ef up to 64, 128), as
// beam_regs() picks for the pass, mode, bound on ef and vector count.
int beam_regs(bool overflow_pass, int ls_mode, int ef_bound, int64_t n);
hipError_t launch_search(int D, int R, bool overflow_pass, int ls_mode, int nb, int lb, const SearchArgs& a, int grid,
                         int wpb, size_t lds, hipStream_t st);
int search_occupancy(int D, int R, bool overflow_pass, int ls_mode, int nb, int lb, int wpb, size_t lds);
constexpr size_t mlp_lds_bytes() { return 2 * 64 * 16 + 8 * 64 * 16 + 3 * 128 + 16; }
hipError_t launch_estimate(int D, int R, const EstimateArgs& a, int64_t nq, hipStream_t st);

}  // namespace qgk
