// qg_layout.h -- byte layouts shared by the host side of libqg and its kernels.
//
// Vertex block (Sec. 3.1.3 of the SymphonyQG paper: raw vector, FastScan data,
// neighbours, in one contiguous segment), for dimension D and out-degree R:
//   [0, 4D)                 raw vector, fp32
//   [4D, 4D + R*D/8)        codes: neighbour j's D-bit RaBitQ code at j*D/8, dim i in byte i/8 bit i%8
//   next 4R bytes           f_add[R]      fp32
//   next 4R bytes           f_rescale[R]  fp32
//   next 4R bytes           nbr[R]        int32 (-1 = empty slot)
//   zero padding to a multiple of 128 bytes (one HBM-friendly aligned segment).
#pragma once
#include <stdint.h>

namespace qgl {

__host__ __device__ constexpr int64_t block_bytes(int D, int R) {
  return (4LL * D + (int64_t)R * (D / 8) + 12LL * R + 127) / 128 * 128;
}
__host__ __device__ constexpr int off_codes(int D) { return 4 * D; }
__host__ __device__ constexpr int off_fadd(int D, int R) { return 4 * D + R * (D / 8); }
__host__ __device__ constexpr int off_fres(int D, int R) { return off_fadd(D, R) + 4 * R; }
__host__ __device__ constexpr int off_nbr(int D, int R) { return off_fadd(D, R) + 8 * R; }

// Per-wavefront LDS of the search kernel (bytes).  ef_cap and k_cap are
// multiples of 4 so every piece stays 16-byte aligned.
struct SearchLds {
  int lut, beam, cand, hash, nkey, nid, qv, aux, total;
};

__host__ __device__ constexpr int align16(int x) { return (x + 15) & ~15; }

// Wide vectors keep the raw query in LDS instead of registers.
__host__ __device__ constexpr bool query_in_lds(int D) { return D > 256; }

// LUT rows are 16 int16 entries (32 bytes).  With two lanes per neighbour the
// second lane's rows start one padding row later so that the two halves of a
// wavefront read different LDS banks.
__host__ __device__ constexpr int lut_rows_padded(int D, int R) { return D / 4 + (64 / R) - 1; }

// cand: one expansion's candidates (R words + 4 of padding), reused for their
// insertion points; beam: packed (key, id | checked) words kept sorted; hash:
// visited ids; nkey/nid: the k nearest vertices found so far; qv: the raw
// query when D > 256; aux: 256 bytes through which the learned stop's MLP
// passes its features and first hidden layer.  The pieces
// indexed by lane (LUT, candidates, beam) come first, at offsets fixed by D
// and R, so one address register serves them with immediate offsets.  With R
// even, D and the caps multiples of 4 (the host rounds them), the hash and the
// whole area are multiples of 16 bytes, so the hash can be read 16 bytes at a
// time in every wavefront's area.
__host__ __device__ inline SearchLds search_lds(int D, int R, int ef_cap, int hash_cap, int k_cap,
                                                int lut_entry_bytes = 2) {
  SearchLds s{};
  int o = 0;
  s.lut = o;   o += align16(lut_rows_padded(D, R) * 16 * lut_entry_bytes);
  s.cand = o;  o += 8 * (R + 4);
  s.beam = o;  o += 8 * ef_cap;
  s.hash = o;  o += 4 * hash_cap;
  s.nkey = o;  o += 4 * k_cap;
  s.nid = o;   o += 4 * k_cap;
  s.qv = o;    o += query_in_lds(D) ? 4 * D : 0;
  s.aux = o;   o += 256;
  s.total = o;
  return s;
}

}  // namespace qgl
