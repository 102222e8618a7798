// qg_kernels.hip -- gfx950 kernels of the SymphonyQG query path.
//
//  rotate_kernel  : Y = X M^T on the matrix cores (fp64 MFMA 16x16x4, k ascending).
//  encode_kernel  : RaBitQ codes and factors of every edge, one wavefront per vertex.
//  search_kernel  : Algorithm 1, one query per wavefront; LUT, beam and visited
//                   hash live in LDS, the top-k in registers (k <= 64) or LDS,
//                   vertex blocks stream from HBM.
//  estimate_kernel: the estimator alone for (query, vertex) pairs.
//
// Compiled with -ffp-contract=off: every fused multiply-add below is explicit.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "qg_kernels.h"
#include "qg_layout.h"

namespace qgk {

// Fixed device scratch of the allocation-free search entry point (queue
// counters, rotated queries, overflow list), one copy per device for as long
// as the library is loaded.  Host code must not pass `scratch` itself to a
// kernel (in host code it names a host-side stand-in); it takes the device
// address from noalloc_scratch().
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(int device, uint8_t** out) {
  static std::mutex mu;
  static uint8_t* addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[device]) {  // once per device, with that device current
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = static_cast<uint8_t*>(p);
  }
  *out = addr[device];
  return hipSuccess;
}

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr uint32_t kChecked = 0x80000000u;
constexpr uint32_t kIdMask = 0x7fffffffu;
// Register-resident beams also flag entries whose vertex has been expanded
// through another entry (consumed duplicates); ids then take 30 bits.
constexpr uint32_t kDup = 0x40000000u;
constexpr uint32_t kIdMask30 = 0x3fffffffu;
constexpr uint32_t kEmpty = 0xffffffffu;

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ int first_lane(uint64_t m) { return __ffsll((unsigned long long)m) - 1; }

__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_wave_barrier(); }

// Values every lane of the wavefront holds identically (broadcast LDS reads,
// ballot-derived counts, butterfly results) are moved to scalar registers so
// control flow on them is a scalar branch.
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint32_t uni(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }
__device__ __forceinline__ float uni(float x) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x))); }

// (key, id) lexicographic order, without branches.
__device__ __forceinline__ bool kv_less(float ka, uint32_t ia, float kb, uint32_t ib) {
  return (ka < kb) | ((ka == kb) & (ia < ib));
}

// (key, id) packed into one unsigned 64-bit integer whose order is the
// lexicographic (key, id) order of the floats: -0 is first mapped to +0 (the
// two compare equal), then the usual sign flip makes the bits sortable.
__device__ __forceinline__ uint32_t sortable(float x) {
  const uint32_t u = __float_as_uint(x + 0.0f);
  return u ^ ((uint32_t)((int32_t)u >> 31) | 0x80000000u);
}
__device__ __forceinline__ float unsortable(uint32_t s) {
  return __uint_as_float((s & 0x80000000u) ? (s ^ 0x80000000u) : ~s);
}
__device__ __forceinline__ uint64_t pack_kv(float key, uint32_t id) { return ((uint64_t)sortable(key) << 32) | id; }

// Minimum over the wavefront of an unsigned value, through DPP: within each
// row of 16 lanes by quad permutes and row rotations, then across rows by the
// row broadcasts of lanes 15 and 31; lane 63 ends with the minimum.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_min_step(uint32_t v) {
  const uint32_t o = (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFFu, (int)v, CTRL, ROWS, 0xF, false);
  return o < v ? o : v;
}
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  v = dpp_min_step<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v = dpp_min_step<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v = dpp_min_step<0x124, 0xF>(v);  // row_ror:4
  v = dpp_min_step<0x128, 0xF>(v);  // row_ror:8
  v = dpp_min_step<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_min_step<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// x from lane (lane ^ s) for s = 1, 2 (DPP quad permutes).  Pure data movement.
template <int S>
__device__ __forceinline__ int xor_lane_i(int v) {
  static_assert(S == 1 || S == 2, "xor distance");
  if constexpr (S == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);
  return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);
}
template <int S>
__device__ __forceinline__ float xor_lane(float x) { return __int_as_float(xor_lane_i<S>(__float_as_int(x))); }

// x from lane (lane + s) mod 16 within its row of 16 lanes (DPP row rotation),
// s = 4 or 8.  For s = 8 that lane is lane ^ 8.
template <int S>
__device__ __forceinline__ float row_ror(float x) {
  static_assert(S == 4 || S == 8, "rotation");
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x120 | S, 0xF, 0xF, false));
}

// The pair {x[l], x[l ^ 32]} (pair32) or {x[l], x[l ^ 16]} (pair16) in every
// lane l, through the gfx950 swaps of the two wavefront halves and of the odd
// and even rows of 16 lanes (which of the two comes first depends on the lane;
// only symmetric combinations of the pair are used).
__device__ __forceinline__ void pair32(float x, float& a, float& b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  a = __uint_as_float(r[0]);
  b = __uint_as_float(r[1]);
}
__device__ __forceinline__ void pair16(float x, float& a, float& b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  a = __uint_as_float(r[0]);
  b = __uint_as_float(r[1]);
}

// Butterfly sum p[l] + p[l ^ s] for s = 32, 16, ..., 1; every lane ends with
// the total.  Floating-point addition is commutative, so each stage adds
// exactly the pair the stage names whatever the order within the pair.  The
// stage of 4 takes its partner from the rotation by 4: after the stage of 8,
// lanes l and l ^ 8 hold the same bits, and the rotated-in lane (l + 4) mod 16
// is l ^ 4 or l ^ 12.  No stage goes through LDS.
__device__ __forceinline__ float butterfly_f(float p) {
  float a, b;
  pair32(p, a, b);
  p = a + b;
  pair16(p, a, b);
  p = a + b;
  p = p + row_ror<8>(p);
  p = p + row_ror<4>(p);
  p = p + xor_lane<2>(p);
  p = p + xor_lane<1>(p);
  return p;
}

__device__ __forceinline__ float wave_max(float v) {
  float a, b;
  pair32(v, a, b);
  v = fmaxf(a, b);
  pair16(v, a, b);
  v = fmaxf(a, b);
  v = fmaxf(v, row_ror<8>(v));
  v = fmaxf(v, row_ror<4>(v));
  v = fmaxf(v, xor_lane<2>(v));
  v = fmaxf(v, xor_lane<1>(v));
  return v;
}

// Exact squared distance |q - x|^2 (implicit re-ranking, Sec. 3.1.2): dim i
// into lane i mod 64 by a fused multiply-add chain in ascending i, then the
// xor butterfly p[l] + p[l^s], s = 32 ... 1.  Every lane ends with the result.
template <int DPL>
__device__ __forceinline__ float exact_dist(const float (&qv)[DPL], const float (&xv)[DPL]) {
  float p = 0.0f;
#pragma unroll
  for (int t = 0; t < DPL; ++t) {
    float d = qv[t] - xv[t];
    p = __builtin_fmaf(d, d, p);
  }
  return butterfly_f(p);
}

// ---------------------------------------------------------------- rotation

// out[r][i] = fl32(sum_j M[i][j] in[r][j]), fp64 products accumulated over j
// ascending (each 16x16x4 MFMA applies its four k terms in order as fused
// multiply-adds onto the accumulator).  A wavefront computes an NT x NT block
// of 16x16 output tiles (NT = 2: each staged fragment of the queries and of M
// feeds two products).  Workgroup b takes row block 8 (b / 8 / T) + b % 8 and
// column block (b / 8) % T (T = D / 16 NT): workgroups are dealt to the 8 XCDs
// round robin, so the T column blocks of one row block run on one XCD and read
// those rows through its L2 once.  Workgroup 0 also clears `nzero` ints at
// `zero` for the kernels that follow.  V4: the input rows start 16-byte
// aligned, so each lane moves four columns per load and per LDS store.
template <bool V4, int NT>
__global__ __launch_bounds__(64) void rotate_kernel(const float* __restrict__ in, int64_t n, int D,
                                                    const float* __restrict__ M, float* __restrict__ out,
                                                    int* __restrict__ zero, int nzero) {
  // the block's 16 NT input rows and 16 NT rows of M, 64 columns at a time,
  // staged through LDS with coalesced loads (rows padded to 68 floats); the
  // next chunk's loads are issued before this chunk's products
  constexpr int KC = 64, LD = KC + 4, RB = 16 * NT;
  __shared__ __align__(16) float As[RB * LD];
  __shared__ __align__(16) float Bs[RB * LD];
  const int lane = threadIdx.x;
  if (zero && blockIdx.x == 0 && lane < nzero) zero[lane] = 0;
  const int T = D / RB;
  const int64_t rest = blockIdx.x >> 3;
  const int64_t r0 = ((rest / T) * 8 + (blockIdx.x & 7)) * RB;
  const int i0 = (int)(rest % T) * RB;
  if (r0 >= n) return;  // the grid's padding to a multiple of 8 row blocks (or an empty batch)
  const int rl = lane & 15, kk = lane >> 4;
  v4d acc[NT][NT];
#pragma unroll
  for (int m = 0; m < NT; ++m)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[m][j] = v4d{0.0, 0.0, 0.0, 0.0};
  // V4: lane l moves columns 4 (l % 16) .. + 3 of rows l / 16 + 4 t; otherwise
  // column l of every row.  Columns past kw (a multiple of 16) re-read the
  // last valid ones into the unread part of the row.
  float va[RB], vb[RB];
  auto load = [&](int k0) __attribute__((always_inline)) {
    const int kw = D - k0 < KC ? D - k0 : KC;
    if constexpr (V4) {
      const int c = min(4 * (lane & 15), kw - 4);
#pragma unroll
      for (int t = 0; t < RB / 4; ++t) {
        const int r = 4 * t + (lane >> 4);
        const int64_t ra = r0 + r < n ? r0 + r : 0;  // rows past n only feed outputs that are not stored
        const float4 x = *reinterpret_cast<const float4*>(in + ra * D + k0 + c);
        const float4 y = *reinterpret_cast<const float4*>(M + (int64_t)(i0 + r) * D + k0 + c);
        va[4 * t] = x.x, va[4 * t + 1] = x.y, va[4 * t + 2] = x.z, va[4 * t + 3] = x.w;
        vb[4 * t] = y.x, vb[4 * t + 1] = y.y, vb[4 * t + 2] = y.z, vb[4 * t + 3] = y.w;
      }
    } else {
      const int c = min(lane, kw - 1);
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const int64_t ra = r0 + r < n ? r0 + r : 0;
        va[r] = in[ra * D + k0 + c];
        vb[r] = M[(int64_t)(i0 + r) * D + k0 + c];
      }
    }
  };
  load(0);
  for (int k0 = 0; k0 < D; k0 += KC) {
    const int kw = D - k0 < KC ? D - k0 : KC;
    if constexpr (V4) {
#pragma unroll
      for (int t = 0; t < RB / 4; ++t) {
        const int o = (4 * t + (lane >> 4)) * LD + 4 * (lane & 15);
        *reinterpret_cast<float4*>(&As[o]) = make_float4(va[4 * t], va[4 * t + 1], va[4 * t + 2], va[4 * t + 3]);
        *reinterpret_cast<float4*>(&Bs[o]) = make_float4(vb[4 * t], vb[4 * t + 1], vb[4 * t + 2], vb[4 * t + 3]);
      }
    } else {
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        As[r * LD + lane] = va[r];
        Bs[r * LD + lane] = vb[r];
      }
    }
    __syncthreads();
    if (k0 + KC < D) load(k0 + KC);
    for (int kb = 0; kb < kw; kb += 4) {
      double a[NT], b[NT];
#pragma unroll
      for (int m = 0; m < NT; ++m) a[m] = (double)As[(16 * m + rl) * LD + kb + kk];
#pragma unroll
      for (int j = 0; j < NT; ++j) b[j] = (double)Bs[(16 * j + rl) * LD + kb + kk];
#pragma unroll
      for (int m = 0; m < NT; ++m)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[m][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], b[j], acc[m][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int m = 0; m < NT; ++m)
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t rr = r0 + 16 * m + (lane >> 4) + 4 * v;
        if (rr < n) out[rr * D + i0 + 16 * j + (lane & 15)] = (float)acc[m][j][v];
      }
}

// ------------------------------------------------------------------ encode

__device__ __forceinline__ double butterfly_d(double p) {
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) p = p + __shfl_xor(p, s, 64);
  return p;
}

// One wavefront per holder vertex c.  For every edge c -> o (Sec. 3.1.1,
// centre = c): y = rot(o) - rot(c) in fp32, bit i = [y_i > 0]; fp64 sums
// |r|^2, sum |y_i| and xc = sum (2b_i - 1) rot(c)_i with dim i in lane i mod
// 64 and a butterfly; f_rescale = -2|r|^2 / sum|y|, f_add = |r|^2 - f_rescale*xc
// (Eq. normalization with Eq. 3.1; degenerate edge: f_rescale = 0,
// f_add = |r|^2).  The block buffer must be zeroed beforehand.
__global__ __launch_bounds__(256) void encode_kernel(const float* __restrict__ X, const float* __restrict__ ROT,
                                                     int64_t N, int D, const int32_t* __restrict__ G, int R,
                                                     uint8_t* __restrict__ blocks, int64_t B) {
  const int lane = lane_id();
  const int64_t c = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (c >= N) return;
  const int DPL = (D + 63) >> 6;
  uint8_t* blk = blocks + c * B;
  const float* xc = X + c * D;
  const float* rc = ROT + c * D;
  for (int i = lane; i < D; i += 64) reinterpret_cast<float*>(blk)[i] = xc[i];
  uint8_t* codes = blk + qgl::off_codes(D);
  float* fadd = reinterpret_cast<float*>(blk + qgl::off_fadd(D, R));
  float* fres = reinterpret_cast<float*>(blk + qgl::off_fres(D, R));
  int32_t* nbr = reinterpret_cast<int32_t*>(blk + qgl::off_nbr(D, R));
  for (int j = 0; j < R; ++j) {
    const int32_t o = G[c * R + j];
    if (o < 0) {
      if (lane == 0) {
        fadd[j] = 0.0f;
        fres[j] = 0.0f;
        nbr[j] = -1;
      }
      continue;
    }
    const float* xo = X + (int64_t)o * D;
    const float* ro = ROT + (int64_t)o * D;
    double pr = 0.0, pa = 0.0, px = 0.0;
    uint8_t* code = codes + (int64_t)j * (D / 8);
    for (int t = 0; t < DPL; ++t) {
      const int i = lane + 64 * t;
      bool bit = false;
      if (i < D) {
        double d = (double)xo[i] - (double)xc[i];
        pr = __builtin_fma(d, d, pr);
        float y = ro[i] - rc[i];
        bit = y > 0.0f;
        pa = pa + __builtin_fabs((double)y);
        px = bit ? px + (double)rc[i] : px - (double)rc[i];
      }
      uint64_t m = ballot(bit);
      const int nbytes = (D - 64 * t) >= 64 ? 8 : (D - 64 * t) / 8;
      if (lane < nbytes) code[8 * t + lane] = (uint8_t)(m >> (8 * lane));
    }
    pr = butterfly_d(pr);
    pa = butterfly_d(pa);
    px = butterfly_d(px);
    if (lane == 0) {
      if (pa == 0.0) {
        fres[j] = 0.0f;
        fadd[j] = (float)pr;
      } else {
        double fr = (-2.0 * pr) / pa;
        double fa = pr - fr * px;
        fres[j] = (float)fr;
        fadd[j] = (float)fa;
      }
      nbr[j] = o;
    }
  }
}

// ------------------------------------------------------------- query side

// Per-query quantisation and LUT (Sec. 2.2 FastScan with the query-only LUT
// of Eq. 3.1b): m = max|q'_i|, inv = fl32(127/m), q_s = clamp(rint(q'_i*inv)),
// Delta = fl32(m/127); LUT[k][p] = sum_t (bit t of p ? q_s[4k+t] : -q_s[4k+t]),
// stored as int16 rows of 16.  Layout: with pad = 1 one padding row sits
// before each later lane group's rows (when two lanes share a neighbour their
// lookups then fall in different banks), with pad = 0 the rows are packed.
// Entries are int16 (LB = 2) or int32 (LB = 4, the same values).  Returns
// Delta.
template <int D, int R, int LB = 2>
__device__ __forceinline__ float build_lut(const float* __restrict__ qrot, void* lut, int pad) {
  constexpr int ROWS = D / 4;
  constexpr int RPG = D / 4 / (64 / R);
  const int lane = lane_id();
  float m = 0.0f;
  for (int i = lane; i < D; i += 64) m = fmaxf(m, __builtin_fabsf(qrot[i]));
  m = wave_max(m);
  float inv = 0.0f, delta = 0.0f;
  if (m != 0.0f) {
    inv = 127.0f / m;
    delta = m / 127.0f;
  }
  for (int w = lane; w < 2 * ROWS; w += 64) {
    const int k = w >> 1, half = w & 1;
    int s[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      float v = (m != 0.0f) ? __builtin_rintf(qrot[4 * k + t] * inv) : 0.0f;
      v = fminf(fmaxf(v, -127.0f), 127.0f);
      s[t] = (int)v;
    }
    const int r = k + pad * (k / RPG);
#pragma unroll
    for (int pp = 0; pp < 8; ++pp) {
      const int p = half * 8 + pp;
      int acc = 0;
#pragma unroll
      for (int t = 0; t < 4; ++t) acc += ((p >> t) & 1) ? s[t] : -s[t];
      if constexpr (LB == 4)
        static_cast<int32_t*>(lut)[r * 16 + p] = acc;
      else
        static_cast<int16_t*>(lut)[r * 16 + p] = (int16_t)acc;
    }
  }
  wave_sync();
  return delta;
}

// Vertex block fields as one lane sees them: its dims of the raw vector, its
// share of one neighbour's code, that neighbour's factors and id.
// LDS (address space 3) views: 32-bit byte addresses of shared memory.
typedef __attribute__((address_space(3))) const int16_t lds_i16;
__device__ __forceinline__ uint32_t lds_addr(const int16_t* p) {
  return (uint32_t)(uintptr_t)(lds_i16*)p;  // generic -> LDS address-space cast
}

// base + byte K of x in one instruction (SDWA source select).
template <int K>
__device__ __forceinline__ uint32_t add_byte(uint32_t base, uint32_t x) {
  uint32_t r;
  if constexpr (K == 0)
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_0"
        : "=v"(r) : "v"(base), "v"(x));
  else if constexpr (K == 1)
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_1"
        : "=v"(r) : "v"(base), "v"(x));
  else if constexpr (K == 2)
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_2"
        : "=v"(r) : "v"(base), "v"(x));
  else
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_3"
        : "=v"(r) : "v"(base), "v"(x));
  return r;
}

// Sum of the LUT entries of nibbles T .. N-1 of one code unit: nibble t of
// the unit indexes row t (16 entries of LB bytes), at byte (t >> 1) of ev
// (even t) or od (odd t), which hold the nibbles times LB.
typedef __attribute__((address_space(3))) const int32_t lds_i32;
template <int T, int N, int LB>
__device__ __forceinline__ int lut_sum(uint32_t b8, uint32_t ev, uint32_t od) {
  const uint32_t a = add_byte<(T >> 1)>(b8, (T & 1) ? od : ev);
  int v;
  if constexpr (LB == 4)
    v = *(lds_i32*)(uintptr_t)(a + T * 64);
  else
    v = *(lds_i16*)(uintptr_t)(a + T * 32);
  if constexpr (T + 1 < N)
    return v + lut_sum<T + 1, N, LB>(b8, ev, od);
  else
    return v;
}

template <int D, int R>
struct BlockView {
  static constexpr int LPN = 64 / R;        // lanes per neighbour
  static constexpr int CB = D / 8;          // code bytes per neighbour
  static constexpr int BPL = CB / LPN;      // code bytes per lane
  static constexpr int DPL = (D + 63) / 64; // raw dims per lane
  static constexpr bool WORDS = (BPL % 4) == 0;
  static constexpr int NW = WORDS ? BPL / 4 : BPL / 2;  // 32- or 16-bit code units per lane
  // Whether a second block (the next vertex, prefetched) is held in registers
  // beside this one (every shape built here: at most 45 words per lane);
  // wider shapes would load the block when it is used instead.
  static constexpr bool kRegPrefetch = NW + DPL <= 48;
  float x[DPL];
  uint32_t cw[NW];
  float fa, fr;
  int32_t nb;

  __device__ __forceinline__ void load(const uint8_t* __restrict__ blk, int lane) {
    const float* raw = reinterpret_cast<const float*>(blk);
#pragma unroll
    for (int t = 0; t < DPL; ++t) {
      const int i = lane + 64 * t;
      x[t] = (i < D) ? raw[i] : 0.0f;
    }
    const int j = lane / LPN, h = lane % LPN;
    const uint8_t* cp = blk + qgl::off_codes(D) + j * CB + h * BPL;
    if constexpr (WORDS) {
#pragma unroll
      for (int w = 0; w < NW; ++w) cw[w] = reinterpret_cast<const uint32_t*>(cp)[w];
    } else {
#pragma unroll
      for (int w = 0; w < NW; ++w) cw[w] = reinterpret_cast<const uint16_t*>(cp)[w];
    }
    fa = reinterpret_cast<const float*>(blk + qgl::off_fadd(D, R))[j];
    fr = reinterpret_cast<const float*>(blk + qgl::off_fres(D, R))[j];
    nb = reinterpret_cast<const int32_t*>(blk + qgl::off_nbr(D, R))[j];
  }

  // FastScan sum of this lane's nibbles; the LPN lanes of one neighbour are
  // then combined (integer, exact) so every lane holds S_j.
  template <int LB = 2>
  __device__ __forceinline__ int fastscan(const void* lut, int lane, int pad) const {
    constexpr int RPG = D / 4 / LPN;
    constexpr int UNIT_NIB = WORDS ? 8 : 4;
    const int h = lane % LPN;
    // group h starts after h padding rows (pad = 1)
    const uint32_t b8 = lds_addr(static_cast<const int16_t*>(lut)) + (uint32_t)((h * RPG + pad * h) * 16 * LB);
    int s = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      // byte offsets (LB x nibble) of the even and odd nibbles, one per byte:
      // each lookup address is the base plus one byte of a register
      const uint32_t ev = LB == 4 ? (cw[w] << 2) & 0x3C3C3C3Cu : (cw[w] << 1) & 0x1E1E1E1Eu;
      const uint32_t od = LB == 4 ? (cw[w] >> 2) & 0x3C3C3C3Cu : (cw[w] >> 3) & 0x1E1E1E1Eu;
      s += lut_sum<0, UNIT_NIB, LB>(b8 + w * UNIT_NIB * 16 * LB, ev, od);
      // wide codes: keep the lookups of one unit together, so that not all of
      // them are in flight (and in registers) at once
      if constexpr (NW > 4) {
        // the running sum passes through here: this unit's lookups are summed
        // (and their registers free) before the next unit's are issued
        asm volatile("" : "+v"(s)::"memory");
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    if constexpr (LPN == 2) s += xor_lane_i<1>(s);
    return s;
  }
};

// ------------------------------------------------------------------ search

struct Visited {
  // LDS hash (open addressing, linear probing) or, in the overflow path, a
  // global bitset of N bits private to this wavefront.
  uint32_t* tab;
  uint32_t mask;
  int hbits;
  uint32_t* bits;

  // First slot of id's probe sequence: a multiplicative hash.
  __device__ __forceinline__ uint32_t slot0(uint32_t id) const {
    return (id * 0x9E3779B1u) >> (32 - hbits);
  }
  // The register-beam search starts every probe sequence at a multiple of 4
  // instead, so that a probe tests four slots with one 16-byte LDS read (the
  // table is 16-byte aligned).  An id sits before the first empty slot of its
  // sequence (ids are never removed), so a probe ends at the first group of
  // four that holds the id or an empty slot.  (The LDS-beam search probes one
  // slot at a time per lane, where the wider read measured slower.)
  __device__ __forceinline__ uint32_t slot4(uint32_t id) const { return slot0(id) & ~3u; }
  __device__ __forceinline__ uint4 group(uint32_t slot) const { return *reinterpret_cast<const uint4*>(tab + slot); }
};
__device__ __forceinline__ bool group_has(const uint4& w, uint32_t id) {
  return min(min(w.x ^ id, w.y ^ id), min(w.z ^ id, w.w ^ id)) == 0u;
}
__device__ __forceinline__ bool group_full(const uint4& w) {  // no empty slot (ids are below kEmpty)
  return max(max(w.x, w.y), max(w.z, w.w)) != kEmpty;
}

// Membership test.  For the LDS hash, end receives the slot where the probe
// stopped: when id is absent, the first empty slot of its probe sequence,
// which is where inserting id puts it.
template <bool GV>
__device__ __forceinline__ bool visited_probe(const Visited& v, uint32_t id, uint32_t& end) {
  if constexpr (GV) {
    uint32_t w = __hip_atomic_load(v.bits + (id >> 5), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return (w >> (id & 31)) & 1u;
  } else {
    uint32_t s = v.slot0(id);
    uint32_t e = v.tab[s];
    while (e != id && e != kEmpty) {  // most probes end at the first slot
      s = (s + 1) & v.mask;
      e = v.tab[s];
    }
    end = s;
    return e == id;
  }
}
template <bool GV>
__device__ __forceinline__ bool visited_contains(const Visited& v, uint32_t id) {
  uint32_t end;
  return visited_probe<GV>(v, id, end);
}

// Insert id (wave-uniform); returns true if it was already present.
template <bool GV>
__device__ __forceinline__ bool visited_insert(const Visited& v, uint32_t id, int lane) {
  if constexpr (GV) {
    uint32_t old = 0;
    if (lane == 0) old = atomicOr(v.bits + (id >> 5), 1u << (id & 31));
    old = (uint32_t)__builtin_amdgcn_readlane((int)old, 0);
    return (old >> (id & 31)) & 1u;
  } else {
    uint32_t base = v.slot0(id);
    for (;;) {
      const uint32_t s = (base + lane) & v.mask;
      const uint32_t e = v.tab[s];
      const uint64_t fm = ballot(e == id), em = ballot(e == kEmpty);
      if (fm | em) {
        const int ff = fm ? first_lane(fm) : 64, fe = em ? first_lane(em) : 64;
        if (ff < fe) return true;
        if (lane == fe) v.tab[s] = id;
        wave_sync();
        return false;
      }
      base += 64;
    }
  }
}

// Insert id (wave-uniform), known to be absent, into the LDS hash: the first
// empty slot of its probe sequence (which starts at `base`), found by reads of
// 64 consecutive slots.
__device__ __forceinline__ void visited_add_absent(const Visited& v, uint32_t id, uint32_t base, int lane) {
  for (;;) {
    const uint32_t s = (base + lane) & v.mask;
    const uint64_t em = ballot(v.tab[s] == kEmpty);
    if (em) {
      if (lane == first_lane(em)) v.tab[s] = id;
      break;
    }
    base += 64;
  }
  wave_sync();
}

// Per-lane insert into the set of estimated vertices (w/o ME); true if id was
// absent, so this lane's estimate is its first.  Lanes holding the same id see
// exactly one true.  The LDS table must keep an empty slot for every lane that
// inserts: the caller checks the count before.
template <bool GV>
__device__ __forceinline__ bool seen_insert(const Visited& v, uint32_t id) {
  if constexpr (GV) {
    const uint32_t old = atomicOr(v.bits + (id >> 5), 1u << (id & 31));
    return !((old >> (id & 31)) & 1u);
  } else {
    uint32_t s = v.slot0(id);
    for (;;) {
      const uint32_t old = atomicCAS(v.tab + s, kEmpty, id);
      if (old == kEmpty) return true;
      if (old == id) return false;
      s = (s + 1) & v.mask;
    }
  }
}

__device__ __forceinline__ uint32_t rdlane(uint32_t v, int l) { return (uint32_t)__builtin_amdgcn_readlane((int)v, l); }
__device__ __forceinline__ float rdlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// ------------------------------------------------------------ learned stop

// Learned early stop (an extension beyond the paper, whose Algorithm 1 runs
// until no unchecked beam entry is left): after the t-th expansion, for
// t >= t_min with (t - t_min) divisible by t_every, 16 state features feed a
// 16-64-64-1 ReLU MLP (bf16 parameters, fp32 arithmetic); the query stops when
// the output exceeds theta.  Hidden unit j runs on lane j as an fma chain over
// its inputs in ascending order from its bias; the output is the butterfly sum
// of w3[j] * h2[j] plus the output bias.  Parameter layout: W1[64][16], b1[64],
// W2[64][64], b2[64], W3[64], b3.
// learned-stop modes of the search kernels
// Kernel modes: plain search, learned stop (MLP in LDS), learned stop with
// trace, per-query k / ef (a mixed batch), and a mixed batch with the learned
// stop, and the "w/o ME" ablation of Sec. 4.2.3 (a vertex enters the beam only
// on its first estimate).  Each is its own instantiation, so the plain kernel
// carries none of the others' state.
constexpr int kLsOff = 0, kLsStop = 1, kLsTrace = 2, kMixed = 3, kMixedStop = 4, kNoMe = 5;
template <int LS>
constexpr bool has_stop = LS == kLsStop || LS == kLsTrace || LS == kMixedStop;
template <int LS>
constexpr bool is_mixed = LS == kMixed || LS == kMixedStop;
template <int LS>
constexpr bool mlp_in_lds = LS == kLsStop || LS == kMixedStop;
// w/o ME the set holds every vertex estimated so far (the entry included)
// rather than the visited ones: each vertex enters the beam at most once, so a
// pop never meets a visited vertex and the set is tested only on appends
template <int LS>
constexpr bool no_me = LS == kNoMe;

constexpr int kLsW1 = 0, kLsB1 = 64 * 16, kLsW2 = kLsB1 + 64, kLsB2 = kLsW2 + 64 * 64, kLsW3 = kLsB2 + 64,
              kLsB3 = kLsW3 + 64;

__device__ __forceinline__ float bf16lo(uint32_t u) { return __uint_as_float(u << 16); }
__device__ __forceinline__ float bf16hi(uint32_t u) { return __uint_as_float(u & 0xffff0000u); }
__device__ __forceinline__ float bf16at(const uint16_t* w, int i) { return __uint_as_float((uint32_t)w[i] << 16); }
__device__ __forceinline__ float ratio(float a, float b) { return b > 0.0f ? a / b : 0.0f; }
__device__ __forceinline__ float clamp8(float x) { return x < 0.0f ? 0.0f : (x > 8.0f ? 8.0f : x); }

// The 16 features of the search state, each a quotient num / den (0 when
// den <= 0) clamped to [0, 8].  Lane i (i < 16) forms feature i with one
// division; the MLP reads feature i from lane i as it needs it.  The lane
// index is made opaque here so that the compiler cannot hoist the 15 lane
// compares out of the search loop (they would hold 30 scalar registers).
struct StopFeatures {
  float mine;  // feature (lane & 15) of this lane
  __device__ __forceinline__ void compute(int E, int P, int nnc, int k, int since, float de, float nn1, float nnk,
                                          float bf, int size, int ef, float dp, int app, int R) {
    int i = lane_id() & 15;
    asm volatile("" : "+v"(i));
    float n = (float)E, d = 64.0f;                                         // 0: expansions
    n = i == 1 ? (float)P : n;                                             // 1: pops
    n = i == 2 ? (float)nnc : n;    d = i == 2 ? (float)k : d;             // 2: NN fill
    n = i == 3 ? (float)since : n;  d = i == 3 ? 16.0f : d;                // 3: expansions since NN changed
    n = i == 4 ? nn1 : n;           d = i == 4 ? de : d;                   // 4: best / entry distance
    n = i == 5 ? nnk : n;           d = i == 5 ? de : d;                   // 5: k-th / entry distance
    n = i == 6 ? bf : n;            d = i == 6 ? nnk : d;                  // 6: next estimate / k-th distance
    n = i == 7 ? bf : n;            d = i == 7 ? nn1 : d;                  // 7: next estimate / best distance
    n = i == 8 ? (float)size : n;   d = i == 8 ? (float)ef : d;            // 8: beam fill
    n = i == 9 ? dp : n;            d = i == 9 ? nnk : d;                  // 9: last exact distance / k-th
    n = i == 10 ? (float)app : n;   d = i == 10 ? (float)R : d;            // 10: fraction of neighbours appended
    n = i == 11 ? nnk - nn1 : n;    d = i == 11 ? nnk : d;                 // 11: relative spread of NN
    n = i == 12 ? (float)ef : n;    d = i == 12 ? 256.0f : d;              // 12: beam size
    n = i == 13 ? bf : n;           d = i == 13 ? de : d;                  // 13: next estimate / entry distance
    n = i == 14 ? (float)E : n;     d = i == 14 ? (float)ef : d;           // 14: expansions / beam size
    n = i == 15 ? 1.0f : n;         d = i == 15 ? 1.0f : d;                // 15: bias input
    mine = clamp8(ratio(n, d));
  }
};

__device__ __forceinline__ float stop_mlp(const uint16_t* __restrict__ w, const StopFeatures& F, int lane) {
  // layer 1: this lane's row of W1 (16 bf16 = two 16-byte loads)
  const uint4* r1 = reinterpret_cast<const uint4*>(w + kLsW1 + lane * 16);
  const uint4 a0 = r1[0], a1 = r1[1];
  const uint32_t wr[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
  float acc = bf16at(w, kLsB1 + lane);
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    acc = __builtin_fmaf(bf16lo(wr[i]), rdlane(F.mine, 2 * i), acc);
    acc = __builtin_fmaf(bf16hi(wr[i]), rdlane(F.mine, 2 * i + 1), acc);
  }
  const float h1 = acc > 0.0f ? acc : 0.0f;
  // layer 2: every lane needs all 64 h1 values; they come through scalar registers
  const uint4* r2 = reinterpret_cast<const uint4*>(w + kLsW2 + lane * 64);
  acc = bf16at(w, kLsB2 + lane);
#pragma unroll 2
  for (int c = 0; c < 8; ++c) {
    const uint4 v = r2[c];
    const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      acc = __builtin_fmaf(bf16lo(u[h]), rdlane(h1, 8 * c + 2 * h), acc);
      acc = __builtin_fmaf(bf16hi(u[h]), rdlane(h1, 8 * c + 2 * h + 1), acc);
    }
  }
  const float h2 = acc > 0.0f ? acc : 0.0f;
  const float pr = bf16at(w, kLsW3 + lane) * h2;
  return uni(butterfly_f(pr) + bf16at(w, kLsB3));
}

// The stop-only kernels keep the MLP in LDS, staged once per workgroup and
// laid out so that lane j's 16-byte chunk c of a weight row sits at chunk
// c * 64 + j (consecutive lanes read consecutive chunks, no bank conflicts):
// W1 as 2 x 64 chunks, W2 as 8 x 64 chunks, then b1[64], b2[64], W3[64], b3.
constexpr int kMlpW2 = 2 * 64 * 16, kMlpB1 = kMlpW2 + 8 * 64 * 16, kMlpB2 = kMlpB1 + 128, kMlpW3 = kMlpB2 + 128,
              kMlpB3 = kMlpW3 + 128;

__device__ __forceinline__ void stage_mlp(const uint16_t* __restrict__ w, uint8_t* m) {
  for (int t = threadIdx.x; t < 10 * 64; t += blockDim.x) {
    const int c = t < 128 ? t >> 6 : (t - 128) >> 6, j = t & 63;
    const uint4* src = t < 128 ? reinterpret_cast<const uint4*>(w + kLsW1 + j * 16) + c
                               : reinterpret_cast<const uint4*>(w + kLsW2 + j * 64) + c;
    reinterpret_cast<uint4*>(m)[t] = *src;
  }
  uint16_t* m16 = reinterpret_cast<uint16_t*>(m + kMlpB1);
  for (int t = threadIdx.x; t < 64 + 129; t += blockDim.x)
    m16[t] = t < 64 ? w[kLsB1 + t] : w[kLsB2 + (t - 64)];  // b2, W3 and b3 are contiguous
}

// bc: 256 bytes of this wavefront's LDS free during the evaluation; the
// features and then the first hidden layer pass through it, so every lane
// reads them back four at a time (broadcast reads) instead of one readlane each.
__device__ __forceinline__ float stop_mlp_lds(const uint8_t* m, float f, int lane, float* bc) {
  const uint4* W = reinterpret_cast<const uint4*>(m);
  const uint16_t* m16 = reinterpret_cast<const uint16_t*>(m + kMlpB1);
  if (lane < 16) bc[lane] = f;
  wave_sync();
  float acc = __uint_as_float((uint32_t)m16[lane] << 16);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const uint4 v = W[c * 64 + lane];
    const float4 x0 = reinterpret_cast<const float4*>(bc)[2 * c], x1 = reinterpret_cast<const float4*>(bc)[2 * c + 1];
    acc = __builtin_fmaf(bf16lo(v.x), x0.x, acc);
    acc = __builtin_fmaf(bf16hi(v.x), x0.y, acc);
    acc = __builtin_fmaf(bf16lo(v.y), x0.z, acc);
    acc = __builtin_fmaf(bf16hi(v.y), x0.w, acc);
    acc = __builtin_fmaf(bf16lo(v.z), x1.x, acc);
    acc = __builtin_fmaf(bf16hi(v.z), x1.y, acc);
    acc = __builtin_fmaf(bf16lo(v.w), x1.z, acc);
    acc = __builtin_fmaf(bf16hi(v.w), x1.w, acc);
  }
  const float h1 = acc > 0.0f ? acc : 0.0f;
  wave_sync();
  bc[lane] = h1;  // the features have been read
  wave_sync();
  acc = __uint_as_float((uint32_t)m16[64 + lane] << 16);
#pragma unroll 1
  for (int c = 0; c < 8; ++c) {
    const uint4 v = W[(2 + c) * 64 + lane];
    const float4 x0 = reinterpret_cast<const float4*>(bc)[2 * c], x1 = reinterpret_cast<const float4*>(bc)[2 * c + 1];
    acc = __builtin_fmaf(bf16lo(v.x), x0.x, acc);
    acc = __builtin_fmaf(bf16hi(v.x), x0.y, acc);
    acc = __builtin_fmaf(bf16lo(v.y), x0.z, acc);
    acc = __builtin_fmaf(bf16hi(v.y), x0.w, acc);
    acc = __builtin_fmaf(bf16lo(v.z), x1.x, acc);
    acc = __builtin_fmaf(bf16hi(v.z), x1.y, acc);
    acc = __builtin_fmaf(bf16lo(v.w), x1.z, acc);
    acc = __builtin_fmaf(bf16hi(v.w), x1.w, acc);
  }
  const float h2 = acc > 0.0f ? acc : 0.0f;
  const float pr = __uint_as_float((uint32_t)m16[128 + lane] << 16) * h2;
  return uni(butterfly_f(pr) + __uint_as_float((uint32_t)m16[192] << 16));
}

__device__ __forceinline__ uint64_t rdlane64(uint64_t v, int l) {
  return ((uint64_t)rdlane((uint32_t)(v >> 32), l) << 32) | rdlane((uint32_t)v, l);
}

// Element r (wave-uniform) of a small register array, by selects (no dynamic
// register indexing).
template <int NB>
__device__ __forceinline__ uint64_t pick(const uint64_t (&b)[NB], int r) {
  uint64_t v = b[0];
#pragma unroll
  for (int i = 1; i < NB; ++i) v = r == i ? b[i] : v;
  return v;
}

template <int D, int R, bool GV, int LS, int LB>
__device__ void search_one(const SearchArgs& a, int64_t q, uint8_t* lds, const qgl::SearchLds& L, uint32_t* gbits,
                           const uint8_t* mlp) {
  using BV = BlockView<D, R>;
  constexpr int DPL = BV::DPL;
  constexpr int LPN = BV::LPN;
  constexpr uint64_t kNone = ~0ull;  // sorts after every real entry
  const int lane = lane_id();
  int ef = a.ef, k = a.k;
  if constexpr (is_mixed<LS>) {
    // a beam size and result count of its own; a.ef and a.k are the bounds
    ef = uni(a.ef_q[q]);
    k = uni(a.k_q[q]);
    if (k < 1 || k > a.k || ef < 1 || ef > a.ef) {  // rejected: an all-padding row, stats[3] = -1
      for (int i = lane; i < a.k_out; i += 64) {
        a.out_ids[q * a.k_out + i] = -1;
        a.out_dists[q * a.k_out + i] = __builtin_inff();
      }
      if (a.out_stats && lane < 4) a.out_stats[4 * q + lane] = lane == 3 ? -1 : 0;
      return;
    }
  }
  void* lut = lds + L.lut;
  // beam entries: sortable(key) << 32 | id | checked, kept in ascending order
  uint64_t* beam = reinterpret_cast<uint64_t*>(lds + L.beam);
  uint32_t* beam_lo = reinterpret_cast<uint32_t*>(lds + L.beam);  // low words (id | checked)
  float* nkey = reinterpret_cast<float*>(lds + L.nkey);
  uint32_t* nid = reinterpret_cast<uint32_t*>(lds + L.nid);

  Visited vis;
  vis.tab = reinterpret_cast<uint32_t*>(lds + L.hash);
  vis.hbits = a.hash_bits;
  vis.mask = (1u << a.hash_bits) - 1u;
  vis.bits = gbits;
  int nvis = 0;
  const int vis_limit = GV ? 0x7fffffff : (1 << a.hash_bits) / 2;
  if constexpr (GV) {
    for (int64_t w = lane; w < a.fb_words; w += 64)
      __hip_atomic_store(gbits + w, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
  } else {
    for (int i = lane; i < (1 << a.hash_bits); i += 64) vis.tab[i] = kEmpty;
  }

  // the raw query: in registers, or for the wide shapes (D > 256) in LDS,
  // read back dim by dim (same arithmetic either way)
  constexpr bool kQvLds = qgl::query_in_lds(D);
  float qv[kQvLds ? 1 : DPL];
  float* qs = reinterpret_cast<float*>(lds + L.qv);
  const float* qr = a.queries + q * D;
  if constexpr (kQvLds) {
    static_assert(D % 64 == 0, "wide shapes have D a multiple of 64");
    for (int i = lane; i < D; i += 64) qs[i] = qr[i];
  } else {
#pragma unroll
    for (int t = 0; t < DPL; ++t) {
      const int i = lane + 64 * t;
      qv[t] = (i < D) ? qr[i] : 0.0f;
    }
  }
  auto dist = [&](const float(&xv)[DPL]) {
    if constexpr (kQvLds) {
      float p = 0.0f;
#pragma unroll
      for (int t = 0; t < DPL; ++t) {
        const float d = qs[lane + 64 * t] - xv[t];
        p = __builtin_fmaf(d, d, p);
      }
      return butterfly_f(p);
    } else {
      return exact_dist<DPL>(qv, xv);
    }
  };
  const float delta = build_lut<D, R, LB>(a.qrot + q * D, lut, a.lut_pad);

  // S starts with the entry, keyed by its exact distance (no estimate exists for it).
  float de;
  {
    BV e;
    e.load(a.blocks + (int64_t)a.entry * a.block_bytes, lane);
    de = uni(dist(e.x));
  }
  uint64_t tail = pack_kv(de, (uint32_t)a.entry);  // beam[ef - 1] whenever the beam is full
  beam[0] = tail;
  wave_sync();
  int size = 1, cursor = 0, nnc = 0;
  if constexpr (no_me<LS>) {  // the entry counts as estimated: it never enters the beam again
    visited_insert<GV>(vis, (uint32_t)a.entry, lane);
    nvis = 1;
  }
  float nn_wk = 0.0f;  // worst (distance, id) of NN once it holds k entries
  uint32_t nn_wi = 0;
  int expansions = 0, pops = 0, appended = 0;
  // Next-vertex prefetch (Sec. 3.1.4): the next vertex to expand is the smaller
  // of the best new candidate and the next unchecked, unvisited old entry; its
  // block is loaded while NN and the beam are updated.
  BV nxt;
  uint32_t nxt_id = kEmpty;
  int since = 0, nevals = 0;  // learned stop: expansions since NN changed, evaluations so far
  // NN (ascending (distance, id)): for k <= 64 lane i holds entry i in
  // registers; larger k keep it in LDS (nkey, nid).
  const bool nn_in_regs = k <= 64;
  float nrk = 0.0f;
  uint32_t nri = 0;

  for (;;) {
    // pop the first unchecked entry whose vertex is not visited yet.  Unchecked
    // entries before it are further estimates of visited vertices: popping
    // them only marks them checked, so they are consumed here in one step (each
    // counts as a pop).  The same chunk read gives the next unchecked entry
    // (o2u, for the stop features) and the next one still to be expanded (o2f,
    // the prefetch target).
    int c = -1;
    uint32_t p = 0, p_slot = 0;  // p_slot: p's free hash slot, found by the probe below
    uint64_t o2u = kNone, o2f = kNone;
    bool o2u_known = false, o2f_known = false;
    while (cursor < size) {
      const int i = cursor + lane;
      const uint64_t e = (i < size) ? beam[i] : (uint64_t)kChecked;
      const bool un = !((uint32_t)e & kChecked);
      const uint64_t mu = ballot(un);
      if (!mu) {
        cursor += 64;
        continue;
      }
      bool fresh = false;
      uint32_t vend = 0;
      if (un) fresh = no_me<LS> || !visited_probe<GV>(vis, (uint32_t)e, vend);
      const uint64_t mf = ballot(fresh);
      const uint64_t dups = mf ? mu & ((1ull << first_lane(mf)) - 1) : mu;
      if (dups) {
        if ((dups >> lane) & 1) beam_lo[2 * i] = (uint32_t)e | kChecked;
        pops += __popcll(dups);
      }
      if (!mf) {
        cursor += 64;
        continue;
      }
      const int f = first_lane(mf);
      c = cursor + f;
      p = rdlane((uint32_t)e, f);
      if constexpr (!GV) p_slot = rdlane(vend, f);
      const uint64_t later = f == 63 ? 0ull : ~0ull << (f + 1);
      const uint64_t mu2 = mu & later, mf2 = mf & later & ballot((uint32_t)e != p);
      if (mu2) {
        o2u = rdlane64(e, first_lane(mu2));
        o2u_known = true;
      }
      if (mf2) {
        o2f = rdlane64(e, first_lane(mf2));
        o2f_known = true;
      }
      if (cursor + 64 >= size) o2u_known = o2f_known = true;  // nothing after this chunk
      break;
    }
    if (c < 0) break;
    beam_lo[2 * c] = p | kChecked;  // every lane stores the same word
    cursor = c + 1;
    ++pops;
    if constexpr (!no_me<LS>) {
      if constexpr (GV) {
        visited_insert<GV>(vis, p, lane);
      } else {
        if (lane == 0) vis.tab[p_slot] = p;  // p is absent: its probe ended at this empty slot
        wave_sync();
      }
      if (++nvis > vis_limit) {  // on-chip visited set full: hand the query to the overflow path
        if (lane == 0) {
          const int slot = atomicAdd(a.counters + 1, 1);
          a.overflow_list[slot] = (int32_t)q;
        }
        return;
      }
    }
    ++expansions;

    BV b;
    if (p == nxt_id)
      b = nxt;
    else
      b.load(a.blocks + (int64_t)p * a.block_bytes, lane);
    nxt_id = kEmpty;
    const float dp = uni(dist(b.x));

    // FastScan estimates of all neighbours (Eq. normalization with Eq. 3.1)
    const int S = b.template fastscan<LB>(lut, lane, a.lut_pad);
    const float est = __builtin_fmaf(b.fr, (float)S * delta, b.fa + dp);
    const uint32_t nb = (uint32_t)b.nb;
    const uint64_t cand = pack_kv(est, nb);
    bool valid = (lane % LPN == 0) && b.nb >= 0;
    if constexpr (no_me<LS>) {
      if constexpr (!GV) {
        if (nvis + (int)__popcll(ballot(valid)) > vis_limit) {  // the set could fill: overflow path
          if (lane == 0) {
            const int slot = atomicAdd(a.counters + 1, 1);
            a.overflow_list[slot] = (int32_t)q;
          }
          return;
        }
      }
      if (valid) valid = seen_insert<GV>(vis, nb);
      nvis += (int)__popcll(ballot(valid));
    } else {
      if (valid) valid = !visited_contains<GV>(vis, nb);
    }
    const int app = uni((int)__popcll(ballot(valid)));
    appended += app;
    if (size == ef) valid = valid && cand < tail;  // would fall past the cut anyway
    const uint64_t V = ballot(valid);
    const int nv = uni((int)__popcll(V));

    // best candidate (the smallest (estimate, id) among them)
    uint64_t best = kNone;
    if (nv > 0) {
      const uint32_t hk = wave_min_u32(valid ? (uint32_t)(cand >> 32) : 0xFFFFFFFFu);
      const uint64_t tie = ballot(valid && (uint32_t)(cand >> 32) == hk);
      const uint32_t lo = (tie & (tie - 1)) ? wave_min_u32((tie >> lane) & 1 ? (uint32_t)cand : 0xFFFFFFFFu)
                                            : rdlane((uint32_t)cand, first_lane(tie));
      best = ((uint64_t)hk << 32) | lo;
    }
    // o2f (and o2u, for the stop features) beyond the popped chunk
    if (!o2f_known || (has_stop<LS> && !o2u_known)) {
      for (int base = cursor; base < size && !(o2f_known && (!has_stop<LS> || o2u_known)); base += 64) {
        const int i = base + lane;
        const uint64_t e = (i < size) ? beam[i] : (uint64_t)kChecked;
        const bool un = !((uint32_t)e & kChecked);
        const uint64_t mu = ballot(un);
        if (!mu) continue;
        if (has_stop<LS> && !o2u_known) {
          o2u = rdlane64(e, first_lane(mu));
          o2u_known = true;
        }
        if (!o2f_known) {
          bool fresh = false;
          if (un) fresh = no_me<LS> || !visited_contains<GV>(vis, (uint32_t)e);
          const uint64_t mf = ballot(fresh);
          if (mf) {
            o2f = rdlane64(e, first_lane(mf));
            o2f_known = true;
          }
        }
      }
    }
    // the next pop is the smaller of the best candidate and o2u; the next
    // expansion the smaller of the best candidate and o2f: prefetch its block
    const uint64_t nxt_u = best < o2u ? best : o2u;
    const float bfk = nxt_u == kNone ? __builtin_inff() : unsortable((uint32_t)(nxt_u >> 32));
    const uint64_t nxt_f = best < o2f ? best : o2f;
    if (nxt_f != kNone) {
      const uint32_t nx = (uint32_t)nxt_f & kIdMask;
      if constexpr (BV::kRegPrefetch) {
        nxt.load(a.blocks + (int64_t)nx * a.block_bytes, lane);
        nxt_id = nx;
      }
    }

    // implicit re-ranking: NN keeps the k smallest (distance, id) seen
    ++since;
    if (nnc < k || kv_less(dp, p, nn_wk, nn_wi)) {
      since = 0;
      if (nn_in_regs) {
        // entries [pos, last) move up one lane (DPP shift of the wavefront by one lane)
        const int pos = (int)__popcll(ballot(lane < nnc && kv_less(nrk, nri, dp, p)));
        const int last = nnc < k ? nnc : k - 1;
        const float upk = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(nrk), 0x138, 0xF, 0xF, false));
        const uint32_t upi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)nri, 0x138, 0xF, 0xF, false);
        if (lane > pos && lane <= last) {
          nrk = upk;
          nri = upi;
        }
        if (lane == pos) {
          nrk = dp;
          nri = p;
        }
        nnc = nnc < k ? nnc + 1 : k;
        if (nnc == k) {
          nn_wk = rdlane(nrk, k - 1);
          nn_wi = rdlane(nri, k - 1);
        }
      } else {
        int pos = 0;
        for (int base = 0; base < nnc; base += 64) {
          const int i = base + lane;
          const bool lt = (i < nnc) && kv_less(nkey[i < nnc ? i : 0], nid[i < nnc ? i : 0], dp, p);
          pos += __popcll(ballot(lt));
        }
        const int last = nnc < k ? nnc : k - 1;  // entries [pos, last) move up by one
        for (int base = ((last - 1) >> 6) << 6; base >= 0 && last > pos; base -= 64) {
          const int i = base + lane;
          float kk = 0.0f;
          uint32_t ii = 0;
          const bool mv = (i >= pos) && (i < last);
          if (mv) {
            kk = nkey[i];
            ii = nid[i];
          }
          wave_sync();
          if (mv) {
            nkey[i + 1] = kk;
            nid[i + 1] = ii;
          }
          wave_sync();
          if (base < pos) break;
        }
        pos = uni(pos);
        nkey[pos] = dp;  // same value from every lane
        nid[pos] = p;
        wave_sync();
        nnc = nnc < k ? nnc + 1 : k;
        if (nnc == k) {
          nn_wk = uni(nkey[k - 1]);
          nn_wi = uni(nid[k - 1]);
        }
      }
    }

    if (nv > 0) {
      // Merge, truncated to ef: old entry i moves to i + cnt_i (cnt_i = number of
      // candidates strictly before it); the candidate of rank r lands at r + lb_r
      // (lb_r = number of old entries <= it, so an old entry precedes an equal
      // new one).  The candidates are compacted into LDS and read back at
      // uniform addresses (broadcast reads); all old entries are read before
      // any is written.
      uint64_t* cbuf = reinterpret_cast<uint64_t*>(lds + L.cand);
      int32_t* lbarr = reinterpret_cast<int32_t*>(lds + L.cand);  // reused once the ranks are known
      if (valid) cbuf[lanes_below(V)] = cand;
      if (lane < 4) cbuf[nv + lane] = kNone;  // padding: compares below nothing
      wave_sync();
      const int nv4 = (nv + 3) & ~3;
      int sidx = 0;  // rank of this lane's candidate
      int lbv;       // lb of this lane's candidate
      if (size <= 128) {
        const bool live0 = lane < size, live1 = lane + 64 < size;
        const uint64_t e0 = live0 ? beam[lane] : kNone, e1 = live1 ? beam[lane + 64] : kNone;
        const uint64_t k0 = e0 & ~(uint64_t)kChecked, k1 = e1 & ~(uint64_t)kChecked;
        int c0 = 0, c1 = 0;
        if (size > 64) {
          for (int t = 0; t < nv4; t += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const uint64_t ct = cbuf[t + u];
              c0 += ct < k0;
              c1 += ct < k1;
              sidx += ct < cand;
            }
          }
        } else {
          for (int t = 0; t < nv4; t += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const uint64_t ct = cbuf[t + u];
              c0 += ct < k0;
              sidx += ct < cand;
            }
          }
        }
        // lb from the counts: the candidates of ranks [cnt_{i-1}, cnt_i) come
        // right before old entry i (cnt_{-1} = 0); ranks from cnt_{size-1} on
        // come after every old entry
        // cnt of the entry before (DPP wave_shr:1; lane 0 keeps the old value 0)
        int p0 = __builtin_amdgcn_update_dpp(0, c0, 0x138, 0xF, 0xF, false);
        int p1 = __builtin_amdgcn_update_dpp(0, c1, 0x138, 0xF, 0xF, false);
        if (lane == 0) p1 = (int)rdlane((uint32_t)c0, 63);
        if (live0)
          for (int r = p0; r < c0; ++r) lbarr[r] = lane;
        if (live1)
          for (int r = p1; r < c1; ++r) lbarr[r] = lane + 64;
        const int clast = size > 64 ? (int)rdlane((uint32_t)c1, size - 65) : (int)rdlane((uint32_t)c0, size - 1);
        wave_sync();
        lbv = (valid && sidx < clast) ? lbarr[sidx] : size;
        const int np0 = lane + c0, np1 = lane + 64 + c1;
        const uint64_t t0m = ballot(live0 && np0 == ef - 1), t1m = ballot(live1 && np1 == ef - 1);
        if (t0m) tail = rdlane64(k0, first_lane(t0m));
        if (t1m) tail = rdlane64(k1, first_lane(t1m));
        if (live0 && np0 < ef) beam[np0] = e0;
        if (live1 && np1 < ef) beam[np1] = e1;
      } else {
        // Beams above 128 entries.  Each candidate finds lb (old entries <= it)
        // by a binary search over the sorted beam; then the candidates are
        // stored in rank order and each old entry finds cnt (candidates below
        // it) by a binary search over them.  Old entries are moved top down, a
        // chunk at a time; once a chunk lies wholly below the smallest
        // candidate, it and every chunk under it stay where they are.
        for (int t = 0; t < nv4; t += 4) {
#pragma unroll
          for (int u = 0; u < 4; ++u) sidx += cbuf[t + u] < cand;
        }
        lbv = 0;
        if (valid) {
          int lo = 0, hi = size;  // beam[0, lo) <= cand < beam[hi, size)
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if ((beam[mid] & ~(uint64_t)kChecked) <= cand)
              lo = mid + 1;
            else
              hi = mid;
          }
          lbv = lo;
        }
        wave_sync();  // every read of the unsorted candidates is done
        if (valid) cbuf[sidx] = cand;
        wave_sync();
        const uint64_t cmin = cbuf[0];  // the same word for every lane
        for (int base = ((size - 1) >> 6) << 6; base >= 0; base -= 64) {  // top down
          const int i = base + lane;
          const bool live = i < size;
          const uint64_t e = live ? beam[i] : kNone;
          const uint64_t ke = e & ~(uint64_t)kChecked;
          const int top = size - 1 - base < 63 ? size - 1 - base : 63;
          if (rdlane64(ke, top) < cmin) break;  // nothing here or below moves
          int lo = 0, hi = nv;  // cbuf[0, lo) < ke <= cbuf[hi, nv)
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (cbuf[mid] < ke)
              lo = mid + 1;
            else
              hi = mid;
          }
          const int np = i + lo;
          if (live && lo > 0 && np < ef) beam[np] = e;
        }
      }
      const int npos = sidx + lbv;
      if (valid && npos < ef) beam[npos] = cand;
      const uint64_t tm = ballot(valid && npos == ef - 1);
      if (tm) tail = rdlane64(cand, first_lane(tm));
      wave_sync();
      const int first = (int)rdlane((uint32_t)npos, first_lane(ballot(valid && sidx == 0)));
      if (first < cursor) cursor = first;
      if (size > 128 && size + nv >= ef) tail = beam[ef - 1] & ~(uint64_t)kChecked;  // the same word for every lane
      size = (size + nv < ef) ? size + nv : ef;
    }

    if constexpr (has_stop<LS>) {
      if (expansions >= a.ls_t_min && (expansions - a.ls_t_min) % a.ls_t_every == 0) {
        StopFeatures F;
        const float nn1 = nn_in_regs ? rdlane(nrk, 0) : uni(nkey[0]);
        const float nnk = nn_in_regs ? rdlane(nrk, nnc - 1) : uni(nkey[nnc - 1]);
        F.compute(expansions, pops, nnc, k, since, de, nn1, nnk, bfk, size, ef, dp, app, R);
        float out;
        if constexpr (mlp_in_lds<LS>)
          out = stop_mlp_lds(mlp, F.mine, lane, reinterpret_cast<float*>(lds + L.cand));
        else
          out = a.ls_w ? stop_mlp(a.ls_w, F, lane) : __builtin_nanf("");
        if constexpr (LS == kLsTrace) {
          if (nevals < a.tr_max) {
            const int64_t slot = q * a.tr_max + nevals;
            if (lane < 16) a.tr_feat[slot * 16 + lane] = F.mine;
            for (int i = lane; i < k; i += 64) {
              int32_t id = -1;
              if (i < nnc) id = nn_in_regs ? (int32_t)nri : (int32_t)nid[i];
              a.tr_nn[slot * k + i] = id;
            }
            if (lane == 0) a.tr_out[slot] = out;
          }
          ++nevals;
        }
        if (out > a.ls_theta) break;  // false for NaN: no model, no stop
      }
    }
  }
  if constexpr (LS == kLsTrace) {
    if (a.tr_max > 0 && lane == 0) a.tr_count[q] = nevals < a.tr_max ? nevals : a.tr_max;
  }

  // answer: NN ascending by (distance, id), padded with (-1, inf)
  const int k_out = is_mixed<LS> ? a.k_out : k;  // a mixed batch's rows are k_out wide
  for (int i = lane; i < k_out; i += 64) {
    int32_t id = -1;
    float d = __builtin_inff();
    if (i < nnc) {
      id = nn_in_regs ? (int32_t)nri : (int32_t)nid[i];
      d = nn_in_regs ? nrk : nkey[i];
    }
    a.out_ids[q * k_out + i] = id;
    a.out_dists[q * k_out + i] = d;
  }
  if (a.out_stats && lane == 0) {
    int32_t* st = a.out_stats + 4 * q;
    st[0] = expansions;
    st[1] = pops;
    st[2] = appended;
    st[3] = GV ? 1 : 0;
  }
}

// Algorithm 1 with the beam in registers (ef up to 64 NB): lane i holds beam
// entries i and 64 + i, each with a checked flag and a consumed-duplicate flag
// (its vertex was expanded through another entry).  The loop is
// software-pipelined.  The next vertex to expand is known before the merge:
// it is the smaller of the best new candidate and the first old entry neither
// checked nor consumed.  Its block is prefetched, and at the top of the next
// iteration its exact distance, FastScan lookups and visited probes are issued
// while the previous merge's read-back is still in flight; the pop's
// bookkeeping (flags, pop count, the next unconsumed entry) then runs on the
// merged beam.  Results and counters equal those of search_one.
template <int D, int R, int LS, int NB, int LB>
__device__ void search_one_rb(const SearchArgs& a, int64_t q, uint8_t* lds, const qgl::SearchLds& L,
                              const uint8_t* mlp) {
  using BV = BlockView<D, R>;
  constexpr int DPL = BV::DPL;
  constexpr int LPN = BV::LPN;
  constexpr uint64_t kNone = ~0ull;  // sorts after every real entry
  constexpr uint64_t kFlags = (uint64_t)(kChecked | kDup);
  const int lane = lane_id();
  int ef = a.ef, k = a.k;
  if constexpr (is_mixed<LS>) {
    ef = uni(a.ef_q[q]);
    k = uni(a.k_q[q]);
    if (k < 1 || k > a.k || ef < 1 || ef > a.ef) {  // rejected: an all-padding row, stats[3] = -1
      for (int i = lane; i < a.k_out; i += 64) {
        a.out_ids[q * a.k_out + i] = -1;
        a.out_dists[q * a.k_out + i] = __builtin_inff();
      }
      if (a.out_stats && lane < 4) a.out_stats[4 * q + lane] = lane == 3 ? -1 : 0;
      return;
    }
  }
  void* lut = lds + L.lut;
  uint64_t* sc = reinterpret_cast<uint64_t*>(lds + L.beam);    // merge output range (ef_cap words)
  uint64_t* cbuf = reinterpret_cast<uint64_t*>(lds + L.cand);  // candidates (R + 4 words)
  float* nkey = reinterpret_cast<float*>(lds + L.nkey);
  uint32_t* nid = reinterpret_cast<uint32_t*>(lds + L.nid);
  Visited vis;
  vis.tab = reinterpret_cast<uint32_t*>(lds + L.hash);
  vis.hbits = a.hash_bits;
  vis.mask = (1u << a.hash_bits) - 1u;
  vis.bits = nullptr;
  const int vis_limit = (1 << a.hash_bits) / 2;
  for (int i = lane; i < (1 << a.hash_bits); i += 64) vis.tab[i] = kEmpty;

  constexpr bool kQvLds = qgl::query_in_lds(D);
  float qv[kQvLds ? 1 : DPL];
  float* qs = reinterpret_cast<float*>(lds + L.qv);
  const float* qr = a.queries + q * D;
  if constexpr (kQvLds) {
    for (int i = lane; i < D; i += 64) qs[i] = qr[i];
  } else {
#pragma unroll
    for (int t = 0; t < DPL; ++t) {
      const int i = lane + 64 * t;
      qv[t] = (i < D) ? qr[i] : 0.0f;
    }
  }
  auto dist = [&](const float(&xv)[DPL]) {
    if constexpr (kQvLds) {
      float pp = 0.0f;
#pragma unroll
      for (int t = 0; t < DPL; ++t) {
        const float d = qs[lane + 64 * t] - xv[t];
        pp = __builtin_fmaf(d, d, pp);
      }
      return butterfly_f(pp);
    } else {
      return exact_dist<DPL>(qv, xv);
    }
  };
  const float delta = build_lut<D, R, LB>(a.qrot + q * D, lut, a.lut_pad);

  // the entry starts the beam, keyed by its exact distance; it is the first
  // vertex expanded, so its block serves both
  BV b;
  b.load(a.blocks + (int64_t)a.entry * a.block_bytes, lane);
  float dp = uni(dist(b.x));
  const float de = dp;
  uint32_t p = (uint32_t)a.entry;
  uint64_t pword = pack_kv(de, p);  // p's beam word
  uint64_t tail = pword;            // beam[ef - 1] whenever the beam is full
  uint64_t bw[NB];
#pragma unroll
  for (int r = 0; r < NB; ++r) bw[r] = (r == 0 && lane == 0) ? pword : kNone;
  int size = 1;
  bool pending = false;  // a merge whose read-back has not been done yet
  int pend_nv = 0;       // its number of candidates
  int nvis = 0, nnc = 0, expansions = 0, pops = 0, appended = 0, since = 0;
  float nn_wk = 0.0f;
  uint32_t nn_wi = 0;
  const bool nn_in_regs = k <= 64;
  float nrk = 0.0f;
  uint32_t nri = 0;
  BV nxt;

  for (;;) {
    // ---- expansion of p (block b, exact distance dp)
    // read-back of the pending merge's range, into the beam registers (their
    // old values died with the merge's scatter)
    if (pending) {
#pragma unroll
      for (int r = 0; r < NB; ++r) {
        const int i = 64 * r + lane;
        bw[r] = i < size ? sc[i] : kNone;
      }
    }
    // visited probes: p's insertion run (64 consecutive slots) and each
    // neighbour's first group of four slots (p itself is excluded explicitly:
    // it is inserted below, after these reads)
    const uint32_t pslot = vis.slot4(p);
    const uint32_t prun = vis.tab[(pslot + lane) & vis.mask];
    const uint32_t nb = (uint32_t)b.nb;
    const bool probe = (lane % LPN == 0) && b.nb >= 0 && nb != p;
    uint32_t ns = vis.slot4(probe ? nb : 0u);
    uint4 ne = vis.group(ns);
    // FastScan estimates of all neighbours (Eq. normalization with Eq. 3.1)
    const int S = b.template fastscan<LB>(lut, lane, a.lut_pad);
    // finish the pending merge: range slots still holding the sentinel take
    // the candidates in rank order
    if (pending) {
      int holes = 0;
#pragma unroll
      for (int r = 0; r < NB; ++r) {
        const bool hole = 64 * r + lane < size && bw[r] == kNone;
        const uint64_t hm = ballot(hole);
        if (hole) bw[r] = cbuf[holes + lanes_below(hm)];
        holes += __popcll(hm);
      }
      if (size == ef) tail = rdlane64(pick<NB>(bw, (ef - 1) >> 6), (ef - 1) & 63) & ~kFlags;
    }
    const float est = __builtin_fmaf(b.fr, (float)S * delta, b.fa + dp);
    const uint64_t cand = pack_kv(est, nb);

    // pop p: its entry is the first entry neither checked nor consumed; the
    // unchecked entries before it are consumed duplicates, each a pop
    uint64_t um[NB], pm[NB];
#pragma unroll
    for (int r = 0; r < NB; ++r) {
      um[r] = ballot(!((uint32_t)bw[r] & kChecked));
      pm[r] = ballot(bw[r] == pword);
    }
    int rs = NB - 1, f = 0;
#pragma unroll
    for (int r = NB - 1; r >= 0; --r)
      if (pm[r]) {
        rs = r;
        f = first_lane(pm[r]);
      }
    const uint64_t before = (1ull << f) - 1ull;
#pragma unroll
    for (int r = 0; r < NB; ++r) {
      const uint64_t dup = r < rs ? um[r] : (r == rs ? (um[r] & before) : 0ull);
      pops += __popcll(dup);
      const uint64_t take = dup | (r == rs ? 1ull << f : 0ull);
      if ((take >> lane) & 1ull) bw[r] |= kChecked;
    }
    ++pops;
    // p's other unchecked entries become consumed duplicates; the next
    // unconsumed entry (o2f, a prefetch candidate) and the next unchecked one
    // (o2u, for the stop features) follow p's entry
    uint64_t o2f = kNone, o2u = kNone;
    {
      int rf = -1, ru = -1;
      uint64_t mf = 0, mu = 0;
#pragma unroll
      for (int r = NB - 1; r >= 0; --r) {
        const uint32_t lo = (uint32_t)bw[r];
        if ((lo & (kChecked | kDup | kIdMask30)) == p) bw[r] |= kDup;
        const uint64_t fr_ = ballot(!((uint32_t)bw[r] & (kChecked | kDup)));
        const uint64_t ur_ = ballot(!((uint32_t)bw[r] & kChecked));
        if (fr_) {
          rf = r;
          mf = fr_;
        }
        if (ur_) {
          ru = r;
          mu = ur_;
        }
      }
      if (rf >= 0) o2f = rdlane64(pick<NB>(bw, rf), first_lane(mf)) & ~kFlags;
      if (has_stop<LS> && ru >= 0) o2u = rdlane64(pick<NB>(bw, ru), first_lane(mu)) & ~kFlags;
    }

    // insert p into the visited set: the first empty slot of its probe run
    {
      uint64_t em = ballot(prun == kEmpty);
      if (em) {
        if (lane == first_lane(em)) vis.tab[(pslot + lane) & vis.mask] = p;
      } else {
        visited_add_absent(vis, p, pslot, lane);  // 64 occupied slots in a row (the table is at most half full)
      }
    }
    if (++nvis > vis_limit) {  // on-chip visited set full: hand the query to the overflow path
      if (lane == 0) {
        const int slot = atomicAdd(a.counters + 1, 1);
        a.overflow_list[slot] = (int32_t)q;
      }
      return;
    }
    ++expansions;

    // visited filter: the probes that met four other ids go on to the next
    // group
    bool seen = probe && group_has(ne, nb);
    bool more = probe && !seen && group_full(ne);
    while (ballot(more)) {
      if (more) {
        ns = (ns + 4) & vis.mask;
        ne = vis.group(ns);
        seen = group_has(ne, nb);
        more = !seen && group_full(ne);
      }
    }
    bool valid = probe && !seen;
    const int app = uni((int)__popcll(ballot(valid)));
    appended += app;
    if (size == ef) valid = valid && cand < tail;  // would fall past the cut anyway
    const uint64_t V = ballot(valid);
    const int nv = uni((int)__popcll(V));
    if (nv > 0 && valid) cbuf[lanes_below(V)] = cand;  // compacted for the merge's broadcast reads (after
                                                         // the read-back above: LDS keeps order)

    // best candidate (the smallest (estimate, id) among them)
    uint64_t best = kNone;
    if (nv > 0) {
      const uint32_t hk = wave_min_u32(valid ? (uint32_t)(cand >> 32) : 0xFFFFFFFFu);
      const uint64_t tie = ballot(valid && (uint32_t)(cand >> 32) == hk);
      const uint32_t lo = (tie & (tie - 1)) ? wave_min_u32((tie >> lane) & 1 ? (uint32_t)cand : 0xFFFFFFFFu)
                                            : rdlane((uint32_t)cand, first_lane(tie));
      best = ((uint64_t)hk << 32) | lo;
    }
    // the next vertex to expand: prefetch its block (Sec. 3.1.4)
    const uint64_t nxt_f = best < o2f ? best : o2f;
    if (nxt_f != kNone) nxt.load(a.blocks + (int64_t)((uint32_t)nxt_f & kIdMask30) * a.block_bytes, lane);
    const uint64_t nxt_u = best < o2u ? best : o2u;
    const float bfk = nxt_u == kNone ? __builtin_inff() : unsortable((uint32_t)(nxt_u >> 32));

    // implicit re-ranking: NN keeps the k smallest (distance, id) seen
    ++since;
    if (nnc < k || kv_less(dp, p, nn_wk, nn_wi)) {
      since = 0;
      if (nn_in_regs) {
        const int pos = (int)__popcll(ballot(lane < nnc && kv_less(nrk, nri, dp, p)));
        const int last = nnc < k ? nnc : k - 1;
        const float upk = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(nrk), 0x138, 0xF, 0xF, false));
        const uint32_t upi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)nri, 0x138, 0xF, 0xF, false);
        if (lane > pos && lane <= last) {
          nrk = upk;
          nri = upi;
        }
        if (lane == pos) {
          nrk = dp;
          nri = p;
        }
        nnc = nnc < k ? nnc + 1 : k;
        if (nnc == k) {
          nn_wk = rdlane(nrk, k - 1);
          nn_wi = rdlane(nri, k - 1);
        }
      } else {
        int pos = 0;
        for (int base = 0; base < nnc; base += 64) {
          const int i = base + lane;
          const bool lt = (i < nnc) && kv_less(nkey[i < nnc ? i : 0], nid[i < nnc ? i : 0], dp, p);
          pos += __popcll(ballot(lt));
        }
        const int last = nnc < k ? nnc : k - 1;  // entries [pos, last) move up by one
        for (int base = ((last - 1) >> 6) << 6; base >= 0 && last > pos; base -= 64) {
          const int i = base + lane;
          float kk = 0.0f;
          uint32_t ii = 0;
          const bool mv = (i >= pos) && (i < last);
          if (mv) {
            kk = nkey[i];
            ii = nid[i];
          }
          wave_sync();
          if (mv) {
            nkey[i + 1] = kk;
            nid[i + 1] = ii;
          }
          wave_sync();
          if (base < pos) break;
        }
        pos = uni(pos);
        nkey[pos] = dp;
        nid[pos] = p;
        wave_sync();
        nnc = nnc < k ? nnc + 1 : k;
        if (nnc == k) {
          nn_wk = uni(nkey[k - 1]);
          nn_wi = uni(nid[k - 1]);
        }
      }
    }

    // Merge, truncated to ef (its read-back happens at the top of the next
    // iteration).  Every old entry counts the candidates below it (cnt) and
    // every candidate its rank among them, from broadcast reads of the
    // compacted candidates.  The new range is filled with a sentinel, old
    // entry i is written at i + cnt_i and the candidates by rank to the
    // candidate array; the range slots still holding the sentinel are then the
    // candidates' places in rank order (an old entry equal to a candidate
    // precedes it, since cnt counts strictly smaller candidates).
    pending = nv > 0;
    if (nv > 0) {
      uint64_t bm[NB];
      int cnt[NB];
#pragma unroll
      for (int r = 0; r < NB; ++r) {
        bm[r] = bw[r] & ~kFlags;
        cnt[r] = 0;
      }
      int rank = 0;
      auto count = [&](uint64_t ct) {
#pragma unroll
        for (int r = 0; r < NB; ++r) cnt[r] += ct < bm[r];
        rank += ct < cand;
      };
      int t = 0;
      for (; t + 4 <= nv; t += 4) {  // four broadcast reads in flight
        const uint64_t c0 = cbuf[t], c1 = cbuf[t + 1], c2 = cbuf[t + 2], c3 = cbuf[t + 3];
        count(c0);
        count(c1);
        count(c2);
        count(c3);
      }
      for (; t < nv; ++t) count(cbuf[t]);  // the last one to three
      const int nsz = (size + nv < ef) ? size + nv : ef;
#pragma unroll
      for (int r = 0; r < NB; ++r)
        if (64 * r + lane < nsz) sc[64 * r + lane] = kNone;
#pragma unroll
      for (int r = 0; r < NB; ++r) {
        const int np = 64 * r + lane + cnt[r];
        if (64 * r + lane < size && np < ef) sc[np] = bw[r];
      }
      if (valid) cbuf[rank] = cand;  // after the count loop's reads (LDS keeps order)
      size = nsz;
      pend_nv = nv;
    }

    if constexpr (has_stop<LS>) {
      if (expansions >= a.ls_t_min && (expansions - a.ls_t_min) % a.ls_t_every == 0) {
        StopFeatures F;
        const float nn1 = nn_in_regs ? rdlane(nrk, 0) : uni(nkey[0]);
        const float nnk = nn_in_regs ? rdlane(nrk, nnc - 1) : uni(nkey[nnc - 1]);
        F.compute(expansions, pops, nnc, k, since, de, nn1, nnk, bfk, size, ef, dp, app, R);
        float out;
        if constexpr (mlp_in_lds<LS>)
          out = stop_mlp_lds(mlp, F.mine, lane, reinterpret_cast<float*>(lds + L.aux));
        else
          out = a.ls_w ? stop_mlp(a.ls_w, F, lane) : __builtin_nanf("");
        if (out > a.ls_theta) break;  // false for NaN: no model, no stop
      }
    }

    if (nxt_f == kNone) {
      // no unconsumed entry is left (and no candidate, so no merge): every
      // remaining unchecked entry is a consumed duplicate, popped in turn
#pragma unroll
      for (int r = 0; r < NB; ++r) pops += __popcll(ballot(!((uint32_t)bw[r] & kChecked)));
      break;
    }
    p = (uint32_t)nxt_f & kIdMask30;
    pword = nxt_f;
    b = nxt;
    dp = uni(dist(b.x));
  }
  (void)pend_nv;

  // answer: NN ascending by (distance, id), padded with (-1, inf)
  const int k_out = is_mixed<LS> ? a.k_out : k;
  for (int i = lane; i < k_out; i += 64) {
    int32_t id = -1;
    float d = __builtin_inff();
    if (i < nnc) {
      id = nn_in_regs ? (int32_t)nri : (int32_t)nid[i];
      d = nn_in_regs ? nrk : nkey[i];
    }
    a.out_ids[q * k_out + i] = id;
    a.out_dists[q * k_out + i] = d;
  }
  if (a.out_stats && lane == 0) {
    int32_t* st = a.out_stats + 4 * q;
    st[0] = expansions;
    st[1] = pops;
    st[2] = appended;
    st[3] = 0;
  }
}

// Minimum wavefronts per SIMD the register allocator must allow (1: no
// constraint).  LDS-beam kernels with D <= 256: 6 for the stop-only and
// mixed-batch modes.  Register-beam kernels with R = 32, plain or mixed
// batches, D = 128 (but the one-word plain kernel, which fits in 80 registers
// anyway) and D = 96: 6, where the allocator would otherwise take 82-96
// registers and drop to 5 wavefronts per SIMD; the few values it then keeps in
// scratch (16-56 bytes per lane) cost less than the lost wavefront (5-17%
// faster at 10,000 and 80,000 queries).  The stop kernels with the beam in
// registers at D = 128, R = 32 (one query or a mixed batch): 6 as well (107-115
// registers and 4 wavefronts otherwise; 48-84 bytes of scratch; 6-16% faster).  Measured not to pay: 4 for D = 768 (32
// bytes of scratch, 1-2% slower); R = 64 would spill over 100 bytes.
template <int D, int R, int LS, int NB>
constexpr int waves_hint() {
  if constexpr (NB > 0) {
    constexpr bool mode = LS == kLsOff || LS == kMixed;
    if constexpr (R == 32 && D == 128 && (LS == kLsStop || LS == kMixedStop)) return 6;
    if constexpr (R == 32 && D == 128) return mode && !(NB == 1 && LS == kLsOff) ? 6 : 1;
    if constexpr (R == 32 && D == 96) return mode ? 6 : 1;
    return 1;
  }
  return D > 256 ? 1 : (mlp_in_lds<LS> || LS == kMixed) ? 6 : 1;
}

// Each wavefront takes queries until none is left: first its own index, then
// from a shared counter.
// GV = false: main pass over all queries with the LDS visited hash.
// GV = true : overflow pass over the queries the main pass handed over, with
//             a global bitset per wavefront.
// The stop-only kernels share one MLP image per workgroup of 8 wavefronts.
// For the narrow shapes the stop-only and mixed-batch kernels hold their
// registers to 80, so that 6 wavefronts per SIMD fit (LDS sets residency for
// the stop-only kernels anyway).
template <int D, int R, bool GV, int LS, int NB, int LB>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(waves_hint<D, R, LS, NB>()))) void search_kernel(
    SearchArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int wave = uni((int)(threadIdx.x >> 6));
  const int lane = lane_id();
  const qgl::SearchLds L = qgl::search_lds(D, R, a.ef_cap, GV ? 0 : (1 << a.hash_bits), a.k_cap, LB);
  uint8_t* lds = smem + wave * L.total;
  uint8_t* mlp = smem + (blockDim.x >> 6) * L.total;  // after every wavefront's area
  if constexpr (mlp_in_lds<LS>) {
    stage_mlp(a.ls_w, mlp);
    __syncthreads();
  }
  const int wid = blockIdx.x * (blockDim.x >> 6) + wave;
  uint32_t* gbits = GV ? a.fb_bits + (int64_t)wid * a.fb_words : nullptr;
  int* ctr = a.counters + (GV ? 2 : 0);
  const int64_t limit = GV ? (int64_t)__hip_atomic_load(a.counters + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                           : a.nq;
  // A wavefront's first query is its own index; the later ones come from the
  // shared counter, offset by the number of wavefronts.  (A device-wide atomic
  // on one address is served one at a time, so taking every first query from
  // it would start the wavefronts only gradually.)
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t qi = wid; qi < limit;) {
    const int64_t q = GV ? (int64_t)a.overflow_list[qi] : qi;
    if constexpr (NB > 0)
      search_one_rb<D, R, LS, NB, LB>(a, q, lds, L, mlp);
    else
      search_one<D, R, GV, LS, LB>(a, q, lds, L, gbits, mlp);
    int c = 0;
    if (lane == 0) c = atomicAdd(ctr, 1);
    qi = nwaves + __builtin_amdgcn_readlane(c, 0);
  }
}

// -------------------------------------------------------------- estimator

template <int D, int R>
__global__ __launch_bounds__(64) void estimate_kernel(EstimateArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  using BV = BlockView<D, R>;
  const int lane = lane_id();
  const int64_t q = blockIdx.x;
  int16_t* lut = reinterpret_cast<int16_t*>(smem);
  const float delta = build_lut<D, R>(a.qrot + q * D, lut, a.lut_pad);
  float qv[BV::DPL];
  for (int t = 0; t < BV::DPL; ++t) {
    const int i = lane + 64 * t;
    qv[t] = (i < D) ? a.queries[q * D + i] : 0.0f;
  }
  BV b;
  b.load(a.blocks + (int64_t)a.vertex[q] * a.block_bytes, lane);
  const float dp = exact_dist<BV::DPL>(qv, b.x);
  const int S = b.fastscan(lut, lane, a.lut_pad);
  const float est = __builtin_fmaf(b.fr, (float)S * delta, b.fa + dp);
  if (lane % BV::LPN == 0) {
    a.out_S[q * R + lane / BV::LPN] = S;
    a.out_est[q * R + lane / BV::LPN] = est;
  }
  if (lane == 0) a.out_dist[q] = dp;
}

// --------------------------------------------------------------- launchers

#define QG_SHAPES(X) X(96, 32) X(96, 64) X(128, 32) X(128, 64) X(768, 32) X(768, 64) X(960, 32) X(960, 64)

bool shape_supported(int D, int R) {
#define QG_CASE(d, r) if (D == d && R == r) return true;
  QG_SHAPES(QG_CASE)
#undef QG_CASE
  return false;
}

hipError_t launch_rotate(const float* in, int64_t n, int D, const float* M, float* out, int* zero, int nzero,
                         hipStream_t st) {
  if (n <= 0) {
    if (zero && nzero > 0)
      hipLaunchKernelGGL((rotate_kernel<false, 1>), dim3(1), dim3(64), 0, st, in, 0, D, M, out, zero, nzero);
    return hipGetLastError();
  }
  // four columns per lane when every row starts 16-byte aligned (M is the
  // library's own allocation); 2 x 2 tiles per wavefront for the wide shapes
  // (D = 768: 5-9% faster; D = 128: 3% slower at 10,000 rows, with a quarter
  // as many wavefronts)
  const bool v4 = (reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(M)) % 16 == 0 && D % 4 == 0;
  const int nt = v4 && D % 32 == 0 && D > 256 ? 2 : 1;
  const int64_t blocks = (n + 16 * nt - 1) / (16 * nt);  // row blocks, padded to a multiple of 8 (one per XCD)
  const dim3 grid((unsigned)(((blocks + 7) / 8) * 8 * (D / (16 * nt))));
  if (nt == 2)
    hipLaunchKernelGGL((rotate_kernel<true, 2>), grid, dim3(64), 0, st, in, n, D, M, out, zero, nzero);
  else if (v4)
    hipLaunchKernelGGL((rotate_kernel<true, 1>), grid, dim3(64), 0, st, in, n, D, M, out, zero, nzero);
  else
    hipLaunchKernelGGL((rotate_kernel<false, 1>), grid, dim3(64), 0, st, in, n, D, M, out, zero, nzero);
  return hipGetLastError();
}

hipError_t launch_encode(const float* X, const float* ROT, int64_t N, int D, const int32_t* G, int R,
                         uint8_t* blocks, int64_t B, hipStream_t st) {
  const int wpb = 4;
  dim3 grid((unsigned)((N + wpb - 1) / wpb));
  hipLaunchKernelGGL(encode_kernel, grid, dim3(64 * wpb), 0, st, X, ROT, N, D, G, R, blocks, B);
  return hipGetLastError();
}

template <int D, int R, bool GV, int LS, int NB, int LB>
static hipError_t launch_search_t(const SearchArgs& a, int grid, int wpb, size_t lds, hipStream_t st) {
  auto kern = search_kernel<D, R, GV, LS, NB, LB>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * wpb), lds, st, a);
  return hipGetLastError();
}

template <int D, int R, bool GV, int LS, int NB, int LB>
static int occupancy_t(int wpb, size_t lds) {
  int nb = 0;
  auto kern = search_kernel<D, R, GV, LS, NB, LB>;
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, 64 * wpb, lds) != hipSuccess) return 0;
  return nb;
}

struct LaunchOp {
  const SearchArgs* a;
  int grid, wpb;
  size_t lds;
  hipStream_t st;
  template <int D, int R, bool GV, int LS, int NB, int LB>
  hipError_t run() const {
    return launch_search_t<D, R, GV, LS, NB, LB>(*a, grid, wpb, lds, st);
  }
};

struct OccupancyOp {
  int wpb;
  size_t lds;
  template <int D, int R, bool GV, int LS, int NB, int LB>
  int run() const {
    return occupancy_t<D, R, GV, LS, NB, LB>(wpb, lds);
  }
};

// The kernel instantiation for (D, R), pass, mode, beam storage and LUT
// entry width.  Register beams (nb 1, 2) exist for the main pass of the
// plain, stop-only and mixed modes; the traced, "w/o ME" and overflow-pass
// kernels keep the beam in LDS.  The int32 LUT (lb 4) exists for the main
// pass of the plain and mixed modes (the ones the autotuner times).
template <int D, int R, class Op, class Ret>
static Ret dispatch_mode(bool gv, int ls, int nb, int lb, const Op& op, Ret bad) {
  if (gv) {
    if (lb != 2) return bad;
    switch (ls) {
      case kLsOff: return op.template run<D, R, true, kLsOff, 0, 2>();
      case kLsStop: return op.template run<D, R, true, kLsStop, 0, 2>();
      case kLsTrace: return op.template run<D, R, true, kLsTrace, 0, 2>();
      case kMixed: return op.template run<D, R, true, kMixed, 0, 2>();
      case kMixedStop: return op.template run<D, R, true, kMixedStop, 0, 2>();
      case kNoMe: return op.template run<D, R, true, kNoMe, 0, 2>();
      default: return bad;
    }
  }
#define QG_NB(ls_, lb_)                                                                         \
  (nb == 1 ? op.template run<D, R, false, ls_, 1, lb_>()                                        \
           : nb == 2 ? op.template run<D, R, false, ls_, 2, lb_>() : op.template run<D, R, false, ls_, 0, lb_>())
  if (lb == 4) {
    switch (ls) {
      case kLsOff: return QG_NB(kLsOff, 4);
      case kMixed: return QG_NB(kMixed, 4);
      default: return bad;
    }
  }
  if (lb != 2) return bad;
  switch (ls) {
    case kLsOff: return QG_NB(kLsOff, 2);
    case kLsStop: return QG_NB(kLsStop, 2);
    case kLsTrace: return op.template run<D, R, false, kLsTrace, 0, 2>();
    case kMixed: return QG_NB(kMixed, 2);
    case kMixedStop: return QG_NB(kMixedStop, 2);
    case kNoMe: return op.template run<D, R, false, kNoMe, 0, 2>();
    default: return bad;
  }
#undef QG_NB
}

// Measured on the SIFT-shaped 1M x 128 index (10,000 queries): one beam
// register is 11-14% faster than the LDS beam in the plain, mixed and
// stop-only kernels; two registers tie with it in the plain and mixed kernels
// and lose 6% in the stop-only kernel (whose MLP already holds many registers).
int beam_regs(bool overflow_pass, int ls_mode, int ef_bound, int64_t n) {
  if (overflow_pass || ls_mode == kLsTrace || ls_mode == kNoMe || n > (int64_t)kIdMask30) return 0;
  if (ef_bound <= 64) return 1;
  return (ef_bound <= 128 && (ls_mode == kLsOff || ls_mode == kMixed)) ? 2 : 0;
}

hipError_t launch_search(int D, int R, bool overflow_pass, int ls_mode, int nb, int lb, const SearchArgs& a,
                         int grid, int wpb, size_t lds, hipStream_t st) {
  const LaunchOp op{&a, grid, wpb, lds, st};
#define QG_CASE(d, r) \
  if (D == d && R == r) return dispatch_mode<d, r>(overflow_pass, ls_mode, nb, lb, op, hipErrorInvalidValue);
  QG_SHAPES(QG_CASE)
#undef QG_CASE
  return hipErrorInvalidValue;
}

int search_occupancy(int D, int R, bool overflow_pass, int ls_mode, int nb, int lb, int wpb, size_t lds) {
  const OccupancyOp op{wpb, lds};
#define QG_CASE(d, r) \
  if (D == d && R == r) return dispatch_mode<d, r>(overflow_pass, ls_mode, nb, lb, op, 0);
  QG_SHAPES(QG_CASE)
#undef QG_CASE
  return 0;
}

hipError_t launch_estimate(int D, int R, const EstimateArgs& a, int64_t nq, hipStream_t st) {
  const size_t lds = (size_t)qgl::align16(qgl::lut_rows_padded(D, R) * 32);
#define QG_CASE(d, r)                                                                           \
  if (D == d && R == r) {                                                                       \
    hipLaunchKernelGGL((estimate_kernel<d, r>), dim3((unsigned)nq), dim3(64), lds, st, a);      \
    return hipGetLastError();                                                                   \
  }
  QG_SHAPES(QG_CASE)
#undef QG_CASE
  return hipErrorInvalidValue;
}

}  // namespace qgk
