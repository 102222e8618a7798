// qg_graph.hip -- gfx950 kernels of the index construction (Algorithm 2,
// Sec. 3.2): candidate lists with exact distances, the NSG pruning rule, the
// angle-based refinement to exactly R edges with random fill, and the helpers
// of the connectivity repair.
//
// Arithmetic: every distance, norm and inner product the decisions rest on is
// an fp64 sum over dimensions 0 .. D-1 in ascending order, with a separate
// multiply and add per term (compiled with -ffp-contract=off), of differences
// of fp32 coordinates widened to fp64; cosines divide by the product of two
// square roots.  One lane computes one such sum, so its order is the
// sequential one.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qg_graph.h"

namespace qgg {

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ int lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ int first_lane(uint64_t m) { return __ffsll((unsigned long long)m) - 1; }

// sum_t ((double)a[t] - (double)b[t])^2, t ascending
__device__ __forceinline__ double dist2_seq(const float* __restrict__ a, const float* __restrict__ b, int D) {
  double s = 0.0;
  for (int t = 0; t < D; t += 4) {
    const float4 x = *reinterpret_cast<const float4*>(a + t);
    const float4 y = *reinterpret_cast<const float4*>(b + t);
    double d = (double)x.x - (double)y.x;
    s = s + d * d;
    d = (double)x.y - (double)y.y;
    s = s + d * d;
    d = (double)x.z - (double)y.z;
    s = s + d * d;
    d = (double)x.w - (double)y.w;
    s = s + d * d;
  }
  return s;
}

// (d, id) ascending
__device__ __forceinline__ bool cand_greater(double da, int32_t ia, double db, int32_t ib) {
  return da > db || (da == db && ia > ib);
}

// Candidates of vertex u (Alg. 2, the search step of each iteration): the
// search results for x_u that are not u, then u's current neighbours not among
// them and not u; each with its exact squared distance to u; sorted by
// (distance, id).  One wavefront per vertex of the chunk; P = the candidate
// capacity rounded up to a power of two (LDS: P ids and P distances).
__global__ __launch_bounds__(64) void candidates_kernel(const float* __restrict__ X, int D,
                                                        const int32_t* __restrict__ sids, int EF,
                                                        const int32_t* __restrict__ G, int R, int64_t u0, int C, int P,
                                                        int32_t* __restrict__ cid, double* __restrict__ cd,
                                                        int32_t* __restrict__ ncand) {
  extern __shared__ __align__(16) uint8_t sm[];
  double* ld = reinterpret_cast<double*>(sm);
  int32_t* li = reinterpret_cast<int32_t*>(sm + 8 * (size_t)P);
  const int lane = lane_id();
  const int64_t u = u0 + blockIdx.x;
  const int32_t* srow = sids + (int64_t)blockIdx.x * EF;
  int n = 0;
  for (int a0 = 0; a0 < EF; a0 += 64) {
    const int a = a0 + lane;
    const int32_t v = a < EF ? srow[a] : -1;
    const bool ok = v >= 0 && v != (int32_t)u;
    const uint64_t m = ballot(ok);
    if (ok) li[n + lanes_below(m)] = v;
    n += __popcll(m);
  }
  __syncthreads();
  for (int j = 0; j < R; ++j) {
    const int32_t v = G[u * R + j];
    if (v < 0 || v == (int32_t)u) continue;
    bool dup = false;
    for (int i = lane; i < n; i += 64) dup |= li[i] == v;
    if (ballot(dup)) continue;
    if (lane == 0) li[n] = v;
    ++n;
    __syncthreads();
  }
  const float* xu = X + u * D;
  for (int i = lane; i < P; i += 64) {
    if (i < n) {
      ld[i] = dist2_seq(xu, X + (int64_t)li[i] * D, D);
    } else {
      ld[i] = __builtin_inf();
      li[i] = 0x7fffffff;
    }
  }
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = lane; i < P; i += 64) {
        const int l = i ^ j;
        if (l > i) {
          const bool up = (i & k) == 0;
          const double di = ld[i], dl = ld[l];
          const int32_t ii = li[i], il = li[l];
          if (cand_greater(di, ii, dl, il) == up) {
            ld[i] = dl;
            ld[l] = di;
            li[i] = il;
            li[l] = ii;
          }
        }
      }
      __syncthreads();
    }
  for (int i = lane; i < n; i += 64) {
    cid[u * C + i] = li[i];
    cd[u * C + i] = ld[i];
  }
  if (lane == 0) ncand[u] = n;
}

// NSG pruning rule (Sec. 3.2.1): scan the sorted candidates and keep v unless
// an already kept w is closer to v than u is, until R are kept.  The 64
// candidates of a chunk are tested against the kept set in parallel, then
// resolved in order: the first undecided one is kept and tests the later ones.
__global__ __launch_bounds__(64) void nsg_kernel(const float* __restrict__ X, int D, int R, int64_t N, int C,
                                                 const int32_t* __restrict__ cid, const double* __restrict__ cd,
                                                 const int32_t* __restrict__ ncand, int32_t* __restrict__ Gout,
                                                 int32_t* __restrict__ kidx, int32_t* __restrict__ nkept) {
  extern __shared__ __align__(16) uint8_t sm[];
  int32_t* kept = reinterpret_cast<int32_t*>(sm);  // R ids
  const int lane = lane_id();
  const int64_t u = blockIdx.x;
  if (u >= N) return;
  const int n = ncand[u];
  int nk = 0;
  for (int base = 0; base < n && nk < R; base += 64) {
    const int i = base + lane;
    const bool active = i < n;
    const int32_t c = active ? cid[u * C + i] : 0;
    const double di = active ? cd[u * C + i] : 0.0;
    const float* xc = X + (int64_t)c * D;
    bool decided = !active;  // occluded, kept, or past the list
    for (int a = 0; a < nk; ++a) {
      const int32_t w = kept[a];
      if (!decided) decided = dist2_seq(X + (int64_t)w * D, xc, D) < di;
    }
    for (;;) {
      const uint64_t m = ballot(!decided);
      if (!m || nk >= R) break;
      const int f = first_lane(m);
      const int32_t w = __builtin_amdgcn_readlane(c, f);
      if (lane == 0) {
        kept[nk] = w;
        kidx[u * R + nk] = base + f;
      }
      ++nk;
      if (lane == f) decided = true;
      if (!decided) decided = dist2_seq(X + (int64_t)w * D, xc, D) < di;
      __syncthreads();
    }
  }
  for (int j = lane; j < R; j += 64) Gout[u * R + j] = j < nk ? kept[j] : -1;
  if (lane == 0) nkept[u] = nk;
}

// Graph refinement (Sec. 3.2.2) and random fill.  For a vertex with fewer than
// R kept neighbours, each pruned candidate v gets t_v = the largest cosine, at
// u, between v and a candidate w closer to u (by (distance, id)); v survives an
// angle threshold theta iff t_v <= cos(theta).  The largest threshold leaving
// R - nk survivors has cos(theta*) = the (R - nk)-th smallest t_v (the limit of
// the paper's binary search); survivors are added in distance order.  Then
// fill[u] supplies neighbours while fewer than R are held (the paper's
// footnote: random neighbours when candidates are too few).  LDS: P pruned
// candidate indices, P t values, P sort slots.
__global__ __launch_bounds__(64) void refine_kernel(const float* __restrict__ X, int D, int R, int64_t N, int C, int P,
                                                    int do_refine, const int32_t* __restrict__ cid,
                                                    const int32_t* __restrict__ ncand, const int32_t* __restrict__ kidx,
                                                    const int32_t* __restrict__ nkept,
                                                    const int32_t* __restrict__ fill, int32_t* __restrict__ G) {
  extern __shared__ __align__(16) uint8_t sm[];
  double* tv = reinterpret_cast<double*>(sm);
  double* srt = tv + P;
  int32_t* pr = reinterpret_cast<int32_t*>(srt + P);
  int32_t* row = pr + P;  // R
  const int lane = lane_id();
  const int64_t u = blockIdx.x;
  if (u >= N) return;
  const int n = ncand[u];
  int nk = nkept[u];
  for (int j = lane; j < R; j += 64) row[j] = G[u * R + j];
  __syncthreads();
  const int need = R - nk;
  if (do_refine && need > 0) {
    // the pruned candidates, in distance order (every candidate was scanned: fewer than R were kept)
    int np = 0;
    for (int b = 0; b < n; b += 64) {
      const int i = b + lane;
      bool isk = false;
      for (int a = 0; a < nk; ++a) isk |= kidx[u * R + a] == i;
      const bool p = i < n && !isk;
      const uint64_t m = ballot(p);
      if (p) pr[np + lanes_below(m)] = i;
      np += __popcll(m);
    }
    __syncthreads();
    const float* xu = X + u * D;
    for (int a = lane; a < np; a += 64) {
      const int i = pr[a];
      const float* xv = X + (int64_t)cid[u * C + i] * D;
      double nv = 0.0;
      for (int t = 0; t < D; ++t) {
        const double du = (double)xv[t] - (double)xu[t];
        nv = nv + du * du;
      }
      double best = -2.0;
      for (int w = 0; w < i; ++w) {
        const float* xw = X + (int64_t)cid[u * C + w] * D;
        double nw = 0.0, dot = 0.0;
        for (int t = 0; t < D; t += 4) {
          const float4 w4 = *reinterpret_cast<const float4*>(xw + t);
          const float4 v4 = *reinterpret_cast<const float4*>(xv + t);
          const float4 u4 = *reinterpret_cast<const float4*>(xu + t);
          double dw = (double)w4.x - (double)u4.x, dv = (double)v4.x - (double)u4.x;
          nw = nw + dw * dw;
          dot = dot + dw * dv;
          dw = (double)w4.y - (double)u4.y;
          dv = (double)v4.y - (double)u4.y;
          nw = nw + dw * dw;
          dot = dot + dw * dv;
          dw = (double)w4.z - (double)u4.z;
          dv = (double)v4.z - (double)u4.z;
          nw = nw + dw * dw;
          dot = dot + dw * dv;
          dw = (double)w4.w - (double)u4.w;
          dv = (double)v4.w - (double)u4.w;
          nw = nw + dw * dw;
          dot = dot + dw * dv;
        }
        const double cs = (nv > 0.0 && nw > 0.0) ? dot / (__builtin_sqrt(nv) * __builtin_sqrt(nw)) : 1.0;
        if (cs > best) best = cs;
      }
      tv[a] = best;
    }
    __syncthreads();
    if (np > 0) {
      int Q = 1;
      while (Q < np) Q <<= 1;
      for (int a = lane; a < Q; a += 64) srt[a] = a < np ? tv[a] : __builtin_inf();
      __syncthreads();
      for (int k = 2; k <= Q; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
          for (int a = lane; a < Q; a += 64) {
            const int l = a ^ j;
            if (l > a) {
              const bool up = (a & k) == 0;
              const double x = srt[a], y = srt[l];
              if ((x > y) == up) {
                srt[a] = y;
                srt[l] = x;
              }
            }
          }
          __syncthreads();
        }
      const double cstar = srt[(need <= np ? need : np) - 1];
      for (int a = 0; a < np && nk < R; ++a)
        if (tv[a] <= cstar) {
          if (lane == 0) row[nk] = cid[u * C + pr[a]];
          ++nk;
        }
      __syncthreads();
    }
  }
  if (do_refine) {
    // too few candidates: random neighbours
    for (int f = 0; nk < R && f < R; ++f) {
      const int32_t v = fill[u * R + f];
      if (v < 0 || v == (int32_t)u) continue;
      bool dup = false;
      for (int a = lane; a < nk; a += 64) dup |= row[a] == v;
      if (ballot(dup)) continue;
      if (lane == 0) row[nk] = v;
      ++nk;
      __syncthreads();
    }
  }
  __syncthreads();
  for (int j = lane; j < R; j += 64) G[u * R + j] = row[j];
}

// Repair helper: rows of X listed in ids, gathered into out[n][D].
__global__ __launch_bounds__(256) void gather_kernel(const float* __restrict__ X, int D, const int32_t* __restrict__ ids,
                                                     int64_t n, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n * D) return;
  const int64_t r = i / D, c = i % D;
  out[i] = X[(int64_t)ids[r] * D + c];
}

// Repair helper: for each listed vertex w, the squared distances from x_w to
// its R neighbours (+inf for an empty slot).
__global__ __launch_bounds__(256) void rows_dist_kernel(const float* __restrict__ X, int D, int R,
                                                        const int32_t* __restrict__ ws, int64_t nw,
                                                        const int32_t* __restrict__ G, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nw * R) return;
  const int64_t w = ws[i / R];
  const int32_t v = G[w * R + i % R];
  out[i] = v >= 0 ? dist2_seq(X + w * D, X + (int64_t)v * D, D) : __builtin_inf();
}

int pow2_at_least(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

hipError_t launch_candidates(const float* X, int D, const int32_t* sids, int EF, const int32_t* G, int R, int64_t u0,
                             int64_t nu, int C, int32_t* cid, double* cd, int32_t* ncand, hipStream_t st) {
  const int P = pow2_at_least(C);
  const size_t lds = 12 * (size_t)P;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(candidates_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(candidates_kernel, dim3((unsigned)nu), dim3(64), lds, st, X, D, sids, EF, G, R, u0, C, P, cid,
                     cd, ncand);
  return hipGetLastError();
}

hipError_t launch_nsg(const float* X, int D, int R, int64_t N, int C, const int32_t* cid, const double* cd,
                      const int32_t* ncand, int32_t* Gout, int32_t* kidx, int32_t* nkept, hipStream_t st) {
  hipLaunchKernelGGL(nsg_kernel, dim3((unsigned)N), dim3(64), 4 * (size_t)R, st, X, D, R, N, C, cid, cd, ncand, Gout,
                     kidx, nkept);
  return hipGetLastError();
}

hipError_t launch_refine(const float* X, int D, int R, int64_t N, int C, int do_refine, const int32_t* cid,
                         const int32_t* ncand, const int32_t* kidx, const int32_t* nkept, const int32_t* fill,
                         int32_t* G, hipStream_t st) {
  const int P = pow2_at_least(C);
  const size_t lds = 20 * (size_t)P + 4 * (size_t)R;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(refine_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(refine_kernel, dim3((unsigned)N), dim3(64), lds, st, X, D, R, N, C, P, do_refine, cid, ncand, kidx,
                     nkept, fill, G);
  return hipGetLastError();
}

hipError_t launch_gather(const float* X, int D, const int32_t* ids, int64_t n, float* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((n * D + 255) / 256)), dim3(256), 0, st, X, D, ids, n, out);
  return hipGetLastError();
}

hipError_t launch_rows_dist(const float* X, int D, int R, const int32_t* ws, int64_t nw, const int32_t* G, double* out,
                            hipStream_t st) {
  if (nw <= 0) return hipSuccess;
  hipLaunchKernelGGL(rows_dist_kernel, dim3((unsigned)((nw * R + 255) / 256)), dim3(256), 0, st, X, D, R, ws, nw, G,
                     out);
  return hipGetLastError();
}

}  // namespace qgg
