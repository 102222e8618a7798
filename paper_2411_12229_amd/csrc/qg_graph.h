// qg_graph.h -- launch interface of the index-construction kernels (Algorithm 2).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qgg {

int pow2_at_least(int x);
// Sorted candidate lists (ids, fp64 squared distances) of vertices u0 .. u0+nu-1
// from their search results sids[nu][EF] and the current graph G[N][R].
hipError_t launch_candidates(const float* X, int D, const int32_t* sids, int EF, const int32_t* G, int R, int64_t u0,
                             int64_t nu, int C, int32_t* cid, double* cd, int32_t* ncand, hipStream_t st);
// NSG pruning of every vertex: Gout rows (-1 padded), kept candidate indices, kept counts.
hipError_t launch_nsg(const float* X, int D, int R, int64_t N, int C, const int32_t* cid, const double* cd,
                      const int32_t* ncand, int32_t* Gout, int32_t* kidx, int32_t* nkept, hipStream_t st);
// Refinement to R edges and random fill, in place on G (the NSG rows).
hipError_t launch_refine(const float* X, int D, int R, int64_t N, int C, int do_refine, const int32_t* cid,
                         const int32_t* ncand, const int32_t* kidx, const int32_t* nkept, const int32_t* fill,
                         int32_t* G, hipStream_t st);
// Rows ids[0..n) of X gathered into out[n][D].
hipError_t launch_gather(const float* X, int D, const int32_t* ids, int64_t n, float* out, hipStream_t st);
// For each w in ws[0..nw): squared distances from x_w to its R neighbours in G (+inf for -1), out[nw][R].
hipError_t launch_rows_dist(const float* X, int D, int R, const int32_t* ws, int64_t nw, const int32_t* G, double* out,
                            hipStream_t st);

}  // namespace qgg
