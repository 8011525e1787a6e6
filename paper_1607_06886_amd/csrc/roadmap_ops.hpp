// BuildGraph (Alg. 3) over a cached roadmap.  Near and the optimal
// connections depend only on the samples, not on the obstacles, so they are
// computed once per sample set (the paper caches neighbours and edge
// controls offline, Sec. V-A) together with each connection's nominal
// position range; a query then only runs the box stages of pass 1 on the
// cached connections, plus all stages for the pairs at its own x_init
// (node 0).  The per-connection decisions are the ones the scratch build
// takes (same cubic, same range, same box tests), so the graph is identical.
#pragma once

#include "device_math.hpp"
#include "pump_internal.hpp"
#include "setup_ops.hpp"

namespace pump {

// Nominal position range of roadmap connection e (the cubic's extremes).
__device__ __forceinline__ void rm_bbox_dev(const float* __restrict__ X, const int32_t* __restrict__ esrc,
                                            const int32_t* __restrict__ col,
                                            const double* __restrict__ tau, double* __restrict__ bbox,
                                            int E) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < E; e += gridDim.x * blockDim.x) {
        Cubic cs[3];
        hermite(X + (size_t)esrc[e] * 6, X + (size_t)col[e] * 6, tau[e], cs);
        for (int a = 0; a < 3; ++a) cubic_range(cs[a], tau[e], bbox[(size_t)e * 6 + a],
                                                bbox[(size_t)e * 6 + 3 + a]);
    }
}

// Samples of the query (nodes 1..n of X) equal to the roadmap's?  Sets
// `bit` in *bad otherwise.
__device__ __forceinline__ void rm_check_dev(const float* __restrict__ X, const float* __restrict__ Xr,
                                             int n_nodes, int32_t* __restrict__ bad, int bit) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 6 || t >= n_nodes * 6) return;
    if (__float_as_uint(X[t]) != __float_as_uint(Xr[t])) atomicOr(bad, bit);
}

// tau* and c* of each final edge: cached for sample-to-sample edges (binary
// search of the roadmap row), computed for edges at node 0.
__device__ __forceinline__ void rm_fill_dev(const float* __restrict__ X, int n_nodes, double r_steer,
                                            const int32_t* __restrict__ row_ptr,
                                            const int32_t* __restrict__ col,
                                            const int32_t* __restrict__ esrc, const RoadmapDev& rm,
                                            double* __restrict__ etau, double* __restrict__ ecost) {
    const int E = row_ptr[n_nodes];
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < E; e += gridDim.x * blockDim.x) {
        const int src = esrc[e], dst = col[e];
        if (src == 0 || dst == 0) {
            double tau, c;
            steer64(X + (size_t)src * 6, X + (size_t)dst * 6, r_steer, tau, c);
            etau[e] = tau;
            ecost[e] = c;
            continue;
        }
        int lo = rm.row_ptr[src], hi = rm.row_ptr[src + 1];   // col sorted within a row
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (rm.col[mid] < dst) lo = mid + 1; else hi = mid;
        }
        etau[e] = rm.tau[lo];
        ecost[e] = rm.cost[lo];
    }
}

}  // namespace pump
