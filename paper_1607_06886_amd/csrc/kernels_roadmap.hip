// BuildGraph (Alg. 3) over a cached roadmap: kernels and launchers.  The
// bodies live in roadmap_ops.hpp.
#include "roadmap_ops.hpp"

namespace pump {

__global__ __launch_bounds__(256) void k_rm_bbox(const float* __restrict__ X,
                                                 const int32_t* __restrict__ esrc,
                                                 const int32_t* __restrict__ col,
                                                 const double* __restrict__ tau,
                                                 double* __restrict__ bbox, int E) {
    rm_bbox_dev(X, esrc, col, tau, bbox, E);
}

__global__ __launch_bounds__(256) void k_rm_check(const float* __restrict__ X,
                                                  const float* __restrict__ Xr, int n_nodes,
                                                  int32_t* __restrict__ bad) {
    rm_check_dev(X, Xr, n_nodes, bad, 4);
}

__global__ __launch_bounds__(256) void k_rm_fill(const float* __restrict__ X, int n_nodes,
                                                 double r_steer,
                                                 const int32_t* __restrict__ row_ptr,
                                                 const int32_t* __restrict__ col,
                                                 const int32_t* __restrict__ esrc, RoadmapDev rm,
                                                 double* __restrict__ etau,
                                                 double* __restrict__ ecost) {
    rm_fill_dev(X, n_nodes, r_steer, row_ptr, col, esrc, rm, etau, ecost);
}

namespace {
int grid_for(long long items) {
    long long b = (items + 255) / 256;
    if (b < 1) b = 1;
    if (b > 8192) b = 8192;
    return (int)b;
}
}  // namespace

void launch_rm_bbox(hipStream_t s, const float* X, const int32_t* esrc, const int32_t* col,
                    const double* tau, double* bbox, int E) {
    k_rm_bbox<<<grid_for(E), 256, 0, s>>>(X, esrc, col, tau, bbox, E);
}

void launch_rm_query(hipStream_t s, const float* X, const uint8_t* valid, int n_nodes,
                     const float* obs, int n_obs, double r_steer, double r_conn,
                     const RoadmapDev& rm, uint32_t* ebits, int words, int32_t* deg, int32_t* bad,
                     const GraphWork& gw) {
    k_rm_check<<<(n_nodes * 6 + 255) / 256, 256, 0, s>>>(X, rm.X, n_nodes, bad);
    launch_graph_pass1_roadmap(s, X, valid, n_nodes, obs, n_obs, r_steer, r_conn, rm.esrc, rm.col,
                               rm.tau, rm.bbox, rm.n_edges, ebits, deg, words, gw);
}

void launch_rm_fill(hipStream_t s, const float* X, int n_nodes, double r_steer,
                    const int32_t* row_ptr, const int32_t* col, const int32_t* esrc,
                    const RoadmapDev& rm, double* etau, double* ecost, int n_edges) {
    k_rm_fill<<<grid_for(n_edges), 256, 0, s>>>(X, n_nodes, r_steer, row_ptr, col, esrc, rm, etau,
                                                ecost);
}

}  // namespace pump
