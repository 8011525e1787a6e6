// Per-query setup kernels: the particle deviation table and BuildGraph (Alg. 3).
// The bodies live in setup_ops.hpp.
#include "setup_ops.hpp"

namespace pump {

__global__ void k_dev_local(const float* __restrict__ noise, double* __restrict__ E, int N, int S,
                            DevCoef m) {
    dev_local_dev(noise, E, N, S, m);
}

__global__ void k_dev_carry(const double* __restrict__ E, double* __restrict__ X0, int N, int S,
                            DevCoef m) {
    dev_carry_dev(E, X0, N, S, m);
}

__global__ void k_dev_final(const float* __restrict__ noise, const double* __restrict__ X0,
                            float* __restrict__ D, int N, int S, DevCoef m) {
    dev_final_dev(noise, X0, D, N, S, m);
}

__global__ void k_lqg_local(const float* __restrict__ noise, const float* __restrict__ meas,
                            double* __restrict__ E, int N, int S, LqgCoef q) {
    lqg_local_dev(noise, meas, E, N, S, q);
}

__global__ void k_lqg_carry(const double* __restrict__ E, double* __restrict__ X0, int N, int S,
                            LqgCoef q) {
    lqg_carry_dev(E, X0, N, S, q);
}

__global__ void k_lqg_final(const float* __restrict__ noise, const float* __restrict__ meas,
                            const double* __restrict__ X0, float* __restrict__ D, int N, int S,
                            LqgCoef q) {
    lqg_final_dev(noise, meas, X0, D, N, S, q);
}

__global__ void k_cloud(const float* __restrict__ D, float* __restrict__ cloud, int N) {
    cloud_dev(D, cloud, N);
}

__global__ void k_gcloud(const float* __restrict__ cloud, float* __restrict__ g, int S1) {
    gcloud_dev(cloud, g, S1);
}

void launch_deviation_table(hipStream_t s, const float* noise, float* D, float* cloud,
                            float* gcloud, int N, int S_max, const double* Acl, const double* L,
                            double* scratch) {
    const DevCoef m{Acl[0], Acl[1], Acl[2], Acl[3], L[0], L[2], L[3]};
    const int K = (S_max + kDevChunk - 1) / kDevChunk;
    double* E = scratch;
    double* X0 = scratch + (size_t)2 * K * 3 * N;
    const int threads = K * 3 * N;
    k_dev_local<<<(threads + 255) / 256, 256, 0, s>>>(noise, E, N, S_max, m);
    k_dev_carry<<<(3 * N + 63) / 64, 64, 0, s>>>(E, X0, N, S_max, m);
    k_dev_final<<<(threads + 255) / 256, 256, 0, s>>>(noise, X0, D, N, S_max, m);
    k_cloud<<<S_max + 1, 256, 0, s>>>(D, cloud, N);
    k_gcloud<<<1, 256, 0, s>>>(cloud, gcloud, S_max + 1);
}

void launch_deviation_table_lqg(hipStream_t s, const float* noise, const float* noise_meas,
                                float* D, float* cloud, float* gcloud, int N, int S_max,
                                const LqgCoef& q, double* scratch) {
    const int K = (S_max + kDevChunk - 1) / kDevChunk;
    double* E = scratch;
    double* X0 = scratch + (size_t)4 * K * 3 * N;
    const int threads = K * 3 * N;
    k_lqg_local<<<(threads + 255) / 256, 256, 0, s>>>(noise, noise_meas, E, N, S_max, q);
    k_lqg_carry<<<(3 * N + 63) / 64, 64, 0, s>>>(E, X0, N, S_max, q);
    k_lqg_final<<<(threads + 255) / 256, 256, 0, s>>>(noise, noise_meas, X0, D, N, S_max, q);
    k_cloud<<<S_max + 1, 256, 0, s>>>(D, cloud, N);
    k_gcloud<<<1, 256, 0, s>>>(cloud, gcloud, S_max + 1);
}

__global__ void k_mark_valid(const float* __restrict__ X, int n, const float* __restrict__ obs,
                             int n_obs, float g0, float g1, float g2, float g3, float g4, float g5,
                             uint8_t* __restrict__ valid, uint8_t* __restrict__ goal,
                             int32_t* __restrict__ bad) {
    mark_valid_dev(X, n, obs, n_obs, g0, g1, g2, g3, g4, g5, valid, goal, bad);
}

void launch_mark_valid(hipStream_t s, const float* X, int n_nodes, const float* obs, int n_obs,
                       const float* gb, uint8_t* valid, uint8_t* goal, int32_t* bad) {
    int n = n_nodes > n_obs ? n_nodes : n_obs;
    k_mark_valid<<<(n + 255) / 256, 256, 0, s>>>(X, n_nodes, obs, n_obs, gb[0], gb[1], gb[2],
                                                 gb[3], gb[4], gb[5], valid, goal, bad);
}

// ---- BuildGraph pass 1 stages (setup_ops.hpp) ----
__global__ __launch_bounds__(kNearThreads) void k_gw_near_rows(const float* __restrict__ X,
                                                      const uint8_t* __restrict__ valid, int n,
                                                      int row0, double r_steer, double r_conn,
                                                      GraphWork gw) {
    __shared__ int s_list[2 * kNearChunk];
    __shared__ int s_cnt[3 + 17];
    gw_near_row(X, valid, n, row0 + blockIdx.x, r_steer, r_conn, gw, s_list, s_cnt);
}

__global__ __launch_bounds__(256) void k_gw_near_col0(const float* __restrict__ X,
                                                      const uint8_t* __restrict__ valid, int n,
                                                      double r_steer, double r_conn,
                                                      GraphWork gw) {
    gw_near_col0(X, valid, n, blockIdx.x * blockDim.x + threadIdx.x, r_steer, r_conn, gw);
}

// boxes over the near list (count on the device) or a cached list (count given)
// (three waves per SIMD: the compiler spills about 40 VGPRs there, which
// measured faster than two waves without spills -- indoor query, pass 1
// 7.36 -> 6.96 ms -- and than four waves with more spills)
__global__ __launch_bounds__(kBoxThreads, 3) void k_gw_boxes(const float* __restrict__ X,
                                                          const uint8_t* __restrict__ valid,
                                                          const int32_t* __restrict__ src,
                                                          const int32_t* __restrict__ dst,
                                                          const double* __restrict__ tau,
                                                          const double* __restrict__ bbox,
                                                          int count, int near_list,
                                                          const float* __restrict__ obs,
                                                          int n_obs, GraphWork gw,
                                                          uint32_t* __restrict__ ebits,
                                                          int words) {
    __shared__ float s_obs[kMaxObs * 6];
    __shared__ uint32_t s_q[kBoxThreads / 64 * kBoxQueue];
    __shared__ int s_src[kBoxThreads], s_dst[kBoxThreads], s_blk[kBoxThreads];
    __shared__ double s_tau[kBoxThreads];
    __shared__ BoxBins s_bins;
    for (int t = threadIdx.x; t < n_obs * 6; t += blockDim.x) s_obs[t] = obs[t];
    __syncthreads();
    box_bins_build(s_obs, n_obs, &s_bins);
    const int N = near_list ? min(gw.counts[0], gw.near_cap) : count;
    gw_boxes(X, valid, src, dst, tau, bbox, N, near_list != 0, near_list == 0, s_obs, n_obs, &s_bins, gw,
             ebits, words, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x, s_q,
             s_src, s_dst, s_tau, s_blk);
}

__global__ __launch_bounds__(256) void k_gw_exact(const float* __restrict__ X,
                                                  const float* __restrict__ obs, GraphWork gw,
                                                  const int32_t* __restrict__ rm_src,
                                                  const int32_t* __restrict__ rm_dst,
                                                  const double* __restrict__ rm_tau,
                                                  uint32_t* __restrict__ ebits, int words) {
    gw_exact(X, obs, gw, rm_src, rm_dst, rm_tau, ebits, words, blockIdx.x * blockDim.x + threadIdx.x,
             gridDim.x * blockDim.x);
}

__global__ __launch_bounds__(256) void k_row_deg(const uint32_t* __restrict__ ebits, int n_nodes,
                                                 int words, int32_t* __restrict__ deg) {
    row_deg_dev(ebits, n_nodes, words, deg, blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
}

__global__ __launch_bounds__(256) void k_graph_fill(int n, const uint32_t* __restrict__ ebits,
                                                    const int32_t* __restrict__ row_ptr,
                                                    int32_t* __restrict__ col,
                                                    int32_t* __restrict__ esrc, int words) {
    graph_fill_dev(n, ebits, row_ptr, col, esrc, words);
}

__global__ __launch_bounds__(256) void k_edge_steer(const float* __restrict__ X, int n,
                                                    double r_steer,
                                                    const int32_t* __restrict__ row_ptr,
                                                    const int32_t* __restrict__ col,
                                                    const int32_t* __restrict__ esrc,
                                                    double* __restrict__ etau,
                                                    double* __restrict__ ecost) {
    edge_steer_dev(X, n, r_steer, row_ptr, col, esrc, etau, ecost);
}

__global__ __launch_bounds__(256) void k_word_start(int n, const uint32_t* __restrict__ ebits,
                                                    const int32_t* __restrict__ row_ptr,
                                                    int32_t* __restrict__ wstart, int words) {
    word_start_dev(n, ebits, row_ptr, wstart, words);
}

__global__ __launch_bounds__(256) void k_near_to_slot(GraphWork gw, const uint32_t* __restrict__ ebits,
                                                      const int32_t* __restrict__ wstart, int words,
                                                      double* __restrict__ slot_tau) {
    near_to_slot_dev(gw, ebits, wstart, words, slot_tau);
}

__global__ __launch_bounds__(256) void k_edge_cost(const float* __restrict__ X, int n, double r_steer,
                                                   const int32_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col,
                                                   const int32_t* __restrict__ esrc,
                                                   double* __restrict__ etau, double* __restrict__ ecost) {
    edge_cost_dev(X, n, r_steer, row_ptr, col, esrc, etau, ecost);
}

namespace {
constexpr int kStageBlocks = 2048;   // grid of the grid-stride stages
}

void launch_graph_mark(hipStream_t s, const float* X, const uint8_t* valid, int n_nodes,
                       const float* obs, int n_obs, double r_steer, double r_conn,
                       uint32_t* ebits, int32_t* deg, int words, const GraphWork& gw) {
    (void)hipMemsetAsync(ebits, 0, (size_t)n_nodes * words * sizeof(uint32_t), s);
    k_gw_near_rows<<<n_nodes, kNearThreads, 0, s>>>(X, valid, n_nodes, 0, r_steer, r_conn, gw);
    k_gw_boxes<<<kStageBlocks, kBoxThreads, 0, s>>>(X, valid, gw.near_src, gw.near_dst, gw.near_tau,
                                            nullptr, 0, 1, obs, n_obs, gw, ebits, words);
    k_gw_exact<<<kStageBlocks, 256, 0, s>>>(X, obs, gw, nullptr, nullptr, nullptr, ebits, words);
    k_row_deg<<<(n_nodes + 3) / 4, 256, 0, s>>>(ebits, n_nodes, words, deg);
}

void launch_graph_pass1_roadmap(hipStream_t s, const float* X, const uint8_t* valid, int n_nodes,
                                const float* obs, int n_obs, double r_steer, double r_conn,
                                const int32_t* rm_src, const int32_t* rm_dst,
                                const double* rm_tau, const double* rm_bbox, int rm_edges,
                                uint32_t* ebits, int32_t* deg, int words, const GraphWork& gw) {
    (void)hipMemsetAsync(ebits, 0, (size_t)n_nodes * words * sizeof(uint32_t), s);
    // the pairs at node 0: its row, then its column
    k_gw_near_rows<<<1, kNearThreads, 0, s>>>(X, valid, n_nodes, 0, r_steer, r_conn, gw);
    const int col = n_nodes - 1;
    k_gw_near_col0<<<(col + 255) / 256 > 0 ? (col + 255) / 256 : 1, 256, 0, s>>>(
        X, valid, n_nodes, r_steer, r_conn, gw);
    k_gw_boxes<<<64, kBoxThreads, 0, s>>>(X, valid, gw.near_src, gw.near_dst, gw.near_tau, nullptr, 0, 1, obs,
                                  n_obs, gw, ebits, words);
    int blocks = (rm_edges + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > kStageBlocks) blocks = kStageBlocks;
    k_gw_boxes<<<blocks, kBoxThreads, 0, s>>>(X, valid, rm_src, rm_dst, rm_tau, rm_bbox, rm_edges, 0, obs,
                                      n_obs, gw, ebits, words);
    k_gw_exact<<<kStageBlocks, 256, 0, s>>>(X, obs, gw, rm_src, rm_dst, rm_tau, ebits, words);
    k_row_deg<<<(n_nodes + 3) / 4, 256, 0, s>>>(ebits, n_nodes, words, deg);
}

void launch_graph_cols(hipStream_t s, int n_nodes, const uint32_t* ebits, const int32_t* row_ptr,
                       int32_t* col, int32_t* esrc, int words) {
    k_graph_fill<<<(n_nodes + 3) / 4, 256, 0, s>>>(n_nodes, ebits, row_ptr, col, esrc, words);
}

void launch_graph_fill_near(hipStream_t s, const float* X, int n_nodes, double r_steer,
                            const uint32_t* ebits, const int32_t* row_ptr, int32_t* col,
                            int32_t* esrc, double* etau, double* ecost, int32_t* wstart, int words,
                            int n_edges, const GraphWork& gw) {
    // the near list lives in esrc / col / etau: its tau* go to their slots
    // (in ecost) before the CSR fill overwrites it
    k_word_start<<<(n_nodes + 3) / 4, 256, 0, s>>>(n_nodes, ebits, row_ptr, wstart, words);
    k_near_to_slot<<<kStageBlocks, 256, 0, s>>>(gw, ebits, wstart, words, ecost);
    k_graph_fill<<<(n_nodes + 3) / 4, 256, 0, s>>>(n_nodes, ebits, row_ptr, col, esrc, words);
    int blocks = (n_edges + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 8192) blocks = 8192;
    k_edge_cost<<<blocks, 256, 0, s>>>(X, n_nodes, r_steer, row_ptr, col, esrc, etau, ecost);
}

void launch_graph_fill(hipStream_t s, const float* X, int n_nodes, double r_steer,
                       const uint32_t* ebits, const int32_t* row_ptr, int32_t* col,
                       int32_t* esrc, double* etau, double* ecost, int words, int n_edges) {
    k_graph_fill<<<(n_nodes + 3) / 4, 256, 0, s>>>(n_nodes, ebits, row_ptr, col, esrc, words);
    int blocks = (n_edges + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 8192) blocks = 8192;
    k_edge_steer<<<blocks, 256, 0, s>>>(X, n_nodes, r_steer, row_ptr, col, esrc, etau, ecost);
}

}  // namespace pump
