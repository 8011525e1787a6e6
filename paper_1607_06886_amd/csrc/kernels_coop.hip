// Explore (Alg. 4) of one query as a single launch: the whole grid is one
// team (explore_team.hpp), so every round runs inside the kernel with
// grid-wide barriers between its phases and no host round trip.
#include "explore_team.hpp"

namespace pump {

// Workgroup size: 512 threads, two waves per SIMD with one workgroup per CU
// (the launch bound holds every N to 256 VGPRs).  More waves per workgroup
// hide the latency of the wave-per-pair phases without adding workgroups to
// the grid barriers.
template <int N>
constexpr int coop_threads() { return 512; }

template <int N>
__global__ __launch_bounds__(coop_threads<N>()) void k_explore_coop(const RoundArgs* __restrict__ ra,
                                                                   CoopArgs ca) {
    __shared__ float s_raw[kMaxObs * 6];
    __shared__ float s_in[kMaxObs * 6];
    __shared__ float s_out[kMaxObs * 6];
    __shared__ int s_w[16];
    __shared__ unsigned long long s_m[16];
    __shared__ long long s_ll[16];
    __shared__ int s_fail;
    TeamCtx t;
    t.arrive = ca.sync.arrive;
    t.release = ca.sync.release;
    t.fail = ca.sync.fail;
    t.patience = ca.sync.patience;
    t.rank = blockIdx.x;
    t.size = gridDim.x;
    t.xa = ca.xa;
    t.xb = ca.xb;
    t.b_deg = ca.b_deg;
    t.open_cur = ca.open_cur;
    t.open_next = ca.open_next;
    t.cap_pairs = ca.cap_pairs;
    explore_team<N>(ra, t, false, 0, s_raw, s_in, s_out, s_w, s_m, s_ll, &s_fail);
}

namespace {
struct CoopFn {
    const void* fn;
    int threads;
};
CoopFn coop_fn(int N) {
    switch (N) {
        case 32: return {(const void*)k_explore_coop<32>, coop_threads<32>()};
        case 64: return {(const void*)k_explore_coop<64>, coop_threads<64>()};
        case 128: return {(const void*)k_explore_coop<128>, coop_threads<128>()};
        default: return {(const void*)k_explore_coop<256>, coop_threads<256>()};
    }
}
}  // namespace

hipError_t launch_explore_coop(hipStream_t s, const RoundArgs* ra_dev, const CoopArgs& ca, int N,
                               int blocks) {
    const RoundArgs* ra = ra_dev;
    void* args[2] = {(void*)&ra, (void*)&ca};
    const CoopFn f = coop_fn(N);
    // An ordinary launch: `blocks` never exceeds what the occupancy query
    // says fits on the device at once, so on an otherwise idle stream every
    // workgroup is resident and the barriers complete (a wait that runs out
    // of patience still ends the kernel with an error).
    return hipLaunchKernel(f.fn, dim3(blocks), dim3(f.threads), args, 0, s);
}

int coop_max_blocks(int N) {
    int per_cu = 0, dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return 0;
    const CoopFn f = coop_fn(N);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f.fn, f.threads, 0) != hipSuccess)
        return 0;
    return per_cu * prop.multiProcessorCount;
}

}  // namespace pump
