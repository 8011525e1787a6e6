// C ABI of the cached roadmap: BuildGraph's obstacle-independent part
// (Near and the optimal connections over a fixed sample set), built once
// with the graph kernels of kernels_setup.hip and no obstacles, plus each
// connection's nominal position range (kernels_roadmap.hip).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "pump_internal.hpp"

using namespace pump;

namespace {

template <class T>
hipError_t ralloc(T** p, size_t n) {
    if (n == 0) n = 1;
    return hipMalloc((void**)p, n * sizeof(T));
}

void free_all(pump_roadmap* rm) {
    void* ptrs[] = {rm->X, rm->row_ptr, rm->col, rm->esrc, rm->tau, rm->cost, rm->bbox};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
}

// Temporaries of the build.
struct Temp {
    uint8_t *valid = nullptr, *goal = nullptr;
    uint32_t* ebits = nullptr;
    int32_t *deg = nullptr, *ints = nullptr, *blk = nullptr;
    int32_t *w_ns = nullptr, *w_nd = nullptr, *w_xe = nullptr, *w_xb = nullptr;
    double* w_nt = nullptr;
    ~Temp() {
        void* ptrs[] = {valid, goal, ebits, deg, ints, blk, w_ns, w_nd, w_xe, w_xb, w_nt};
        for (void* p : ptrs)
            if (p) (void)hipFree(p);
    }
};

}  // namespace

int pump_roadmap_create(const pump_config* cfg, const float* samples, int32_t n, int32_t mem,
                        void* hip_stream, pump_roadmap** out) {
    if (!out) return PUMP_E_ARG;
    *out = nullptr;
    if (!cfg || !samples || n < 1 || n + 1 > cfg->max_nodes || cfg->max_nodes > 65535)
        return PUMP_E_ARG;
    if (mem != PUMP_MEM_HOST && mem != PUMP_MEM_DEVICE) return PUMP_E_ARG;
    if (!(cfg->r_steer > 0) || !(cfg->r_conn > 0)) return PUMP_E_ARG;
    if (cfg->cap_pairs < 1 || cfg->cap_pairs > (1ll << 26) || cfg->cap_edges < 1) return PUMP_E_ARG;
    hipStream_t s = (hipStream_t)hip_stream;
    const int nn = n + 1;
    const int words = ((nn + 63) / 64) * 2;
    pump_roadmap* rm = new pump_roadmap();
    rm->n = n;
    rm->r_steer = cfg->r_steer;
    rm->r_conn = cfg->r_conn;
    Temp t;
    bool ok = true;
    auto A = [&](hipError_t e) { ok = ok && (e == hipSuccess); };
    A(ralloc(&rm->X, (size_t)nn * 6));
    A(ralloc(&rm->row_ptr, (size_t)nn + 1));
    A(ralloc(&t.valid, nn));
    A(ralloc(&t.goal, nn));
    A(ralloc(&t.ebits, (size_t)nn * words));
    A(ralloc(&t.deg, (size_t)nn + 1));
    A(ralloc(&t.ints, 8));
    A(ralloc(&t.blk, (size_t)2 * 65536));
    const size_t ncap = (size_t)std::min<int64_t>(cfg->cap_edges, (1ll << 31) - 1);
    A(ralloc(&t.w_ns, ncap)); A(ralloc(&t.w_nd, ncap)); A(ralloc(&t.w_nt, ncap));
    A(ralloc(&t.w_xe, 1)); A(ralloc(&t.w_xb, 1));   // no boxes: the exact queue stays empty
    hipEvent_t e0 = nullptr, e1 = nullptr;
    A(hipEventCreate(&e0));
    A(hipEventCreate(&e1));
    auto bail = [&](int code) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipStreamSynchronize(s);
        free_all(rm);
        delete rm;
        return code;
    };
    if (!ok) return bail(PUMP_E_HIP);
    const hipMemcpyKind kind = mem == PUMP_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    const float zeros[6] = {0, 0, 0, 0, 0, 0};
    int32_t ints_h[8] = {nn, 0, 0, 0, 0, 0, 0, 0};
    A(hipEventRecord(e0, s));
    A(hipMemcpyAsync(rm->X, zeros, 6 * sizeof(float), hipMemcpyHostToDevice, s));
    A(hipMemcpyAsync(rm->X + 6, samples, (size_t)n * 6 * sizeof(float), kind, s));
    A(hipMemcpyAsync(t.ints, ints_h, sizeof(ints_h), hipMemcpyHostToDevice, s));
    // every sample valid (no obstacles; bit 1 of ints[1] flags a bad sample),
    // the placeholder node 0 excluded
    launch_mark_valid(s, rm->X, nn, nullptr, 0, zeros, t.valid, t.goal, t.ints + 1);
    A(hipMemsetAsync(t.valid, 0, 1, s));
    A(hipMemsetAsync(t.deg, 0, ((size_t)nn + 1) * sizeof(int32_t), s));
    const GraphWork gw{t.w_ns, t.w_nd, t.w_nt, t.w_xe, t.w_xb, t.ints + 4, (int32_t)ncap, 1};
    launch_graph_mark(s, rm->X, t.valid, nn, nullptr, 0, (double)cfg->r_steer, (double)cfg->r_conn,
                      t.ebits, t.deg, words, gw);
    scan_exclusive(s, t.deg, rm->row_ptr, t.ints, nn, t.ints + 2, t.blk);
    A(hipMemcpyAsync(ints_h, t.ints, sizeof(ints_h), hipMemcpyDeviceToHost, s));
    A(hipStreamSynchronize(s));
    A(hipGetLastError());
    if (!ok) return bail(PUMP_E_HIP);
    if (ints_h[1] & 1) return bail(PUMP_E_ARG);
    if ((size_t)ints_h[4] > ncap) return bail(PUMP_E_CAPACITY);
    const int32_t E = ints_h[2];
    if ((long long)E > cfg->cap_edges) return bail(PUMP_E_CAPACITY);
    A(hipMemcpyAsync(rm->row_ptr + nn, &E, sizeof(int32_t), hipMemcpyHostToDevice, s));
    A(ralloc(&rm->col, (size_t)E));
    A(ralloc(&rm->esrc, (size_t)E));
    A(ralloc(&rm->tau, (size_t)E));
    A(ralloc(&rm->cost, (size_t)E));
    A(ralloc(&rm->bbox, (size_t)E * 6));
    if (!ok) return bail(PUMP_E_HIP);
    launch_graph_fill(s, rm->X, nn, (double)cfg->r_steer, t.ebits, rm->row_ptr, rm->col, rm->esrc,
                      rm->tau, rm->cost, words, E);
    launch_rm_bbox(s, rm->X, rm->esrc, rm->col, rm->tau, rm->bbox, E);
    A(hipEventRecord(e1, s));
    A(hipEventSynchronize(e1));
    A(hipGetLastError());
    if (!ok) return bail(PUMP_E_HIP);
    (void)hipEventElapsedTime(&rm->ms_build, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    rm->d = RoadmapDev{rm->X, rm->row_ptr, rm->col, rm->esrc, rm->tau, rm->cost, rm->bbox, nn, E};
    *out = rm;
    return PUMP_OK;
}

int pump_roadmap_destroy(pump_roadmap* rm) {
    if (!rm) return PUMP_OK;
    (void)hipDeviceSynchronize();
    free_all(rm);
    delete rm;
    return PUMP_OK;
}

int pump_roadmap_info(const pump_roadmap* rm, int32_t* n, int64_t* n_edges, float* ms_build) {
    if (!rm) return PUMP_E_ARG;
    if (n) *n = rm->n;
    if (n_edges) *n_edges = rm->d.n_edges;
    if (ms_build) *ms_build = rm->ms_build;
    return PUMP_OK;
}
