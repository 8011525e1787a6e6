// Workspace partition for range queries against the obstacle boxes (the
// broad phase the paper suggests for cluttered maps, Sec. V-C).
//
// Along each axis the span of the boxes is cut into kBins equal bins, with
// bin(x) = clamp(floor((x - org) * scale), 0, kBins - 1), a non-decreasing
// function of x (each floating-point step is monotone).  Per axis and bin b
// two bit sets over the boxes are kept:
//   lo_le[b] = { o : bin(lo_o) <= b },   hi_ge[b] = { o : bin(hi_o) >= b }.
// A box that meets the interval [p, q] on an axis (lo_o <= q, hi_o >= p) has
// bin(lo_o) <= bin(q) and bin(hi_o) >= bin(p), so it is in
// lo_le[bin(q)] & hi_ge[bin(p)]; the AND over the three axes is a superset of
// the boxes a 3-D range meets, found with six shared-memory reads per word of
// the bit set.  The exact range test then runs over that superset only, so
// the boxes found are exactly those of a test over every box.
//
// One workgroup builds the table in LDS from the boxes it already holds
// there; a range that is not finite gets every box.
#pragma once

#include "device_math.hpp"
#include "pump_internal.hpp"

namespace pump {

constexpr int kBins = 64;

struct BoxBins {
    float org[3], scale[3];
    int n;                                               // boxes
    int nw;                                              // bit-set words in use
    unsigned long long lo_le[3][kBins][kMaxObsWords];
    unsigned long long hi_ge[3][kBins][kMaxObsWords];
};

__device__ __forceinline__ int box_bin(const BoxBins* s, int a, float x) {
    const float f = (x - s->org[a]) * s->scale[a];
    // fmaxf(NaN, 0) = 0; the clamp keeps the conversion in range
    return (int)fminf(fmaxf(f, 0.0f), (float)(kBins - 1));
}

// All threads of the workgroup call it; boxes b[o * 6 + (lo xyz, hi xyz)].
__device__ __forceinline__ void box_bins_build(const float* b, int n, BoxBins* s) {
    if (threadIdx.x < 3) {
        const int a = threadIdx.x;
        float lo = INFINITY, hi = -INFINITY;
        for (int o = 0; o < n; ++o) {
            lo = fminf(lo, b[o * 6 + a]);
            hi = fmaxf(hi, b[o * 6 + 3 + a]);
        }
        if (n > 0 && hi > lo) {
            s->org[a] = lo;
            s->scale[a] = (float)kBins / (hi - lo);
        } else {
            s->org[a] = 0.0f;   // every box in bin 0
            s->scale[a] = 0.0f;
        }
    }
    if (threadIdx.x == 0) {
        s->n = n;
        s->nw = (n + 63) / 64;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < 3 * kBins * kMaxObsWords; t += blockDim.x) {
        const int a = t / (kBins * kMaxObsWords);
        const int bn = (t / kMaxObsWords) % kBins;
        const int w = t % kMaxObsWords;
        unsigned long long le = 0ull, ge = 0ull;
        for (int k = 0; k < 64 && w * 64 + k < n; ++k) {
            const int o = w * 64 + k;
            if (box_bin(s, a, b[o * 6 + a]) <= bn) le |= 1ull << k;
            if (box_bin(s, a, b[o * 6 + 3 + a]) >= bn) ge |= 1ull << k;
        }
        s->lo_le[a][bn][w] = le;
        s->hi_ge[a][bn][w] = ge;
    }
    __syncthreads();
}

// Candidate boxes of the range [lo3, hi3]: bits o < s->n of cand[0 .. kMaxObsWords).
__device__ __forceinline__ void box_bins_query(const BoxBins* s, const float* lo3, const float* hi3,
                                               unsigned long long* cand) {
    const int n = s->n, nw = s->nw;
    bool finite = true;
    for (int a = 0; a < 3; ++a) finite &= isfinite(lo3[a]) && isfinite(hi3[a]);
    for (int w = 0; w < kMaxObsWords; ++w) {
        const int left = n - w * 64;   // boxes from this word on
        cand[w] = left >= 64 ? ~0ull : (left > 0 ? (1ull << left) - 1ull : 0ull);
    }
    if (!finite) return;
    for (int a = 0; a < 3; ++a) {
        const int b0 = box_bin(s, a, lo3[a]), b1 = box_bin(s, a, hi3[a]);
        for (int w = 0; w < nw; ++w) cand[w] &= s->lo_le[a][b1][w] & s->hi_ge[a][b0][w];
    }
}

}  // namespace pump
