// FP64 device math of the double-integrator connection (Sec. II cost c,
// Sec. IV Cost / Collision primitives).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace pump {

constexpr int kMaxObsWords = 4;   // 64-bit words of a box bit set (256 boxes)

// Boundary sums of a connection x0 -> x1:
//   S_PP = sum P_a^2, S_Pv = sum P_a (v0_a + v1_a), S_vv = sum v0^2 + v0 v1 + v1^2
// with P = p1 - p0.  The minimum-effort cost of duration tau is
//   c(tau) = tau + r (12 S_PP / tau^3 - 12 S_Pv / tau^2 + 4 S_vv / tau).
struct BSums {
    double pp, pv, vv;
};

// boundary_sums and cost_of round every operation on its own (no fused
// multiply-adds), so that each kernel that inlines them -- the near stage's
// steering, the edge costs of pass 2, the batched engine's -- gets the same
// bits from the same inputs.
__device__ __forceinline__ BSums boundary_sums(const float* x0, const float* x1) {
#pragma clang fp contract(off)
    BSums s{0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double P = (double)x1[a] - (double)x0[a];
        double v0 = (double)x0[3 + a];
        double v1 = (double)x1[3 + a];
        s.pp += P * P;
        s.pv += P * (v0 + v1);
        s.vv += v0 * v0 + v0 * v1 + v1 * v1;
    }
    return s;
}

__device__ __forceinline__ double cost_of(double t, const BSums& s, double r) {
#pragma clang fp contract(off)
    const double it = 1.0 / t;
    return t + r * (it * (it * (12.0 * s.pp * it - 12.0 * s.pv) + 4.0 * s.vv));
}

// a / b for a Newton or Halley step: the hardware reciprocal refined by one
// Newton step (relative error far below what the step needs; the iteration's
// fixed point, where the numerator vanishes, does not depend on it).
__device__ __forceinline__ double step_div(double a, double b) {
    double r = __builtin_amdgcn_rcp(b);
    r = fma(fma(-b, r, 1.0), r, r);
    return a * r;
}

// An upper bound of the cube root of x >= 0 (for root bounds, where any
// larger value also bounds): an FP32 estimate raised by 0.1 %, far above its
// error; below 1e-30 the bound 1e-10, above 1e30 the FP64 cube root.
__device__ __forceinline__ double cbrt_upper(double x) {
    if (!(x >= 1e-30)) return 1e-10;
    if (x > 1e30) return cbrt(x);
    return (double)exp2f(log2f((float)x) * (1.0f / 3.0f)) * 1.001;
}

// Stationarity of c: f(t) = t^4 + a2 t^2 + a1 t + a0 with a2 = -4 r S_vv <= 0,
// a1 = 24 r S_Pv, a0 = -36 r S_PP <= 0; f' = 4 t^3 + 2 a2 t + a1, f'' = 12 t^2 + 2 a2.
struct Quartic {
    double a2, a1, a0;
    __device__ double f(double t) const { return ((t * t + a2) * t + a1) * t + a0; }
    __device__ double g(double t) const { return (4.0 * t * t + 2.0 * a2) * t + a1; }
    __device__ double gp(double t) const { return 12.0 * t * t + 2.0 * a2; }
};

// Root of a function monotone on [lo, hi] whose values at the ends have
// opposite signs: Halley steps (cubic convergence) from the end where
// h * h'' > 0, kept inside the shrinking bracket (bisection when a step
// leaves it); stops once a step moves t by at most 4 ulp.  `which` selects f
// (0) or f' (1) of the quartic.
__device__ __forceinline__ double bracket_root(const Quartic& q, int which, double lo, double hi) {
    auto h0 = [&](double t) { return which ? q.g(t) : q.f(t); };
    auto h1 = [&](double t) { return which ? q.gp(t) : q.g(t); };
    auto h2 = [&](double t) { return which ? 24.0 * t : q.gp(t); };
    double flo = h0(lo);
    double fhi = h0(hi);
    if (flo == 0.0) return lo;
    if (fhi == 0.0) return hi;
    if ((flo < 0.0) == (fhi < 0.0)) return fabs(flo) < fabs(fhi) ? lo : hi;
    const bool rising = flo < 0.0;
    double t = flo * h2(lo) > 0.0 ? lo : (fhi * h2(hi) > 0.0 ? hi : 0.5 * (lo + hi));
    for (int it = 0; it < 200; ++it) {
        const double v = h0(t);
        if (v == 0.0) return t;
        if ((v < 0.0) == rising) lo = t; else hi = t;
        const double d = h1(t);
        const double tn = t - step_div(2.0 * v * d, 2.0 * d * d - v * h2(t));
        if (fabs(tn - t) <= 4.0 * 2.220446049250313e-16 * fabs(t)) return tn;
        const double tb = (tn > lo && tn < hi) ? tn : 0.5 * (lo + hi);
        if (tb == t || !(hi > lo)) break;
        // stop once the bracket is down to a few ulps
        if (hi - lo <= 4.0 * 2.220446049250313e-16 * hi) { t = tb; break; }
        t = tb;
    }
    return t;
}

// Which branch steer64 takes for these boundary sums: true when f' >= 0 at its
// inflection point ti, so f has one upward crossing and one root solve
// settles it; false for the branch with up to four root solves.  (The same
// arithmetic as steer64, so the two always agree.)
__device__ __forceinline__ bool steer_one_root(const BSums& s, double r) {
    if (s.pp == 0.0 && s.vv == 0.0) return true;
    const Quartic q{-4.0 * r * s.vv, 24.0 * r * s.pv, -36.0 * r * s.pp};
    const double ti = sqrt(-q.a2 * (1.0 / 6.0));
    return q.g(ti) >= 0.0;
}

// Optimal duration and cost of the connection x0 -> x1 (FP64).  The global
// minimiser of c over tau > 0 is one of the upward zero crossings of f
// (local minima of c).  f is concave on (0, ti) and convex on (ti, inf) with
// ti = sqrt(-a2/6), so f' has at most one zero t1 on (0, ti) (only when
// f'(0) = a1 > 0) and one zero t2 on (ti, inf); the upward crossings lie in
// (0, t1) and (t2, inf).  Identical states give tau = cost = 0.
__device__ __forceinline__ void steer64(const float* x0, const float* x1, double r,
                                        double& tau, double& cost) {
    BSums s = boundary_sums(x0, x1);
    if (s.pp == 0.0 && s.vv == 0.0) { tau = 0.0; cost = 0.0; return; }
    Quartic q{-4.0 * r * s.vv, 24.0 * r * s.pv, -36.0 * r * s.pp};
    // Fujiwara bound on the roots of f and of f'/4
    // (cube roots raised to an upper bound: the bounds only need to bound)
    double Bf = 2.0 * fmax(fmax(sqrt(fabs(q.a2)), cbrt_upper(fabs(q.a1))), sqrt(sqrt(0.5 * fabs(q.a0))));
    double Bg = 2.0 * fmax(sqrt(0.5 * fabs(q.a2)), cbrt_upper(0.25 * fabs(q.a1)));
    double ti = sqrt(-q.a2 * (1.0 / 6.0));
    double cand[2];
    int nc = 0;
    if (q.g(ti) >= 0.0) {
        cand[nc++] = bracket_root(q, 0, 0.0, Bf);
    } else {
        double t2 = bracket_root(q, 1, ti, fmax(Bg, ti));
        if (q.f(t2) < 0.0) cand[nc++] = bracket_root(q, 0, t2, fmax(Bf, t2));
        if (q.a1 > 0.0) {
            double t1 = bracket_root(q, 1, 0.0, ti);
            if (q.f(t1) > 0.0) cand[nc++] = bracket_root(q, 0, 0.0, t1);
        }
    }
    double bt = 0.0, bc = INFINITY;
    for (int k = 0; k < nc; ++k) {
        double t = cand[k];
        if (!(t > 0.0)) continue;
        double c = cost_of(t, s, r);
        if (c < bc || (c == bc && t < bt)) { bc = c; bt = t; }
    }
    tau = bt;
    cost = bc;
}

// Exact rejection test for Near: true only if c(tau) > R for every tau > 0,
// so the pair cannot be an edge with c* < R.  For tau >= R, c(tau) >= tau >= R.
// On (0, R), c(tau) < R iff g(tau) = tau^3 (c(tau) - R) < 0 with
//   g(tau) = tau^4 - R tau^3 + 4 r S_vv tau^2 - 12 r S_Pv tau + 12 r S_PP.
// A polynomial whose Bernstein coefficients on an interval are all positive is
// positive there; the test splits [0, R] into halves and quarters (de
// Casteljau) where needed and demands a margin far above the rounding error.
__device__ __forceinline__ bool bern_pos(const double* b, double m) {
    return fmin(fmin(fmin(b[0], b[1]), fmin(b[2], b[3])), b[4]) > m;
}

__device__ __forceinline__ void bern_split(const double* b, double* L, double* Rr) {
    double c[5] = {b[0], b[1], b[2], b[3], b[4]};
    L[0] = c[0];
    Rr[4] = c[4];
    for (int lvl = 1; lvl <= 4; ++lvl) {
        for (int i = 0; i <= 4 - lvl; ++i) c[i] = 0.5 * (c[i] + c[i + 1]);
        L[lvl] = c[0];
        Rr[4 - lvl] = c[4 - lvl];
    }
}

__device__ __forceinline__ bool surely_not_near(const BSums& s, double r, double R) {
    const double R2 = R * R, R4 = R2 * R2;
    const double a0 = 12.0 * r * s.pp, a1 = -12.0 * r * s.pv * R, a2 = 4.0 * r * s.vv * R2;
    const double a3 = -R4, a4 = R4;
    const double m = 1e-9 * (fabs(a0) + fabs(a1) + fabs(a2) + fabs(a3) + fabs(a4));
    double b[5] = {a0, a0 + 0.25 * a1, a0 + 0.5 * a1 + a2 * (1.0 / 6.0),
                   a0 + 0.75 * a1 + 0.5 * a2 + 0.25 * a3, a0 + a1 + a2 + a3 + a4};
    if (bern_pos(b, m)) return true;
    double h[2][5];
    bern_split(b, h[0], h[1]);
    for (int k = 0; k < 2; ++k) {
        if (bern_pos(h[k], m)) continue;
        double q0[5], q1[5];
        bern_split(h[k], q0, q1);
        if (!(bern_pos(q0, m) && bern_pos(q1, m))) return false;
    }
    return true;
}

// A cheap first look, in FP32, at the level-0 Bernstein bound that
// surely_not_near starts with: true only where the FP64 test is true too.
// Every FP32 coefficient is within about 20 units of 2^-24 of the magnitudes
// that enter it (tv bounds those of S_Pv, whose terms can cancel), which is
// far below the margin of 1e-4 times their sum, while the FP64 test's margin
// is 1e-9 times a smaller sum; pairs the bound cannot settle go to the FP64
// test.  r and R are FP32 values (the configuration's), so their casts are
// exact.
__device__ __forceinline__ bool surely_not_near32(const float* x0, const float* x1, float r,
                                                  float R) {
    float pp = 0.f, pv = 0.f, tv = 0.f, vv = 0.f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float P = x1[a] - x0[a];
        const float v0 = x0[3 + a], v1 = x1[3 + a];
        const float sv = v0 + v1;
        pp += P * P;
        pv += P * sv;
        tv += fabsf(P * sv);
        vv += v0 * v0 + v0 * v1 + v1 * v1;
    }
    const float R2 = R * R, R4 = R2 * R2;
    const float a0 = 12.f * r * pp, a1 = -12.f * r * pv * R, a2 = 4.f * r * vv * R2;
    const float m = 1e-4f * (fabsf(a0) + 12.f * r * tv * R + fabsf(a2) + 2.f * R4);
    const float b1 = a0 + 0.25f * a1;
    const float b2 = a0 + 0.5f * a1 + a2 * (1.f / 6.f);
    const float b3 = a0 + 0.75f * a1 + 0.5f * a2 - 0.25f * R4;
    const float b4 = a0 + a1 + a2;                 // + a3 + a4 = 0
    return fminf(fminf(fminf(a0, b1), fminf(b2, b3)), b4) > m;
}

// Minimum-effort nominal trajectory per axis (cubic Hermite):
//   p(t) = p0 + v0 t + c2 t^2 + c3 t^3,
//   c2 = (3P - (2 v0 + v1) tau) / tau^2,  c3 = (-2P + (v0 + v1) tau) / tau^3.
struct Cubic {
    double c0, c1, c2, c3;
    __device__ double at(double t) const { return c0 + t * (c1 + t * (c2 + t * c3)); }
};

// 1 / b from the hardware reciprocal and two Newton steps: within an ulp or
// two of the rounded quotient, for values that need no exact rounding.
__device__ __forceinline__ double recip_fast(double b) {
    double r = __builtin_amdgcn_rcp(b);
    r = fma(fma(-b, r, 1.0), r, r);
    return fma(fma(-b, r, 1.0), r, r);
}

// The same coefficients with it = 1 / tau given.
__device__ __forceinline__ void hermite_r(const float* x0, const float* x1, double tau, double it,
                                          Cubic* out) {
    const double it2 = it * it, it3 = it2 * it;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double p0 = (double)x0[a], v0 = (double)x0[3 + a], v1 = (double)x1[3 + a];
        double P = (double)x1[a] - p0;
        out[a].c0 = p0;
        out[a].c1 = v0;
        out[a].c2 = (3.0 * P - (2.0 * v0 + v1) * tau) * it2;
        out[a].c3 = (-2.0 * P + (v0 + v1) * tau) * it3;
    }
}

__device__ __forceinline__ void hermite(const float* x0, const float* x1, double tau, Cubic* out) {
    hermite_r(x0, x1, tau, 1.0 / tau, out);   // one division for all six coefficients
}

// Interior stationary points of a cubic on (0, tau), ascending; returns count.
__device__ __forceinline__ int stationary_points(const Cubic& c, double tau, double* br) {
    double A = 3.0 * c.c3, B = 2.0 * c.c2, C = c.c1;
    double r0 = NAN, r1 = NAN;
    if (A == 0.0) {
        if (B != 0.0) r0 = -C / B;
    } else {
        double disc = B * B - 4.0 * A * C;
        if (disc >= 0.0) {
            double sq = sqrt(disc);
            double qv = -0.5 * (B + (B >= 0.0 ? sq : -sq));
            if (qv != 0.0) { r0 = qv / A; r1 = C / qv; }
            else { r0 = 0.0; }
        }
    }
    int n = 0;
    if (r0 > 0.0 && r0 < tau) br[n++] = r0;
    if (r1 > 0.0 && r1 < tau) br[n++] = r1;
    if (n == 2 && br[1] < br[0]) { double t = br[0]; br[0] = br[1]; br[1] = t; }
    return n;
}

// On a monotone piece [ta, tb] bracketing `level`: the crossing as a bracket
// (lo, hi) with p(lo) on the start side of the level and p(hi) past it.
// Up to 8 Newton steps kept inside the shrinking bracket (bisection when a
// step leaves it); once a step moves t by at most 4 ulp the bracket is
// closed by testing t -/+ 8 ulp.  Otherwise (slow convergence, e.g. a level
// grazing a stationary point) the bracket is bisected until it is a few ulp
// wide (at most 64 halvings).
__device__ __forceinline__ void crossing(const Cubic& c, double ta, double tb, double level,
                                         bool rising, double& lo, double& hi) {
    constexpr double kEps = 2.220446049250313e-16;
    lo = ta; hi = tb;
    auto on_start = [&](double t) {
        const bool below = c.at(t) < level;
        return rising ? below : !below;
    };
    double t = 0.5 * (lo + hi);
    bool conv = false;
    for (int it = 0; it < 8; ++it) {
        const double p = c.at(t);
        const bool below = p < level;
        if (rising ? below : !below) lo = t; else hi = t;
        const double d = c.c1 + t * (2.0 * c.c2 + 3.0 * c.c3 * t);
        double tn = t - (p - level) / d;
        if (!(tn >= lo && tn <= hi)) tn = 0.5 * (lo + hi);
        if (fabs(tn - t) <= 4.0 * kEps * fabs(t)) {
            t = tn;
            conv = true;
            break;
        }
        t = tn;
    }
    if (conv) {
        const double dl = 8.0 * kEps * fmax(fabs(t), 1e-300);
        const double a = fmax(t - dl, ta), b = fmin(t + dl, tb);
        if (on_start(a) && !on_start(b)) {
            lo = fmax(lo, a);
            hi = fmin(hi, b);
            return;
        }
    }
    for (int it = 0; it < 64 && hi - lo > 2.0 * kEps * fabs(hi); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (on_start(mid)) lo = mid; else hi = mid;
    }
}

// The set {t in [0, tau] : lo <= p(t) <= hi} as up to 3 closed intervals,
// one per monotone piece between the stationary points: interval k is
// [s[k], e[k]] when ok[k].  Fixed slots (no dynamic indexing), so the
// intervals stay in registers.
__device__ __forceinline__ void slab_set(const Cubic& c, double tau, double lo, double hi,
                                         double* s, double* e, bool* ok) {
    double br[2];
    const int nb = stationary_points(c, tau, br);
    const double edge[4] = {0.0, nb > 0 ? br[0] : tau, nb > 1 ? br[1] : tau, tau};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        ok[k] = false;
        s[k] = 0.0;
        e[k] = 0.0;
        if (k > nb) continue;
        const double ta = k == 0 ? 0.0 : edge[k], tb = k == nb ? tau : edge[k + 1];
        const double pa = c.at(ta), pb = c.at(tb);
        const bool rising = pb >= pa;
        const double pmin = fmin(pa, pb), pmax = fmax(pa, pb);
        if (!(pmax >= lo && pmin <= hi)) continue;
        double l0, l1, h0, h1;
        double st, en;
        if (rising) {
            if (pmin >= lo) st = ta; else { crossing(c, ta, tb, lo, true, l0, l1); st = l1; }
            if (pmax <= hi) en = tb; else { crossing(c, ta, tb, hi, true, h0, h1); en = h0; }
        } else {
            if (pmax <= hi) st = ta; else { crossing(c, ta, tb, hi, false, h0, h1); st = h1; }
            if (pmin >= lo) en = tb; else { crossing(c, ta, tb, lo, false, l0, l1); en = l0; }
        }
        s[k] = st;
        e[k] = en;
        ok[k] = true;
    }
}

// Range of a cubic over [0, tau] (endpoints and stationary points).
__device__ __forceinline__ void cubic_range(const Cubic& c, double tau, double& mn, double& mx) {
    double br[2];
    int nb = stationary_points(c, tau, br);
    double p0 = c.at(0.0), p1 = c.at(tau);
    mn = fmin(p0, p1); mx = fmax(p0, p1);
    for (int k = 0; k < nb; ++k) { double v = c.at(br[k]); mn = fmin(mn, v); mx = fmax(mx, v); }
}

// Does the nominal trajectory (three axis cubics on [0, tau]) meet the closed
// box? It is inside at time t iff all three coordinates are in their slabs,
// so it meets the box iff the three per-axis in-slab sets intersect
// (trajectory_hits_box_exact).
//
// Two cheap tests settle most cases first (trajectory_box_quick).  The
// trajectory is swept over 8 equal pieces: a sample point (interior piece
// ends) inside the box proves a hit; and on each piece a cubic lies in the
// hull of its Bernstein coefficients p(ta), p(ta) + h p'(ta)/3,
// p(tb) - h p'(tb)/3, p(tb), so a piece whose hull (widened by kHullMargin,
// far above the rounding of these values) misses the box on some axis
// cannot meet it.  A piece whose hull does meet the box is split once more
// into 4 (more sample points, tighter hulls).  When every piece is cleared
// the trajectory misses the box.  Both tests only settle cases the exact
// test decides the same way.
constexpr double kHullMargin = 1e-9;
enum BoxTest : int { kBoxMiss = 0, kBoxHit = 1, kBoxUnsure = 2 };

// Does the hull of the piece with end values (pa, da), (pb, db) and length
// 3 * h3 miss the box on some axis?
__device__ __forceinline__ bool piece_clear(const double* pa, const double* da, const double* pb,
                                            const double* db, double h3, const float* box) {
    bool sep = false;
    for (int a = 0; a < 3; ++a) {
        const double b1 = pa[a] + h3 * da[a], b2 = pb[a] - h3 * db[a];
        const double lo = fmin(fmin(pa[a], pb[a]), fmin(b1, b2)) - kHullMargin;
        const double hi = fmax(fmax(pa[a], pb[a]), fmax(b1, b2)) + kHullMargin;
        sep |= (hi < (double)box[a]) | (lo > (double)box[3 + a]);
    }
    return sep;
}

__device__ __forceinline__ bool point_in_box(const double* p, const float* box) {
    bool in = true;
    for (int a = 0; a < 3; ++a) in &= (p[a] >= (double)box[a]) & (p[a] <= (double)box[3 + a]);
    return in;
}

__device__ __forceinline__ void eval_pd(const Cubic* cs, double t, double* p, double* d) {
    for (int a = 0; a < 3; ++a) {
        p[a] = cs[a].at(t);
        d[a] = cs[a].c1 + t * (2.0 * cs[a].c2 + t * 3.0 * cs[a].c3);
    }
}

// The piecewise test with `pieces` equal pieces (each split into 4 when its
// hull meets the box).  The quick test uses 8 pieces; the exact stage first
// tries 64 before solving for the slab crossings.
__device__ __forceinline__ int trajectory_box_pieces(const Cubic* cs, double tau, const float* box,
                                                     int pieces) {
    const double inv = 1.0 / (double)pieces;
    const double h = inv * tau;
    const double h3 = h * (1.0 / 3.0);          // piece length / 3 (within the margin)
    const double q3 = 0.25 * h3;                // the same for a quarter piece
    double pa[3], da[3];
    for (int a = 0; a < 3; ++a) {
        pa[a] = cs[a].c0;
        da[a] = cs[a].c1;
    }
    bool ambiguous = false;
    for (int k = 1; k <= pieces; ++k) {
        const double ta = tau * (inv * (double)(k - 1));
        const double t = k == pieces ? tau : tau * (inv * (double)k);
        double pb[3], db[3];
        eval_pd(cs, t, pb, db);
        if (k < pieces && point_in_box(pb, box)) return kBoxHit;
        if (!piece_clear(pa, da, pb, db, h3, box)) {
            // split the piece into 4
            double qa[3] = {pa[0], pa[1], pa[2]}, qd[3] = {da[0], da[1], da[2]};
            for (int j = 1; j <= 4; ++j) {
                double qb[3], qe[3];
                if (j == 4) {
                    for (int a = 0; a < 3; ++a) { qb[a] = pb[a]; qe[a] = db[a]; }
                } else {
                    eval_pd(cs, ta + 0.25 * (double)j * h, qb, qe);
                    if (point_in_box(qb, box)) return kBoxHit;
                }
                ambiguous |= !piece_clear(qa, qd, qb, qe, q3, box);
                for (int a = 0; a < 3; ++a) { qa[a] = qb[a]; qd[a] = qe[a]; }
            }
        }
        for (int a = 0; a < 3; ++a) {
            pa[a] = pb[a];
            da[a] = db[a];
        }
    }
    return ambiguous ? kBoxUnsure : kBoxMiss;
}

__device__ __forceinline__ int trajectory_box_quick(const Cubic* cs, double tau, const float* box) {
    return trajectory_box_pieces(cs, tau, box, 8);
}

__device__ __forceinline__ bool trajectory_hits_box_exact(const Cubic* cs, double tau,
                                                          const float* box) {
    double s[3][3], e[3][3];
    bool ok[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        slab_set(cs[a], tau, (double)box[a], (double)box[3 + a], s[a], e[a], ok[a]);
        if (!(ok[a][0] || ok[a][1] || ok[a][2])) return false;
    }
    bool hit = false;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double st = fmax(fmax(s[0][i], s[1][j]), s[2][k]);
                const double en = fmin(fmin(e[0][i], e[1][j]), e[2][k]);
                hit |= ok[0][i] && ok[1][j] && ok[2][k] && st <= en;
            }
    return hit;
}

__device__ __forceinline__ bool trajectory_hits_box(const Cubic* cs, double tau, const float* box) {
    const int q = trajectory_box_quick(cs, tau, box);
    if (q != kBoxUnsure) return q == kBoxHit;
    return trajectory_hits_box_exact(cs, tau, box);
}

// ---------------------------------------------------------------------------
// Half-Space Monte Carlo (Sec. III-B): the local convex region around a
// workspace point y is built one plane at a time.  Each step takes the
// closest point of the remaining boxes (ties: lowest box index), d = that
// point - y, and drops every remaining box that lies in the closed
// half-space d.(z - y) >= d.d (always the box that gave d).  `rem` holds the
// remaining boxes as bits; returns false when none remains.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool hs_next(const double* y, const float* boxes, int n_obs,
                                        unsigned long long* rem, double* d) {
#pragma clang fp contract(off)
    int best = -1;
    double best_d2 = INFINITY;
    double bd[3] = {0.0, 0.0, 0.0};
    for (int w = 0; w * 64 < n_obs; ++w) {
        unsigned long long m = rem[w];
        while (m) {
            const int o = w * 64 + __ffsll((long long)m) - 1;
            m &= m - 1ull;
            const float* b = boxes + o * 6;
            double dv[3];
            for (int a = 0; a < 3; ++a)
                dv[a] = fmin(fmax(y[a], (double)b[a]), (double)b[3 + a]) - y[a];
            const double d2 = (dv[0] * dv[0] + dv[1] * dv[1]) + dv[2] * dv[2];
            if (d2 < best_d2) {
                best_d2 = d2;
                best = o;
                bd[0] = dv[0]; bd[1] = dv[1]; bd[2] = dv[2];
            }
        }
    }
    if (best < 0) return false;
    d[0] = bd[0]; d[1] = bd[1]; d[2] = bd[2];
    const double dd = (bd[0] * bd[0] + bd[1] * bd[1]) + bd[2] * bd[2];
    const double dy = (bd[0] * y[0] + bd[1] * y[1]) + bd[2] * y[2];
    for (int w = 0; w * 64 < n_obs; ++w) {
        unsigned long long m = rem[w];
        while (m) {
            const int o = w * 64 + __ffsll((long long)m) - 1;
            m &= m - 1ull;
            const float* b = boxes + o * 6;
            double lo_part = 0.0;
            for (int a = 0; a < 3; ++a)
                lo_part += fmin(bd[a] * (double)b[a], bd[a] * (double)b[3 + a]);
            if (o == best || lo_part - dy >= dd) rem[w] &= ~(1ull << (o & 63));
        }
    }
    return true;
}

// hs_next for a wave whose lanes share y and rem (all 64 lanes call it, in
// uniform control flow): lane l takes box w * 64 + l, the nearest box is the
// wave minimum of the same squared distances, taken at its lowest box index
// (as the loop above, which keeps the first strict minimum in box order), and
// the boxes the new plane removes are one ballot per word.  Every value is
// the same expression as in hs_next, so the planes and the boxes left are
// identical.
__device__ __forceinline__ bool hs_next_wave(const double* y, const float* boxes, int n_obs,
                                             unsigned long long* rem, double* d) {
#pragma clang fp contract(off)
    const int lane = threadIdx.x & 63;
    int best = -1;
    double best_d2 = INFINITY;
    for (int w = 0; w * 64 < n_obs; ++w) {
        double d2 = INFINITY;
        if ((rem[w] >> lane) & 1ull) {
            const float* b = boxes + (w * 64 + lane) * 6;
            double dv[3];
            for (int a = 0; a < 3; ++a)
                dv[a] = fmin(fmax(y[a], (double)b[a]), (double)b[3 + a]) - y[a];
            d2 = (dv[0] * dv[0] + dv[1] * dv[1]) + dv[2] * dv[2];
            if (!(d2 < INFINITY)) d2 = INFINITY;   // never chosen, as in the loop
        }
        double m = d2;
        for (int off = 32; off >= 1; off >>= 1) m = fmin(m, __shfl_xor(m, off, 64));
        if (m < best_d2) {
            best_d2 = m;
            best = w * 64 + __ffsll((long long)__ballot(d2 == m)) - 1;
        }
    }
    if (best < 0) return false;
    double bd[3];
    {
        const float* b = boxes + best * 6;
        for (int a = 0; a < 3; ++a) bd[a] = fmin(fmax(y[a], (double)b[a]), (double)b[3 + a]) - y[a];
    }
    d[0] = bd[0]; d[1] = bd[1]; d[2] = bd[2];
    const double dd = (bd[0] * bd[0] + bd[1] * bd[1]) + bd[2] * bd[2];
    const double dy = (bd[0] * y[0] + bd[1] * y[1]) + bd[2] * y[2];
    for (int w = 0; w * 64 < n_obs; ++w) {
        const int o = w * 64 + lane;
        bool drop = false;
        if ((rem[w] >> lane) & 1ull) {
            const float* b = boxes + o * 6;
            double lo_part = 0.0;
            for (int a = 0; a < 3; ++a)
                lo_part += fmin(bd[a] * (double)b[a], bd[a] * (double)b[3 + a]);
            drop = o == best || lo_part - dy >= dd;
        }
        rem[w] &= ~__ballot(drop);
    }
    return true;
}

// eq. (7): the plane normal made perpendicular to the nominal velocity v
// (unchanged at rest); b = a.a.
__device__ __forceinline__ void hs_project(const double* d, const double* v, double* a, double& b) {
#pragma clang fp contract(off)
    const double vv = (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2];
    if (vv > 0.0) {
        const double f = ((d[0] * v[0] + d[1] * v[1]) + d[2] * v[2]) / vv;
        for (int k = 0; k < 3; ++k) a[k] = d[k] - f * v[k];
    } else {
        for (int k = 0; k < 3; ++k) a[k] = d[k];
    }
    b = (a[0] * a[0] + a[1] * a[1]) + a[2] * a[2];
}

__device__ __forceinline__ void all_boxes(int n_obs, unsigned long long* rem) {
    for (int w = 0; w < kMaxObsWords; ++w) {
        const int lo = w * 64;
        rem[w] = n_obs >= lo + 64 ? ~0ull : (n_obs > lo ? ((1ull << (n_obs - lo)) - 1ull) : 0ull);
    }
}

}  // namespace pump
