// Host-side constants of a query shared by the single-query and batched
// entry points: the tracking controller of eq. (2) for the double
// integrator (steady-state discrete LQR per axis), the Cholesky factor of the
// per-step process noise covariance, and the eta rule tying alpha_min and
// alpha_max to alpha.
#pragma once

#include <math.h>
#include <string.h>

#include <algorithm>

namespace pump {

// Steady-state discrete LQR for one axis of the double integrator: iterate
// P <- Q + A'PA - A'PB (R + B'PB)^-1 B'PA to a relative change below 1e-14,
// K = (R + B'PB)^-1 B'PA, du = -K dx.
inline void lqr_axis(double dt, double q_pos, double q_vel, double r, double K[2]) {
    const double A[2][2] = {{1.0, dt}, {0.0, 1.0}};
    const double B[2] = {0.5 * dt * dt, dt};
    double P[2][2] = {{q_pos, 0.0}, {0.0, q_vel}};
    for (int it = 0; it < 1000000; ++it) {
        double PA[2][2], PB[2];
        for (int i = 0; i < 2; ++i) {
            for (int j = 0; j < 2; ++j) PA[i][j] = P[i][0] * A[0][j] + P[i][1] * A[1][j];
            PB[i] = P[i][0] * B[0] + P[i][1] * B[1];
        }
        const double G = r + B[0] * PB[0] + B[1] * PB[1];
        double BPA[2];  // B'PA
        for (int j = 0; j < 2; ++j) BPA[j] = B[0] * PA[0][j] + B[1] * PA[1][j];
        double Pn[2][2];
        double dmax = 0.0, pmax = 0.0;
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                const double APA = A[0][i] * PA[0][j] + A[1][i] * PA[1][j];
                const double v = (i == j ? (i == 0 ? q_pos : q_vel) : 0.0) + APA - BPA[i] * BPA[j] / G;
                Pn[i][j] = v;
                dmax = std::max(dmax, fabs(v - P[i][j]));
                pmax = std::max(pmax, fabs(v));
            }
        memcpy(P, Pn, sizeof(P));
        if (dmax <= 1e-14 * pmax) break;
    }
    double PA[2][2], PB[2];
    for (int i = 0; i < 2; ++i) {
        for (int j = 0; j < 2; ++j) PA[i][j] = P[i][0] * A[0][j] + P[i][1] * A[1][j];
        PB[i] = P[i][0] * B[0] + P[i][1] * B[1];
    }
    const double G = r + B[0] * PB[0] + B[1] * PB[1];
    for (int j = 0; j < 2; ++j) K[j] = (B[0] * PA[0][j] + B[1] * PA[1][j]) / G;
}

// Closed-loop deviation dynamics of one axis, dx' = A_cl dx + w with
// w ~ N(0, sigma^2 V) for the integrated white acceleration noise of one step
// (V = [[dt + dt^3/3, dt^2/2], [dt^2/2, dt]]); L is the lower Cholesky factor
// of sigma^2 V, row-major with L[1] = 0.
inline void tracking_constants(double dt, double q_pos, double q_vel, double r, double sigma,
                               double K[2], double Acl[4], double L[4]) {
    lqr_axis(dt, q_pos, q_vel, r, K);
    const double s2 = sigma * sigma;
    const double Bd[2] = {0.5 * dt * dt, dt};
    Acl[0] = 1.0 - Bd[0] * K[0];
    Acl[1] = dt - Bd[0] * K[1];
    Acl[2] = -Bd[1] * K[0];
    Acl[3] = 1.0 - Bd[1] * K[1];
    const double V00 = s2 * (dt + dt * dt * dt / 3.0), V10 = s2 * (0.5 * dt * dt), V11 = s2 * dt;
    L[0] = sqrt(V00);
    L[1] = 0.0;
    L[2] = L[0] > 0.0 ? V10 / L[0] : 0.0;
    L[3] = sqrt(std::max(0.0, V11 - L[2] * L[2]));
}

// eta: 2 at alpha >= 1e-2, 10 at alpha <= 1e-3, log-linear in between.
inline double eta_rule(double alpha) {
    if (alpha >= 0.01) return 2.0;
    if (alpha <= 0.001) return 10.0;
    const double w = (log(0.01) - log(alpha)) / (log(0.01) - log(0.001));
    return exp(log(2.0) + w * (log(10.0) - log(2.0)));
}

// Integer forms of the cp_hat tests for N particles (pop / N is exact for N a
// power of 2): a plan is cut once pop >= c_cut, and a goal plan stops the
// search once pop < c_min.
inline void cp_thresholds(double alpha, double eta, int N, int* c_cut, int* c_min) {
    *c_cut = (int)std::min<double>(ceil(eta * alpha * N), (double)(N + 1));
    *c_min = (int)std::min<double>(ceil(alpha / eta * N), (double)(N + 1));
}

}  // namespace pump
