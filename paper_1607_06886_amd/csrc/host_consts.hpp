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
// w ~ N(0, V), V the one-step integral of eq. (2) for V_c = sigma^2 I:
// V = sigma^2 [[dt + dt^3/3, dt^2/2], [dt^2/2, dt]]; L is the lower Cholesky
// factor of V, row-major with L[1] = 0.
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

// Steady-state Kalman gain of one axis for the position measurement
// y = [1 0] dx + w, w ~ N(0, Wm) (eq. (2)): iterate the predicted covariance
// P <- A (P - P C' C P / (C P C' + Wm)) A' + V from P = V to a relative change
// below 1e-14; G = P C' / (C P C' + Wm).  V is the process covariance above.
inline void kalman_axis(double dt, const double V[3], double Wm, double G[2]) {
    const double A[2][2] = {{1.0, dt}, {0.0, 1.0}};
    double P[2][2] = {{V[0], V[1]}, {V[1], V[2]}};
    for (int it = 0; it < 1000000; ++it) {
        const double S = P[0][0] + Wm;
        double U[2][2];  // filtered covariance P - P C' C P / S
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) U[i][j] = P[i][j] - P[i][0] * P[0][j] / S;
        double AU[2][2];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) AU[i][j] = A[i][0] * U[0][j] + A[i][1] * U[1][j];
        double Pn[2][2];
        double dmax = 0.0, pmax = 0.0;
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                const double Vij = (i == 0 && j == 0) ? V[0] : (i == 1 && j == 1) ? V[2] : V[1];
                const double v = AU[i][0] * A[j][0] + AU[i][1] * A[j][1] + Vij;
                Pn[i][j] = v;
                dmax = std::max(dmax, fabs(v - P[i][j]));
                pmax = std::max(pmax, fabs(v));
            }
        memcpy(P, Pn, sizeof(P));
        if (dmax <= 1e-14 * std::max(pmax, 1e-300)) break;
    }
    const double S = P[0][0] + Wm;
    G[0] = P[0][0] / S;
    G[1] = P[1][0] / S;
}

// LQG closed loop of one axis on z = (dx, x_hat), both 2-vectors:
//   dx'    = A dx - B K x_hat + L xi_p
//   x_hat' = x_pred + G (y' - C x_pred),  x_pred = A x_hat - B K x_hat,
//            y' = C dx' + sqrt(Wm) xi_m
// i.e. z' = M z + E (xi_p0, xi_p1, xi_m) with M, E row-major (4x4, 4x3).
// Wm = sigma_meas^2 / dt (W = W_c / dt of eq. (2)).  The controller is the
// LQR gain acting on the estimate (certainty equivalence).
inline void lqg_constants(double dt, double q_pos, double q_vel, double r, double sigma,
                          double sigma_meas, double M[16], double E[12]) {
    double K[2], Acl[4], L[4];
    tracking_constants(dt, q_pos, q_vel, r, sigma, K, Acl, L);
    const double s2 = sigma * sigma;
    const double V[3] = {s2 * (dt + dt * dt * dt / 3.0), s2 * (0.5 * dt * dt), s2 * dt};
    const double Wm = sigma_meas * sigma_meas / dt;
    double G[2];
    kalman_axis(dt, V, Wm, G);
    const double A[2][2] = {{1.0, dt}, {0.0, 1.0}};
    const double B[2] = {0.5 * dt * dt, dt};
    for (int i = 0; i < 2; ++i) {
        for (int j = 0; j < 2; ++j) {
            M[i * 4 + j] = A[i][j];                       // true state
            M[i * 4 + 2 + j] = -B[i] * K[j];              // control from the estimate
            M[(2 + i) * 4 + j] = G[i] * A[0][j];          // G C A
            const double IGCA = A[i][j] - G[i] * A[0][j]; // (I - G C) A
            M[(2 + i) * 4 + 2 + j] = IGCA - B[i] * K[j];
        }
    }
    const double sw = sqrt(Wm);
    E[0] = L[0]; E[1] = 0.0; E[2] = 0.0;
    E[3] = L[2]; E[4] = L[3]; E[5] = 0.0;
    E[6] = G[0] * L[0]; E[7] = 0.0; E[8] = G[0] * sw;
    E[9] = G[1] * L[0]; E[10] = 0.0; E[11] = G[1] * sw;
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
