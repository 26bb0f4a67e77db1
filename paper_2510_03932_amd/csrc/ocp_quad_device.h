// Per-node values of the quadrotor model (device code): attitude
// trigonometry, the right-hand side, its first derivatives on the Jacobian
// support and the multiplier-weighted second derivatives on the Hessian
// pattern.  Numbering and patterns are those of ocp_quad_model.h.
#pragma once

#include <hip/hip_runtime.h>

#include "ocp_quad_model.h"

namespace ocp {
namespace quad {

// Trigonometric values of one node's attitude.
struct Trig {
    double s7, c7, s8, c8, s9, c9;
    double sec, t8, sec2;  // 1 / c8, s8 / c8, 1 / c8^2
};

__device__ __forceinline__ Trig node_trig(double roll, double pitch, double yaw)
{
    Trig t;
    sincos(roll, &t.s7, &t.c7);
    sincos(pitch, &t.s8, &t.c8);
    sincos(yaw, &t.s9, &t.c9);
    t.sec = 1.0 / t.c8;
    t.t8 = t.s8 * t.sec;
    t.sec2 = t.sec * t.sec;
    return t;
}

// Right-hand side F (9 values) at one node.
__device__ __forceinline__ void rhs(const double *x, const double *u, double g, double *F)
{
    const Trig t = node_trig(x[6], x[7], x[8]);
    const double p = u[1] * t.c7 + u[2] * t.s7;
    F[0] = x[1];
    F[1] = u[0] * (t.c7 * t.s8 * t.c9 + t.s7 * t.s9);
    F[2] = x[3];
    F[3] = u[0] * (t.c7 * t.s8 * t.s9 - t.s7 * t.c9);
    F[4] = x[5];
    F[5] = u[0] * t.c7 * t.c8 - g;
    F[6] = p * t.sec;
    F[7] = -u[1] * t.s7 + u[2] * t.c7;
    F[8] = p * t.t8 + u[3];
}

// dF_i / dv for pair q = (row i, p-th support variable).  With q a
// compile-time constant (unrolled loops) the switch folds away.
__device__ __forceinline__ double partial(int q, const Trig &t, const double *u)
{
    const double p = u[1] * t.c7 + u[2] * t.s7;   // d p / d roll = w
    const double w = -u[1] * t.s7 + u[2] * t.c7;  // d w / d roll = -p
    switch (q) {
    // row 0, x1' = x2: (x1, x2)
    case 0: return 0.0;
    case 1: return 1.0;
    // row 1, x2': (x2, x7, x8, x9, u1)
    case 2: return 0.0;
    case 3: return u[0] * (t.c7 * t.s9 - t.s7 * t.s8 * t.c9);
    case 4: return u[0] * t.c7 * t.c8 * t.c9;
    case 5: return u[0] * (t.s7 * t.c9 - t.c7 * t.s8 * t.s9);
    case 6: return t.c7 * t.s8 * t.c9 + t.s7 * t.s9;
    // row 2, x3' = x4: (x3, x4)
    case 7: return 0.0;
    case 8: return 1.0;
    // row 3, x4': (x4, x7, x8, x9, u1)
    case 9: return 0.0;
    case 10: return -u[0] * (t.s7 * t.s8 * t.s9 + t.c7 * t.c9);
    case 11: return u[0] * t.c7 * t.c8 * t.s9;
    case 12: return u[0] * (t.c7 * t.s8 * t.c9 + t.s7 * t.s9);
    case 13: return t.c7 * t.s8 * t.s9 - t.s7 * t.c9;
    // row 4, x5' = x6: (x5, x6)
    case 14: return 0.0;
    case 15: return 1.0;
    // row 5, x6': (x6, x7, x8, u1)
    case 16: return 0.0;
    case 17: return -u[0] * t.s7 * t.c8;
    case 18: return -u[0] * t.c7 * t.s8;
    case 19: return t.c7 * t.c8;
    // row 6, x7': (x7, x8, u2, u3)
    case 20: return w * t.sec;
    case 21: return p * t.s8 * t.sec2;
    case 22: return t.c7 * t.sec;
    case 23: return t.s7 * t.sec;
    // row 7, x8': (x7, x8, u2, u3)
    case 24: return -p;
    case 25: return 0.0;
    case 26: return -t.s7;
    case 27: return t.c7;
    // row 8, x9': (x7, x8, x9, u2, u3, u4)
    case 28: return w * t.t8;
    case 29: return p * t.sec2;
    case 30: return 0.0;
    case 31: return t.c7 * t.t8;
    case 32: return t.s7 * t.t8;
    default: return 1.0;  // 33: u4
    }
}

// Hessian entries of one node: H[s] = sw C_s - hh S_s, where sw = sigma w_k,
// C_s the cost's constant second derivative (1 on x1, x3, x5, x7, x8, x9; r on
// the controls) and S_s = sum_i Y_i d2F_i / (dv_a dv_b) with Y the node
// multipliers ytilde (only rows 2, 4, 6, 7, 8, 9 of the ODE are nonlinear).
__device__ __forceinline__ void hess_values(const Trig &t, const double *u, const double *Y,
                                            double sw, double r, double hh, double *H)
{
    const double p = u[1] * t.c7 + u[2] * t.s7;
    const double w = -u[1] * t.s7 + u[2] * t.c7;
    const double A2 = Y[1] * u[0], A4 = Y[3] * u[0];
    const double a2 = t.c7 * t.s8 * t.c9 + t.s7 * t.s9;  // F2 / u1
    const double a4 = t.c7 * t.s8 * t.s9 - t.s7 * t.c9;  // F4 / u1
    const double sec3 = t.sec2 * t.sec;
    const double Srr = -A2 * a2 - A4 * a4 - Y[5] * u[0] * t.c7 * t.c8 - Y[6] * p * t.sec - Y[7] * w -
                       Y[8] * p * t.t8;
    const double Spr = -A2 * t.s7 * t.c8 * t.c9 - A4 * t.s7 * t.c8 * t.s9 + Y[5] * u[0] * t.s7 * t.s8 +
                       Y[6] * w * t.s8 * t.sec2 + Y[8] * w * t.sec2;
    const double Spp = -A2 * t.c7 * t.s8 * t.c9 - A4 * t.c7 * t.s8 * t.s9 - Y[5] * u[0] * t.c7 * t.c8 +
                       Y[6] * p * (1.0 + t.s8 * t.s8) * sec3 + Y[8] * 2.0 * p * t.s8 * sec3;
    const double Syr = A2 * (t.s7 * t.s8 * t.s9 + t.c7 * t.c9) + A4 * (t.c7 * t.s9 - t.s7 * t.s8 * t.c9);
    const double Syp = -A2 * t.c7 * t.c8 * t.s9 + A4 * t.c7 * t.c8 * t.c9;
    const double Syy = -A2 * a2 - A4 * a4;
    const double S1r = Y[1] * (t.c7 * t.s9 - t.s7 * t.s8 * t.c9) - Y[3] * (t.s7 * t.s8 * t.s9 + t.c7 * t.c9) -
                       Y[5] * t.s7 * t.c8;
    const double S1p = Y[1] * t.c7 * t.c8 * t.c9 + Y[3] * t.c7 * t.c8 * t.s9 - Y[5] * t.c7 * t.s8;
    const double S1y = Y[1] * (t.s7 * t.c9 - t.c7 * t.s8 * t.s9) + Y[3] * a2;
    const double S2r = -Y[6] * t.s7 * t.sec - Y[7] * t.c7 - Y[8] * t.s7 * t.t8;
    const double S2p = Y[6] * t.c7 * t.s8 * t.sec2 + Y[8] * t.c7 * t.sec2;
    const double S3r = Y[6] * t.c7 * t.sec - Y[7] * t.s7 + Y[8] * t.c7 * t.t8;
    const double S3p = Y[6] * t.s7 * t.s8 * t.sec2 + Y[8] * t.s7 * t.sec2;
    const double swr = sw * r;
    H[0] = sw;
    H[1] = 0.0;
    H[2] = sw;
    H[3] = 0.0;
    H[4] = sw;
    H[5] = 0.0;
    H[6] = sw - hh * Srr;
    H[7] = -hh * Spr;
    H[8] = sw - hh * Spp;
    H[9] = -hh * Syr;
    H[10] = -hh * Syp;
    H[11] = sw - hh * Syy;
    H[12] = -hh * S1r;
    H[13] = -hh * S1p;
    H[14] = -hh * S1y;
    H[15] = swr;
    H[16] = -hh * S2r;
    H[17] = -hh * S2p;
    H[18] = swr;
    H[19] = -hh * S3r;
    H[20] = -hh * S3p;
    H[21] = swr;
    H[22] = swr;
}

}  // namespace quad
}  // namespace ocp
