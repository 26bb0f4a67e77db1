// The quadrotor model of the paper's benchmark set (Appendix A), transcribed
// with the trapezoidal scheme of Sec. 5.
//
// Node-local variables v = 0..12: states x1..x9 are v = 0..8 (positions x1,
// x3, x5; velocities x2, x4, x6; Euler angles x7 = roll, x8 = pitch, x9 =
// yaw), controls u1..u4 are v = 9..12 (thrust, then three rates).  Every
// variable lives on the N+1 nodes, so its global index at node k is
// v (N+1) + k.  Dynamics (c = cos, s = sin, t = tan, digits = state index):
//   x1' = x2,  x3' = x4,  x5' = x6,
//   x2' = u1 (c7 s8 c9 + s7 s9),  x4' = u1 (c7 s8 s9 - s7 c9),  x6' = u1 c7 c8 - g,
//   x7' = (u2 c7 + u3 s7) / c8,  x8' = -u2 s7 + u3 c7,  x9' = (u2 c7 + u3 s7) t8 + u4.
// Cost: one half of the integral of (x1 - sin 2 pi t)^2 + (x3 - 2 sin 4 pi t)^2
// + (x5 - 2t)^2 + x7^2 + x8^2 + x9^2 + r |u|^2 on t in [0, 1].
//
// This header holds the pattern tables, which the host index layer and the
// kernels share; the per-node values are in ocp_quad_device.h.
#pragma once

#include <cstdint>

namespace ocp {
namespace quad {

constexpr int kStates = 9;
constexpr int kControls = 4;
constexpr int kVars = 13;

// Jacobian support of defect row i: its own state and the variables its
// right-hand side depends on, ascending.  Row i holds two entries per
// support variable (node k, node k+1), so the row's entries are in
// ascending column order.
constexpr int kSupLen[kStates] = {2, 5, 2, 5, 2, 4, 4, 4, 6};
constexpr int kSup[kStates][6] = {
    {0, 1, 0, 0, 0, 0},    {1, 6, 7, 8, 9, 0},  {2, 3, 0, 0, 0, 0},
    {3, 6, 7, 8, 9, 0},    {4, 5, 0, 0, 0, 0},  {5, 6, 7, 9, 0, 0},
    {6, 7, 10, 11, 0, 0},  {6, 7, 10, 11, 0, 0}, {6, 7, 8, 10, 11, 12},
};
// First Jacobian slot of row i within an interval (twice the support sizes
// of the rows before it); kRowSlot[9] is the number of slots per interval.
constexpr int kRowSlot[kStates + 1] = {0, 4, 14, 18, 28, 32, 40, 48, 56, 68};
constexpr int kSlots = 68;
// (row, support variable) pairs: pair kRowSlot[i] / 2 + p.
constexpr int kPairs = 34;

// Hessian: the 23 lower-triangle entries of one node, sorted by (row, col),
// each variable's row ending with its diagonal.  Entry s of node k sits at
// COO position s (N+1) + k.
constexpr int kHessNode = 23;
constexpr int kHessRow[kHessNode] = {0, 1, 2, 3, 4, 5, 6, 7, 7, 8, 8, 8, 9, 9, 9, 9,
                                     10, 10, 10, 11, 11, 11, 12};
constexpr int kHessCol[kHessNode] = {0, 1, 2, 3, 4, 5, 6, 6, 7, 6, 7, 8, 6, 7, 8, 9,
                                     6, 7, 10, 6, 7, 11, 12};
// First Hessian entry of variable v's row; kHessFirst[13] = 23.
constexpr int kHessFirst[kVars + 1] = {0, 1, 2, 3, 4, 5, 6, 7, 9, 12, 16, 19, 22, 23};

constexpr int pair_index(int i, int p) { return kRowSlot[i] / 2 + p; }
constexpr bool pair_is_own_state(int i, int p) { return kSup[i][p] == i; }

}  // namespace quad
}  // namespace ocp
