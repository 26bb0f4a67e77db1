// Derivatives of the Lagrangian L(z, y) = sigma f(z) + y^T c(z) beyond the
// interior-point evaluations: its value, grad_z L, Hessian-vector and
// Jacobian-vector products, and the gradient with respect to the dynamics
// coefficients (A, B, gamma) -- the pieces a differentiable-programming
// wrapper needs (the paper names tighter integration with differentiable
// programming as future work, Sec. 8).
//
// With the node multiplier yt_ik = y_{i,k-1}[k >= 1] + y_ik[k < N] (node k
// closes interval k-1 and opens interval k):
//   grad_z L at X_jk  = 2 sigma w_k q_j X_jk + y_{j,k-1} - y_jk
//                       - hh (cos X_jk (A^T yt)_j + yt_j gamma_j X_{p(j)k}
//                             + yt_{j-1} gamma_{j-1} X_{j-1,k})
//   grad_z L at U_lk  = 2 sigma w_k r_l U_lk - hh (B^T yt)_l
//   (H v) at node k   = diag_j v_j + P_j v_{p(j)} + P_{j-1} v_{j-1},
//                       diag_j = 2 sigma w_k q_j + hh sin X_jk (A^T yt)_j,
//                       P_i = -hh yt_i gamma_i;  controls 2 sigma w_k r_l v
//   (J v)_ik          = (v_{i,k+1} - v_ik) - hh (D_i(k) + D_i(k+1)),
//                       D_i = sum_j A_ij cos X_j v_j + sum_l B_il v_l
//                             + gamma_i (X_p v_i + X_i v_p)
//   dL/dA_ij = -hh sum_k yt_ik sin X_jk,  dL/dB_il = -hh sum_k yt_ik U_lk,
//   dL/dgamma_i = -hh sum_k yt_ik X_ik X_{p(i)k}.
// Forward Euler (Sec. 3), c_ik = X_{i,k+1} - X_ik - h F_i(k): the same with
// hh replaced by h and the node multiplier yt_ik = y_ik [k < N] (F at node k
// enters only row (i, k)); controls exist on nodes k < N.  Generally the
// defect is X_{i,k+1} - X_ik - al F_i(k) - be F_i(k+1) with (al, be) =
// (hh, hh) or (h, 0).  Boundary rows (the state itself at node 0, and at node
// N) add their multiplier to grad_z L at that state and v at that state to
// J v; they are linear, so H v and dL/dtheta do not see them.
// Every sum over nodes is a fixed-shape two-pass reduction (deterministic).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "ocp_device.h"
#include "ocp_internal.h"
#include "ocp_problem.h"
#include "ocp_quad.h"

using namespace ocp;
using namespace ocp::dev;

// The coefficient gradient needs the synthetic family's coefficient arrays
// (either scheme, any boundary option); the quadrotor model has none.
static int check_coefficients(const ocp_problem *p, const char *what)
{
    if (p->model != 0)
        return fail(OCP_ERR_ARG, std::string(what) + ": supports the synthetic dynamics family only");
    return OCP_OK;
}

namespace {


// Lagrangian value, pass 1.  Chunk c covers nodes [c (B-1), c (B-1) + B) and
// closes the B-1 intervals starting there (one node of overlap, as in the
// defect kernel); workgroups take chunks c = blockIdx.x, + gridDim.x, ...
// A node's cost term is counted by the chunk that owns it (lane < B-1, or
// the last node N).
template <int NB>
__global__ __launch_bounds__(kBlock) void lag_partial_kernel(KP P, const double *__restrict__ z,
                                                             const double *__restrict__ y,
                                                             double sigma, int nchunks,
                                                             double *__restrict__ partials)
{
    __shared__ double Ms[NB][kBlock];
    const int tid = threadIdx.x;
    const int n = P.n, m = P.m;
    const int64_t N = P.N, N1 = P.N1, NU = P.NU;
    const double *U = z + (int64_t)n * N1;
    const double *yb = y + (int64_t)n * N;  // boundary-row multipliers
    const bool euler = P.scheme != 0;
    const double al = euler ? P.h : P.hh, be = euler ? 0.0 : P.hh;
    double acc = 0.0;
    for (int ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int64_t k = (int64_t)ch * (kBlock - 1) + tid;
        // the multipliers of this lane's interval, loaded up front so that
        // they arrive while the node's dynamics are evaluated (index clamped
        // into the row; used only for k < N)
        double yv[NB];
        const int64_t ky = k < N ? k : N - 1;
#pragma unroll
        for (int i = 0; i < NB; i++) yv[i] = y[(int64_t)(i < n ? i : 0) * N + ky];
        double Pk[NB];
        if (k <= N) {
            double x[NB], F[NB];
            if (k < NU) {
                dyn_node<NB>(P, z, k, x, F);
            } else {  // forward Euler, node N: F(N) enters no row
#pragma unroll
                for (int i = 0; i < NB; i++) {
                    x[i] = (i < n) ? z[i * N1 + k] : 0.0;
                    F[i] = 0.0;
                }
            }
#pragma unroll
            for (int i = 0; i < NB; i++) {
                if (i < n) {
                    Ms[i][tid] = x[i] - be * F[i];
                    Pk[i] = x[i] + al * F[i];
                }
            }
            if (tid < kBlock - 1 || k == N) {
                double s = 0.0;
#pragma unroll
                for (int i = 0; i < NB; i++)
                    if (i < n) s += P.q[i] * x[i] * x[i];
                if (k < NU) {
                    for (int l = 0; l < m; l++) {
                        const double u = U[l * NU + k];
                        s += P.r[l] * u * u;
                    }
                }
                acc += sigma * node_weight(P, (int)k) * s;
                // boundary rows: the state at node 0 (and at node N)
                if (P.nb >= n && k == 0) {
#pragma unroll
                    for (int i = 0; i < NB; i++)
                        if (i < n) acc += yb[i] * x[i];
                }
                if (P.nb >= 2 * n && k == N) {
#pragma unroll
                    for (int i = 0; i < NB; i++)
                        if (i < n) acc += yb[n + i] * x[i];
                }
            }
        }
        __syncthreads();
        if (tid < kBlock - 1 && k < N) {
#pragma unroll
            for (int i = 0; i < NB; i++)
                if (i < n) acc += yv[i] * (Ms[i][tid + 1] - Pk[i]);
        }
        __syncthreads();
    }
    const double t = block_sum<kBlock>(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ __launch_bounds__(kBlock) void sum_partials_kernel(const double *__restrict__ partials,
                                                              int count, double *__restrict__ out)
{
    double acc = 0.0;
    for (int i = threadIdx.x; i < count; i += kBlock) acc += partials[i];
    const double t = block_sum<kBlock>(acc);
    if (threadIdx.x == 0) out[0] = t;
}

// Loads shared by grad_z L and H v at node k: states and node multipliers.
template <int NB>
__device__ __forceinline__ void node_x_yt(const KP &P, const double *__restrict__ z,
                                          const double *__restrict__ y, int k, double (&x)[NB],
                                          double (&yl)[NB], double (&yr)[NB])
{
    const int n = P.n;
    const int64_t N = P.N, N1 = P.N1;
#pragma unroll
    for (int i = 0; i < NB; i++) {
        x[i] = yl[i] = yr[i] = 0.0;
        if (i < n) {
            x[i] = z[i * N1 + k];
            const double *yi = y + i * N + k;
            if (k >= 1) yl[i] = yi[-1];
            if (k < P.N) yr[i] = yi[0];
        }
    }
}

// The node's first NB control entries of a z-shaped array a (zero past m and
// at a node without controls), loaded with the node's other values (J v:
// 11.1-11.3 against 11.9-12.0 us at N = 2e5, n = 8, m = 4; grad_z L and H v
// measured the same either way and load theirs at the stores).
template <int NB>
__device__ __forceinline__ void node_controls(const KP &P, const double *__restrict__ a, int64_t k,
                                              double (&u)[NB])
{
    const double *U = a + (int64_t)P.n * P.N1;
#pragma unroll
    for (int l = 0; l < NB; l++) u[l] = (l < P.m && k < P.NU) ? U[(int64_t)l * P.NU + k] : 0.0;
}

template <int NB>
__global__ __launch_bounds__(kBlock) void lag_grad_kernel(KP P, const double *__restrict__ z,
                                                          const double *__restrict__ y, double sigma,
                                                          double *__restrict__ g)
{
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k > P.N) return;
    const int n = P.n, m = P.m;
    const int64_t N = P.N, N1 = P.N1, NU = P.NU;
    const bool euler = P.scheme != 0;
    const double wF = euler ? P.h : P.hh;
    const double w = node_weight(P, k);
    double x[NB], yl[NB], yr[NB], yt[NB];
    node_x_yt<NB>(P, z, y, k, x, yl, yr);
#pragma unroll
    for (int i = 0; i < NB; i++) yt[i] = euler ? yr[i] : yl[i] + yr[i];
    const double x_last = last_of<NB>(x, n), yt_last = last_of<NB>(yt, n);
    // boundary rows at this node add their multiplier to the state's entry
    const double *yb = nullptr;
    if (P.nb >= n && k == 0) yb = y + (int64_t)n * N;
    if (P.nb >= 2 * n && k == N) yb = y + (int64_t)n * N + n;
#pragma unroll
    for (int j = 0; j < NB; j++) {
        if (j < n) {
            const double *a = P.AT + j * kLd;
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < NB; i++) s = __builtin_fma(yt[i], a[i], s);
            const double xn = (j + 1 < n) ? x[(j + 1) % NB] : x[0];
            const int jm = (j == 0) ? n - 1 : j - 1;
            const double xm = (j == 0) ? x_last : x[(j + NB - 1) % NB];
            const double ym = (j == 0) ? yt_last : yt[(j + NB - 1) % NB];
            const double G = cos(x[j]) * s + yt[j] * P.gam[j] * xn + ym * P.gam[jm] * xm;
            double val = 2.0 * sigma * w * P.q[j] * x[j] + (yl[j] - yr[j]) - wF * G;
            if (yb) val += yb[j];
            st_nt(g + j * N1 + k, val);
        }
    }
    if (k >= NU) return;  // forward Euler: no controls at node N
    const double *U = z + (int64_t)n * N1;
    for (int l = 0; l < m; l++) {
        const double *b = P.BT + l * kLd;
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < NB; i++) s = __builtin_fma(yt[i], b[i], s);
        st_nt(g + n * N1 + l * NU + k, 2.0 * sigma * w * P.r[l] * U[l * NU + k] - wF * s);
    }
}

template <int NB>
__global__ __launch_bounds__(kBlock) void hvp_kernel(KP P, const double *__restrict__ z,
                                                     const double *__restrict__ y, double sigma,
                                                     const double *__restrict__ v,
                                                     double *__restrict__ out)
{
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k > P.N) return;
    const int n = P.n, m = P.m;
    const int64_t N1 = P.N1, NU = P.NU;
    const bool euler = P.scheme != 0;
    const double wF = euler ? P.h : P.hh;
    const double w = node_weight(P, k);
    double x[NB], yl[NB], yr[NB], vx[NB], pr[NB];
    node_x_yt<NB>(P, z, y, k, x, yl, yr);
    double *yt = yl;  // node multiplier, in place: y_{i,k-1} + y_ik, or y_ik under Euler
#pragma unroll
    for (int i = 0; i < NB; i++) {
        yt[i] = euler ? yr[i] : yl[i] + yr[i];
        vx[i] = (i < n) ? v[i * N1 + k] : 0.0;
        pr[i] = (i < n) ? -wF * yt[i] * P.gam[i] : 0.0;
    }
    const double v_last = last_of<NB>(vx, n), p_last = last_of<NB>(pr, n);
#pragma unroll
    for (int j = 0; j < NB; j++) {
        if (j < n) {
            const double *a = P.AT + j * kLd;
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < NB; i++) s = __builtin_fma(yt[i], a[i], s);
            const double d = 2.0 * sigma * w * P.q[j] + wF * sin(x[j]) * s;
            const double vn = (j + 1 < n) ? vx[(j + 1) % NB] : vx[0];
            const double vm = (j == 0) ? v_last : vx[(j + NB - 1) % NB];
            const double pm = (j == 0) ? p_last : pr[(j + NB - 1) % NB];
            st_nt(out + j * N1 + k, d * vx[j] + pr[j] * vn + pm * vm);
        }
    }
    if (k >= NU) return;  // forward Euler: no controls at node N
    for (int l = 0; l < m; l++) {
        const int64_t e = (int64_t)n * N1 + l * NU + k;
        st_nt(out + e, 2.0 * sigma * w * P.r[l] * v[e]);
    }
}

// J v, laid out like the defects: lane k publishes v_ik - be D_i(k) for lane
// k-1 and keeps v_ik + al D_i(k).
template <int NB>
__global__ __launch_bounds__(kBlock) void jvp_kernel(KP P, const double *__restrict__ z,
                                                     const double *__restrict__ v,
                                                     double *__restrict__ out)
{
    __shared__ double Ms[NB][kBlock];
    const int tid = threadIdx.x;
    const int64_t k = (int64_t)blockIdx.x * (kBlock - 1) + tid;
    const int n = P.n, m = P.m;
    const int64_t N = P.N, N1 = P.N1, NU = P.NU;
    const bool euler = P.scheme != 0;
    const double al = euler ? P.h : P.hh, be = euler ? 0.0 : P.hh;
    double Pk[NB];
    if (k <= N) {
        double x[NB], vx[NB], D[NB], vu[NB];
#pragma unroll
        for (int i = 0; i < NB; i++) {
            x[i] = (i < n) ? z[i * N1 + k] : 0.0;
            vx[i] = (i < n) ? v[i * N1 + k] : 0.0;
            D[i] = 0.0;
        }
        node_controls<NB>(P, v, k, vu);
#pragma unroll
        for (int j = 0; j < NB; j++) {
            if (j < n) {
                const double t = cos(x[j]) * vx[j];
                const double *a = P.AT + j * kLd;
#pragma unroll
                for (int i = 0; i < NB; i++) D[i] = __builtin_fma(a[i], t, D[i]);
            }
        }
#pragma unroll
        for (int l = 0; l < NB; l++) {
            if (l < m && k < NU) {
                const double *b = P.BT + l * kLd;
#pragma unroll
                for (int i = 0; i < NB; i++) D[i] = __builtin_fma(b[i], vu[l], D[i]);
            }
        }
        for (int l = NB; l < m && k < NU; l++) {
            const double u = v[n * N1 + l * NU + k];
            const double *b = P.BT + l * kLd;
#pragma unroll
            for (int i = 0; i < NB; i++) D[i] = __builtin_fma(b[i], u, D[i]);
        }
#pragma unroll
        for (int i = 0; i < NB; i++) {
            if (i < n) {
                const double xp = (i + 1 < n) ? x[(i + 1) % NB] : x[0];
                const double vp = (i + 1 < n) ? vx[(i + 1) % NB] : vx[0];
                D[i] += P.gam[i] * (xp * vx[i] + x[i] * vp);
                Ms[i][tid] = vx[i] - be * D[i];
                Pk[i] = vx[i] + al * D[i];
            }
        }
    }
    __syncthreads();
    if (tid < kBlock - 1 && k < N) {
#pragma unroll
        for (int i = 0; i < NB; i++)
            if (i < n) st_nt(out + i * N + k, Ms[i][tid + 1] - Pk[i]);
    }
}

// Boundary rows of J v: row n N + b holds the state X_{b mod n} at node 0
// (b < n) or at node N.
__global__ __launch_bounds__(kBlock) void bnd_jvp_kernel(KP P, const double *__restrict__ v,
                                                         double *__restrict__ out)
{
    const int b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= P.nb) return;
    const int i = b % P.n;
    const int64_t node = b < P.n ? 0 : P.N;
    out[(int64_t)P.n * P.N + b] = v[(int64_t)i * P.N1 + node];
}

// Coefficient gradient, pass 1.  With yt_i(k) the multiplier weight of node
// k in row block i (y_{i,k-1} + y_{i,k} for the trapezoid, y_{i,k} for
// forward Euler), the sums S_ij = sum_k yt_i sin X_j and S_il = sum_k yt_i
// U_l are the product of the (n x N+1) matrix yt with the (N+1 x n+m)
// matrix [sin X | U]: a contraction over the nodes, done here on the FP64
// matrix cores.  The gamma sums S_i = sum_k yt_i X_i X_p(i) are one per row
// and are summed on the vector units.
//
// Workgroup b takes the chunks of kCoefChunk nodes b, b + G, ...  Per chunk,
// two phases split by one barrier:
// (1) staging: the workgroup is split into Q = kBlock / kCoefChunk parts of
// one node per lane; part h loads columns h, h + Q, h + 2Q, ... of [X | U]
// (so that every part holds about the same number of state columns) and a
// run of the rows of y, all loads coalesced and issued together.  The lanes
// take the sines of their state entries in registers and store sin X | U,
// the raw X rows (for the gamma terms) and y to LDS;
// (2) each lane adds the gamma terms X_i X_p(i) yt_i of its node for the
// rows of its part, and wave w feeds its kCoefChunk / 4 nodes to
// v_mfma_f64_16x16x4f64, 4 nodes per instruction (lane l supplies row or
// column l mod 16 at node l / 16 of the step), accumulating every 16 x 16
// block of the product.
// At the end the 4 waves' blocks are added in order in LDS and workgroup b
// writes its n (n+m+1) sums as one contiguous run, cpart[b n (n+m+1) +
// i (n+m+1) + col] (col n+m: the gamma sum).  MB = ceil(n / 16) row blocks,
// NBK = ceil((n+m) / 16) column blocks.
//
// MIXED: the derivative of the same sums along a direction v of z (the mixed
// second derivatives d2L/(dtheta dz) v): the columns become [cos X * V_X |
// V_U] and the gamma terms yt_i (V_X,i X_p(i) + X_i V_X,p(i)); the parts load
// the state rows of X and the rows of v (the control rows of z are not
// needed), and stage the raw V_X rows beside the raw X rows.
template <int MB, int NBK, bool MIXED>
__global__ __launch_bounds__(kBlock) void coef_partial_kernel(
    KP P, const double *__restrict__ z, const double *__restrict__ y, const double *__restrict__ v, int G,
    double *__restrict__ cpart)
{
    constexpr int W = kBlock / 64, CH = kCoefChunk, LD = CH + 2;  // LD: row stride, spreads LDS banks
    constexpr int Q = kBlock / CH;                               // staging parts (lanes per node)
    constexpr int HR = 16 * MB / Q, HC = 16 * NBK / Q;           // rows and columns per part
    static_assert(kBlock % CH == 0 && CH % 64 == 0 && (16 % Q) == 0, "whole waves per staging part");
    // staging: [sin X | U] (16 NBK rows), raw X (16 MB rows), y (16 MB rows);
    // MIXED: raw V_X (16 MB rows) after y
    constexpr int STAGE = (16 * NBK + (MIXED ? 48 : 32) * MB) * LD, RED = W * MB * NBK * 256;
    __shared__ double sh[STAGE > RED ? STAGE : RED];  // staging area, then the block sums
    __shared__ double gs[W][HR];
    double(*Vl)[LD] = reinterpret_cast<double(*)[LD]>(sh);
    double(*Xl)[LD] = reinterpret_cast<double(*)[LD]>(sh + 16 * NBK * LD);
    double(*Yl)[LD] = reinterpret_cast<double(*)[LD]>(sh + (16 * NBK + 16 * MB) * LD);
    double(*Wl)[LD] = reinterpret_cast<double(*)[LD]>(sh + (16 * NBK + 32 * MB) * LD);
    const int n = P.n, m = P.m, ncol = n + m + 1;
    // w and h are the same across a wave: readfirstlane lets the compiler
    // keep what derives from them (row and column pointers) in scalar
    // registers
    const int t = threadIdx.x, lane = t & 63, w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int slot = t % CH, h = __builtin_amdgcn_readfirstlane(t / CH);  // staging: node slot, part
    const int j16 = lane & 15, kq = lane >> 4;
    const int64_t N = P.N, N1 = P.N1, NU = P.NU;
    const bool euler = P.scheme != 0;
    d4 acc[MB][NBK];
#pragma unroll
    for (int mb = 0; mb < MB; mb++)
#pragma unroll
        for (int cb = 0; cb < NBK; cb++) acc[mb][cb] = d4{0.0, 0.0, 0.0, 0.0};
    double gam[HR];
#pragma unroll
    for (int rr = 0; rr < HR; rr++) gam[rr] = 0.0;
    // Every load is unconditional, from an index clamped into its row, and
    // all are issued before the first LDS store, so that they are in flight
    // together; values past a row's end (and the last chunk's tail) are
    // scaled to 0 when stored (a multiply, not a select, which the compiler
    // would turn into a branch per load).  The rows of y are staged shifted
    // by one slot: Yl[r][s + 1] = y_{r, base + s} (0 from node N on) and
    // Yl[r][0] = y_{r, base - 1}, so that yt = Yl[r][s + 1] + Yl[r][s] for
    // the trapezoid.
    double xv[HC], vv[MIXED ? HC : 1], yv[HR], hv[HR];
    // Each load is a uniform row pointer at the chunk's first node (or at
    // the row's start when the row ends before the chunk) plus a 32-bit lane
    // offset clamped to the row's last node, so that no per-lane 64-bit
    // address has to stay live across the chunk loop.
    auto row_load = [&](const double *src, int64_t last, int64_t b0) {
        const int64_t span = last - b0;  // lanes slot <= span hold nodes of the row
        const double *pb = span >= 0 ? src + b0 : src;
        const uint32_t lim = span >= 0 ? (uint32_t)(span < CH - 1 ? span : CH - 1) : 0u;
        return pb[(uint32_t)slot < lim ? (uint32_t)slot : lim];
    };
    auto issue = [&](int64_t b0) {
#pragma unroll
        for (int jj = 0; jj < HC; jj++) {
            const int c = Q * jj + h;
            const bool isx = c < n, isu = !isx && c < n + m;
            const int64_t last = isx ? N : isu ? NU - 1 : -1;
            if (MIXED) {
                // the state row itself (a column past the states reloads the
                // last state row, an L2 hit; its value is unused), and v's row
                xv[jj] = row_load(z + (isx ? c : n - 1) * N1, N, b0);
                vv[jj] = row_load(isx ? v + c * N1 : isu ? v + n * N1 + (c - n) * NU : v, last, b0);
            } else {
                xv[jj] = row_load(isx ? z + c * N1 : isu ? z + n * N1 + (c - n) * NU : z, last, b0);
            }
        }
        const int64_t rspan = N - 1 - b0;  // lanes slot <= rspan hold nodes k < N
        const uint32_t rlim = rspan >= 0 ? (uint32_t)(rspan < CH - 1 ? rspan : CH - 1) : 0u;
        const uint32_t ri = (uint32_t)slot < rlim ? (uint32_t)slot : rlim;
#pragma unroll
        for (int rr = 0; rr < HR; rr++) {
            const int r = HR * h + rr;
            const double *yi = y + (int64_t)(r < n ? r : 0) * N;
            yv[rr] = (rspan >= 0 ? yi + b0 : yi)[ri];
            hv[rr] = yi[b0 >= 1 ? b0 - 1 : 0];
        }
    };
    auto stage = [&](int64_t b0) {
        const int64_t k = b0 + slot;
#pragma unroll
        for (int jj = 0; jj < HC; jj++) {
            const int c = Q * jj + h;
            const int64_t last = c < n ? N : c < n + m ? NU - 1 : -1;
            const double live = k <= last ? 1.0 : 0.0;
            if (MIXED) {
                const double x = xv[jj] * live, d = vv[jj] * live;
                if (c < n) {
                    Xl[c][slot] = x;
                    Wl[c][slot] = d;
                    Vl[c][slot] = cos(x) * d;
                } else {
                    Vl[c][slot] = d;
                }
            } else {
                const double x = xv[jj] * live;
                if (c < n) {
                    Xl[c][slot] = x;
                    Vl[c][slot] = sin(x);
                } else {
                    Vl[c][slot] = x;
                }
            }
        }
        const double fr = k < N ? 1.0 : 0.0, fh = b0 >= 1 ? 1.0 : 0.0;
#pragma unroll
        for (int rr = 0; rr < HR; rr++) {
            const int r = HR * h + rr;
            const double live = r < n ? 1.0 : 0.0;
            Yl[r][slot + 1] = yv[rr] * (fr * live);
            if (slot == 0) Yl[r][0] = hv[rr] * (fh * live);
        }
    };
    const double fl = euler ? 0.0 : 1.0;  // weight of the left neighbour
    for (int64_t base = (int64_t)blockIdx.x * CH; base <= N; base += (int64_t)G * CH) {
        issue(base);
        asm volatile("" ::: "memory");  // every load issued before the first store
        stage(base);
        __syncthreads();
        // gamma terms X_i X_p(i) yt_i of this lane's node
#pragma unroll
        for (int rr = 0; rr < HR; rr++) {
            const int i = HR * h + rr;
            if (i < n) {
                const int p = (i + 1 == n) ? 0 : i + 1;
                const double yt = __builtin_fma(fl, Yl[i][slot], Yl[i][slot + 1]);
                const double pr = MIXED ? __builtin_fma(Wl[i][slot], Xl[p][slot], Xl[i][slot] * Wl[p][slot])
                                        : Xl[i][slot] * Xl[p][slot];
                gam[rr] = __builtin_fma(yt, pr, gam[rr]);
            }
        }
        // the contraction
#pragma unroll 2
        for (int st = 0; st < CH / (4 * W); st++) {
            const int s = w * (CH / W) + 4 * st + kq;
            double a[MB];
#pragma unroll
            for (int mb = 0; mb < MB; mb++)
                a[mb] = __builtin_fma(fl, Yl[mb * 16 + j16][s], Yl[mb * 16 + j16][s + 1]);
#pragma unroll
            for (int cb = 0; cb < NBK; cb++) {
                const double b = Vl[cb * 16 + j16][s];
#pragma unroll
                for (int mb = 0; mb < MB; mb++)
                    acc[mb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mb], b, acc[mb][cb], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // D[i][j] of a block sits in lane 16 (i mod 4) + j, element i / 4
    double(*red)[MB][NBK][256] = reinterpret_cast<double(*)[MB][NBK][256]>(sh);
#pragma unroll
    for (int mb = 0; mb < MB; mb++)
#pragma unroll
        for (int cb = 0; cb < NBK; cb++)
#pragma unroll
            for (int r = 0; r < 4; r++) red[w][mb][cb][(4 * r + kq) * 16 + j16] = acc[mb][cb][r];
#pragma unroll
    for (int rr = 0; rr < HR; rr++) {
        if (HR * h + rr < n) {
            const double v = wave_sum(gam[rr]);
            if (lane == 0) gs[w][rr] = v;
        }
    }
    __syncthreads();
    double *out = cpart + (int64_t)blockIdx.x * n * ncol;
#pragma unroll
    for (int mb = 0; mb < MB; mb++)
#pragma unroll
        for (int cb = 0; cb < NBK; cb++) {
            const int i = mb * 16 + (t >> 4), col = cb * 16 + (t & 15);
            if (i >= n || col >= n + m) continue;
            double sum = red[0][mb][cb][t];
#pragma unroll
            for (int v = 1; v < W; v++) sum += red[v][mb][cb][t];
            out[i * ncol + col] = sum;
        }
    if (t < n) {
        constexpr int WP = W / Q;  // waves per staging part
        const int hh = t / HR, rr = t - hh * HR;
        double sum = gs[WP * hh][rr];
#pragma unroll
        for (int v = 1; v < WP; v++) sum += gs[WP * hh + v][rr];
        out[t * ncol + n + m] = sum;
    }
}

// Pass 2: one workgroup per coefficient; lane b < G holds workgroup b's
// partial and a fixed-shape tree adds them.
__global__ __launch_bounds__(kBlock) void coef_final_kernel(KP P, const double *__restrict__ cpart,
                                                            int G, double *__restrict__ gA,
                                                            double *__restrict__ gB,
                                                            double *__restrict__ gg)
{
    const int n = P.n, m = P.m, ncol = n + m + 1, nc = n * ncol;
    const int idx = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < G; b += kBlock) s += cpart[(int64_t)b * nc + idx];
    s = block_sum<kBlock>(s);
    if (threadIdx.x != 0) return;
    const double val = -(P.scheme != 0 ? P.h : P.hh) * s;
    const int i = idx / ncol, col = idx - i * ncol;
    if (col < n) gA[i * n + col] = val;
    else if (col < n + m) gB[i * m + (col - n)] = val;
    else gg[i] = val;
}

// ---------------------------------------------------------------------------
// Adjoint of the coefficient gradient: for cotangents t = (tA, tB, tg) of
// (dL/dA, dL/dB, dL/dgamma), the gradients in z and in y of t . dL/dtheta.
// The defects are linear in theta, so t . dL/dtheta = sum_ik y_ik D_ik, D
// being the defects' theta part with theta := t:
//   Ft_i(k) = sum_j tA_ij sin X_jk + sum_l tB_il U_lk + tg_i X_ik X_p(i)k,
//   D_ik    = -al Ft_i(k) - be Ft_i(k+1)   ((al, be) = (hh, hh) or (h, 0)).
// The y-gradient is D on the defect rows and 0 on the boundary rows; the
// z-gradient is the coefficient part of J^T y with theta := t:
//   at X_jk  -wF (cos X_jk (tA^T yt)_j + yt_j tg_j X_p(j)k + yt_q tg_q X_qk),
//   at U_lk  -wF (tB^T yt)_l,
// q = (j-1) mod n being the row whose bilinear partner is j.  Chunks of B
// nodes close B-1 intervals, as in the defect kernel: lane k publishes
// Ft(k) in LDS for lane k-1, and node k's z-entries are written by the chunk
// in which it is not the overlap node.  Every workgroup copies t from the
// caller's row-major arrays into zero-padded columns in LDS (the same region
// later holds the exchange), so the call reads no coefficients of the handle.
// ---------------------------------------------------------------------------
template <int NB>
__global__ __launch_bounds__(kBlock) void coef_adjoint_kernel(KP P, const double *__restrict__ z,
                                                              const double *__restrict__ y,
                                                              const double *__restrict__ tA,
                                                              const double *__restrict__ tB,
                                                              const double *__restrict__ tg,
                                                              double *__restrict__ gz,
                                                              double *__restrict__ gy)
{
    // columns: tA's n (of NB rows), then tB's m (kLd slots), then tg
    constexpr int kCoef = (NB + kLd + 1) * NB, kExch = NB * kBlock;
    __shared__ double lds[kCoef > kExch ? kCoef : kExch];
    const double *cA = lds, *cB = lds + NB * NB, *cg = lds + (NB + kLd) * NB;
    const int tid = threadIdx.x;
    const int n = P.n, m = P.m;
    const int64_t N = P.N, N1 = P.N1, NU = P.NU;
    const int64_t k = (int64_t)blockIdx.x * (kBlock - 1) + tid;
    const bool live = k <= N;
    const bool euler = P.scheme != 0;
    const double wF = euler ? P.h : P.hh;
    // The node's state and multiplier loads come first, at clamped indices
    // (every lane issues them unconditionally; a lane past node N computes
    // values it never stores), so that the staging of t below overlaps their
    // latency.  (Loading the controls here too doubled the registers.)
    const int64_t kc = live ? k : N;
    const int64_t kr = kc < N ? kc : N - 1, kl = kc >= 1 ? kc - 1 : 0;
    double x[NB], yt[NB], Ft[NB];
#pragma unroll
    for (int i = 0; i < NB; i++) {
        x[i] = yt[i] = Ft[i] = 0.0;
        if (i < n) {
            x[i] = z[i * N1 + kc];
            const double yr = y[i * N + kr], yl = y[i * N + kl];
            yt[i] = (kc < N ? yr : 0.0) + (euler || kc < 1 ? 0.0 : yl);
        }
    }
    for (int e = tid; e < kCoef; e += kBlock) {
        const int c = e / NB, i = e - c * NB;  // column c, row i
        double v = 0.0;
        if (i < n) {
            if (c < NB) v = c < n ? tA[i * n + c] : 0.0;
            else if (c < NB + kLd) v = c - NB < m ? tB[i * m + (c - NB)] : 0.0;
            else v = tg[i];
        }
        lds[e] = v;
    }
    if (gy && blockIdx.x == 0 && tid < P.nb) gy[(int64_t)n * N + tid] = 0.0;  // boundary rows
    __syncthreads();
    if (live) {
        if (gz && (tid < kBlock - 1 || k == N)) {
            const double x_last = last_of<NB>(x, n), yt_last = last_of<NB>(yt, n);
#pragma unroll
            for (int j = 0; j < NB; j++) {
                if (j < n) {
                    double s = 0.0;
#pragma unroll
                    for (int i = 0; i < NB; i++) s = __builtin_fma(yt[i], cA[j * NB + i], s);
                    const double xn = (j + 1 < n) ? x[(j + 1) % NB] : x[0];
                    const int jm = (j == 0) ? n - 1 : j - 1;
                    const double xm = (j == 0) ? x_last : x[(j + NB - 1) % NB];
                    const double ym = (j == 0) ? yt_last : yt[(j + NB - 1) % NB];
                    const double G = cos(x[j]) * s + yt[j] * cg[j] * xn + ym * cg[jm] * xm;
                    gz[j * N1 + k] = -wF * G;
                }
            }
            if (k < NU) {
                for (int l = 0; l < m; l++) {
                    double s = 0.0;
#pragma unroll
                    for (int i = 0; i < NB; i++) s = __builtin_fma(yt[i], cB[l * NB + i], s);
                    gz[n * N1 + l * NU + k] = -wF * s;
                }
            }
        }
        if (gy && (!euler || k < N)) {
#pragma unroll
            for (int j = 0; j < NB; j++) {
                if (j < n) {
                    const double sx = sin(x[j]);
#pragma unroll
                    for (int i = 0; i < NB; i++) Ft[i] = __builtin_fma(cA[j * NB + i], sx, Ft[i]);
                }
            }
            if (k < NU) {
                const double *U = z + (int64_t)n * N1;
                for (int l = 0; l < m; l++) {
                    const double ul = U[l * NU + k];
#pragma unroll
                    for (int i = 0; i < NB; i++) Ft[i] = __builtin_fma(cB[l * NB + i], ul, Ft[i]);
                }
            }
#pragma unroll
            for (int i = 0; i < NB; i++) {
                if (i < n) {
                    const double xp = (i + 1 < n) ? x[(i + 1) % NB] : x[0];
                    Ft[i] = __builtin_fma(cg[i] * x[i], xp, Ft[i]);
                }
            }
        }
    }
    if (!gy) return;  // uniform: no barrier follows for any lane
    __syncthreads();  // every read of the coefficient columns is done
    if (!euler) {
#pragma unroll
        for (int i = 0; i < NB; i++)
            if (i < n) lds[i * kBlock + tid] = Ft[i];
    }
    __syncthreads();
    if (tid < kBlock - 1 && k < N) {
#pragma unroll
        for (int i = 0; i < NB; i++) {
            if (i < n) {
                const double v = euler ? -P.h * Ft[i] : -P.hh * (Ft[i] + lds[i * kBlock + tid + 1]);
                gy[i * N + k] = v;
            }
        }
    }
}

// Up to five device arrays scaled in place by one device double (the
// incoming gradient of a backward pass), in one launch over their
// concatenation; end[j] is the cumulative length through array j.
struct ScaleSegs {
    double *p[5];
    int64_t end[5];
    int count;
};

__global__ __launch_bounds__(kBlock) void scale_kernel(ScaleSegs s, const double *__restrict__ g)
{
    const int64_t total = s.end[s.count - 1];
    const double f = *g;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
        double *dst = s.p[0];
        int64_t off = i;
#pragma unroll
        for (int j = 1; j < 5; j++) {
            if (j < s.count && i >= s.end[j - 1]) {
                dst = s.p[j];
                off = i - s.end[j - 1];
            }
        }
        dst[off] *= f;
    }
}

int nb_of(int n) { return n <= 4 ? 4 : n <= 8 ? 8 : n <= 16 ? 16 : 32; }

// A coefficient update in one launch: the row-major copies of A, B and gamma
// and the padded columns AT, BT (kLd rows each, zero below row n), built from
// the caller's device arrays, on the caller's stream (asynchronous).
__global__ __launch_bounds__(kBlock) void set_coefficients_kernel(int n, int m, const double *__restrict__ A,
                                                                  const double *__restrict__ B,
                                                                  const double *__restrict__ gam,
                                                                  double *__restrict__ hA, double *__restrict__ hB,
                                                                  double *__restrict__ hgam,
                                                                  double *__restrict__ AT,
                                                                  double *__restrict__ BT)
{
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e < (n + m) * kLd) {
        const int c = e / kLd, i = e % kLd;
        if (c < n) AT[e] = i < n ? A[i * n + c] : 0.0;
        else BT[e - n * kLd] = i < n ? B[i * m + (c - n)] : 0.0;
    }
    if (e < n * n) hA[e] = A[e];
    if (e < n * m) hB[e] = B[e];
    if (e < n) hgam[e] = gam[e];
}

}  // namespace

// The allocation-free coefficient gradient keeps its per-workgroup partial
// sums in this array instead of the handle's workspace.  Each device holds
// its own copy (for the life of the process); host code never passes the
// array's name to a kernel, only the device address that
// hipGetSymbolAddress returns on that device.
static __device__ __align__(256) double scratch[OCP_NOALLOC_SCRATCH];

namespace {
std::mutex scratch_mu;
std::vector<double *> scratch_addr;  // by device ordinal; null until looked up
}  // namespace

double *noalloc_scratch(int device)
{
    if (device < 0) return nullptr;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if ((size_t)device >= scratch_addr.size()) scratch_addr.resize((size_t)device + 1, nullptr);
    if (!scratch_addr[device]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess || cur != device) {
            (void)hipGetLastError();
            return nullptr;
        }
        void *addr = nullptr;
        if (hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch)) != hipSuccess || !addr) {
            (void)hipGetLastError();  // leave no sticky error for the next launch check
            return nullptr;
        }
        scratch_addr[device] = static_cast<double *>(addr);
    }
    return scratch_addr[device];
}

static int launch_coef_grad(const ocp_problem *p, const double *z, const double *y, const double *v, double *gA,
                            double *gB, double *ggamma, double *cpart, hipStream_t stream, const char *fn);

#define OCP_DISPATCH_NB(n, KERNEL, grid, ...)                                                   \
    do {                                                                                        \
        switch (nb_of(n)) {                                                                     \
        case 4: hipLaunchKernelGGL(KERNEL<4>, grid, dim3(kBlock), 0, __VA_ARGS__); break;      \
        case 8: hipLaunchKernelGGL(KERNEL<8>, grid, dim3(kBlock), 0, __VA_ARGS__); break;      \
        case 16: hipLaunchKernelGGL(KERNEL<16>, grid, dim3(kBlock), 0, __VA_ARGS__); break;    \
        default: hipLaunchKernelGGL(KERNEL<32>, grid, dim3(kBlock), 0, __VA_ARGS__); break;    \
        }                                                                                       \
    } while (0)

extern "C" {

int ocp_set_coefficients(ocp_problem *p, const double *A, const double *B, const double *gamma,
                         hipStream_t stream)
{
    clear_error();
    if (int rc = check_handle(p, "ocp_set_coefficients")) return rc;
    if (p->model != 0)
        return fail(OCP_ERR_ARG, "ocp_set_coefficients: the handle's model has no coefficients");
    if (!A || !gamma || (p->d.m > 0 && !B)) return fail(OCP_ERR_ARG, "ocp_set_coefficients: NULL array");
    const int n = p->d.n, m = p->d.m;
    const int64_t work = std::max<int64_t>((int64_t)(n + m) * kLd, (int64_t)n * n);
    hipLaunchKernelGGL(set_coefficients_kernel, dim3(blocks_for(work, kBlock)), dim3(kBlock), 0, stream, n, m, A,
                       B, gamma, const_cast<double *>(p->kp.A), const_cast<double *>(p->kp.B),
                       const_cast<double *>(p->kp.gam), const_cast<double *>(p->kp.AT),
                       const_cast<double *>(p->kp.BT));
    return check_launch("ocp_set_coefficients");
}

int ocp_eval_lagrangian(const ocp_problem *p, const double *z, const double *y, double sigma,
                        double *L, hipStream_t stream)
{
    clear_error();
    if (int rc = check_handle(p, "ocp_eval_lagrangian")) return rc;
    if (!z || !y || !L) return fail(OCP_ERR_ARG, "ocp_eval_lagrangian: null array");
    if (!std::isfinite(sigma)) return fail(OCP_ERR_ARG, "ocp_eval_lagrangian: sigma is not finite");
    if (p->model == quad::kModel) return quad::eval_lagrangian(p, z, y, sigma, L, stream);
    const int nchunks = (int)blocks_for(p->d.N, kBlock - 1);
    const int g = std::min(nchunks, kObjBlocks);
    OCP_DISPATCH_NB(p->d.n, lag_partial_kernel, dim3(g), stream, p->kp, z, y, sigma, nchunks, p->partials);
    if (int rc = check_launch("ocp_eval_lagrangian")) return rc;
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(kBlock), 0, stream, p->partials, g, L);
    return check_launch("ocp_eval_lagrangian");
}

int ocp_eval_lag_grad(const ocp_problem *p, const double *z, const double *y, double sigma,
                      double *g, hipStream_t stream)
{
    clear_error();
    if (int rc = check_handle(p, "ocp_eval_lag_grad")) return rc;
    if (!z || !y || !g) return fail(OCP_ERR_ARG, "ocp_eval_lag_grad: null array");
    if (!std::isfinite(sigma)) return fail(OCP_ERR_ARG, "ocp_eval_lag_grad: sigma is not finite");
    if (p->model == quad::kModel) return quad::eval_lag_grad(p, z, y, sigma, g, stream);
    OCP_DISPATCH_NB(p->d.n, lag_grad_kernel, dim3(blocks_for(p->d.N1, kBlock)), stream, p->kp, z, y,
                    sigma, g);
    return check_launch("ocp_eval_lag_grad");
}

int ocp_eval_hvp(const ocp_problem *p, const double *z, const double *y, double sigma,
                 const double *v, double *out, hipStream_t stream)
{
    clear_error();
    if (int rc = check_handle(p, "ocp_eval_hvp")) return rc;
    if (!z || !y || !v || !out) return fail(OCP_ERR_ARG, "ocp_eval_hvp: null array");
    if (!std::isfinite(sigma)) return fail(OCP_ERR_ARG, "ocp_eval_hvp: sigma is not finite");
    if (p->model == quad::kModel) return quad::eval_hvp(p, z, y, sigma, v, out, stream);
    OCP_DISPATCH_NB(p->d.n, hvp_kernel, dim3(blocks_for(p->d.N1, kBlock)), stream, p->kp, z, y, sigma,
                    v, out);
    return check_launch("ocp_eval_hvp");
}

int ocp_eval_jvp(const ocp_problem *p, const double *z, const double *v, double *out,
                 hipStream_t stream)
{
    clear_error();
    if (int rc = check_handle(p, "ocp_eval_jvp")) return rc;
    if (!z || !v || !out) return fail(OCP_ERR_ARG, "ocp_eval_jvp: null array");
    if (p->model == quad::kModel) return quad::eval_jvp(p, z, v, out, stream);
    OCP_DISPATCH_NB(p->d.n, jvp_kernel, dim3(blocks_for(p->d.N, kBlock - 1)), stream, p->kp, z, v,
                    out);
    if (int rc = check_launch("ocp_eval_jvp")) return rc;
    if (p->d.nb > 0)
        hipLaunchKernelGGL(bnd_jvp_kernel, dim3(blocks_for(p->d.nb, kBlock)), dim3(kBlock), 0, stream,
                           p->kp, v, out);
    return check_launch("ocp_eval_jvp");
}

int ocp_eval_coef_grad(const ocp_problem *p, const double *z, const double *y, double *gA,
                       double *gB, double *ggamma, hipStream_t stream)
{
    clear_error();
    if (int rc = check_handle(p, "ocp_eval_coef_grad")) return rc;
    if (int rc = check_coefficients(p, "ocp_eval_coef_grad")) return rc;
    if (!z || !y || !gA || !ggamma || (p->d.m > 0 && !gB))
        return fail(OCP_ERR_ARG, "ocp_eval_coef_grad: null array");
    return launch_coef_grad(p, z, y, nullptr, gA, gB, ggamma, p->cpart, stream, "ocp_eval_coef_grad");
}

int ocp_eval_coef_mixed(const ocp_problem *p, const double *z, const double *y, const double *v, double *gA,
                        double *gB, double *ggamma, hipStream_t stream)
{
    clear_error();
    if (int rc = check_handle(p, "ocp_eval_coef_mixed")) return rc;
    if (int rc = check_coefficients(p, "ocp_eval_coef_mixed")) return rc;
    if (!z || !y || !v || !gA || !ggamma || (p->d.m > 0 && !gB))
        return fail(OCP_ERR_ARG, "ocp_eval_coef_mixed: null array");
    return launch_coef_grad(p, z, y, v, gA, gB, ggamma, p->cpart, stream, "ocp_eval_coef_mixed");
}

int ocp_eval_lagrangian_backward(const ocp_problem *p, const double *z, const double *y, double sigma,
                                 const double *gL, double *gz, double *gy, double *gA, double *gB, double *ggamma,
                                 hipStream_t stream)
{
    const char *fn = "ocp_eval_lagrangian_backward";
    clear_error();
    if (int rc = check_handle(p, fn)) return rc;
    if (!z || !y || !gL) return fail(OCP_ERR_ARG, std::string(fn) + ": null array");
    if (!std::isfinite(sigma)) return fail(OCP_ERR_ARG, std::string(fn) + ": sigma is not finite");
    const bool coef = gA || gB || ggamma;
    if (coef) {
        if (int rc = check_coefficients(p, fn)) return rc;
        if (!gA || !ggamma || (p->d.m > 0 && !gB))
            return fail(OCP_ERR_ARG, std::string(fn) + ": gA and ggamma (and gB when m > 0) go together");
    }
    if (!gz && !gy && !coef) return fail(OCP_ERR_ARG, std::string(fn) + ": no output");
    // the same kernels as the three separate calls, then one scale
    if (gz)
        if (int rc = ocp_eval_lag_grad(p, z, y, sigma, gz, stream)) return rc;
    if (gy)
        if (int rc = ocp_eval_cons(p, z, gy, stream)) return rc;
    if (coef)
        if (int rc = ocp_eval_coef_grad(p, z, y, gA, gB, ggamma, stream)) return rc;
    ScaleSegs segs{};
    int64_t total = 0;
    auto add = [&](double *ptr, int64_t len) {
        if (!ptr || len <= 0) return;
        total += len;
        segs.p[segs.count] = ptr;
        segs.end[segs.count++] = total;
    };
    const int64_t n = p->d.n, m = p->d.m;
    add(gz, p->d.nvar);
    add(gy, p->d.ncon);
    if (coef) {
        add(gA, n * n);
        add(gB, n * m);
        add(ggamma, n);
    }
    if (segs.count == 0) return OCP_OK;
    const unsigned grid = std::min<unsigned>(blocks_for(total, kBlock), 4096u);
    hipLaunchKernelGGL(scale_kernel, dim3(grid), dim3(kBlock), 0, stream, segs, gL);
    return check_launch(fn);
}

int ocp_eval_coef_adjoint(const ocp_problem *p, const double *z, const double *y, const double *tA,
                          const double *tB, const double *tgamma, double *gz, double *gy, hipStream_t stream)
{
    const char *fn = "ocp_eval_coef_adjoint";
    clear_error();
    if (int rc = check_handle(p, fn)) return rc;
    if (int rc = check_coefficients(p, fn)) return rc;
    if (!z || !y || !tA || !tgamma || (p->d.m > 0 && !tB)) return fail(OCP_ERR_ARG, std::string(fn) + ": null array");
    if (!gz && !gy) return fail(OCP_ERR_ARG, std::string(fn) + ": no output (gz and gy are both NULL)");
    OCP_DISPATCH_NB(p->d.n, coef_adjoint_kernel, dim3(blocks_for(p->d.N, kBlock - 1)), stream, p->kp, z, y, tA, tB,
                    tgamma, gz, gy);
    return check_launch(fn);
}

int ocp_eval_coef_grad_noalloc(const ocp_problem *p, const double *z, const double *y, double *gA,
                               double *gB, double *ggamma, hipStream_t stream)
{
    const char *fn = "ocp_eval_coef_grad_noalloc";
    clear_error();
    if (int rc = check_handle(p, fn)) return rc;
    if (int rc = check_coefficients(p, fn)) return rc;
    if (!z || !y || !gA || !ggamma || (p->d.m > 0 && !gB)) return fail(OCP_ERR_ARG, std::string(fn) + ": null array");
    const int64_t need = (int64_t)p->d.n * (p->d.n + p->d.m + 1) * coef_blocks(p->d.N1);
    if (need > OCP_NOALLOC_SCRATCH)
        return fail(OCP_ERR_ARG, std::string(fn) + ": the partial sums need " + std::to_string(need) +
                                     " doubles, more than the " + std::to_string(OCP_NOALLOC_SCRATCH) +
                                     " of the fixed scratch array");
    int dev = -1;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail("ocp_eval_coef_grad_noalloc: hipGetDevice", e);
    if (dev != p->device)
        return fail(OCP_ERR_ARG, std::string(fn) + ": the current device is not the handle's");
    double *ws = noalloc_scratch(dev);
    if (!ws) return fail(OCP_ERR_HIP, std::string(fn) + ": the scratch array's device address is unknown");
    return launch_coef_grad(p, z, y, nullptr, gA, gB, ggamma, ws, stream, fn);
}

}  // extern "C"

template <bool MIXED>
static void launch_coef_partial(const ocp_problem *p, const double *z, const double *y, const double *v, int G,
                                double *cpart, hipStream_t stream)
{
    const int n = p->d.n, m = p->d.m;
    // 16-row blocks of yt (n <= 32) and 16-column blocks of [sin X | U] (n + m <= 64)
    const int mb = (n + 15) / 16, nbk = (n + m + 15) / 16;
#define OCP_COEF_LAUNCH(MB_, NBK_)                                                                       \
    hipLaunchKernelGGL((coef_partial_kernel<MB_, NBK_, MIXED>), dim3(G), dim3(kBlock), 0, stream, p->kp, z, \
                       y, v, G, cpart)
    if (mb == 1) {
        if (nbk == 1) OCP_COEF_LAUNCH(1, 1);
        else if (nbk == 2) OCP_COEF_LAUNCH(1, 2);
        else OCP_COEF_LAUNCH(1, 3);
    } else {
        if (nbk == 2) OCP_COEF_LAUNCH(2, 2);
        else if (nbk == 3) OCP_COEF_LAUNCH(2, 3);
        else OCP_COEF_LAUNCH(2, 4);
    }
#undef OCP_COEF_LAUNCH
}

// v == nullptr: the coefficient gradient; otherwise its derivative along v.
static int launch_coef_grad(const ocp_problem *p, const double *z, const double *y, const double *v, double *gA,
                            double *gB, double *ggamma, double *cpart, hipStream_t stream, const char *fn)
{
    const int n = p->d.n, m = p->d.m, ncol = n + m + 1;
    const int G = coef_blocks(p->d.N1);
    if (v) launch_coef_partial<true>(p, z, y, v, G, cpart, stream);
    else launch_coef_partial<false>(p, z, y, nullptr, G, cpart, stream);
    if (int rc = check_launch(fn)) return rc;
    hipLaunchKernelGGL(coef_final_kernel, dim3(n * ncol), dim3(kBlock), 0, stream, p->kp, cpart, G,
                       gA, gB, ggamma);
    return check_launch(fn);
}
