// Quadrotor model (paper Appendix A, trapezoidal transcription of Sec. 5):
// HIP kernels for gfx950 and the handle constructor.  The evaluations keep
// the single-instance layout (structure of arrays, node index fastest, COO
// values slot-major) and the same entry points; only the pattern differs:
// 68 Jacobian entries per interval in 9 rows of 4 to 12 entries, and 23
// Hessian entries per node.  Everything is HBM-bound: no MFMA.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "ocp_device.h"
#include "ocp_problem.h"
#include "ocp_quad.h"
#include "ocp_quad_device.h"

using namespace ocp;
using namespace ocp::dev;
using namespace ocp::quad;

namespace {

struct QP {
    int N, N1, nb;
    double h, hh, g, r;
};

__device__ __forceinline__ double q_weight(const QP &P, int k) { return (k == 0 || k == P.N) ? P.hh : P.h; }

// Attitude and controls of node k: the only inputs of the dynamics'
// derivatives.
__device__ __forceinline__ void load_att(const QP &P, const double *__restrict__ z, int64_t k, double *a,
                                         double *u)
{
    const int64_t N1 = P.N1;
#pragma unroll
    for (int j = 0; j < 3; j++) a[j] = z[(6 + j) * N1 + k];
#pragma unroll
    for (int l = 0; l < 4; l++) u[l] = z[(9 + l) * N1 + k];
}

// ---------------------------------------------------------------------------
// Jacobian values.  2-D grid: blockIdx.y is the defect row i, blockIdx.x
// picks NPT intervals per lane.  Row i's 2 kSupLen[i] slots are stored as
// unit-stride runs across lanes (16-byte pairs for NPT = 2).  Rows 1, 3, 5,
// 6, 7, 8 need the attitude trigonometry of NPT + 1 nodes; rows 0, 2, 4 are
// constants.
// ---------------------------------------------------------------------------
template <int I, int NPT>
__device__ __forceinline__ void jac_row(const QP &P, const double *__restrict__ z, double *__restrict__ jac,
                                        int64_t k)
{
    constexpr bool kTrig = !(I == 0 || I == 2 || I == 4);
    constexpr int L = kSupLen[I];
    Trig t[NPT + 1];
    double u[NPT + 1][4];
    if constexpr (kTrig) {
#pragma unroll
        for (int j = 0; j <= NPT; j++) {
            double a[3];
            load_att(P, z, k + j, a, u[j]);
            t[j] = node_trig(a[0], a[1], a[2]);
        }
    } else {
#pragma unroll
        for (int j = 0; j <= NPT; j++) {
            t[j] = Trig{};
#pragma unroll
            for (int l = 0; l < 4; l++) u[j][l] = 0.0;
        }
    }
    const int64_t N = P.N;
#pragma unroll
    for (int p = 0; p < L; p++) {
        const int q = pair_index(I, p);
        const bool own = pair_is_own_state(I, p);
#pragma unroll
        for (int s = 0; s < 2; s++) {
            const double id = own ? (s ? 1.0 : -1.0) : 0.0;
            double v[NPT];
#pragma unroll
            for (int j = 0; j < NPT; j++) v[j] = id - P.hh * partial(q, t[j + s], u[j + s]);
            double *o = jac + (int64_t)(kRowSlot[I] + 2 * p + s) * N + k;
            if constexpr (NPT == 2) st_nt2(o, dbl2{v[0], v[1]});
            else st_nt(o, v[0]);
        }
    }
}

template <int NPT>
__global__ __launch_bounds__(kBlock) void quad_jac_kernel(QP P, const double *__restrict__ z,
                                                          double *__restrict__ jac)
{
    const int64_t k = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * NPT;
    if (k >= P.N) return;
    switch (blockIdx.y) {
    case 0: jac_row<0, NPT>(P, z, jac, k); break;
    case 1: jac_row<1, NPT>(P, z, jac, k); break;
    case 2: jac_row<2, NPT>(P, z, jac, k); break;
    case 3: jac_row<3, NPT>(P, z, jac, k); break;
    case 4: jac_row<4, NPT>(P, z, jac, k); break;
    case 5: jac_row<5, NPT>(P, z, jac, k); break;
    case 6: jac_row<6, NPT>(P, z, jac, k); break;
    case 7: jac_row<7, NPT>(P, z, jac, k); break;
    default: jac_row<8, NPT>(P, z, jac, k); break;
    }
}

// Boundary rows: one Jacobian entry 1.0 each, after the defect entries.
__global__ __launch_bounds__(kBlock) void quad_bnd_jac_kernel(QP P, double *__restrict__ jac)
{
    const int b = blockIdx.x * kBlock + threadIdx.x;
    if (b < P.nb) jac[(int64_t)kSlots * P.N + b] = 1.0;
}

// ---------------------------------------------------------------------------
// Hessian values, one lane per node: loads first (attitude, controls and the
// multipliers of the six nonlinear rows at intervals k-1 and k), then the 23
// entries as unit-stride stores.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void quad_hess_kernel(QP P, const double *__restrict__ z,
                                                           const double *__restrict__ y, double sigma,
                                                           double *__restrict__ hv)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k > P.N) return;
    const int64_t N = P.N, N1 = P.N1;
    double a[3], u[4], Y[kStates];
    load_att(P, z, k, a, u);
#pragma unroll
    for (int i = 0; i < kStates; i++) {
        if (i == 0 || i == 2 || i == 4) {  // linear rows: no curvature
            Y[i] = 0.0;
            continue;
        }
        double s = 0.0;
        if (k >= 1) s += y[i * N + k - 1];
        if (k < N) s += y[i * N + k];
        Y[i] = s;
    }
    const Trig t = node_trig(a[0], a[1], a[2]);
    double H[kHessNode];
    hess_values(t, u, Y, sigma * q_weight(P, (int)k), P.r, P.hh, H);
#pragma unroll
    // ordinary stores (23 slot rows of 8 bytes per lane), as for the
    // synthetic model's Hessian kernel: 66 -> 57 us at N = 1e6 in the step
    for (int s = 0; s < kHessNode; s++) hv[s * N1 + k] = H[s];
}

// ---------------------------------------------------------------------------
// Defects.  Workgroup b owns nodes [b (B-1), b (B-1) + B): every lane reads
// its node once, evaluates F there and leaves (x, F) in LDS; lane t < B-1
// then forms the defect of interval k = b (B-1) + t from its own node and
// its neighbour's.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void quad_cons_kernel(QP P, const double *__restrict__ z,
                                                           double *__restrict__ c)
{
    __shared__ double Xs[kStates][kBlock];
    __shared__ double Fs[kStates][kBlock];
    const int tid = threadIdx.x;
    const int64_t k = (int64_t)blockIdx.x * (kBlock - 1) + tid;
    const int64_t N = P.N, N1 = P.N1;
    double x[kStates], F[kStates];
    if (k <= N) {
        double u[4];
#pragma unroll
        for (int j = 0; j < kStates; j++) x[j] = z[j * N1 + k];
#pragma unroll
        for (int l = 0; l < 4; l++) u[l] = z[(9 + l) * N1 + k];
        rhs(x, u, P.g, F);
#pragma unroll
        for (int j = 0; j < kStates; j++) {
            Xs[j][tid] = x[j];
            Fs[j][tid] = F[j];
        }
    }
    __syncthreads();
    if (tid < kBlock - 1 && k < N) {
#pragma unroll
        for (int i = 0; i < kStates; i++)
            st_nt(c + i * N + k, (Xs[i][tid + 1] - x[i]) - P.hh * (F[i] + Fs[i][tid + 1]));
    }
}

// Boundary rows: the state itself (X_i0, then X_iN).
__global__ __launch_bounds__(kBlock) void quad_bnd_cons_kernel(QP P, const double *__restrict__ z,
                                                               double *__restrict__ c)
{
    const int b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= P.nb) return;
    const int64_t node = b < kStates ? 0 : P.N;
    c[(int64_t)kStates * P.N + b] = z[(int64_t)(b % kStates) * P.N1 + node];
}

// ---------------------------------------------------------------------------
// Objective and gradient.  Reference trajectory at t_k = k h: sin(2 pi t),
// 2 sin(4 pi t), 2 t for x1, x3, x5.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void refs(const QP &P, int64_t k, double *d)
{
    constexpr double kPi = 3.14159265358979323846;
    const double t = (double)k * P.h;
    d[0] = sin(2.0 * kPi * t);
    d[1] = 2.0 * sin(4.0 * kPi * t);
    d[2] = 2.0 * t;
}

__global__ __launch_bounds__(kBlock) void quad_obj_partial_kernel(QP P, const double *__restrict__ z,
                                                                  double *__restrict__ partials)
{
    const int64_t N1 = P.N1;
    double acc = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < N1; k += (int64_t)gridDim.x * kBlock) {
        double d[3];
        refs(P, k, d);
        const double e0 = z[k] - d[0], e2 = z[2 * N1 + k] - d[1], e4 = z[4 * N1 + k] - d[2];
        double L = e0 * e0 + e2 * e2 + e4 * e4;
#pragma unroll
        for (int j = 6; j < 9; j++) {
            const double v = z[j * N1 + k];
            L += v * v;
        }
        double uu = 0.0;
#pragma unroll
        for (int l = 0; l < 4; l++) {
            const double v = z[(9 + l) * N1 + k];
            uu += v * v;
        }
        L += P.r * uu;
        acc += q_weight(P, (int)k) * (0.5 * L);
    }
    const double t = block_sum<kBlock>(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ __launch_bounds__(kBlock) void quad_obj_final_kernel(const double *__restrict__ partials, int count,
                                                                double *__restrict__ obj)
{
    double acc = 0.0;
    for (int i = threadIdx.x; i < count; i += kBlock) acc += partials[i];
    const double t = block_sum<kBlock>(acc);
    if (threadIdx.x == 0) obj[0] = t;
}

__global__ __launch_bounds__(kBlock) void quad_grad_kernel(QP P, const double *__restrict__ z,
                                                           double *__restrict__ g)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k > P.N) return;
    const int64_t N1 = P.N1;
    const double w = q_weight(P, (int)k);
    double d[3];
    refs(P, k, d);
    double v[kVars];
#pragma unroll
    for (int q = 0; q < 3; q++) {
        v[2 * q] = w * (z[2 * q * N1 + k] - d[q]);
        v[2 * q + 1] = 0.0;
    }
#pragma unroll
    for (int j = 6; j < 9; j++) v[j] = w * z[j * N1 + k];
#pragma unroll
    for (int l = 0; l < 4; l++) v[9 + l] = w * P.r * z[(9 + l) * N1 + k];
#pragma unroll
    for (int j = 0; j < kVars; j++) st_nt(g + j * N1 + k, v[j]);
}

// ---------------------------------------------------------------------------
// KKT assembly, table-driven by row group.  Group g < 9 is defect row i: its
// N KKT rows nvar + i N + k hold the row's Jacobian slots then a diagonal
// (reg, or zero).  Group 9 + v is variable v: its N+1 KKT rows v (N+1) + k
// hold the Hessian entries of v's row, the last being the diagonal (+ reg).
// A workgroup owns KT consecutive rows of one group; their CSR range
// [base, base + ext) is staged in LDS from the slot maps and written with
// contiguous stores when the tile's values cover it exactly, as the
// closed-form maps do; otherwise the tile stores each value directly, so any
// injective slot map gives the same result.  Blocks after the groups handle
// the boundary rows.
// ---------------------------------------------------------------------------
constexpr int kGroups = kStates + kVars;
constexpr int kTileCap = 2048;  // values staged per workgroup (16 KiB of LDS)

struct AsmGroups {
    int tile0[kGroups + 1];  // first workgroup of each group; tile0[kGroups] = first boundary workgroup
    int KT[kGroups];         // rows per tile (even)
};

__global__ __launch_bounds__(kBlock) void quad_assemble_kernel(
    QP P, AsmGroups G, int nnzk, bool vec_j, bool vec_h, const int32_t *__restrict__ perm_j,
    const int32_t *__restrict__ perm_h, const int32_t *__restrict__ rowptr, const double *__restrict__ jv,
    const double *__restrict__ hv, const double *__restrict__ reg, double *__restrict__ kkt)
{
    __shared__ double tile[kTileCap];
    __shared__ int filled;
    const int64_t N = P.N, N1 = P.N1;
    const int64_t nvar = (int64_t)kVars * N1;
    const int bid = blockIdx.x;
    if (bid >= G.tile0[kGroups]) {
        const int b = (bid - G.tile0[kGroups]) * kBlock + threadIdx.x;
        if (b >= P.nb) return;
        const int64_t e = (int64_t)kSlots * N + b;
        const uint32_t q = (uint32_t)perm_j[e];
        if (q < (uint32_t)nnzk) kkt[q] = jv[e];
        const int64_t d = nvar + (int64_t)kStates * N + b;
        const uint32_t dq = (uint32_t)(rowptr[d + 1] - 1);
        if (dq < (uint32_t)nnzk) kkt[dq] = reg ? reg[d] : 0.0;
        return;
    }
    int g = 0;
    while (g + 1 < kGroups && bid >= G.tile0[g + 1]) g++;
    const bool is_h = g >= kStates;
    const int gi = is_h ? g - kStates : g;
    const int first = is_h ? kHessFirst[gi] : kRowSlot[gi];
    const int count = is_h ? kHessFirst[gi + 1] - first : kRowSlot[gi + 1] - first;
    const int64_t rows = is_h ? N1 : N;
    const int64_t stride = rows;
    const int KT = G.KT[g];
    const int64_t k0 = (int64_t)(bid - G.tile0[g]) * KT;
    const int kn = (int)std::min<int64_t>(KT, rows - k0);
    const int64_t d0 = is_h ? gi * N1 + k0 : nvar + gi * N + k0;  // first KKT row of the tile
    const int32_t *perm = is_h ? perm_h : perm_j;
    const double *src = is_h ? hv : jv;
    const bool vec = is_h ? vec_h : vec_j;
    const int32_t base = rowptr[d0];
    const int32_t ext = (int32_t)((uint32_t)rowptr[d0 + kn] - (uint32_t)base);
    // stage only a range inside [0, nnzk) (a corrupt rowptr falls back to
    // bounds-checked direct stores)
    const bool staged = ext >= 0 && ext <= kTileCap && base >= 0 && (int64_t)base + ext <= nnzk;
    if (threadIdx.x == 0) filled = 0;
    __syncthreads();
    const int half = KT / 2;

    // Visit every (slot, value) of the tile; `put` decides where it goes.
    auto visit = [&](auto put) {
        for (int w = threadIdx.x; w < count * half; w += kBlock) {
            const int t = w / half;
            const int kl = 2 * (w - t * half);
            if (kl >= kn) continue;
            const int64_t e = (int64_t)(first + t) * stride + k0 + kl;
            const bool diag = is_h && t == count - 1;
            const bool two = kl + 1 < kn;
            double v0, v1 = 0.0;
            int32_t q0, q1 = 0;
            if (vec && two && (e & 1) == 0) {
                const dbl2 v = __builtin_nontemporal_load(reinterpret_cast<const dbl2 *>(src + e));
                const int2v q = __builtin_nontemporal_load(reinterpret_cast<const int2v *>(perm + e));
                v0 = v.x;
                v1 = v.y;
                q0 = q.x;
                q1 = q.y;
            } else {
                v0 = src[e];
                q0 = perm[e];
                if (two) {
                    v1 = src[e + 1];
                    q1 = perm[e + 1];
                }
            }
            if (diag && reg) {
                v0 += reg[d0 + kl];
                if (two) v1 += reg[d0 + kl + 1];
            }
            put(q0, v0);
            if (two) put(q1, v1);
        }
        if (!is_h)
            for (int x = threadIdx.x; x < kn; x += kBlock) {
                const int64_t d = d0 + x;
                put(rowptr[d + 1] - 1, reg ? reg[d] : 0.0);
            }
    };
    int mine = 0;
    visit([&](int32_t q, double v) {
        const uint32_t loc = (uint32_t)q - (uint32_t)base;
        if (staged && loc < (uint32_t)ext) {
            tile[loc] = v;
            mine++;
        } else if ((uint32_t)q < (uint32_t)nnzk) {
            kkt[q] = v;
        }
    });
    if (mine) atomicAdd(&filled, mine);
    __syncthreads();
    if (!staged) return;
    if (filled == ext) {
        double *out = kkt + base;
        for (int x = threadIdx.x; x < ext; x += kBlock) st_nt(out + x, tile[x]);
    } else {
        visit([&](int32_t q, double v) {
            if ((uint32_t)q < (uint32_t)nnzk) kkt[q] = v;
        });
    }
}

// ---------------------------------------------------------------------------
// Lagrangian derivatives, L = sigma f + y^T c (the same set as the synthetic
// family's, without the coefficient gradient: the model has no coefficient
// arrays).  With the node multiplier yt_i = y_{i,k-1} [k >= 1] + y_ik [k < N]
// and the right-hand side's partials dF_i/dv on the Jacobian support:
//   grad_z L at (v, k) = sigma df/dv + (y_{v,k-1} - y_vk) [v state]
//                        - hh sum_i yt_i dF_i/dv (k) + boundary multipliers
//   (J v)_ik = (v_{i,k+1} - v_ik) - hh (D_i(k) + D_i(k+1)),
//              D_i = sum over the support of dF_i/dv v
//   (H v) at node k: the node's 23 Hessian entries (lower triangle) times v.
// ---------------------------------------------------------------------------

// Node k's variables (states then controls) from a vector in the layout of z.
__device__ __forceinline__ void load_node(const QP &P, const double *__restrict__ z, int64_t k, double *v)
{
#pragma unroll
    for (int j = 0; j < kVars; j++) v[j] = z[j * (int64_t)P.N1 + k];
}

// sigma times the running cost's gradient at node k (weight included).
__device__ __forceinline__ void cost_grad(const QP &P, int64_t k, const double *x, double sw, double *g)
{
    double d[3];
    refs(P, k, d);
#pragma unroll
    for (int q = 0; q < 3; q++) {
        g[2 * q] = sw * (x[2 * q] - d[q]);
        g[2 * q + 1] = 0.0;
    }
#pragma unroll
    for (int j = 6; j < 9; j++) g[j] = sw * x[j];
#pragma unroll
    for (int l = 0; l < 4; l++) g[9 + l] = sw * P.r * x[9 + l];
}

// D_i = sum over row i's support of dF_i/dv v (all nine rows).
__device__ __forceinline__ void dir_deriv(const Trig &t, const double *u, const double *v, double *D)
{
#pragma unroll
    for (int i = 0; i < kStates; i++) {
        double s = 0.0;
#pragma unroll
        for (int p = 0; p < kSupLen[i]; p++) s += partial(pair_index(i, p), t, u) * v[kSup[i][p]];
        D[i] = s;
    }
}

__global__ __launch_bounds__(kBlock) void quad_lag_partial_kernel(QP P, const double *__restrict__ z,
                                                                  const double *__restrict__ y, double sigma,
                                                                  int nchunks, double *__restrict__ partials)
{
    __shared__ double Ms[kStates][kBlock];
    const int tid = threadIdx.x;
    const int64_t N = P.N;
    double acc = 0.0;
    for (int ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int64_t k = (int64_t)ch * (kBlock - 1) + tid;
        double x[kVars], F[kStates];
        if (k <= N) {
            load_node(P, z, k, x);
            rhs(x, x + kStates, P.g, F);
#pragma unroll
            for (int i = 0; i < kStates; i++) Ms[i][tid] = x[i] - P.hh * F[i];
            if (tid < kBlock - 1 || k == N) {
                double d[3];
                refs(P, k, d);
                const double e0 = x[0] - d[0], e2 = x[2] - d[1], e4 = x[4] - d[2];
                double Lk = e0 * e0 + e2 * e2 + e4 * e4 + x[6] * x[6] + x[7] * x[7] + x[8] * x[8];
                double uu = 0.0;
#pragma unroll
                for (int l = 0; l < 4; l++) uu += x[9 + l] * x[9 + l];
                Lk += P.r * uu;
                acc += sigma * (q_weight(P, (int)k) * (0.5 * Lk));
                const double *yb = y + (int64_t)kStates * N;  // boundary-row multipliers
                if (P.nb >= kStates && k == 0) {
#pragma unroll
                    for (int i = 0; i < kStates; i++) acc += yb[i] * x[i];
                }
                if (P.nb >= 2 * kStates && k == N) {
#pragma unroll
                    for (int i = 0; i < kStates; i++) acc += yb[kStates + i] * x[i];
                }
            }
        }
        __syncthreads();
        if (tid < kBlock - 1 && k < N) {
#pragma unroll
            for (int i = 0; i < kStates; i++)
                acc += y[i * N + k] * (Ms[i][tid + 1] - (x[i] + P.hh * F[i]));
        }
        __syncthreads();
    }
    const double t = block_sum<kBlock>(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ __launch_bounds__(kBlock) void quad_lag_grad_kernel(QP P, const double *__restrict__ z,
                                                               const double *__restrict__ y, double sigma,
                                                               double *__restrict__ g)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k > P.N) return;
    const int64_t N = P.N, N1 = P.N1;
    double x[kVars], yl[kStates], yr[kStates], G[kVars];
    load_node(P, z, k, x);
#pragma unroll
    for (int i = 0; i < kStates; i++) {
        yl[i] = k >= 1 ? y[i * N + k - 1] : 0.0;
        yr[i] = k < N ? y[i * N + k] : 0.0;
    }
    cost_grad(P, k, x, sigma * q_weight(P, (int)k), G);
#pragma unroll
    for (int j = 0; j < kStates; j++) G[j] += yl[j] - yr[j];
    const Trig t = node_trig(x[6], x[7], x[8]);
#pragma unroll
    for (int i = 0; i < kStates; i++) {
        const double yt = yl[i] + yr[i];
#pragma unroll
        for (int p = 0; p < kSupLen[i]; p++)
            G[kSup[i][p]] -= P.hh * (yt * partial(pair_index(i, p), t, x + kStates));
    }
    if (P.nb >= kStates && k == 0) {
#pragma unroll
        for (int j = 0; j < kStates; j++) G[j] += y[kStates * N + j];
    }
    if (P.nb >= 2 * kStates && k == N) {
#pragma unroll
        for (int j = 0; j < kStates; j++) G[j] += y[kStates * N + kStates + j];
    }
#pragma unroll
    for (int j = 0; j < kVars; j++) st_nt(g + j * N1 + k, G[j]);
}

__global__ __launch_bounds__(kBlock) void quad_hvp_kernel(QP P, const double *__restrict__ z,
                                                          const double *__restrict__ y, double sigma,
                                                          const double *__restrict__ v,
                                                          double *__restrict__ out)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k > P.N) return;
    const int64_t N = P.N, N1 = P.N1;
    double a[3], u[4], Y[kStates], vv[kVars];
    load_att(P, z, k, a, u);
    load_node(P, v, k, vv);
#pragma unroll
    for (int i = 0; i < kStates; i++) {
        if (i == 0 || i == 2 || i == 4) {  // linear rows: no curvature
            Y[i] = 0.0;
            continue;
        }
        double s = 0.0;
        if (k >= 1) s += y[i * N + k - 1];
        if (k < N) s += y[i * N + k];
        Y[i] = s;
    }
    const Trig t = node_trig(a[0], a[1], a[2]);
    double H[kHessNode];
    hess_values(t, u, Y, sigma * q_weight(P, (int)k), P.r, P.hh, H);
    double o[kVars];
#pragma unroll
    for (int j = 0; j < kVars; j++) o[j] = 0.0;
#pragma unroll
    for (int s = 0; s < kHessNode; s++) {
        const int r = kHessRow[s], c = kHessCol[s];
        o[r] += H[s] * vv[c];
        if (r != c) o[c] += H[s] * vv[r];
    }
#pragma unroll
    for (int j = 0; j < kVars; j++) st_nt(out + j * N1 + k, o[j]);
}

__global__ __launch_bounds__(kBlock) void quad_jvp_kernel(QP P, const double *__restrict__ z,
                                                          const double *__restrict__ v,
                                                          double *__restrict__ out)
{
    __shared__ double Ms[kStates][kBlock];
    const int tid = threadIdx.x;
    const int64_t k = (int64_t)blockIdx.x * (kBlock - 1) + tid;
    const int64_t N = P.N;
    double Pk[kStates];
    if (k <= N) {
        double a[3], u[4], vv[kVars], D[kStates];
        load_att(P, z, k, a, u);
        load_node(P, v, k, vv);
        const Trig t = node_trig(a[0], a[1], a[2]);
        dir_deriv(t, u, vv, D);
#pragma unroll
        for (int i = 0; i < kStates; i++) {
            Ms[i][tid] = vv[i] - P.hh * D[i];
            Pk[i] = vv[i] + P.hh * D[i];
        }
    }
    __syncthreads();
    if (tid < kBlock - 1 && k < N) {
#pragma unroll
        for (int i = 0; i < kStates; i++) st_nt(out + i * N + k, Ms[i][tid + 1] - Pk[i]);
    }
}

// Boundary rows of J v: the direction at the fixed state.
__global__ __launch_bounds__(kBlock) void quad_bnd_jvp_kernel(QP P, const double *__restrict__ v,
                                                              double *__restrict__ out)
{
    const int b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= P.nb) return;
    const int64_t node = b < kStates ? 0 : P.N;
    out[(int64_t)kStates * P.N + b] = v[(int64_t)(b % kStates) * P.N1 + node];
}

// ---------------------------------------------------------------------------
// Fused evaluation into the KKT values (ocp_eval_kkt for a quadrotor
// handle): the values eval_jac, eval_hess and assemble_kkt give with the slot
// maps of ocp_quad_kkt, written straight into the CSR rows.  Row layout (that
// of the host builder): variable v's row at node k holds its len_v Hessian
// entries (the diagonal last, + reg) at var_start[v] + len_v k; defect row
// (i, k) holds its 2 kSupLen[i] Jacobian entries, then its diagonal (reg or
// 0), at def_start[i] + (2 kSupLen[i] + 1) k; boundary row b holds 1 and its
// diagonal at bnd_start + 2 b.
// ---------------------------------------------------------------------------
struct QLayout {
    int64_t var_start[kVars];
    int64_t def_start[kStates];
    int64_t bnd_start;
};

// Variable rows: one lane per node computes the node's 23 Hessian values;
// each variable's rows of the workgroup's nodes with more than one entry are
// staged in LDS and written with contiguous stores.
__global__ __launch_bounds__(kBlock) void quad_kkt_var_kernel(QP P, QLayout Lo, const double *__restrict__ z,
                                                              const double *__restrict__ y, double sigma,
                                                              const double *__restrict__ reg,
                                                              double *__restrict__ kkt)
{
    __shared__ double buf[4 * kBlock];  // one variable's rows of the workgroup (<= 4 entries each)
    const int64_t k0 = (int64_t)blockIdx.x * kBlock, k = k0 + threadIdx.x;
    const bool live = k <= P.N;
    const int kn = (int)min((int64_t)kBlock, (int64_t)P.N1 - k0);
    const int64_t N = P.N, N1 = P.N1;
    double H[kHessNode];
#pragma unroll
    for (int s = 0; s < kHessNode; s++) H[s] = 0.0;
    if (live) {
        double a[3], u[4], Y[kStates];
        load_att(P, z, k, a, u);
#pragma unroll
        for (int i = 0; i < kStates; i++) {
            if (i == 0 || i == 2 || i == 4) {  // linear rows: no curvature
                Y[i] = 0.0;
                continue;
            }
            double sy = 0.0;
            if (k >= 1) sy += y[i * N + k - 1];
            if (k < N) sy += y[i * N + k];
            Y[i] = sy;
        }
        const Trig t = node_trig(a[0], a[1], a[2]);
        hess_values(t, u, Y, sigma * q_weight(P, (int)k), P.r, P.hh, H);
        if (reg) {
#pragma unroll
            for (int v = 0; v < kVars; v++) H[kHessFirst[v + 1] - 1] += reg[v * N1 + k];
        }
    }
#pragma unroll
    for (int v = 0; v < kVars; v++) {
        const int f = kHessFirst[v], len = kHessFirst[v + 1] - f;
        if (len == 1) {  // one entry per row: the lanes' stores are contiguous already
            if (live) st_nt(kkt + Lo.var_start[v] + k, H[f]);
            continue;
        }
        if (live) {
#pragma unroll
            for (int e = 0; e < len; e++) buf[threadIdx.x * len + e] = H[f + e];
        }
        __syncthreads();
        double *out = kkt + Lo.var_start[v] + k0 * len;
        for (int x = threadIdx.x; x < kn * len; x += kBlock) st_nt(out + x, buf[x]);
        __syncthreads();
    }
}

// Defect rows: one lane per interval evaluates the right-hand side's partials
// at its two nodes; each row block's rows of the workgroup are staged in LDS
// and written with contiguous stores.
__global__ __launch_bounds__(kBlock) void quad_kkt_defect_kernel(QP P, QLayout Lo, const double *__restrict__ z,
                                                                 const double *__restrict__ reg,
                                                                 double *__restrict__ kkt)
{
    __shared__ double buf[(2 * 6 + 1) * kBlock];  // one row block's rows (<= 12 entries + diagonal)
    const int64_t k0 = (int64_t)blockIdx.x * kBlock, k = k0 + threadIdx.x;
    const bool live = k < P.N;
    const int kn = (int)min((int64_t)kBlock, (int64_t)P.N - k0);
    const int64_t N = P.N, N1 = P.N1;
    const int64_t nvar = (int64_t)kVars * N1;
    Trig tr[2];
    double u[2][4];
#pragma unroll
    for (int s = 0; s < 2; s++) {
        tr[s] = Trig{};
#pragma unroll
        for (int l = 0; l < 4; l++) u[s][l] = 0.0;
        if (live) {
            double a[3];
            load_att(P, z, k + s, a, u[s]);
            tr[s] = node_trig(a[0], a[1], a[2]);
        }
    }
#pragma unroll
    for (int i = 0; i < kStates; i++) {
        const int L = kSupLen[i], len = 2 * L + 1;
        if (live) {
            double *row = buf + threadIdx.x * len;
#pragma unroll
            for (int p = 0; p < L; p++) {
                const int q = pair_index(i, p);
                const bool own = pair_is_own_state(i, p);
#pragma unroll
                for (int s = 0; s < 2; s++) {
                    const double id = own ? (s ? 1.0 : -1.0) : 0.0;
                    row[2 * p + s] = id - P.hh * partial(q, tr[s], u[s]);
                }
            }
            row[len - 1] = reg ? reg[nvar + i * N + k] : 0.0;
        }
        __syncthreads();
        double *out = kkt + Lo.def_start[i] + k0 * len;
        for (int x = threadIdx.x; x < kn * len; x += kBlock) st_nt(out + x, buf[x]);
        __syncthreads();
    }
}

// Boundary rows: their state entry (1) and their diagonal.
__global__ __launch_bounds__(kBlock) void quad_kkt_bnd_kernel(QP P, QLayout Lo, const double *__restrict__ reg,
                                                              double *__restrict__ kkt)
{
    const int b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= P.nb) return;
    const int64_t row = (int64_t)kVars * P.N1 + (int64_t)kStates * P.N + b;
    kkt[Lo.bnd_start + 2 * b] = 1.0;
    kkt[Lo.bnd_start + 2 * b + 1] = reg ? reg[row] : 0.0;
}

QP make_qp(const ocp_problem *p)
{
    QP P;
    P.N = (int)p->d.N;
    P.N1 = (int)p->d.N1;
    P.nb = (int)p->d.nb;
    P.h = 1.0 / (double)p->d.N;
    P.hh = 0.5 * P.h;
    P.g = p->quad_g;
    P.r = p->quad_r;
    return P;
}

}  // namespace

namespace ocp {
namespace quad {

int eval_obj(const ocp_problem *p, const double *z, double *obj, hipStream_t stream)
{
    const QP P = make_qp(p);
    const unsigned g = (unsigned)std::min<int64_t>(kObjBlocks, blocks_for(p->d.N1, kBlock));
    hipLaunchKernelGGL(quad_obj_partial_kernel, dim3(g), dim3(kBlock), 0, stream, P, z, p->partials);
    if (int rc = check_launch("ocp_eval_obj")) return rc;
    hipLaunchKernelGGL(quad_obj_final_kernel, dim3(1), dim3(kBlock), 0, stream, p->partials, (int)g, obj);
    return check_launch("ocp_eval_obj");
}

int eval_kkt(const ocp_problem *p, const double *z, const double *y, double sigma, const double *reg,
             double *kkt, hipStream_t stream)
{
    const QP P = make_qp(p);
    const int64_t N = p->d.N, N1 = p->d.N1;
    QLayout Lo;
    int64_t o = 0;
    for (int v = 0; v < kVars; v++) {
        Lo.var_start[v] = o;
        o += (int64_t)(kHessFirst[v + 1] - kHessFirst[v]) * N1;
    }
    for (int i = 0; i < kStates; i++) {
        Lo.def_start[i] = o;
        o += (int64_t)(kRowSlot[i + 1] - kRowSlot[i] + 1) * N;
    }
    Lo.bnd_start = o;
    hipLaunchKernelGGL(quad_kkt_defect_kernel, dim3(blocks_for(N, kBlock)), dim3(kBlock), 0, stream, P, Lo, z,
                       reg, kkt);
    if (int rc = check_launch("ocp_eval_kkt")) return rc;
    hipLaunchKernelGGL(quad_kkt_var_kernel, dim3(blocks_for(N1, kBlock)), dim3(kBlock), 0, stream, P, Lo, z, y,
                       sigma, reg, kkt);
    if (int rc = check_launch("ocp_eval_kkt")) return rc;
    if (P.nb > 0)
        hipLaunchKernelGGL(quad_kkt_bnd_kernel, dim3(blocks_for(P.nb, kBlock)), dim3(kBlock), 0, stream, P, Lo,
                           reg, kkt);
    return check_launch("ocp_eval_kkt");
}

int eval_lagrangian(const ocp_problem *p, const double *z, const double *y, double sigma, double *L,
                    hipStream_t stream)
{
    const QP P = make_qp(p);
    const int nchunks = (int)blocks_for(p->d.N, kBlock - 1);
    const int g = std::min(nchunks, kObjBlocks);
    hipLaunchKernelGGL(quad_lag_partial_kernel, dim3(g), dim3(kBlock), 0, stream, P, z, y, sigma, nchunks,
                       p->partials);
    if (int rc = check_launch("ocp_eval_lagrangian")) return rc;
    hipLaunchKernelGGL(quad_obj_final_kernel, dim3(1), dim3(kBlock), 0, stream, p->partials, g, L);
    return check_launch("ocp_eval_lagrangian");
}

int eval_lag_grad(const ocp_problem *p, const double *z, const double *y, double sigma, double *g,
                  hipStream_t stream)
{
    hipLaunchKernelGGL(quad_lag_grad_kernel, dim3(blocks_for(p->d.N1, kBlock)), dim3(kBlock), 0, stream,
                       make_qp(p), z, y, sigma, g);
    return check_launch("ocp_eval_lag_grad");
}

int eval_hvp(const ocp_problem *p, const double *z, const double *y, double sigma, const double *v,
             double *out, hipStream_t stream)
{
    hipLaunchKernelGGL(quad_hvp_kernel, dim3(blocks_for(p->d.N1, kBlock)), dim3(kBlock), 0, stream,
                       make_qp(p), z, y, sigma, v, out);
    return check_launch("ocp_eval_hvp");
}

int eval_jvp(const ocp_problem *p, const double *z, const double *v, double *out, hipStream_t stream)
{
    const QP P = make_qp(p);
    hipLaunchKernelGGL(quad_jvp_kernel, dim3(blocks_for(p->d.N, kBlock - 1)), dim3(kBlock), 0, stream, P, z,
                       v, out);
    if (int rc = check_launch("ocp_eval_jvp")) return rc;
    if (P.nb > 0)
        hipLaunchKernelGGL(quad_bnd_jvp_kernel, dim3(blocks_for(P.nb, kBlock)), dim3(kBlock), 0, stream, P, v,
                           out);
    return check_launch("ocp_eval_jvp");
}

int eval_grad(const ocp_problem *p, const double *z, double *g, hipStream_t stream)
{
    hipLaunchKernelGGL(quad_grad_kernel, dim3(blocks_for(p->d.N1, kBlock)), dim3(kBlock), 0, stream,
                       make_qp(p), z, g);
    return check_launch("ocp_eval_grad");
}

int eval_cons(const ocp_problem *p, const double *z, double *c, hipStream_t stream)
{
    const QP P = make_qp(p);
    hipLaunchKernelGGL(quad_cons_kernel, dim3(blocks_for(p->d.N, kBlock - 1)), dim3(kBlock), 0, stream, P,
                       z, c);
    if (P.nb > 0)
        hipLaunchKernelGGL(quad_bnd_cons_kernel, dim3(blocks_for(P.nb, kBlock)), dim3(kBlock), 0, stream, P,
                           z, c);
    return check_launch("ocp_eval_cons");
}

int eval_jac(const ocp_problem *p, const double *z, double *jvals, hipStream_t stream)
{
    const QP P = make_qp(p);
    // Paired stores need every slot row 16-byte aligned: N even and the
    // output 16-byte aligned.
    const bool pair = P.N % 2 == 0 && (uintptr_t)jvals % 16 == 0;
    if (pair)
        hipLaunchKernelGGL(quad_jac_kernel<2>, dim3(blocks_for(P.N / 2, kBlock), kStates), dim3(kBlock), 0,
                           stream, P, z, jvals);
    else
        hipLaunchKernelGGL(quad_jac_kernel<1>, dim3(blocks_for(P.N, kBlock), kStates), dim3(kBlock), 0,
                           stream, P, z, jvals);
    if (P.nb > 0)
        hipLaunchKernelGGL(quad_bnd_jac_kernel, dim3(blocks_for(P.nb, kBlock)), dim3(kBlock), 0, stream, P,
                           jvals);
    return check_launch("ocp_eval_jac");
}

int eval_hess(const ocp_problem *p, const double *z, const double *y, double sigma, double *hvals,
              hipStream_t stream)
{
    hipLaunchKernelGGL(quad_hess_kernel, dim3(blocks_for(p->d.N1, kBlock)), dim3(kBlock), 0, stream,
                       make_qp(p), z, y, sigma, hvals);
    return check_launch("ocp_eval_hess");
}

int assemble_kkt(const ocp_problem *p, const int32_t *perm_j, const int32_t *perm_h, const int32_t *rowptr,
                 const double *jvals, const double *hvals, const double *reg, double *kkt, hipStream_t stream)
{
    const QP P = make_qp(p);
    AsmGroups G;
    int64_t blocks = 0;
    for (int g = 0; g < kGroups; g++) {
        const bool is_h = g >= kStates;
        const int gi = is_h ? g - kStates : g;
        const int per_row = is_h ? kHessFirst[gi + 1] - kHessFirst[gi] : kRowSlot[gi + 1] - kRowSlot[gi] + 1;
        const int KT = (kTileCap / per_row) & ~1;
        const int64_t rows = is_h ? p->d.N1 : p->d.N;
        G.tile0[g] = (int)blocks;
        G.KT[g] = KT;
        blocks += (rows + KT - 1) / KT;
    }
    G.tile0[kGroups] = (int)blocks;
    blocks += blocks_for(P.nb, kBlock);
    // paired loads need 16-byte aligned values and 8-byte aligned slots
    const bool vec_j = (uintptr_t)jvals % 16 == 0 && (uintptr_t)perm_j % 8 == 0;
    const bool vec_h = (uintptr_t)hvals % 16 == 0 && (uintptr_t)perm_h % 8 == 0;
    hipLaunchKernelGGL(quad_assemble_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, stream, P, G,
                       (int)p->d.nnzk, vec_j, vec_h, perm_j, perm_h, rowptr, jvals, hvals, reg, kkt);
    return check_launch("ocp_assemble_kkt");
}

}  // namespace quad
}  // namespace ocp

extern "C" {

int ocp_quad_create(int64_t N, int32_t boundary, double g, double r, ocp_problem **out)
{
    clear_error();
    if (!out) return fail(OCP_ERR_ARG, "ocp_quad_create: out is NULL");
    *out = nullptr;
    Dims d;
    if (int rc = quad::make_dims(N, boundary, &d)) return rc;
    if (!std::isfinite(g) || !std::isfinite(r))
        return fail(OCP_ERR_ARG, "ocp_quad_create: g and r must be finite");
    ocp_problem *p = new (std::nothrow) ocp_problem();
    if (!p) return fail(OCP_ERR_ALLOC, "ocp_quad_create: out of host memory");
    p->d = d;
    p->model = quad::kModel;
    p->quad_g = g;
    p->quad_r = r;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        delete p;
        return hip_fail("ocp_quad_create: hipGetDevice", e);
    }
    e = hipMalloc(&p->partials, kObjBlocks * sizeof(double));
    if (e != hipSuccess) {
        ocp_destroy(p);
        return fail(OCP_ERR_ALLOC, std::string("ocp_quad_create: hipMalloc: ") + hipGetErrorString(e));
    }
    *out = p;
    return OCP_OK;
}

}  // extern "C"
