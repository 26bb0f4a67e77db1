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
#include <string>

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

constexpr int kCols = 8;  // coefficient-gradient columns per workgroup

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
                if (i < n) acc += y[i * N + k] * (Ms[i][tid + 1] - Pk[i]);
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
        double x[NB], vx[NB], D[NB];
#pragma unroll
        for (int i = 0; i < NB; i++) {
            x[i] = (i < n) ? z[i * N1 + k] : 0.0;
            vx[i] = (i < n) ? v[i * N1 + k] : 0.0;
            D[i] = 0.0;
        }
#pragma unroll
        for (int j = 0; j < NB; j++) {
            if (j < n) {
                const double t = cos(x[j]) * vx[j];
                const double *a = P.AT + j * kLd;
#pragma unroll
                for (int i = 0; i < NB; i++) D[i] = __builtin_fma(a[i], t, D[i]);
            }
        }
        for (int l = 0; l < m && k < NU; l++) {
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

// Coefficient gradient, pass 1.  Grid (G, n, ceil((n+m+1)/kCols)): row i,
// columns c0 .. c0+kCols-1 of [A row i | B row i | gamma_i]; lanes take nodes
// k = blockIdx.x * B + lane + s G B in order; each column's workgroup total
// goes to cpart[(i (n+m+1) + col) G + blockIdx.x].
__global__ __launch_bounds__(kBlock) void coef_partial_kernel(KP P, const double *__restrict__ z,
                                                              const double *__restrict__ y, int G,
                                                              double *__restrict__ cpart)
{
    __shared__ double ws[kCols][kBlock / 64];
    const int n = P.n, m = P.m, ncol = n + m + 1;
    const int i = blockIdx.y, c0 = blockIdx.z * kCols;
    const int p = (i + 1 == n) ? 0 : i + 1;
    const int64_t N = P.N, N1 = P.N1;
    double acc[kCols];
#pragma unroll
    for (int c = 0; c < kCols; c++) acc[c] = 0.0;
    const int64_t NU = P.NU;
    const bool euler = P.scheme != 0;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k <= N; k += (int64_t)G * kBlock) {
        const double *yi = y + i * N + k;
        // node multiplier: F at node k enters rows (i, k-1) and (i, k), or
        // only (i, k) under forward Euler
        const double yt = euler ? (k < N ? yi[0] : 0.0) : (k >= 1 ? yi[-1] : 0.0) + (k < N ? yi[0] : 0.0);
#pragma unroll
        for (int c = 0; c < kCols; c++) {
            const int col = c0 + c;
            if (col < n) acc[c] += yt * sin(z[col * N1 + k]);
            else if (col < n + m) {
                if (k < NU) acc[c] += yt * z[n * N1 + (col - n) * NU + k];
            } else if (col == n + m) acc[c] += yt * (z[i * N1 + k] * z[p * N1 + k]);
        }
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < kCols; c++) {
        const double t = wave_sum(acc[c]);
        if (lane == 0) ws[c][wid] = t;
    }
    __syncthreads();
    if (threadIdx.x < kCols) {
        const int col = c0 + threadIdx.x;
        if (col < ncol) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < kBlock / 64; w++) t += ws[threadIdx.x][w];
            cpart[((int64_t)i * ncol + col) * G + blockIdx.x] = t;
        }
    }
}

// Pass 2: one workgroup per coefficient; lane b < G holds workgroup b's
// partial and a fixed-shape tree adds them.
__global__ __launch_bounds__(kBlock) void coef_final_kernel(KP P, const double *__restrict__ cpart,
                                                            int G, double *__restrict__ gA,
                                                            double *__restrict__ gB,
                                                            double *__restrict__ gg)
{
    const int n = P.n, m = P.m, ncol = n + m + 1;
    const int idx = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < G; b += kBlock) s += cpart[(int64_t)idx * G + b];
    s = block_sum<kBlock>(s);
    if (threadIdx.x != 0) return;
    const double val = -(P.scheme != 0 ? P.h : P.hh) * s;
    const int i = idx / ncol, col = idx - i * ncol;
    if (col < n) gA[i * n + col] = val;
    else if (col < n + m) gB[i * m + (col - n)] = val;
    else gg[i] = val;
}

int nb_of(int n) { return n <= 4 ? 4 : n <= 8 ? 8 : n <= 16 ? 16 : 32; }

// Rebuild the padded columns AT, BT (kLd rows each, zero below row n) from
// the row-major A and B, on the device so that a coefficient update stays
// asynchronous on the caller's stream.
__global__ __launch_bounds__(kBlock) void pack_columns_kernel(int n, int m, const double *__restrict__ A,
                                                              const double *__restrict__ B,
                                                              double *__restrict__ AT,
                                                              double *__restrict__ BT)
{
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= (n + m) * kLd) return;
    const int c = e / kLd, i = e % kLd;
    if (c < n) AT[e] = i < n ? A[i * n + c] : 0.0;
    else BT[e - n * kLd] = i < n ? B[i * m + (c - n)] : 0.0;
}

}  // namespace

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
    hipError_t e = hipMemcpyAsync(const_cast<double *>(p->kp.A), A, sizeof(double) * n * n,
                                  hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess && m)
        e = hipMemcpyAsync(const_cast<double *>(p->kp.B), B, sizeof(double) * n * m,
                           hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(const_cast<double *>(p->kp.gam), gamma, sizeof(double) * n,
                           hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return hip_fail("ocp_set_coefficients", e);
    hipLaunchKernelGGL(pack_columns_kernel, dim3(blocks_for((int64_t)(n + m) * kLd, kBlock)),
                       dim3(kBlock), 0, stream, n, m, p->kp.A, p->kp.B,
                       const_cast<double *>(p->kp.AT), const_cast<double *>(p->kp.BT));
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
    const int n = p->d.n, m = p->d.m, ncol = n + m + 1;
    const int G = (int)std::min<int64_t>(kCoefBlocks, blocks_for(p->d.N1, kBlock));
    const dim3 grid(G, n, (ncol + kCols - 1) / kCols);
    hipLaunchKernelGGL(coef_partial_kernel, grid, dim3(kBlock), 0, stream, p->kp, z, y, G, p->cpart);
    if (int rc = check_launch("ocp_eval_coef_grad")) return rc;
    hipLaunchKernelGGL(coef_final_kernel, dim3(n * ncol), dim3(kBlock), 0, stream, p->kp, p->cpart, G,
                       gA, gB, ggamma);
    return check_launch("ocp_eval_coef_grad");
}

}  // extern "C"
