// Per-node device arithmetic shared by the single-instance kernels and the
// batched persistent kernel of the evaluation library (gfx950, wave64).
//
// Every evaluation maps one grid node (or one interval) to one lane, the SIMD
// structure of direct transcription (paper Sec. 3): the same few functions are
// evaluated at every node.  All arrays are structure-of-arrays with the node
// index fastest, so the lanes of a wavefront touch consecutive doubles.
//
// Formulas (component-major unknowns, h = 1/N, hh = h/2, p(i) = (i+1) mod n):
//   F_i(k)   = sum_j A_ij sin X_jk + sum_l B_il U_lk + gamma_i X_ik X_{p(i)k}
//   c_{ik}   = (X_{i,k+1} - X_ik) - hh (F_i(k) + F_i(k+1))         [Sec. 5]
//   f        = sum_k w_k (sum_j q_j X_jk^2 + sum_l r_l U_lk^2)     [Sec. 5]
//   dF_i/dX_j = A_ij cos X_j + gamma_i (delta_ij X_p(i) + delta_j,p(i) X_i)
//   Hessian of L = sigma f + y^T c at node k uses the node multiplier
//   yt_ik = y_{i,k-1} [k >= 1] + y_{ik} [k < N]  (node k is the right end of
//   interval k-1 and the left end of interval k).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ocp {
namespace dev {

typedef double dbl2 __attribute__((ext_vector_type(2)));
typedef double d4 __attribute__((ext_vector_type(4)));  // FP64 MFMA 16x16 accumulator
typedef int32_t int2v __attribute__((ext_vector_type(2)));

constexpr int kBlock = 256;  // threads per workgroup of the single-instance kernels (4 waves)

// Kernel-side view of one problem: sizes and device coefficient pointers.
struct KP {
    int N;         // intervals
    int N1;        // nodes = N + 1
    int n, m, npair, T, S;
    int nnzk;      // KKT entries
    int NU;        // control nodes: N + 1 (trapezoidal) or N (forward Euler)
    int scheme;    // 0 trapezoidal, 1 forward Euler
    int nb;        // boundary rows after the n N defect rows
    double h, hh;
    const double *A;    // n x n row-major
    const double *B;    // n x m row-major
    const double *gam;  // n
    const double *q;    // n
    const double *r;    // m
    const double *AT;   // n columns of kLd: AT[j kLd + i] = A_ij (i < n), 0 (n <= i < kLd)
    const double *BT;   // m columns of kLd: BT[l kLd + i] = B_il (i < n), 0 (n <= i < kLd)
};

// Column stride of the padded copies AT and BT (the bound on n).  A kernel
// whose register bound NB <= kLd sums a column over all NB rows without a
// guard, the padding adding exact zeros; the column's entries are contiguous
// at offsets known at compile time, so a wavefront fetches them with a few
// wide scalar loads instead of one load per coefficient behind a branch.
constexpr int kLd = 32;

// Host side: the padded copies of one instance's A (n x n) and B (n x m),
// both row-major, into AT (n kLd doubles) and BT (m kLd doubles).
inline void pack_columns(int n, int m, const double *A, const double *B, double *AT, double *BT)
{
    for (int j = 0; j < n; j++)
        for (int i = 0; i < kLd; i++) AT[j * kLd + i] = i < n ? A[i * n + j] : 0.0;
    for (int l = 0; l < m; l++)
        for (int i = 0; i < kLd; i++) BT[l * kLd + i] = i < n ? B[i * m + l] : 0.0;
}

// Cost weight of node k: trapezoidal rule (end nodes h/2), or the forward
// Euler sum over nodes 0..N-1 (weight h, none at node N).
__device__ __forceinline__ double node_weight(const KP &P, int k)
{
    if (P.scheme) return k < P.N ? P.h : 0.0;
    return (k == 0 || k == P.N) ? P.hh : P.h;
}

__device__ __forceinline__ void st_nt(double *p, double v) { __builtin_nontemporal_store(v, p); }
// A store that is non-temporal when NT (the default for outputs), else an
// ordinary one.
template <bool NT>
__device__ __forceinline__ void st_out(double *p, double v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}
__device__ __forceinline__ void st_nt2(double *p, dbl2 v)
{
    __builtin_nontemporal_store(v, reinterpret_cast<dbl2 *>(p));
}

// Fixed-shape sums: over a wavefront (cross-lane shuffles, tree of halving
// offsets) and over a workgroup of BS lanes (wavefront sums, then the BS/64
// wave totals in order).  The order of additions never depends on timing.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

template <int BS>
__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double ws[BS / 64];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) ws[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < BS / 64; i++) t += ws[i];
    }
    return t;  // valid in thread 0
}

// ---------------------------------------------------------------------------
// Jacobian values of one column for NPT consecutive intervals k .. k+NPT-1
// (the caller guarantees k + NPT <= N, and for NPT = 2 a 16-byte aligned
// output with N even).  Column col < n is state column j: slots 2j, 2j+1 of
// every row i; col = n + l is control column l: slots 2n+2l, 2n+2l+1, the
// constant -hh B_il.  NPT = 2 stores a 16-byte pair per lane, so a wavefront
// store is one contiguous KiB of a slot row.  A state column needs NPT+1
// cosines per lane; the bilinear term touches only rows i = j (partner
// X_{j+1}) and i = j-1 (factor X_{j-1}).
// ---------------------------------------------------------------------------
template <int NPT>
__device__ __forceinline__ void jac_column(const KP &P, const double *__restrict__ z,
                                           double *__restrict__ jac, int64_t k, int col)
{
    const int n = P.n, T = P.T;
    const int64_t N = P.N, N1 = P.N1;
    const double hh = P.hh;
    if (col < n) {
        const int j = col;
        const int jn = (j + 1 == n) ? 0 : j + 1;
        const int jp = (j == 0) ? n - 1 : j - 1;
        const double *xj = z + j * N1 + k;
        const double *xn = z + jn * N1 + k;
        const double *xp = z + jp * N1 + k;
        double cs[NPT + 1], dg[NPT + 1], lo[NPT + 1];
#pragma unroll
        for (int u = 0; u <= NPT; u++) {
            cs[u] = cos(xj[u]);
            dg[u] = -hh * P.gam[j] * xn[u];   // row i = j: gamma_j X_{j+1}
            lo[u] = -hh * P.gam[jp] * xp[u];  // row i = j-1: gamma_{j-1} X_{j-1}
        }
        for (int i = 0; i < n; i++) {
            const double a = -hh * P.A[i * n + j];
            double v0[NPT], v1[NPT];
#pragma unroll
            for (int u = 0; u < NPT; u++) {
                v0[u] = a * cs[u];
                v1[u] = a * cs[u + 1];
            }
            if (i == j) {
#pragma unroll
                for (int u = 0; u < NPT; u++) {
                    v0[u] += dg[u] - 1.0;
                    v1[u] += dg[u + 1] + 1.0;
                }
            }
            if (i == jp) {
#pragma unroll
                for (int u = 0; u < NPT; u++) {
                    v0[u] += lo[u];
                    v1[u] += lo[u + 1];
                }
            }
            double *o0 = jac + ((int64_t)i * T + 2 * j) * N + k;
            double *o1 = o0 + N;
            if constexpr (NPT == 2) {
                st_nt2(o0, dbl2{v0[0], v0[1]});
                st_nt2(o1, dbl2{v1[0], v1[1]});
            } else {
                st_nt(o0, v0[0]);
                st_nt(o1, v1[0]);
            }
        }
    } else {
        const int l = col - n, m = P.m;
        for (int i = 0; i < n; i++) {
            const double v = -hh * P.B[i * m + l];
            double *o0 = jac + ((int64_t)i * T + 2 * n + 2 * l) * N + k;
            double *o1 = o0 + N;
            if constexpr (NPT == 2) {
                st_nt2(o0, dbl2{v, v});
                st_nt2(o1, dbl2{v, v});
            } else {
                st_nt(o0, v);
                st_nt(o1, v);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Hessian-of-Lagrangian values at node k <= N.  NB >= n is a compile-time
// bound so the node's states and multipliers stay in registers; all loads are
// issued before the arithmetic, and the control slots (constants) and the
// bilinear slots (multipliers only) are stored before the state diagonals,
// so their stores leave while the sines are computed.
// NT selects non-temporal stores.  The single-instance trapezoidal kernel
// stores ordinarily: a node's values go to S slot rows, one 8-byte store per
// lane and row, and with non-temporal stores that pattern reaches 60 % of HBM
// with no arithmetic at all against 73 % with ordinary ones.  The lines are
// then written back during the next kernel (in an interior-point step the
// assembly, which reads these values).  The batched kernel and the forward
// Euler kernel keep non-temporal stores (with ordinary ones their steps
// measured the same or slower).
// ---------------------------------------------------------------------------
template <int NB, bool NT>
__device__ __forceinline__ void hess_node(const KP &P, const double *__restrict__ z,
                                          const double *__restrict__ y, double sigma,
                                          double *__restrict__ hv, int k)
{
    const int n = P.n, m = P.m;
    const int64_t N = P.N, N1 = P.N1;
    const double w = node_weight(P, k);
    double x[NB], yl[NB], yr[NB];
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
    const int64_t ub = (int64_t)(n + P.npair) * N1 + k;
    for (int l = 0; l < m; l++) st_out<NT>(hv + ub + l * N1, 2.0 * sigma * w * P.r[l]);
    double yt[NB];
#pragma unroll
    for (int i = 0; i < NB; i++) yt[i] = yl[i] + yr[i];
    if (n >= 3) {
#pragma unroll
        for (int i = 0; i < NB; i++)
            if (i < n) st_out<NT>(hv + (n + i) * N1 + k, -P.hh * yt[i] * P.gam[i]);
    } else if (n == 2) {
        st_out<NT>(hv + 2 * N1 + k, -P.hh * (yt[0] * P.gam[0] + yt[1] * P.gam[1]));
    }
#pragma unroll
    for (int j = 0; j < NB; j++) {
        if (j < n) {
            const double sx = sin(x[j]);
            const double *a = P.AT + j * kLd;
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < NB; i++) s = __builtin_fma(yt[i], a[i], s);
            double v = 2.0 * sigma * w * P.q[j] + P.hh * sx * s;
            if (n == 1) v -= P.h * yt[0] * P.gam[0];
            st_out<NT>(hv + j * N1 + k, v);
        }
    }
}

// ---------------------------------------------------------------------------
// Dynamics at node k <= N: the node's states x[i] = X_ik and F_i(k) for every
// i < n (NB >= n, entries beyond n are zero).  F_i sums j ascending, then l
// ascending, then the bilinear term.  The states and the first MB controls
// are loaded before any arithmetic (further controls, when m > MB, after);
// a caller that knows m <= MB < NB saves the registers of NB - MB controls.
// ---------------------------------------------------------------------------
template <int NB, int MB = NB>
__device__ __forceinline__ void dyn_node(const KP &P, const double *__restrict__ z, int64_t k,
                                         double (&x)[NB], double (&F)[NB])
{
    static_assert(MB <= NB, "the control bound is at most the state bound");
    const int n = P.n, m = P.m;
    const int64_t N1 = P.N1;
    const double *U = z + (int64_t)n * N1;
    double u[MB];
#pragma unroll
    for (int i = 0; i < NB; i++) {
        x[i] = (i < n) ? z[i * N1 + k] : 0.0;
        if (i < MB) u[i] = (i < m) ? U[(int64_t)i * P.NU + k] : 0.0;
        F[i] = 0.0;
    }
#pragma unroll
    for (int j = 0; j < NB; j++) {
        if (j < n) {
            const double s = sin(x[j]);
            const double *a = P.AT + j * kLd;
#pragma unroll
            for (int i = 0; i < NB; i++) F[i] = __builtin_fma(a[i], s, F[i]);
        }
    }
#pragma unroll
    for (int l = 0; l < MB; l++) {
        if (l < m) {
            const double *b = P.BT + l * kLd;
#pragma unroll
            for (int i = 0; i < NB; i++) F[i] = __builtin_fma(b[i], u[l], F[i]);
        }
    }
    for (int l = MB; l < m; l++) {
        const double ul = U[(int64_t)l * P.NU + k];
        const double *b = P.BT + l * kLd;
#pragma unroll
        for (int i = 0; i < NB; i++) F[i] = __builtin_fma(b[i], ul, F[i]);
    }
#pragma unroll
    for (int i = 0; i < NB; i++) {
        if (i < n) {
            const double xp = (i + 1 < n) ? x[(i + 1) % NB] : x[0];
            F[i] = __builtin_fma(P.gam[i] * x[i], xp, F[i]);  // explicit: same bits in every kernel
        }
    }
}

// Entry n-1 of a register array (n is a run-time value <= NB), by selects so
// the array stays in registers.
template <int NB>
__device__ __forceinline__ double last_of(const double (&a)[NB], int n)
{
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < NB; i++)
        if (i == n - 1) v = a[i];
    return v;
}

// ---------------------------------------------------------------------------
// Forward Euler (paper Sec. 3): Jacobian values of one column for NPT
// consecutive intervals k .. k+NPT-1 (k + NPT <= N; NPT = 2 needs N even and a
// 16-byte aligned output).  Row i's slots, in ascending column order, are
// X_0..X_i at k (slots 0..i), X_i at k+1 (slot i+1), X_{i+1}..X_{n-1} at k
// (slots i+2..n), U_l at k (slot n+1+l).  State column j writes slot
// (j <= i ? j : j+1) of every row i, -delta_ij - h dF_i/dX_j(k), and the +1
// at slot j+1 of row j; control column l writes -h B_il at slot n+1+l.
// ---------------------------------------------------------------------------
template <int NPT>
__device__ __forceinline__ void jac_column_euler(const KP &P, const double *__restrict__ z,
                                                 double *__restrict__ jac, int64_t k, int col)
{
    const int n = P.n, T = P.T;
    const int64_t N = P.N, N1 = P.N1;
    const double h = P.h;
    auto put = [&](int64_t i, int t, const double (&v)[NPT]) {
        double *o = jac + ((int64_t)i * T + t) * N + k;
        if constexpr (NPT == 2) st_nt2(o, dbl2{v[0], v[1]});
        else st_nt(o, v[0]);
    };
    if (col < n) {
        const int j = col;
        const int jn = (j + 1 == n) ? 0 : j + 1;
        const int jp = (j == 0) ? n - 1 : j - 1;
        const double *xj = z + j * N1 + k;
        const double *xn = z + jn * N1 + k;
        const double *xp = z + jp * N1 + k;
        double cs[NPT], dg[NPT], lo[NPT];
#pragma unroll
        for (int u = 0; u < NPT; u++) {
            cs[u] = cos(xj[u]);
            dg[u] = -h * P.gam[j] * xn[u];   // row i = j: gamma_j X_{j+1}
            lo[u] = -h * P.gam[jp] * xp[u];  // row i = j-1: gamma_{j-1} X_{j-1}
        }
        for (int i = 0; i < n; i++) {
            const double a = -h * P.A[i * n + j];
            double v[NPT];
#pragma unroll
            for (int u = 0; u < NPT; u++) v[u] = a * cs[u];
            if (i == j) {
#pragma unroll
                for (int u = 0; u < NPT; u++) v[u] += dg[u] - 1.0;
            }
            if (i == jp) {
#pragma unroll
                for (int u = 0; u < NPT; u++) v[u] += lo[u];
            }
            put(i, j <= i ? j : j + 1, v);
        }
        double one[NPT];
#pragma unroll
        for (int u = 0; u < NPT; u++) one[u] = 1.0;
        put(j, j + 1, one);
    } else {
        const int l = col - n, m = P.m;
        for (int i = 0; i < n; i++) {
            double v[NPT];
#pragma unroll
            for (int u = 0; u < NPT; u++) v[u] = -h * P.B[i * m + l];
            put(i, n + 1 + l, v);
        }
    }
}

// Forward Euler Hessian-of-Lagrangian values at node k <= N: node k enters
// only the defect of interval k (multiplier y_k, factor h); node N enters no
// defect and carries no cost, so its entries are zero.  Control slots exist
// for k < N only, at (n+npair)(N+1) + l N + k.  NT as for hess_node.
template <int NB, bool NT>
__device__ __forceinline__ void hess_node_euler(const KP &P, const double *__restrict__ z,
                                                const double *__restrict__ y, double sigma,
                                                double *__restrict__ hv, int k)
{
    const int n = P.n, m = P.m;
    const int64_t N = P.N, N1 = P.N1;
    const double w = node_weight(P, k);
    const double h = P.h;
    double x[NB], yt[NB];
#pragma unroll
    for (int i = 0; i < NB; i++) {
        x[i] = yt[i] = 0.0;
        if (i < n) {
            x[i] = z[i * N1 + k];
            if (k < P.N) yt[i] = y[i * N + k];
        }
    }
    // the control and bilinear slots (no sines) are stored first, as in
    // hess_node, then the diagonals
    if (k < P.NU) {
        const int64_t ub = (int64_t)(n + P.npair) * N1 + k;
        for (int l = 0; l < m; l++) st_out<NT>(hv + ub + (int64_t)l * P.NU, 2.0 * sigma * w * P.r[l]);
    }
    if (n >= 3) {
#pragma unroll
        for (int i = 0; i < NB; i++)
            if (i < n) st_out<NT>(hv + (n + i) * N1 + k, -h * yt[i] * P.gam[i]);
    } else if (n == 2) {
        st_out<NT>(hv + 2 * N1 + k, -h * (yt[0] * P.gam[0] + yt[1] * P.gam[1]));
    }
#pragma unroll
    for (int j = 0; j < NB; j++) {
        if (j < n) {
            const double sx = sin(x[j]);
            const double *a = P.AT + j * kLd;
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < NB; i++) s = __builtin_fma(yt[i], a[i], s);
            double v = 2.0 * sigma * w * P.q[j] + h * sx * s;
            if (n == 1) v -= 2.0 * h * yt[0] * P.gam[0];
            st_out<NT>(hv + j * N1 + k, v);
        }
    }
}

// Host-side launchers of the single-instance kernels (ocp_eval.hip,
// ocp_fused.hip); the batched path uses them for its per-instance mode.
// `pair_ok`: the Jacobian output is 16-byte aligned.  launch_obj's
// `partials` holds min(4096, ceil((N+1) / 256)) doubles.  Each covers the
// problem's boundary rows too.
hipError_t launch_jac(const KP &P, const double *z, double *jac, bool pair_ok, hipStream_t stream);
hipError_t launch_hess(const KP &P, const double *z, const double *y, double sigma, double *hv,
                       hipStream_t stream);
hipError_t launch_obj(const KP &P, const double *z, double *partials, double *obj, hipStream_t stream);
hipError_t launch_grad(const KP &P, const double *z, double *g, hipStream_t stream);
hipError_t launch_cons(const KP &P, const double *z, double *c, hipStream_t stream);
hipError_t launch_eval_kkt(const KP &P, const double *z, const double *y, double sigma, const double *reg,
                           double *kkt, hipStream_t stream);

}  // namespace dev
}  // namespace ocp
