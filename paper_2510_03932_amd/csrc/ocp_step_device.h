// Per-tile device arithmetic of a whole interior-point evaluation step, shared
// by the single-instance kernels (ocp_eval.hip, ocp_fused.hip) and the batched
// persistent kernel (ocp_batch.hip): defects, objective gradient, the
// objective's per-node terms and its fixed-shape sums, and the fused
// evaluation of the Jacobian and the Hessian of the Lagrangian straight into
// the lower CSR KKT matrix (paper Sec. 6: the KKT system is assembled in
// device buffers).  A tile is a run of intervals or nodes of one problem; a
// workgroup of BS lanes evaluates it.  The values do not depend on the tile
// shape, so single-instance and batched evaluations agree bit for bit.
#pragma once

#include "ocp_device.h"
#include "ocp_eval.h"

namespace ocp {
namespace dev {

// ---------------------------------------------------------------------------
// Defects, trapezoidal scheme, one wavefront: lane l evaluates the dynamics at
// node k0 + l and closes interval k0 + l (lanes 0..62), with
//   c_ik = (X_{i,k+1} - hh F_i(k+1)) - (X_ik + hh F_i(k)):
// lane l keeps X + hh F of its node and receives X - hh F of node k+1 from
// lane l+1 by a cross-lane shuffle.  Every state value is read once.  Both
// halves are explicit fused multiply-adds, as in the single-instance kernel,
// so the two agree bit for bit whatever the compiler contracts elsewhere.
// ---------------------------------------------------------------------------
template <int NB>
__device__ __forceinline__ void cons_wave(const KP &P, const double *__restrict__ z, double *__restrict__ c,
                                          int64_t k0)
{
    const int lane = threadIdx.x & 63, n = P.n;
    const int64_t k = k0 + lane, N = P.N;
    double x[NB], F[NB];
    if (k <= N) {
        dyn_node<NB>(P, z, k, x, F);
    } else {
#pragma unroll
        for (int i = 0; i < NB; i++) x[i] = F[i] = 0.0;
    }
    const bool store = lane < 63 && k < N;
#pragma unroll
    for (int i = 0; i < NB; i++) {
        if (i < n) {
            const double right = __shfl_down(__builtin_fma(-P.hh, F[i], x[i]), 1, 64);
            const double left = __builtin_fma(P.hh, F[i], x[i]);
            if (store) st_nt(c + i * N + k, right - left);
        }
    }
}

// Forward-Euler defects of interval k < N: c_ik = (X_{i,k+1} - X_ik) - h F_i(k).
// Up to NB = 16 the next node's states are loaded with this node's, before
// any arithmetic; at NB = 32 those registers would leave one wavefront per
// SIMD, so they are loaded at the stores.  (MB: the controls' register
// bound, as in dyn_node.)
template <int NB, int MB = NB>
__device__ __forceinline__ void cons_euler_interval(const KP &P, const double *__restrict__ z,
                                                    double *__restrict__ c, int64_t k)
{
    constexpr bool kEarly = NB <= 16;
    const int n = P.n;
    const int64_t N = P.N, N1 = P.N1;
    double xn[kEarly ? NB : 1], x[NB], F[NB];
    if constexpr (kEarly) {
#pragma unroll
        for (int i = 0; i < NB; i++) xn[i] = (i < n) ? z[i * N1 + k + 1] : 0.0;
    }
    dyn_node<NB, MB>(P, z, k, x, F);
#pragma unroll
    for (int i = 0; i < NB; i++) {
        if (i < n) {
            const double next = kEarly ? xn[kEarly ? i : 0] : z[i * N1 + k + 1];
            st_nt(c + i * N + k, __builtin_fma(-P.h, F[i], next - x[i]));
        }
    }
}

// Boundary rows b < nb after the n N defect rows: row b is X_{b mod n} at
// node 0 (b < n) or node N.
__device__ __forceinline__ double bnd_value(const KP &P, const double *__restrict__ z, int b)
{
    const int i = b % P.n;
    const int64_t node = b < P.n ? 0 : P.N;
    return z[(int64_t)i * P.N1 + node];
}

// Objective gradient at component comp (state j < n, control n + l) and node
// k: 2 w_k q_j X_jk or 2 w_k r_l U_lk (controls exist on NU nodes).
__device__ __forceinline__ void grad_entry(const KP &P, const double *__restrict__ z, double *__restrict__ g,
                                           int comp, int64_t k)
{
    const double coef = comp < P.n ? P.q[comp] : P.r[comp - P.n];
    const int64_t e = comp < P.n ? (int64_t)comp * P.N1 + k
                                 : (int64_t)P.n * P.N1 + (int64_t)(comp - P.n) * P.NU + k;
    const double w = node_weight(P, (int)k);
    st_nt(g + e, 2.0 * w * coef * z[e]);
}

// The objective's term of node k: w_k (sum_j q_j X_jk^2 + sum_l r_l U_lk^2),
// states first (every load issued before the sum), then the controls in
// groups of NB, each in component order.  (Loading the controls together
// with the states measured no faster at n = 16, m = 8 and costs occupancy.)
template <int NB>
__device__ __forceinline__ double obj_node(const KP &P, const double *__restrict__ z, int64_t k)
{
    const int n = P.n, m = P.m;
    const int64_t N1 = P.N1, NU = P.NU;
    const double *U = z + (int64_t)n * N1;
    double v[NB];
#pragma unroll
    for (int c = 0; c < NB; c++) v[c] = c < n ? z[c * N1 + k] : 0.0;
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < NB; c++)
        if (c < n) s += P.q[c] * v[c] * v[c];
    if (k < NU) {
        for (int l0 = 0; l0 < m; l0 += NB) {
#pragma unroll
            for (int u = 0; u < NB; u++) v[u] = l0 + u < m ? U[(l0 + u) * NU + k] : 0.0;
#pragma unroll
            for (int u = 0; u < NB; u++)
                if (l0 + u < m) s += P.r[l0 + u] * v[u] * v[u];
        }
    }
    return node_weight(P, (int)k) * s;
}

// Sum of 256 values, one per virtual lane t = 0..255, in the order of
// block_sum<256>: a wavefront tree over each run of 64 virtual lanes, then the
// four run totals in order.  A workgroup of BS lanes (BS = 128 or 256) holds
// virtual lane t + r BS in v[r], r < 256 / BS.  ws: 4 doubles of LDS.  The
// result is valid in thread 0; the caller synchronizes before reusing ws.
template <int BS>
__device__ __forceinline__ double sum256(const double (&v)[256 / BS], double *ws)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int r = 0; r < 256 / BS; r++) {
        const double t = wave_sum(v[r]);
        if (lane == 0) ws[wid + r * (BS / 64)] = t;
    }
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < 4; i++) t += ws[i];
    }
    return t;
}

// ---------------------------------------------------------------------------
// Fused KKT evaluation.  CSR layout of the variable rows (ocp_build_kkt): the
// rows of state a come first for every a, each holding len[a] entries (its
// bilinear entries, then the diagonal), so state a's block starts at
// pre[a] (N+1); then the control rows (one entry each), the defect rows (T
// Jacobian entries and the diagonal each) and the boundary rows (two each).
// ---------------------------------------------------------------------------
struct KKTLayout {
    int32_t len[OCP_MAX_DIM];
    int32_t pre[OCP_MAX_DIM + 1];
};

inline KKTLayout kkt_layout(int n)
{
    KKTLayout Lo{};
    int s = 0;
    for (int a = 0; a < n; a++) {
        int pairs = 0;
        if (n >= 3) pairs = a == 0 ? 0 : (a == n - 1 ? 2 : 1);
        else if (n == 2) pairs = a == 1 ? 1 : 0;
        Lo.pre[a] = s;
        Lo.len[a] = pairs + 1;
        s += pairs + 1;
    }
    Lo.pre[n] = s;
    return Lo;
}

__device__ __forceinline__ int64_t kkt_ctrl_start(const KP &P, const KKTLayout &Lo)
{
    return (int64_t)Lo.pre[P.n] * P.N1;
}
__device__ __forceinline__ int64_t kkt_cons_start(const KP &P, const KKTLayout &Lo)
{
    return kkt_ctrl_start(P, Lo) + (int64_t)P.m * P.NU;
}
__device__ __forceinline__ int64_t kkt_bnd_start(const KP &P, const KKTLayout &Lo)
{
    return kkt_cons_start(P, Lo) + (int64_t)P.n * P.N * (P.T + 1);
}

// Defect-row tiles: KT intervals per tile (a power of two, 16 to 64), chosen
// per problem by kkt_defect_kt; each row block is computed slot-major into an
// LDS tile and copied out (see kkt_defect_tile).
constexpr int kDefectKTMax = 64;
constexpr size_t kDefectLdsMax = 64 * 1024;  // bytes of LDS a tile may take

// LDS doubles of one defect-row tile of KT intervals (n states, m controls,
// T Jacobian slots per row): states and cosines at KT+1 nodes, the rows'
// diagonals, the scaled coefficients, and the output tile.
inline size_t kkt_defect_lds(int n, int m, int T, int KT)
{
    return 2 * (size_t)n * (KT + 1) + (size_t)n * KT + (size_t)n * (n + m) + (size_t)n + (size_t)KT * (T + 1);
}

// Intervals per defect-row tile: a row block of KT (T+1) entries of about 500
// to 1000 doubles (measured best at n = 16, m = 8: KT = 16, 784 entries; at
// n = 6, m = 3: KT = 32, 608 entries), within the LDS bound.
inline int kkt_defect_kt(int n, int m, int T)
{
    int KT = T + 1 >= 33 ? 16 : (T + 1 >= 17 ? 32 : 64);
    while (KT > 16 && kkt_defect_lds(n, m, T, KT) * sizeof(double) > kDefectLdsMax) KT /= 2;
    return KT;
}

// Entry t of defect row (i, k0 + kk): T Jacobian slots then the diagonal,
// from the tile's LDS arrays (states xs and cosines cs at W = KT + 1 nodes,
// coefficients cf = -w A | -w B, gs = -w gamma, diagonals rg; w = h/2, or h
// under forward Euler).
__device__ __forceinline__ double defect_entry(int i, int t, int kk, int n, int m, int T, int W, int KT,
                                               bool euler, const double *cf, const double *gs,
                                               const double *xs, const double *cs, const double *rg)
{
#pragma clang fp contract(off)
    double v;
    if (euler) {
        // row i: X_0..X_i at k, X_i at k+1, X_{i+1}..X_{n-1} at k, U at k
        if (t == i + 1) {
            v = 1.0;
        } else if (t <= n) {
            const int j = t <= i ? t : t - 1;
            const int jn = (j + 1 == n) ? 0 : j + 1;
            const int jp = (j == 0) ? n - 1 : j - 1;
            v = cf[i * (n + m) + j] * cs[j * W + kk];
            if (i == j) v += gs[j] * xs[jn * W + kk] - 1.0;
            if (i == jp) v += gs[jp] * xs[jp * W + kk];
        } else if (t < T) {
            v = cf[i * (n + m) + n + (t - n - 1)];
        } else {
            v = rg[i * KT + kk];
        }
    } else if (t < 2 * n) {
        const int j = t >> 1, s = t & 1, u = kk + s;
        const int jn = (j + 1 == n) ? 0 : j + 1;
        const int jp = (j == 0) ? n - 1 : j - 1;
        v = cf[i * (n + m) + j] * cs[j * W + u];
        if (i == j) {
            const double dg = gs[j] * xs[jn * W + u];
            v += s ? dg + 1.0 : dg - 1.0;
        }
        if (i == jp) v += gs[jp] * xs[jp * W + u];
    } else if (t < T) {
        v = cf[i * (n + m) + n + ((t - 2 * n) >> 1)];
    } else {
        v = rg[i * KT + kk];
    }
    return v;
}

// Defect rows of intervals [k0, k0 + KT): the tile's states and their cosines
// at nodes k0 .. k0 + KT, the rows' regularization and the scaled
// coefficients -hh A, -hh B, -hh gamma are staged in LDS (the lanes of a
// wavefront span several slots of a row, so coefficient reads from global
// memory would be per-lane loads); then, for each state component i, the rows
// (i, k0 .. k0 + kn - 1) -- one contiguous CSR range of kn (T + 1) entries,
// each row its T Jacobian entries and its diagonal -- are computed slot-major
// (KT lanes share a slot, so a wavefront reads few coefficients and
// conflict-free state columns) into an LDS tile and copied out with
// contiguous stores, two barriers per row block.  (Alternating two tiles, one
// barrier per block, measured 9 % slower at n = 16, m = 8 and 5 % at n = 6,
// m = 3; storing in output order straight from the sweep, no barrier at all,
// 15 % slower: the lanes of a wavefront then mix slot kinds and diverge.)
// KT = 2^LG <= 64 intervals (the caller's grid uses the same KT); reg: the
// problem's dim-entry regularization or null.  Ends with a barrier, so a
// following tile may restage the LDS.
template <int BS>
__device__ __forceinline__ void kkt_defect_tile(const KP &P, const KKTLayout &Lo, const double *__restrict__ z,
                                                const double *__restrict__ reg, double *__restrict__ kkt,
                                                int64_t k0, int LG, double *lds)
{
    // no implicit contraction: the single-instance and the batched kernels
    // inline this body into different code and must produce the same bits
#pragma clang fp contract(off)
    const int KT = 1 << LG, W = KT + 1;  // intervals k0 .. k0+KT-1, nodes k0 .. k0+KT
    const int n = P.n, m = P.m, T = P.T, T1 = P.T + 1;
    const int64_t N = P.N, N1 = P.N1;
    const int64_t nvar = (int64_t)n * N1 + (int64_t)m * P.NU;  // controls on NU nodes
    const int kn = (int)min((int64_t)KT, N - k0);
    double *xs = lds;                     // [n][W] states
    double *cs = lds + n * W;             // [n][W] cosines
    double *rg = lds + 2 * n * W;         // [n][KT] the tile's defect-row diagonals (reg or 0)
    double *cf = rg + n * KT;             // [n][n+m] -hh A | -hh B, then [n] -hh gamma
    double *gs = cf + n * (n + m);
    double *tile = gs + n;                // [KT][T1] output row block
    const bool euler = P.scheme != 0;
    const double hh = euler ? P.h : P.hh;  // the weight of F in a defect row
    // every global load is issued here, before the row loop
    for (int x = threadIdx.x; x < n * W; x += BS) {
        const int j = x / W, u = x - j * W;
        const int64_t k = k0 + u;
        const double v = k <= N ? z[j * N1 + k] : 0.0;
        xs[x] = v;
        cs[x] = cos(v);
    }
    for (int x = threadIdx.x; x < n * KT; x += BS) {
        const int i = x >> LG, kk = x & (KT - 1);
        rg[x] = (reg && kk < kn) ? reg[nvar + i * N + k0 + kk] : 0.0;
    }
    for (int x = threadIdx.x; x < n * (n + m); x += BS) {
        const int i = x / (n + m), j = x - i * (n + m);
        cf[x] = -hh * (j < n ? P.A[i * n + j] : P.B[i * m + (j - n)]);
    }
    for (int x = threadIdx.x; x < n; x += BS) gs[x] = -hh * P.gam[x];
    __syncthreads();
    const int64_t cons_start = kkt_cons_start(P, Lo);
    for (int i = 0; i < n; i++) {
        for (int w = threadIdx.x; w < T1 << LG; w += BS) {
            const int t = w >> LG, kk = w & (KT - 1);
            if (kk < kn) tile[kk * T1 + t] = defect_entry(i, t, kk, n, m, T, W, KT, euler, cf, gs, xs, cs, rg);
        }
        __syncthreads();
        double *out = kkt + cons_start + (i * N + k0) * T1;
        for (int x = threadIdx.x; x < kn * T1; x += BS) st_nt(out + x, tile[x]);
        __syncthreads();
    }
}

// Variable rows of nodes [k0, k0 + BS): one lane per node computes the node's
// Hessian values (+ reg on the diagonals), as in eval_hess; each state
// block's rows of the tile's nodes are one contiguous CSR range, staged in
// LDS (buf: 3 BS doubles) and written with contiguous stores.  Ends with a
// barrier.
template <int NB, int BS>
__device__ __forceinline__ void kkt_var_tile(const KP &P, const KKTLayout &Lo, const double *__restrict__ z,
                                             const double *__restrict__ y, double sigma,
                                             const double *__restrict__ reg, double *__restrict__ kkt,
                                             int64_t k0, double *buf)
{
#pragma clang fp contract(off)  // as in kkt_defect_tile
    const int64_t k = k0 + threadIdx.x;
    const bool live = k <= P.N;
    const int kn = (int)min((int64_t)BS, (int64_t)P.N1 - k0);
    const int n = P.n, m = P.m;
    const int64_t N = P.N, N1 = P.N1, NU = P.NU;
    const bool euler = P.scheme != 0;
    const double w = node_weight(P, (int)k);
    // every load of the node, the diagonals' regularization included, is
    // issued before the arithmetic (the regularization loaded after each
    // diagonal's sine and products made the batched KKT launches 4 % slower)
    double x[NB], yl[NB], yr[NB], rd[NB];
#pragma unroll
    for (int i = 0; i < NB; i++) {
        x[i] = yl[i] = yr[i] = rd[i] = 0.0;
        if (live && i < n) {
            x[i] = z[i * N1 + k];
            const double *yi = y + i * N + k;
            if (k >= 1) yl[i] = yi[-1];
            if (k < P.N) yr[i] = yi[0];
            if (reg) rd[i] = reg[i * N1 + k];
        }
    }
    // node multiplier: F at node k enters rows (i, k-1) and (i, k), or only
    // (i, k) under forward Euler
    double yt[NB];
#pragma unroll
    for (int i = 0; i < NB; i++) yt[i] = euler ? yr[i] : yl[i] + yr[i];
    const double wF = euler ? P.h : P.hh;
    // Hessian values of the node, as in eval_hess: state diagonals and the
    // bilinear entries (pair i couples states i and i+1 mod n)
    double dg[NB], pr[NB];
#pragma unroll
    for (int j = 0; j < NB; j++) {
        dg[j] = 0.0;
        if (j < n) {
            const double sx = sin(x[j]);
            const double *a = P.AT + j * kLd;
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < NB; i++) s = __builtin_fma(yt[i], a[i], s);
            double v = 2.0 * sigma * w * P.q[j] + wF * sx * s;
            if (n == 1) v -= euler ? 2.0 * P.h * yt[0] * P.gam[0] : P.h * yt[0] * P.gam[0];
            if (live && reg) v += rd[j];
            dg[j] = v;
        }
    }
#pragma unroll
    for (int i = 0; i < NB; i++) pr[i] = i < n ? -wF * yt[i] * P.gam[i] : 0.0;
    if (n == 2) pr[0] = -wF * (yt[0] * P.gam[0] + yt[1] * P.gam[1]);
    // state block a: rows (a, k0 .. k0+kn-1) are one contiguous CSR range of
    // kn * len[a] entries, staged in LDS and written with contiguous stores
#pragma unroll
    for (int a = 0; a < NB; a++) {
        if (a < n) {  // uniform across the workgroup
            const int len = Lo.len[a];
            double *row = buf + threadIdx.x * len;
            if (live) {
                row[len - 1] = dg[a];
                if (n >= 3 && a >= 1 && a <= n - 2) row[0] = pr[a - 1];
                if (n >= 3 && a == n - 1) {
                    row[0] = pr[n - 1];  // column 0
                    row[1] = pr[n - 2];  // column n-2
                }
                if (n == 2 && a == 1) row[0] = pr[0];
            }
            __syncthreads();
            double *out = kkt + (int64_t)Lo.pre[a] * N1 + k0 * len;
            for (int t = threadIdx.x; t < kn * len; t += BS) st_nt(out + t, buf[t]);
            __syncthreads();
        }
    }
    if (live && k < NU) {  // controls exist on NU nodes
        const int64_t NX = (int64_t)n * N1, cstart = kkt_ctrl_start(P, Lo);
        for (int l = 0; l < m; l++) {
            double v = 2.0 * sigma * w * P.r[l];
            if (reg) v += reg[NX + l * NU + k];
            st_nt(kkt + cstart + l * NU + k, v);
        }
    }
}

// Boundary row b's two KKT entries: its state entry (1) and its diagonal.
__device__ __forceinline__ void kkt_bnd_row(const KP &P, const KKTLayout &Lo, const double *__restrict__ reg,
                                            double *__restrict__ kkt, int b)
{
    const int64_t bs = kkt_bnd_start(P, Lo);
    const int64_t row0 = (int64_t)P.n * P.N1 + (int64_t)P.m * P.NU + (int64_t)P.n * P.N;  // nvar + n N
    kkt[bs + 2 * b] = 1.0;
    kkt[bs + 2 * b + 1] = reg ? reg[row0 + b] : 0.0;
}

}  // namespace dev
}  // namespace ocp
