// Fused evaluation into the KKT matrix (ocp_eval_kkt): the Jacobian and the
// Hessian of the Lagrangian are evaluated straight into their slots of the
// lower CSR KKT matrix of ocp_build_kkt, with the regularization on the
// diagonal, skipping the COO value arrays.  An interior-point iteration that
// only needs the assembled matrix (paper Sec. 6) then moves the matrix once:
// the state rows, y and reg in, the KKT values out (about 7 GB at N = 1e6,
// n = 16, m = 8, against 23 GB for eval_jac + eval_hess + assemble_kkt).
//
// The values are computed with the same expressions, in the same order, as
// the COO kernels and the assembly.
//
// Defect rows: workgroup b owns intervals [b KT, b KT + KT).  It stages the
// states and their cosines at the KT+1 nodes, the rows' regularization and
// the scaled coefficients -hh A, -hh B, -hh gamma in LDS (a wavefront spans
// four slots of a row, so coefficient reads from global memory would be
// per-lane loads, each waited for); then, for each state
// component i, it computes the tile's KT rows (T Jacobian entries and the
// diagonal each) slot by slot into an LDS tile and writes the rows'
// contiguous CSR range with full-line stores.
// Variable rows: one lane per node computes the node's Hessian values (+ reg
// on the diagonals), as in eval_hess; each state block's rows of the
// workgroup's nodes are staged in LDS and written contiguously.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "ocp_device.h"
#include "ocp_problem.h"
#include "ocp_quad.h"

using namespace ocp;
using namespace ocp::dev;

namespace {

constexpr int kDefectTile = 16;  // intervals per defect-row workgroup

// CSR layout of the state rows: block of state a starts at sb[a]; its rows
// hold len[a] entries (bilinear entries, then the diagonal).
struct KKTLayout {
    int64_t sb[OCP_MAX_DIM];
    int len[OCP_MAX_DIM];
    int64_t ctrl_start, cons_start, bnd_start;
};

__global__ __launch_bounds__(kBlock) void kkt_defect_kernel(KP P, KKTLayout Lo, const double *__restrict__ z,
                                                            const double *__restrict__ reg,
                                                            double *__restrict__ kkt)
{
    extern __shared__ double lds[];
    constexpr int KT = kDefectTile, LG = 4, W = KT + 1;  // intervals k0 .. k0+KT-1, nodes k0 .. k0+KT
    const int n = P.n, m = P.m, T = P.T, T1 = P.T + 1;
    const int64_t N = P.N, N1 = P.N1;
    const int64_t nvar = (int64_t)n * N1 + (int64_t)m * P.NU;  // controls on NU nodes
    const int64_t k0 = (int64_t)blockIdx.x * KT;
    const int kn = (int)min((int64_t)KT, N - k0);
    double *xs = lds;                     // [n][W] states
    double *cs = lds + n * W;             // [n][W] cosines
    double *rg = lds + 2 * n * W;         // [n][KT] the tile's defect-row diagonals (reg or 0)
    double *cf = rg + n * KT;             // [n][n+m] -hh A | -hh B, then [n] -hh gamma
    double *gs = cf + n * (n + m);
    double *tile = gs + n;                // [KT][T1] output rows
    const bool euler = P.scheme != 0;
    const double hh = euler ? P.h : P.hh;  // the weight of F in a defect row
    for (int x = threadIdx.x; x < n * (n + m); x += kBlock) {
        const int i = x / (n + m), j = x - i * (n + m);
        cf[x] = -hh * (j < n ? P.A[i * n + j] : P.B[i * m + (j - n)]);
    }
    for (int x = threadIdx.x; x < n; x += kBlock) gs[x] = -hh * P.gam[x];
    for (int x = threadIdx.x; x < n * W; x += kBlock) {
        const int j = x / W, u = x - j * W;
        const int64_t k = k0 + u;
        const double v = k <= N ? z[j * N1 + k] : 0.0;
        xs[x] = v;
        cs[x] = cos(v);
    }
    // every global load is issued here, before the per-component loop, so no
    // wavefront stalls on memory between that loop's barriers
    for (int x = threadIdx.x; x < n * KT; x += kBlock) {
        const int i = x >> LG, kk = x & (KT - 1);
        rg[x] = (reg && kk < kn) ? reg[nvar + i * N + k0 + kk] : 0.0;
    }
    __syncthreads();
    for (int i = 0; i < n; i++) {
        // slot t of the tile's rows, interval fastest: 16 lanes share t, so
        // a wavefront covers four slots; its coefficients come from LDS
        for (int w = threadIdx.x; w < T1 << LG; w += kBlock) {
            const int t = w >> LG, kk = w & (KT - 1);
            if (kk >= kn) continue;
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
                    v = rg[(i << LG) + kk];
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
                v = rg[(i << LG) + kk];
            }
            tile[kk * T1 + t] = v;
        }
        __syncthreads();
        double *out = kkt + Lo.cons_start + (i * N + k0) * T1;
        for (int x = threadIdx.x; x < kn * T1; x += kBlock) st_nt(out + x, tile[x]);
        __syncthreads();
    }
}

template <int NB>
__global__ __launch_bounds__(kBlock) void kkt_var_kernel(KP P, KKTLayout Lo, const double *__restrict__ z,
                                                         const double *__restrict__ y, double sigma,
                                                         const double *__restrict__ reg,
                                                         double *__restrict__ kkt)
{
    __shared__ double buf[3 * kBlock];  // one state block's rows of this workgroup (<= 3 entries each)
    const int k0 = blockIdx.x * kBlock, k = k0 + threadIdx.x;
    const bool live = k <= P.N;
    const int kn = min(kBlock, P.N1 - k0);
    const int n = P.n, m = P.m;
    const int64_t N = P.N, N1 = P.N1, NU = P.NU;
    const bool euler = P.scheme != 0;
    const double w = node_weight(P, k);
    double x[NB], yl[NB], yr[NB];
#pragma unroll
    for (int i = 0; i < NB; i++) {
        x[i] = yl[i] = yr[i] = 0.0;
        if (live && i < n) {
            x[i] = z[i * N1 + k];
            const double *yi = y + i * N + k;
            if (k >= 1) yl[i] = yi[-1];
            if (k < P.N) yr[i] = yi[0];
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
            if (live && reg) v += reg[j * N1 + k];
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
            double *out = kkt + Lo.sb[a] + (int64_t)k0 * len;
            for (int t = threadIdx.x; t < kn * len; t += kBlock) st_nt(out + t, buf[t]);
            __syncthreads();
        }
    }
    if (live && k < NU) {  // controls exist on NU nodes
        const int64_t NX = (int64_t)n * N1;
        for (int l = 0; l < m; l++) {
            double v = 2.0 * sigma * w * P.r[l];
            if (reg) v += reg[NX + l * NU + k];
            st_nt(kkt + Lo.ctrl_start + l * NU + k, v);
        }
    }
}

// Boundary rows: their state entry (1) and their diagonal.
__global__ __launch_bounds__(kBlock) void kkt_bnd_kernel(KP P, KKTLayout Lo, int64_t row0,
                                                         const double *__restrict__ reg,
                                                         double *__restrict__ kkt)
{
    const int b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= P.nb) return;
    kkt[Lo.bnd_start + 2 * b] = 1.0;
    kkt[Lo.bnd_start + 2 * b + 1] = reg ? reg[row0 + b] : 0.0;
}

}  // namespace

extern "C" {

int ocp_eval_kkt(const ocp_problem *p, const double *z, const double *y, double sigma, const double *reg,
                 double *kkt, hipStream_t stream)
{
    clear_error();
    if (int rc = check_handle(p, "ocp_eval_kkt")) return rc;
    if (!z || !y || !kkt) return fail(OCP_ERR_ARG, "ocp_eval_kkt: null array");
    if (!std::isfinite(sigma)) return fail(OCP_ERR_ARG, "ocp_eval_kkt: sigma is not finite");
    const Dims &d = p->d;
    if (p->model == quad::kModel) return quad::eval_kkt(p, z, y, sigma, reg, kkt, stream);
    // state-row layout of ocp_build_kkt: row (a, k) holds the bilinear
    // entries whose larger index is a, then the diagonal
    KKTLayout Lo;
    int64_t s = 0;
    for (int a = 0; a < d.n; a++) {
        int pairs = 0;
        if (d.n >= 3) pairs = a == 0 ? 0 : (a == d.n - 1 ? 2 : 1);
        else if (d.n == 2) pairs = a == 1 ? 1 : 0;
        Lo.sb[a] = s;
        Lo.len[a] = pairs + 1;
        s += (int64_t)(pairs + 1) * d.N1;
    }
    Lo.ctrl_start = s;
    Lo.cons_start = s + (int64_t)d.m * d.NU;
    Lo.bnd_start = Lo.cons_start + d.ndef * (d.T + 1);
    // defect-row tiles of kDefectTile intervals; LDS holds the tile's states,
    // their cosines and the output rows of one state component
    const size_t lds = ((size_t)kDefectTile * (d.T + 1) + 2 * (size_t)d.n * (kDefectTile + 1) +
                        (size_t)d.n * kDefectTile + (size_t)d.n * (d.n + d.m) + (size_t)d.n) *
                       sizeof(double);
    hipLaunchKernelGGL(kkt_defect_kernel, dim3(blocks_for(d.N, kDefectTile)), dim3(kBlock), lds, stream, p->kp,
                       Lo, z, reg, kkt);
    if (int rc = check_launch("ocp_eval_kkt")) return rc;
    const dim3 g(blocks_for(d.N1, kBlock));
    if (d.n <= 4) hipLaunchKernelGGL(kkt_var_kernel<4>, g, dim3(kBlock), 0, stream, p->kp, Lo, z, y, sigma, reg, kkt);
    else if (d.n <= 8) hipLaunchKernelGGL(kkt_var_kernel<8>, g, dim3(kBlock), 0, stream, p->kp, Lo, z, y, sigma, reg, kkt);
    else if (d.n <= 16) hipLaunchKernelGGL(kkt_var_kernel<16>, g, dim3(kBlock), 0, stream, p->kp, Lo, z, y, sigma, reg, kkt);
    else hipLaunchKernelGGL(kkt_var_kernel<32>, g, dim3(kBlock), 0, stream, p->kp, Lo, z, y, sigma, reg, kkt);
    if (int rc = check_launch("ocp_eval_kkt")) return rc;
    if (d.nb > 0)
        hipLaunchKernelGGL(kkt_bnd_kernel, dim3(blocks_for(d.nb, kBlock)), dim3(kBlock), 0, stream, p->kp, Lo,
                           d.nvar + d.ndef, reg, kkt);
    return check_launch("ocp_eval_kkt");
}

}  // extern "C"
