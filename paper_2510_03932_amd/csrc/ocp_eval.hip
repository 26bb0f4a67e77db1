// Device layer of the evaluation library, single-instance entry points: HIP
// kernels for gfx950 (CDNA4, wave64) and the C ABI functions that validate
// arguments and launch them.  The per-node arithmetic shared with the batched
// path lives in ocp_device.h.  The path is HBM-bound sparse evaluation, not a
// dense contraction: no MFMA.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "ocp_device.h"
#include "ocp_internal.h"
#include "ocp_problem.h"
#include "ocp_quad.h"
#include "ocp_step_device.h"

using namespace ocp;
using namespace ocp::dev;

namespace {

// ---------------------------------------------------------------------------
// Jacobian values.  2-D grid: blockIdx.x picks NPT intervals per lane,
// blockIdx.y the column (state j < n, control n + l).  Many short lanes (a
// grid of (N/NPT) x (n+m)) keep the write stream at the device's
// streaming-store rate.
// ---------------------------------------------------------------------------
template <int NPT>
__global__ __launch_bounds__(kBlock) void jac_kernel(KP P, const double *__restrict__ z,
                                                     double *__restrict__ jac)
{
    const int64_t k = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * NPT;
    if (k >= P.N) return;
    jac_column<NPT>(P, z, jac, k, blockIdx.y);
}

// ---------------------------------------------------------------------------
// Hessian-of-Lagrangian values, one lane per node.
// ---------------------------------------------------------------------------
template <int NB>
__global__ __launch_bounds__(kBlock) void hess_kernel(KP P, const double *__restrict__ z,
                                                      const double *__restrict__ y, double sigma,
                                                      double *__restrict__ hv)
{
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k > P.N) return;
    hess_node<NB, false>(P, z, y, sigma, hv, k);
}

// ---------------------------------------------------------------------------
// Defects.  Workgroup b evaluates the dynamics at nodes [b (B-1), b (B-1) + B),
// one node per lane, and writes the B-1 intervals they close (one node of
// overlap between workgroups).  With
//   c_ik = (X_{i,k+1} - hh F_i(k+1)) - (X_ik + hh F_i(k)),
// lane k keeps X_ik + hh F_i(k) in registers and publishes X_ik - hh F_i(k)
// in LDS for lane k-1, so every state value is read from HBM once.
// ---------------------------------------------------------------------------
template <int NB, int MB>
__global__ __launch_bounds__(kBlock) void cons_kernel(KP P, const double *__restrict__ z,
                                                      double *__restrict__ c)
{
    __shared__ double Ms[NB][kBlock];
    const int tid = threadIdx.x;
    const int64_t k = (int64_t)blockIdx.x * (kBlock - 1) + tid;
    const int n = P.n;
    const int64_t N = P.N;
    double Pk[NB];
    if (k <= N) {
        double x[NB], F[NB];
        dyn_node<NB, MB>(P, z, k, x, F);
#pragma unroll
        for (int i = 0; i < NB; i++) {
            if (i < n) {
                Ms[i][tid] = __builtin_fma(-P.hh, F[i], x[i]);
                Pk[i] = __builtin_fma(P.hh, F[i], x[i]);
            }
        }
    }
    __syncthreads();
    if (tid < kBlock - 1 && k < N) {
#pragma unroll
        for (int i = 0; i < NB; i++)
            if (i < n) st_nt(c + i * N + k, Ms[i][tid + 1] - Pk[i]);
    }
}

// ---------------------------------------------------------------------------
// Forward-Euler defects: one lane per interval k < N,
//   c_ik = (X_{i,k+1} - X_ik) - h F_i(k)  (paper Sec. 3).
// ---------------------------------------------------------------------------
template <int NB, int MB>
__global__ __launch_bounds__(kBlock) void cons_euler_kernel(KP P, const double *__restrict__ z,
                                                            double *__restrict__ c)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= P.N) return;
    cons_euler_interval<NB, MB>(P, z, c, k);
}

// Boundary rows after the n N defect rows: row b holds X_{b mod n} at node 0
// (b < n) or node N; its single Jacobian entry (1.0) follows the defect
// entries.
__global__ __launch_bounds__(kBlock) void bnd_cons_kernel(KP P, const double *__restrict__ z,
                                                          double *__restrict__ c)
{
    const int b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= P.nb) return;
    c[(int64_t)P.n * P.N + b] = bnd_value(P, z, b);
}

__global__ __launch_bounds__(kBlock) void bnd_jac_kernel(KP P, double *__restrict__ jac)
{
    const int b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= P.nb) return;
    jac[(int64_t)P.n * P.N * P.T + b] = 1.0;
}

template <int NPT>
__global__ __launch_bounds__(kBlock) void jac_euler_kernel(KP P, const double *__restrict__ z,
                                                           double *__restrict__ jac)
{
    const int64_t k = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * NPT;
    if (k >= P.N) return;
    jac_column_euler<NPT>(P, z, jac, k, blockIdx.y);
}

template <int NB>
__global__ __launch_bounds__(kBlock) void hess_euler_kernel(KP P, const double *__restrict__ z,
                                                            const double *__restrict__ y,
                                                            double sigma, double *__restrict__ hv)
{
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k > P.N) return;
    hess_node_euler<NB, true>(P, z, y, sigma, hv, k);
}

// ---------------------------------------------------------------------------
// Gradient: g = 2 w_k q_j X_jk, 2 w_k r_l U_lk.  blockIdx.y = component.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void grad_kernel(KP P, const double *__restrict__ z,
                                                      double *__restrict__ g)
{
    const int comp = blockIdx.y;
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k > P.N || (comp >= P.n && k >= P.NU)) return;
    grad_entry(P, z, g, comp, k);
}

// ---------------------------------------------------------------------------
// Objective: deterministic two-pass sum.  Pass 1: min(ceil((N+1)/256), 4096)
// workgroups (so one node per lane up to 1M nodes), each lane summing its
// nodes in order, then a fixed-shape tree over the wavefront (cross-lane
// shuffles) and over the 4 waves; pass 2: one workgroup sums the partials in a
// fixed order.  The grid depends only on N, so the result is reproducible.
// ---------------------------------------------------------------------------
template <int NB>
__global__ __launch_bounds__(kBlock) void obj_partial_kernel(KP P, const double *__restrict__ z,
                                                             double *__restrict__ partials)
{
    const int64_t N1 = P.N1;
    double acc = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < N1; k += (int64_t)gridDim.x * kBlock)
        acc += obj_node<NB>(P, z, k);
    const double t = block_sum<kBlock>(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ __launch_bounds__(kBlock) void obj_final_kernel(const double *__restrict__ partials,
                                                           int count, double *__restrict__ obj)
{
    double acc = 0.0;
    for (int i = threadIdx.x; i < count; i += kBlock) acc += partials[i];
    const double t = block_sum<kBlock>(acc);
    if (threadIdx.x == 0) obj[0] = t;
}

// ---------------------------------------------------------------------------
// KKT assembly.
//
// Jacobian part: the COO values are slot-major (node fastest) while the CSR
// rows of the constraint block are row-major, so the scatter is a transpose.
// Workgroup g < gj owns a tile of up to KT consecutive constraint rows of one
// state component i (intervals k0 .. k0+kn-1).  It reads the tile's T slot rows
// coalesced (one wavefront per slot row), drops each value into LDS at
// perm_j[e] - base, where [base, base + ext) is the tile's CSR range from
// rowptr, adds the tile's diagonals, and then writes the whole range with
// contiguous full-line stores.  A slot outside the range is stored directly.
// If the values that landed in LDS do not cover the range exactly (a slot map
// other than the closed-form one), the tile is redone with direct stores, so
// the result is the same for any injective slot map.
//
// Hessian part: workgroups gj.. take nodes and scatter the S Hessian slots
// directly (rows of 1 to 3 entries, close to contiguous across lanes), adding
// reg on the variable diagonals in the same IEEE add.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void assemble_kernel(
    KP P, int gj, int gh, int KT, bool vec_ok, const int32_t *__restrict__ perm_j, const int32_t *__restrict__ perm_h,
    const int32_t *__restrict__ rowptr, const double *__restrict__ jv,
    const double *__restrict__ hv, const double *__restrict__ reg, double *__restrict__ kkt)
{
    extern __shared__ double tile[];
    __shared__ int filled;
    const int64_t N = P.N, N1 = P.N1;
    const int64_t nvar = (int64_t)P.n * N1 + (int64_t)P.m * P.NU;
    const uint32_t nnzk = (uint32_t)P.nnzk;  // slots outside [0, nnzk) are skipped
    const int T = P.T;
    if ((int)blockIdx.x < gj) {
        const int tiles_per_i = (P.N + KT - 1) / KT;
        const int i = blockIdx.x / tiles_per_i;
        const int k0 = (blockIdx.x - i * tiles_per_i) * KT;
        const int kn = min(KT, P.N - k0);
        const int64_t r0 = nvar + (int64_t)i * N + k0;  // first KKT row of the tile
        const int32_t base = rowptr[r0];
        const int32_t ext = (int32_t)((uint32_t)rowptr[r0 + kn] - (uint32_t)base);
        const int cap = KT * (T + 1);
        // stage only a range inside [0, nnzk) (a corrupt rowptr falls back
        // to bounds-checked direct stores)
        const bool staged = ext >= 0 && ext <= cap && base >= 0 && (int64_t)base + ext <= (int64_t)nnzk;
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        if (threadIdx.x == 0) filled = 0;
        if (staged)
            for (int x = threadIdx.x; x < ext; x += kBlock) tile[x] = 0.0;
        __syncthreads();
        int mine = 0;
        const int64_t e0 = (int64_t)i * T * N + k0;
        // Each lane takes two adjacent intervals of a slot row (16-byte value
        // and 8-byte slot loads when aligned), so KT/2 lanes cover a slot row
        // and a wavefront covers 128/KT slot rows per pass.
        const int lanes_per_row = KT / 2;
        const int rows_per_wave = 64 / lanes_per_row;
        const int kl = (lane % lanes_per_row) * 2;
        const int sub = lane / lanes_per_row;
        auto place = [&](int32_t q, double v) {
            const uint32_t loc = (uint32_t)q - (uint32_t)base;
            if (staged && loc < (uint32_t)ext) {
                tile[loc] = v;
                mine++;
            } else if ((uint32_t)q < nnzk) {
                kkt[q] = v;
            }
        };
        if (kl < kn) {
            for (int t = wave * rows_per_wave + sub; t < T; t += 4 * rows_per_wave) {
                const int64_t e = e0 + (int64_t)t * N + kl;
                if (vec_ok && kl + 1 < kn && (e & 1) == 0) {
                    const int2v q = __builtin_nontemporal_load(reinterpret_cast<const int2v *>(perm_j + e));
                    const dbl2 v = __builtin_nontemporal_load(reinterpret_cast<const dbl2 *>(jv + e));
                    place(q.x, v.x);
                    place(q.y, v.y);
                } else {
                    place(perm_j[e], jv[e]);
                    if (kl + 1 < kn) place(perm_j[e + 1], jv[e + 1]);
                }
            }
        }
        if (threadIdx.x < kn) {
            const int64_t d = r0 + threadIdx.x;
            place(rowptr[d + 1] - 1, reg ? reg[d] : 0.0);
        }
        if (mine) atomicAdd(&filled, mine);
        __syncthreads();
        if (!staged) return;
        if (filled == ext) {
            double *out = kkt + base;
            for (int x = threadIdx.x; x < ext; x += kBlock) st_nt(out + x, tile[x]);
        } else {
            // not an exact cover: store this tile's values directly
            if (kl < kn) {
                for (int t = wave * rows_per_wave + sub; t < T; t += 4 * rows_per_wave) {
                    const int64_t e = e0 + (int64_t)t * N + kl;
                    for (int u = 0; u < 2 && kl + u < kn; u++) {
                        const int32_t q = perm_j[e + u];
                        if ((uint32_t)q < nnzk) kkt[q] = jv[e + u];
                    }
                }
            }
            if (threadIdx.x < kn) {
                const int64_t d = r0 + threadIdx.x;
                const int32_t q = rowptr[d + 1] - 1;
                if ((uint32_t)q < nnzk) kkt[q] = reg ? reg[d] : 0.0;
            }
        }
    } else if ((int)blockIdx.x < gj + gh) {
        const int64_t k = (int64_t)(blockIdx.x - gj) * kBlock + threadIdx.x;
        if (k >= N1) return;
        const int n = P.n, np = P.npair, S = P.S;
        for (int s = 0; s < S; s++) {
            int64_t e, row = -1;  // COO entry; KKT row of a diagonal entry
            if (s < n + np) {
                e = (int64_t)s * N1 + k;
                if (s < n) row = e;
            } else {
                if (k >= P.NU) break;  // control slots exist on NU nodes
                const int64_t l = s - n - np;
                e = (int64_t)(n + np) * N1 + l * P.NU + k;
                row = (int64_t)n * N1 + l * P.NU + k;
            }
            double v = hv[e];
            if (reg && row >= 0) v += reg[row];
            const uint32_t q = (uint32_t)perm_h[e];
            if (q < nnzk) kkt[q] = v;
        }
    } else {
        // boundary rows: their Jacobian entry and their diagonal
        const int b = (blockIdx.x - gj - gh) * kBlock + threadIdx.x;
        if (b >= P.nb) return;
        const int64_t e = (int64_t)P.n * N * T + b;
        const uint32_t q = (uint32_t)perm_j[e];
        if (q < nnzk) kkt[q] = jv[e];
        const int64_t d = nvar + (int64_t)P.n * N + b;
        const uint32_t dq = (uint32_t)(rowptr[d + 1] - 1);
        if (dq < nnzk) kkt[dq] = reg ? reg[d] : 0.0;
    }
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

namespace ocp {
namespace dev {

hipError_t launch_jac(const KP &P, const double *z, double *jac, bool pair_ok, hipStream_t stream)
{
    // Paired 16-byte stores need every slot row 16-byte aligned: N even and
    // the output 16-byte aligned.
    const unsigned cols = (unsigned)(P.n + P.m);
    const bool pair = pair_ok && P.N % 2 == 0;
    const dim3 g2((unsigned)((P.N / 2 + kBlock - 1) / kBlock), cols);
    const dim3 g1((unsigned)((P.N + kBlock - 1) / kBlock), cols);
    if (P.scheme == 0) {
        if (pair) hipLaunchKernelGGL(jac_kernel<2>, g2, dim3(kBlock), 0, stream, P, z, jac);
        else hipLaunchKernelGGL(jac_kernel<1>, g1, dim3(kBlock), 0, stream, P, z, jac);
    } else {
        if (pair) hipLaunchKernelGGL(jac_euler_kernel<2>, g2, dim3(kBlock), 0, stream, P, z, jac);
        else hipLaunchKernelGGL(jac_euler_kernel<1>, g1, dim3(kBlock), 0, stream, P, z, jac);
    }
    if (P.nb > 0)
        hipLaunchKernelGGL(bnd_jac_kernel, dim3((P.nb + kBlock - 1) / kBlock), dim3(kBlock), 0, stream,
                           P, jac);
    return hipGetLastError();
}

template <int NB>
static void launch_hess_nb(const KP &P, const double *z, const double *y, double sigma, double *hv,
                           hipStream_t stream)
{
    const dim3 g((unsigned)((P.N1 + kBlock - 1) / kBlock));
    if (P.scheme == 0) hipLaunchKernelGGL(hess_kernel<NB>, g, dim3(kBlock), 0, stream, P, z, y, sigma, hv);
    else hipLaunchKernelGGL(hess_euler_kernel<NB>, g, dim3(kBlock), 0, stream, P, z, y, sigma, hv);
}

hipError_t launch_hess(const KP &P, const double *z, const double *y, double sigma, double *hv,
                       hipStream_t stream)
{
    if (P.n <= 4) launch_hess_nb<4>(P, z, y, sigma, hv, stream);
    else if (P.n <= 8) launch_hess_nb<8>(P, z, y, sigma, hv, stream);
    else if (P.n <= 16) launch_hess_nb<16>(P, z, y, sigma, hv, stream);
    else launch_hess_nb<32>(P, z, y, sigma, hv, stream);
    return hipGetLastError();
}

hipError_t launch_obj(const KP &P, const double *z, double *partials, double *obj, hipStream_t stream)
{
    const unsigned g = (unsigned)std::min<int64_t>(kObjBlocks, blocks_for(P.N1, kBlock));
    if (P.n <= 4) hipLaunchKernelGGL(obj_partial_kernel<4>, dim3(g), dim3(kBlock), 0, stream, P, z, partials);
    else if (P.n <= 8) hipLaunchKernelGGL(obj_partial_kernel<8>, dim3(g), dim3(kBlock), 0, stream, P, z, partials);
    else if (P.n <= 16) hipLaunchKernelGGL(obj_partial_kernel<16>, dim3(g), dim3(kBlock), 0, stream, P, z, partials);
    else hipLaunchKernelGGL(obj_partial_kernel<32>, dim3(g), dim3(kBlock), 0, stream, P, z, partials);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(obj_final_kernel, dim3(1), dim3(kBlock), 0, stream, partials, (int)g, obj);
    return hipGetLastError();
}

hipError_t launch_grad(const KP &P, const double *z, double *g, hipStream_t stream)
{
    dim3 grid(blocks_for(P.N1, kBlock), P.n + P.m);
    hipLaunchKernelGGL(grad_kernel, grid, dim3(kBlock), 0, stream, P, z, g);
    return hipGetLastError();
}

// The trapezoidal defect kernel for the state bound NB, with the controls'
// register array halved when m <= NB/2 (at n = 16, m = 8: 109 VGPRs instead
// of 125, 4 wavefronts per SIMD either way, 1-3 % faster at N = 1e6).  The
// sums run in the same order, so the values are the same bits.
template <int NB>
void launch_cons_trap(const KP &P, unsigned g, const double *z, double *c, hipStream_t stream)
{
    if (P.m <= NB / 2) hipLaunchKernelGGL((cons_kernel<NB, NB / 2>), dim3(g), dim3(kBlock), 0, stream, P, z, c);
    else hipLaunchKernelGGL((cons_kernel<NB, NB>), dim3(g), dim3(kBlock), 0, stream, P, z, c);
}

// The forward-Euler defect kernel, with the same control bound.
template <int NB>
void launch_cons_euler(const KP &P, unsigned g, const double *z, double *c, hipStream_t stream)
{
    if (P.m <= NB / 2) hipLaunchKernelGGL((cons_euler_kernel<NB, NB / 2>), dim3(g), dim3(kBlock), 0, stream, P, z, c);
    else hipLaunchKernelGGL((cons_euler_kernel<NB, NB>), dim3(g), dim3(kBlock), 0, stream, P, z, c);
}

hipError_t launch_cons(const KP &P, const double *z, double *c, hipStream_t stream)
{
    const int n = P.n;
    if (P.scheme == 0) {
        const unsigned g = blocks_for(P.N, kBlock - 1);
        if (n <= 4) launch_cons_trap<4>(P, g, z, c, stream);
        else if (n <= 8) launch_cons_trap<8>(P, g, z, c, stream);
        else if (n <= 16) launch_cons_trap<16>(P, g, z, c, stream);
        else launch_cons_trap<32>(P, g, z, c, stream);
    } else {
        const unsigned g = blocks_for(P.N, kBlock);
        if (n <= 4) launch_cons_euler<4>(P, g, z, c, stream);
        else if (n <= 8) launch_cons_euler<8>(P, g, z, c, stream);
        else if (n <= 16) launch_cons_euler<16>(P, g, z, c, stream);
        else launch_cons_euler<32>(P, g, z, c, stream);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (P.nb > 0)
        hipLaunchKernelGGL(bnd_cons_kernel, dim3(blocks_for(P.nb, kBlock)), dim3(kBlock), 0, stream, P, z, c);
    return hipGetLastError();
}

}  // namespace dev
}  // namespace ocp

extern "C" {

int ocp_create(int64_t N, int32_t n, int32_t m, const double *A, const double *B,
               const double *gamma, const double *q, const double *r, ocp_problem **out)
{
    return ocp_create_ex(N, n, m, nullptr, A, B, gamma, q, r, out);
}

int ocp_create_ex(int64_t N, int32_t n, int32_t m, const ocp_options *opt, const double *A,
                  const double *B, const double *gamma, const double *q, const double *r,
                  ocp_problem **out)
{
    clear_error();
    if (!out) return fail(OCP_ERR_ARG, "ocp_create: out is NULL");
    *out = nullptr;
    Dims d;
    int rc = make_dims_ex(N, n, m, opt ? opt->scheme : OCP_SCHEME_TRAPEZOIDAL,
                          opt ? opt->boundary : OCP_BOUNDARY_NONE, &d);
    if (rc) return rc;
    if (!A || !gamma || !q || (m > 0 && (!B || !r)))
        return fail(OCP_ERR_ARG, "ocp_create: coefficient pointer is NULL");
    for (int64_t x = 0; x < (int64_t)n * n; x++)
        if (!std::isfinite(A[x])) return fail(OCP_ERR_ARG, "ocp_create: A has a non-finite entry");

    ocp_problem *p = new (std::nothrow) ocp_problem();
    if (!p) return fail(OCP_ERR_ALLOC, "ocp_create: out of host memory");
    p->d = d;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) { delete p; return hip_fail("ocp_create: hipGetDevice", e); }
    // locate this device's scratch array of the allocation-free entry point
    // now, outside any stream capture (a failure only disables that entry)
    (void)noalloc_scratch(p->device);
    static_assert(kLd == OCP_MAX_DIM, "padded coefficient columns hold up to OCP_MAX_DIM rows");
    const size_t nplain = (size_t)n * n + (size_t)n * m + 3 * (size_t)n + (size_t)m;
    const size_t ncoef = nplain + (size_t)(n + m) * kLd;
    e = hipMalloc(&p->coef, ncoef * sizeof(double));
    if (e != hipSuccess) { delete p; return fail(OCP_ERR_ALLOC, std::string("ocp_create: hipMalloc: ") + hipGetErrorString(e)); }
    e = hipMalloc(&p->partials, kObjBlocks * sizeof(double));
    if (e == hipSuccess)
        e = hipMalloc(&p->cpart, (size_t)n * (n + m + 1) * coef_blocks(d.N1) * sizeof(double));
    if (e != hipSuccess) {
        ocp_destroy(p);
        return fail(OCP_ERR_ALLOC, std::string("ocp_create: hipMalloc: ") + hipGetErrorString(e));
    }
    double *host = new (std::nothrow) double[ncoef];
    if (!host) { ocp_destroy(p); return fail(OCP_ERR_ALLOC, "ocp_create: out of host memory"); }
    size_t o = 0;
    std::memcpy(host + o, A, sizeof(double) * n * n); o += (size_t)n * n;
    if (m) std::memcpy(host + o, B, sizeof(double) * n * m); o += (size_t)n * m;
    std::memcpy(host + o, gamma, sizeof(double) * n); o += n;
    std::memcpy(host + o, q, sizeof(double) * n); o += n;
    if (m) std::memcpy(host + o, r, sizeof(double) * m);
    pack_columns(n, m, A, B, host + nplain, host + nplain + (size_t)n * kLd);
    e = hipMemcpy(p->coef, host, ncoef * sizeof(double), hipMemcpyHostToDevice);
    delete[] host;
    if (e != hipSuccess) { ocp_destroy(p); return hip_fail("ocp_create: hipMemcpy", e); }

    KP &kp = p->kp;
    kp.N = (int)d.N;
    kp.N1 = (int)d.N1;
    kp.n = n;
    kp.m = m;
    kp.npair = d.npair;
    kp.T = d.T;
    kp.S = d.S;
    kp.nnzk = (int)d.nnzk;
    kp.NU = (int)d.NU;
    kp.scheme = d.scheme;
    kp.nb = (int)d.nb;
    kp.h = 1.0 / (double)d.N;
    kp.hh = 0.5 * kp.h;
    kp.A = p->coef;
    kp.B = p->coef + (size_t)n * n;
    kp.gam = kp.B + (size_t)n * m;
    kp.q = kp.gam + n;
    kp.r = kp.q + n;
    kp.AT = p->coef + nplain;
    kp.BT = kp.AT + (size_t)n * kLd;
    *out = p;
    return OCP_OK;
}

void ocp_destroy(ocp_problem *p)
{
    if (!p) return;
    if (p->coef) (void)hipFree(p->coef);
    if (p->partials) (void)hipFree(p->partials);
    if (p->cpart) (void)hipFree(p->cpart);
    if (p->mplan) (void)hipFree(p->mplan);
    delete p;
}

int ocp_problem_sizes(const ocp_problem *p, ocp_sizes_t *out)
{
    clear_error();
    if (int rc = check_handle(p, "ocp_problem_sizes")) return rc;
    if (!out) return fail(OCP_ERR_ARG, "ocp_problem_sizes: out is NULL");
    to_public(p->d, out);
    return OCP_OK;
}

int ocp_eval_obj(const ocp_problem *p, const double *z, double *obj, hipStream_t stream)
{
    clear_error();
    if (int rc = check_handle(p, "ocp_eval_obj")) return rc;
    if (!z || !obj) return fail(OCP_ERR_ARG, "ocp_eval_obj: null array");
    if (p->model == quad::kModel) return quad::eval_obj(p, z, obj, stream);
    const hipError_t e = launch_obj(p->kp, z, p->partials, obj, stream);
    if (e != hipSuccess) return hip_fail("ocp_eval_obj", e);
    return OCP_OK;
}

int ocp_eval_grad(const ocp_problem *p, const double *z, double *g, hipStream_t stream)
{
    clear_error();
    if (int rc = check_handle(p, "ocp_eval_grad")) return rc;
    if (!z || !g) return fail(OCP_ERR_ARG, "ocp_eval_grad: null array");
    if (p->model == quad::kModel) return quad::eval_grad(p, z, g, stream);
    const hipError_t e = launch_grad(p->kp, z, g, stream);
    if (e != hipSuccess) return hip_fail("ocp_eval_grad", e);
    return OCP_OK;
}

int ocp_eval_cons(const ocp_problem *p, const double *z, double *c, hipStream_t stream)
{
    clear_error();
    if (int rc = check_handle(p, "ocp_eval_cons")) return rc;
    if (!z || !c) return fail(OCP_ERR_ARG, "ocp_eval_cons: null array");
    if (p->model == quad::kModel) return quad::eval_cons(p, z, c, stream);
    const hipError_t e = launch_cons(p->kp, z, c, stream);
    if (e != hipSuccess) return hip_fail("ocp_eval_cons", e);
    return OCP_OK;
}

int ocp_eval_jac(const ocp_problem *p, const double *z, double *jvals, hipStream_t stream)
{
    clear_error();
    if (int rc = check_handle(p, "ocp_eval_jac")) return rc;
    if (!z || !jvals) return fail(OCP_ERR_ARG, "ocp_eval_jac: null array");
    if (p->model == quad::kModel) return quad::eval_jac(p, z, jvals, stream);
    const hipError_t e = launch_jac(p->kp, z, jvals, (uintptr_t)jvals % 16 == 0, stream);
    if (e != hipSuccess) return hip_fail("ocp_eval_jac", e);
    return OCP_OK;
}

int ocp_eval_hess(const ocp_problem *p, const double *z, const double *y, double sigma,
                  double *hvals, hipStream_t stream)
{
    clear_error();
    if (int rc = check_handle(p, "ocp_eval_hess")) return rc;
    if (!z || !y || !hvals) return fail(OCP_ERR_ARG, "ocp_eval_hess: null array");
    if (!std::isfinite(sigma)) return fail(OCP_ERR_ARG, "ocp_eval_hess: sigma is not finite");
    if (p->model == quad::kModel) return quad::eval_hess(p, z, y, sigma, hvals, stream);
    const hipError_t e = launch_hess(p->kp, z, y, sigma, hvals, stream);
    if (e != hipSuccess) return hip_fail("ocp_eval_hess", e);
    return OCP_OK;
}

int ocp_assemble_kkt(const ocp_problem *p, const int32_t *perm_j, const int32_t *perm_h,
                     const int32_t *rowptr, const double *jvals, const double *hvals,
                     const double *reg, double *kkt, hipStream_t stream)
{
    clear_error();
    if (int rc = check_handle(p, "ocp_assemble_kkt")) return rc;
    if (!perm_j || !perm_h || !rowptr || !jvals || !hvals || !kkt)
        return fail(OCP_ERR_ARG, "ocp_assemble_kkt: null array");
    if (p->model == quad::kModel)
        return quad::assemble_kkt(p, perm_j, perm_h, rowptr, jvals, hvals, reg, kkt, stream);
    // Tile height: 64 constraint rows (one per lane) while the staged CSR
    // range fits in 64 KiB of LDS, else 32.
    const int KT = (64 * (p->d.T + 1) * 8 <= 64 * 1024) ? 64 : 32;
    const unsigned tiles_per_i = (unsigned)((p->d.N + KT - 1) / KT);
    const unsigned gj = tiles_per_i * (unsigned)p->d.n;
    const unsigned gh = blocks_for(p->d.N1, kBlock);
    const unsigned gb = blocks_for(p->d.nb, kBlock);
    const size_t lds = (size_t)KT * (p->d.T + 1) * sizeof(double);
    // paired loads need 16-byte aligned values and 8-byte aligned slots
    const bool vec_ok = ((uintptr_t)jvals % 16 == 0) && ((uintptr_t)perm_j % 8 == 0);
    hipLaunchKernelGGL(assemble_kernel, dim3(gj + gh + gb), dim3(kBlock), lds, stream, p->kp, (int)gj,
                       (int)gh, KT, vec_ok, perm_j, perm_h, rowptr, jvals, hvals, reg, kkt);
    return check_launch("ocp_assemble_kkt");
}

}  // extern "C"
