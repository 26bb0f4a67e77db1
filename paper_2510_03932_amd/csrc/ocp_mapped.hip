// KKT assembly through slot maps alone (ocp_assemble_kkt_mapped): the slot
// maps may come from any symmetric reordering of the KKT matrix, so the
// assembly writes P K P^T directly (paper Sec. 6: the host analysis reorders
// the matrix once; folding the ordering into the slot maps saves a device
// permutation of the values before every factorization).
//
// Work is tiled by grid node: workgroup t owns nodes [t KT, (t+1) KT) and
// every entry whose row, in a node-grouped ordering, belongs to one of those
// nodes -- the Hessian entries of the nodes, the Jacobian entries whose
// column sits at the node (interval k's entries at node k+1 go with node
// k+1), the defect-row diagonals of the intervals starting there and the
// boundary rows fixed there.  A first pass reads the tile's slots and finds
// their range; if the tile fills [min, max] exactly (as under
// ocp_stage_order), the values are staged in LDS and the range is written
// with contiguous stores, else every value is stored at its slot.  The
// ranges depend on the slot maps only, so ocp_mapped_plan can record them
// once and later assemblies skip the first pass.  The result is the same for
// every injective slot map; no atomics touch global memory.
#include <hip/hip_runtime.h>

#include <climits>
#include <mutex>
#include <string>

#include "ocp_device.h"
#include "ocp_problem.h"
#include "ocp_quad.h"
#include "ocp_quad_model.h"

using namespace ocp;
using namespace ocp::dev;

namespace {

constexpr int kMapTarget = 2048;  // values staged per workgroup when a node fits (16 KiB)
constexpr int kMapCap = 7936;     // most values staged per workgroup (62 KiB of LDS)

struct MP {
    int N, N1, NU;
    int n;          // defect rows per interval
    int T;          // Jacobian slots per defect row (synthetic family)
    int nJ;         // Jacobian slot rows per interval
    int sA, sB;     // Hessian slot rows of stride N+1, then of stride NU
    int npair;      // synthetic family: bilinear slots after the n state diagonals
    int euler;      // synthetic family under forward Euler
    int quad;       // quadrotor model
    int nb, bnd;
    int64_t nvar, ndef, nnzj_def;
    int nnzk;
    int KT, lgKT;
    int cap;  // LDS tile capacity (values)
};

// Node offset (0 or 1) of the column of Jacobian slot row sigma.
__device__ __forceinline__ int jac_side(const MP &P, int sigma)
{
    if (!P.euler) return sigma & 1;  // trapezoidal rows alternate (node k, node k+1)
    const int i = sigma / P.T, t = sigma - i * P.T;
    return t == i + 1 ? 1 : 0;       // Euler: only the row's own state at k+1
}

// Variable row of Hessian slot row s at node k if it is a diagonal, else -1.
__device__ __forceinline__ int64_t hess_diag_row(const MP &P, int s, int64_t k)
{
    if (P.quad) {
        return quad::kHessRow[s] == quad::kHessCol[s] ? (int64_t)quad::kHessRow[s] * P.N1 + k : -1;
    }
    if (s < P.n) return (int64_t)s * P.N1 + k;
    if (s < P.sA) return -1;
    return (int64_t)P.n * P.N1 + (int64_t)(s - P.sA) * P.NU + k;
}

// Every entry of tile `tb` (nodes [tb KT, tb KT + KT)) is passed to
// put(slot, value); with_values = false skips the value loads.
template <class F>
__device__ __forceinline__ void tile_visit(const MP &P, int64_t tb, const int32_t *__restrict__ perm_j,
                                           const int32_t *__restrict__ perm_h, const int32_t *__restrict__ diag,
                                           const double *__restrict__ jv, const double *__restrict__ hv,
                                           const double *__restrict__ reg, bool with_values, F put)
{
    const int KT = P.KT, lg = P.lgKT;
    const int64_t k0 = tb * KT;
    const int64_t N = P.N, N1 = P.N1, NU = P.NU;
    const int nJ = P.nJ, sA = P.sA, sB = P.sB, n = P.n;
    // segment sizes of the tile's work list
    const int s1 = nJ << lg, s2 = sA << lg, s3 = sB << lg, s4 = n << lg, s5 = 2 * n;
    const int total = s1 + s2 + s3 + s4 + s5;
    const bool first = k0 == 0, last = k0 + KT > N;
    for (int w = threadIdx.x; w < total; w += kBlock) {
        int32_t q;
        double v = 0.0;
        if (w < s1) {
            const int sigma = w >> lg;
            const int64_t k = k0 - jac_side(P, sigma) + (w & (KT - 1));
            if (k < 0 || k >= N) continue;
            const int64_t e = (int64_t)sigma * N + k;
            q = perm_j[e];
            if (with_values) v = jv[e];
        } else if (w < s1 + s2) {
            const int x = w - s1;
            const int s = x >> lg;
            const int64_t k = k0 + (x & (KT - 1));
            if (k >= N1) continue;
            const int64_t e = (int64_t)s * N1 + k;
            q = perm_h[e];
            if (with_values) {
                v = hv[e];
                if (reg) {
                    const int64_t row = hess_diag_row(P, s, k);
                    if (row >= 0) v += reg[row];
                }
            }
        } else if (w < s1 + s2 + s3) {
            const int x = w - s1 - s2;
            const int l = x >> lg;
            const int64_t k = k0 + (x & (KT - 1));
            if (k >= NU) continue;
            const int64_t e = (int64_t)sA * N1 + (int64_t)l * NU + k;
            q = perm_h[e];
            if (with_values) {
                v = hv[e];
                if (reg) v += reg[(int64_t)n * N1 + (int64_t)l * NU + k];
            }
        } else if (w < s1 + s2 + s3 + s4) {
            const int x = w - s1 - s2 - s3;
            const int i = x >> lg;
            const int64_t k = k0 + (x & (KT - 1));
            if (k >= N) continue;
            const int64_t row = P.nvar + (int64_t)i * N + k;
            q = diag[row];
            if (with_values && reg) v = reg[row];
        } else {
            // boundary rows: the initial ones with node 0, the final ones with node N
            const int b = w - s1 - s2 - s3 - s4;
            if (b >= P.nb) continue;
            if (b < n ? !first : !last) continue;
            const int64_t e = P.nnzj_def + b;
            const int64_t row = P.nvar + P.ndef + b;
            q = perm_j[e];
            if (with_values) v = jv[e];
            put(q, v);
            q = diag[row];
            v = (with_values && reg) ? reg[row] : 0.0;
        }
        put(q, v);
    }
}

// Range of tile blockIdx.x's slots: (base, count) with base = -1 unless the
// slots fill [base, base + count) exactly and the range fits the LDS tile.
__device__ __forceinline__ int2 tile_range(const MP &P, const int32_t *__restrict__ perm_j,
                                           const int32_t *__restrict__ perm_h, const int32_t *__restrict__ diag)
{
    __shared__ int smin, smax, scount;
    if (threadIdx.x == 0) {
        smin = INT_MAX;
        smax = INT_MIN;
        scount = 0;
    }
    __syncthreads();
    int lmin = INT_MAX, lmax = INT_MIN, lcount = 0;
    tile_visit(P, blockIdx.x, perm_j, perm_h, diag, nullptr, nullptr, nullptr, false, [&](int32_t q, double) {
        lmin = min(lmin, (int)q);
        lmax = max(lmax, (int)q);
        lcount++;
    });
    if (lcount) {
        atomicMin(&smin, lmin);
        atomicMax(&smax, lmax);
        atomicAdd(&scount, lcount);
    }
    __syncthreads();
    const int qmin = smin, qmax = smax, count = scount;
    const bool exact = count > 0 && qmin >= 0 && qmax < P.nnzk && count <= P.cap && qmax - qmin + 1 == count;
    return int2{exact ? qmin : -1, count};
}

// The plan of a set of slot maps: tile_range of every tile.
__global__ __launch_bounds__(kBlock) void mapped_plan_kernel(MP P, const int32_t *__restrict__ perm_j,
                                                             const int32_t *__restrict__ perm_h,
                                                             const int32_t *__restrict__ diag,
                                                             int32_t *__restrict__ plan)
{
    const int2 r = tile_range(P, perm_j, perm_h, diag);
    if (threadIdx.x == 0) {
        plan[2 * blockIdx.x] = r.x;
        plan[2 * blockIdx.x + 1] = r.y;
    }
}

__global__ __launch_bounds__(kBlock) void mapped_assemble_kernel(
    MP P, const int32_t *__restrict__ plan, const int32_t *__restrict__ perm_j, const int32_t *__restrict__ perm_h,
    const int32_t *__restrict__ diag, const double *__restrict__ jv, const double *__restrict__ hv,
    const double *__restrict__ reg, double *__restrict__ kkt)
{
    extern __shared__ double tile[];  // the tile's entries (host-sized, <= kMapCap)
    __shared__ int filled;            // tile slots written by this tile's entries
    int base, count;
    if (plan) {
        base = plan[2 * blockIdx.x];
        count = plan[2 * blockIdx.x + 1];
        // a plan from other slot maps must not send stores out of bounds
        if (base < 0 || count < 1 || count > P.cap || (int64_t)base + count > P.nnzk) base = -1;
    } else {
        const int2 r = tile_range(P, perm_j, perm_h, diag);
        base = r.x;
        count = r.y;
    }
    if (base >= 0) {
        if (threadIdx.x == 0) filled = 0;
        __syncthreads();
        int mine = 0;
        tile_visit(P, blockIdx.x, perm_j, perm_h, diag, jv, hv, reg, true, [&](int32_t q, double v) {
            const uint32_t loc = (uint32_t)q - (uint32_t)base;
            if (loc < (uint32_t)count) {
                tile[loc] = v;
                mine++;
            } else if ((uint32_t)q < (uint32_t)P.nnzk) {
                kkt[q] = v;
            }
        });
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) mine += __shfl_down(mine, off, 64);
        if ((threadIdx.x & 63) == 0 && mine) atomicAdd(&filled, mine);
        __syncthreads();
        if (filled == count) {
            // the tile's slots (distinct, the maps being injective) cover the
            // range exactly: write it with contiguous stores
            double *out = kkt + base;
            for (int x = threadIdx.x; x < count; x += kBlock) st_nt(out + x, tile[x]);
            return;
        }
        // else a plan made from other slot maps: the staged values go to
        // their slots one by one below (values stored above are stored again)
    }
    tile_visit(P, blockIdx.x, perm_j, perm_h, diag, jv, hv, reg, true, [&](int32_t q, double v) {
        if ((uint32_t)q < (uint32_t)P.nnzk) kkt[q] = v;
    });
}

// Tile shape for a handle: the largest power of two of nodes whose entries
// fit a 16 KiB tile (small tiles keep several workgroups per CU), but at
// least 4 nodes while they fit the 62 KiB maximum.
MP make_mp(const ocp_problem *p)
{
    const Dims &d = p->d;
    MP P;
    P.N = (int)d.N;
    P.N1 = (int)d.N1;
    P.NU = (int)d.NU;
    P.n = d.n;
    P.quad = p->model == quad::kModel ? 1 : 0;
    P.euler = (!P.quad && d.scheme == OCP_SCHEME_EULER) ? 1 : 0;
    P.T = d.T;
    P.nJ = P.quad ? quad::kSlots : d.n * d.T;
    P.sA = P.quad ? quad::kHessNode : d.n + d.npair;
    P.sB = P.quad ? 0 : d.m;
    P.npair = P.quad ? 0 : d.npair;
    P.nb = (int)d.nb;
    P.bnd = d.bnd;
    P.nvar = d.nvar;
    P.ndef = d.ndef;
    P.nnzj_def = d.nnzj_def;
    P.nnzk = (int)d.nnzk;
    const int64_t per_node = (int64_t)P.nJ + P.sA + P.sB + P.n;
    auto need = [&](int lgk) { return ((int64_t)1 << lgk) * per_node + 2 * P.n; };
    int lg = 0;
    while (lg < 10 && need(lg + 1) <= kMapTarget) lg++;
    while (lg < 2 && need(lg + 1) <= kMapCap) lg++;
    P.KT = 1 << lg;
    P.lgKT = lg;
    P.cap = (int)need(lg);
    return P;
}

}  // namespace

extern "C" {

int ocp_mapped_plan_size(const ocp_problem *p, int64_t *entries)
{
    clear_error();
    if (int rc = check_handle(p, "ocp_mapped_plan_size")) return rc;
    if (!entries) return fail(OCP_ERR_ARG, "ocp_mapped_plan_size: entries is NULL");
    const MP P = make_mp(p);
    *entries = 2 * (int64_t)blocks_for(p->d.N1, P.KT);
    return OCP_OK;
}

int ocp_mapped_plan(const ocp_problem *p, const int32_t *perm_j, const int32_t *perm_h, const int32_t *diag,
                    int32_t *plan, hipStream_t stream)
{
    clear_error();
    if (int rc = check_handle(p, "ocp_mapped_plan")) return rc;
    if (!perm_j || !perm_h || !diag || !plan) return fail(OCP_ERR_ARG, "ocp_mapped_plan: null array");
    const MP P = make_mp(p);
    hipLaunchKernelGGL(mapped_plan_kernel, dim3(blocks_for(p->d.N1, P.KT)), dim3(kBlock), 0, stream, P, perm_j,
                       perm_h, diag, plan);
    return check_launch("ocp_mapped_plan");
}

int ocp_assemble_kkt_mapped(const ocp_problem *p, const int32_t *perm_j, const int32_t *perm_h,
                            const int32_t *diag, const int32_t *plan, const double *jvals, const double *hvals,
                            const double *reg, double *kkt, hipStream_t stream)
{
    clear_error();
    if (int rc = check_handle(p, "ocp_assemble_kkt_mapped")) return rc;
    if (!perm_j || !perm_h || !diag || !jvals || !hvals || !kkt)
        return fail(OCP_ERR_ARG, "ocp_assemble_kkt_mapped: null array");
    const MP P = make_mp(p);
    if (!plan) {
        // the handle keeps the plan of the slot maps it last assembled from
        // (keyed by their addresses; a stale plan is caught per tile by the
        // kernel's exact-cover check and costs speed, not correctness)
        std::lock_guard<std::mutex> lock(p->mplan_mu);
        const int64_t len = 2 * (int64_t)blocks_for(p->d.N1, P.KT);
        if (!p->mplan) {
            if (hipMalloc(&p->mplan, (size_t)len * sizeof(int32_t)) != hipSuccess) {
                (void)hipGetLastError();  // no plan: every tile finds its own range
                p->mplan = nullptr;
            }
            p->mplan_key[0] = p->mplan_key[1] = p->mplan_key[2] = nullptr;
        }
        if (p->mplan) {
            if (p->mplan_key[0] != perm_j || p->mplan_key[1] != perm_h || p->mplan_key[2] != diag) {
                hipLaunchKernelGGL(mapped_plan_kernel, dim3(blocks_for(p->d.N1, P.KT)), dim3(kBlock), 0, stream,
                                   P, perm_j, perm_h, diag, p->mplan);
                if (int rc = check_launch("ocp_assemble_kkt_mapped: plan")) return rc;
                p->mplan_key[0] = perm_j;
                p->mplan_key[1] = perm_h;
                p->mplan_key[2] = diag;
            }
            plan = p->mplan;
        }
    }
    hipLaunchKernelGGL(mapped_assemble_kernel, dim3(blocks_for(p->d.N1, P.KT)), dim3(kBlock),
                       (size_t)P.cap * sizeof(double), stream, P, plan, perm_j, perm_h, diag, jvals, hvals, reg, kkt);
    return check_launch("ocp_assemble_kkt_mapped");
}

}  // extern "C"
