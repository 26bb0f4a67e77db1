// Host index layer of the quadrotor model: sizes, the Jacobian / Hessian COO
// patterns and the lower-triangular CSR of the KKT matrix with its slot maps,
// in closed form from N and the node-local tables of ocp_quad_model.h (the
// one-time host symbolic step of paper Sec. 6).  No HIP call is made here.
#include <algorithm>
#include <string>
#include <thread>
#include <vector>

#include "ocp_internal.h"
#include "ocp_quad.h"
#include "ocp_quad_model.h"

namespace ocp {
namespace quad {

int make_dims(int64_t N, int32_t bnd, Dims *d)
{
    if (!d) return fail(OCP_ERR_ARG, "null output pointer");
    if (N < 1) return fail(OCP_ERR_ARG, "N must be >= 1 (got " + std::to_string(N) + ")");
    if (bnd < OCP_BOUNDARY_NONE || bnd > OCP_BOUNDARY_INITIAL_FINAL)
        return fail(OCP_ERR_ARG, "unknown boundary option " + std::to_string(bnd));
    if (N > INT32_MAX) return fail(OCP_ERR_OVERFLOW, "N does not fit in int32");
    Dims r;
    r.N = N;
    r.n = kStates;
    r.m = kControls;
    r.npair = 0;
    r.T = kSlots;
    r.S = kHessNode;
    r.scheme = OCP_SCHEME_TRAPEZOIDAL;
    r.bnd = bnd;
    r.N1 = N + 1;
    r.NU = N + 1;
    r.nvar = (int64_t)kVars * r.N1;
    r.ndef = (int64_t)kStates * N;
    r.nb = (int64_t)kStates * bnd;
    r.ncon = r.ndef + r.nb;
    r.nnzj_def = (int64_t)kSlots * N;
    r.nnzj = r.nnzj_def + r.nb;
    r.nnzh = (int64_t)kHessNode * r.N1;
    r.nnzk = r.nnzh + r.nnzj + r.ncon;
    r.dim = r.nvar + r.ncon;
    if (r.nnzk > INT32_MAX || r.dim + 1 > INT32_MAX)
        return fail(OCP_ERR_OVERFLOW, "KKT size " + std::to_string(r.nnzk) + " entries / " +
                                          std::to_string(r.dim) + " rows does not fit in int32");
    *d = r;
    return OCP_OK;
}

namespace {

// Run body(lo, hi) over [0, count) split across host threads.
template <class F>
void parallel_range(int64_t count, F body)
{
    unsigned hw = std::thread::hardware_concurrency();
    int64_t nt = std::max<int64_t>(1, std::min<int64_t>(hw ? hw : 1, 64));
    if (count < 65536) nt = 1;
    nt = std::min<int64_t>(nt, count);
    if (nt <= 1) {
        body((int64_t)0, count);
        return;
    }
    std::vector<std::thread> th;
    th.reserve(nt);
    for (int64_t t = 0; t < nt; t++) {
        int64_t lo = count * t / nt, hi = count * (t + 1) / nt;
        th.emplace_back([=] { body(lo, hi); });
    }
    for (auto &x : th) x.join();
}

// Offsets of the KKT's row blocks.  Variable rows come first, grouped by
// variable v (N+1 rows of kHessFirst[v+1] - kHessFirst[v] entries each), then
// the defect rows grouped by state i (N rows of 2 kSupLen[i] + 1 entries),
// then the boundary rows (2 entries each).
struct KktLayout {
    int64_t var_start[kVars];
    int64_t def_start[kStates];
    int64_t bnd_start;
};

KktLayout layout(const Dims &d)
{
    KktLayout L;
    int64_t o = 0;
    for (int v = 0; v < kVars; v++) {
        L.var_start[v] = o;
        o += (int64_t)(kHessFirst[v + 1] - kHessFirst[v]) * d.N1;
    }
    for (int i = 0; i < kStates; i++) {
        L.def_start[i] = o;
        o += (int64_t)(kRowSlot[i + 1] - kRowSlot[i] + 1) * d.N;
    }
    L.bnd_start = o;
    return L;
}

}  // namespace

}  // namespace quad
}  // namespace ocp

using namespace ocp;
using namespace ocp::quad;

extern "C" {

int ocp_quad_sizes(int64_t N, int32_t boundary, ocp_sizes_t *out)
{
    clear_error();
    if (!out) return fail(OCP_ERR_ARG, "ocp_quad_sizes: out is NULL");
    Dims d;
    if (int rc = make_dims(N, boundary, &d)) return rc;
    to_public(d, out);
    return OCP_OK;
}

int ocp_quad_pattern(int64_t N, int32_t boundary, int32_t *jrow, int32_t *jcol, int32_t *hrow,
                     int32_t *hcol)
{
    clear_error();
    Dims d;
    if (int rc = make_dims(N, boundary, &d)) return rc;
    const int64_t N1 = d.N1;
    if (jrow || jcol) {
        // defect entry (i, p-th support variable, side s) of interval k sits at
        // (kRowSlot[i] + 2p + s) N + k
        parallel_range((int64_t)kSlots, [&](int64_t lo, int64_t hi) {
            for (int64_t slot = lo; slot < hi; slot++) {
                int i = 0;
                while (kRowSlot[i + 1] <= slot) i++;
                const int p = (int)(slot - kRowSlot[i]) / 2, s = (int)(slot - kRowSlot[i]) % 2;
                const int64_t v = kSup[i][p];
                for (int64_t k = 0; k < N; k++) {
                    const int64_t e = slot * N + k;
                    if (jrow) jrow[e] = (int32_t)(i * N + k);
                    if (jcol) jcol[e] = (int32_t)(v * N1 + k + s);
                }
            }
        });
        for (int64_t b = 0; b < d.nb; b++) {
            const int64_t e = d.nnzj_def + b;
            if (jrow) jrow[e] = (int32_t)(d.ndef + b);
            if (jcol) jcol[e] = (int32_t)((b % kStates) * N1 + (b < kStates ? 0 : N));
        }
    }
    if (hrow || hcol) {
        parallel_range((int64_t)kHessNode, [&](int64_t lo, int64_t hi) {
            for (int64_t s = lo; s < hi; s++)
                for (int64_t k = 0; k < N1; k++) {
                    if (hrow) hrow[s * N1 + k] = (int32_t)(kHessRow[s] * N1 + k);
                    if (hcol) hcol[s * N1 + k] = (int32_t)(kHessCol[s] * N1 + k);
                }
        });
    }
    return OCP_OK;
}

int ocp_quad_kkt(int64_t N, int32_t boundary, int32_t *rowptr, int32_t *colind, int32_t *perm_j,
                 int32_t *perm_h)
{
    clear_error();
    Dims d;
    if (int rc = make_dims(N, boundary, &d)) return rc;
    const int64_t N1 = d.N1, nvar = d.nvar;
    const KktLayout L = layout(d);
    // variable rows: the Hessian entries of row v at node k, ascending columns
    for (int v = 0; v < kVars; v++) {
        const int f = kHessFirst[v], len = kHessFirst[v + 1] - f;
        parallel_range(N1, [&](int64_t lo, int64_t hi) {
            for (int64_t k = lo; k < hi; k++) {
                const int64_t start = L.var_start[v] + (int64_t)len * k;
                const int64_t row = v * N1 + k;
                if (rowptr) rowptr[row] = (int32_t)start;
                for (int t = 0; t < len; t++) {
                    if (colind) colind[start + t] = (int32_t)(kHessCol[f + t] * N1 + k);
                    if (perm_h) perm_h[(int64_t)(f + t) * N1 + k] = (int32_t)(start + t);
                }
            }
        });
    }
    // defect rows: the row's Jacobian entries, then the diagonal
    for (int i = 0; i < kStates; i++) {
        const int f = kRowSlot[i], len = kRowSlot[i + 1] - f;
        parallel_range(N, [&](int64_t lo, int64_t hi) {
            for (int64_t k = lo; k < hi; k++) {
                const int64_t start = L.def_start[i] + (int64_t)(len + 1) * k;
                const int64_t row = nvar + i * N + k;
                if (rowptr) rowptr[row] = (int32_t)start;
                for (int t = 0; t < len; t++) {
                    if (colind) colind[start + t] = (int32_t)(kSup[i][t / 2] * N1 + k + t % 2);
                    if (perm_j) perm_j[(int64_t)(f + t) * N + k] = (int32_t)(start + t);
                }
                if (colind) colind[start + len] = (int32_t)row;
            }
        });
    }
    // boundary rows: their state entry, then the diagonal
    for (int64_t b = 0; b < d.nb; b++) {
        const int64_t start = L.bnd_start + 2 * b;
        const int64_t row = nvar + d.ndef + b;
        if (rowptr) rowptr[row] = (int32_t)start;
        if (colind) {
            colind[start] = (int32_t)((b % kStates) * N1 + (b < kStates ? 0 : N));
            colind[start + 1] = (int32_t)row;
        }
        if (perm_j) perm_j[d.nnzj_def + b] = (int32_t)start;
    }
    if (rowptr) rowptr[d.dim] = (int32_t)d.nnzk;
    return OCP_OK;
}

}  // extern "C"
