// Host symmetric reordering of the KKT matrix (paper Sec. 6: the one-time
// host analysis reorders the matrix for a sparse LDL^T factorization).
//
//   ocp_stage_order / ocp_quad_stage_order: a fill-reducing ordering in
//     closed form.  Unknowns and rows are grouped by grid node: node k's
//     block holds its states, its controls, the boundary rows fixed at it,
//     then the defect rows of interval k.  The KKT matrix becomes banded with
//     a bandwidth independent of N, so the LDL^T fill grows linearly in N
//     (in the natural component-major order it grows superlinearly).
//   ocp_kkt_permute: the lower CSR of P K P^T for any ordering, with the
//     Jacobian / Hessian slot maps and every row's diagonal slot carried over,
//     so that device-side assembly writes the reordered matrix directly.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "ocp_internal.h"
#include "ocp_quad.h"

namespace ocp {
namespace {

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

void stage_order(const Dims &d, int32_t *order)
{
    const int64_t N = d.N, N1 = d.N1, NU = d.NU, n = d.n, m = d.m;
    // position of node k's block: states and controls of nodes < k, the
    // initial boundary rows (k > 0), the defect rows of intervals < k
    auto block_start = [&](int64_t k) {
        int64_t p = n * k + m * std::min(k, NU) + n * k;
        if (k > 0 && d.bnd >= 1) p += n;
        return p;
    };
    parallel_range(N1, [&](int64_t lo, int64_t hi) {
        for (int64_t k = lo; k < hi; k++) {
            int64_t p = block_start(k);
            for (int64_t j = 0; j < n; j++) order[p++] = (int32_t)(j * N1 + k);
            if (k < NU)
                for (int64_t l = 0; l < m; l++) order[p++] = (int32_t)(n * N1 + l * NU + k);
            if (k == 0 && d.bnd >= 1)
                for (int64_t b = 0; b < n; b++) order[p++] = (int32_t)(d.nvar + d.ndef + b);
            if (k == N && d.bnd == 2)
                for (int64_t b = 0; b < n; b++) order[p++] = (int32_t)(d.nvar + d.ndef + n + b);
            if (k < N)
                for (int64_t i = 0; i < n; i++) order[p++] = (int32_t)(d.nvar + i * N + k);
        }
    });
}

}  // namespace
}  // namespace ocp

using namespace ocp;

extern "C" {

int ocp_stage_order(int64_t N, int32_t n, int32_t m, const ocp_options *opt, int32_t *order)
{
    clear_error();
    Dims d;
    if (int rc = make_dims_ex(N, n, m, opt ? opt->scheme : OCP_SCHEME_TRAPEZOIDAL,
                              opt ? opt->boundary : OCP_BOUNDARY_NONE, &d))
        return rc;
    if (!order) return fail(OCP_ERR_ARG, "ocp_stage_order: order is NULL");
    stage_order(d, order);
    return OCP_OK;
}

int ocp_quad_stage_order(int64_t N, int32_t boundary, int32_t *order)
{
    clear_error();
    Dims d;
    if (int rc = quad::make_dims(N, boundary, &d)) return rc;
    if (!order) return fail(OCP_ERR_ARG, "ocp_quad_stage_order: order is NULL");
    stage_order(d, order);
    return OCP_OK;
}

int ocp_kkt_permute(int64_t dim, const int32_t *rowptr, const int32_t *colind, int64_t nnzj,
                    const int32_t *perm_j, int64_t nnzh, const int32_t *perm_h, const int32_t *order,
                    int32_t *rowptr2, int32_t *colind2, int32_t *perm_j2, int32_t *perm_h2,
                    int32_t *diag2)
{
    clear_error();
    if (dim < 1 || dim >= INT32_MAX) return fail(OCP_ERR_ARG, "ocp_kkt_permute: dim out of range");
    if (!rowptr || !colind || !order || !rowptr2 || !colind2)
        return fail(OCP_ERR_ARG, "ocp_kkt_permute: null array");
    if ((nnzj > 0 && (!perm_j) != (!perm_j2)) || (nnzh > 0 && (!perm_h) != (!perm_h2)) || nnzj < 0 ||
        nnzh < 0)
        return fail(OCP_ERR_ARG, "ocp_kkt_permute: slot maps must be given in pairs");
    const int64_t nnzk = rowptr[dim];
    if (rowptr[0] != 0 || nnzk < dim) return fail(OCP_ERR_ARG, "ocp_kkt_permute: rowptr is not a CSR row pointer");
    std::vector<int32_t> pos;
    std::vector<int32_t> cnt;
    std::unique_ptr<int32_t[]> ent, src, map;  // per new-row columns and old slots; old -> new slot
    try {
        pos.assign((size_t)dim, -1);
        cnt.assign((size_t)dim + 1, 0);
        ent.reset(new int32_t[(size_t)nnzk]);
        src.reset(new int32_t[(size_t)nnzk]);
        map.reset(new int32_t[(size_t)nnzk]);
    } catch (const std::bad_alloc &) {
        return fail(OCP_ERR_ALLOC, "ocp_kkt_permute: out of host memory");
    }
    for (int64_t i = 0; i < dim; i++) {
        const int64_t o = order[i];
        if (o < 0 || o >= dim || pos[o] >= 0) return fail(OCP_ERR_ARG, "ocp_kkt_permute: order is not a permutation");
        pos[o] = (int32_t)i;
    }
    for (int64_t r = 0; r < dim; r++)
        if (rowptr[r + 1] < rowptr[r]) return fail(OCP_ERR_ARG, "ocp_kkt_permute: rowptr decreases");
    // count the entries of every new row (threads over old rows, atomic counters)
    std::atomic<bool> upper{false};
    parallel_range(dim, [&](int64_t lo, int64_t hi) {
        bool local = false;
        for (int64_t r = lo; r < hi; r++)
            for (int64_t q = rowptr[r]; q < rowptr[r + 1]; q++) {
                const int64_t c = colind[q];
                if (c < 0 || c > r) {
                    local = true;
                    continue;
                }
                __atomic_fetch_add(&cnt[std::max(pos[r], pos[c]) + 1], 1, __ATOMIC_RELAXED);
            }
        if (local) upper = true;
    });
    if (upper) return fail(OCP_ERR_ARG, "ocp_kkt_permute: colind is not lower triangular");
    rowptr2[0] = 0;
    for (int64_t i = 0; i < dim; i++) rowptr2[i + 1] = rowptr2[i] + cnt[i + 1];
    // scatter every entry to its new row; the order inside a row is fixed by
    // the per-row sort below, so the result does not depend on the threads
    std::vector<int32_t> fill(rowptr2, rowptr2 + dim);
    parallel_range(dim, [&](int64_t lo, int64_t hi) {
        for (int64_t r = lo; r < hi; r++)
            for (int64_t q = rowptr[r]; q < rowptr[r + 1]; q++) {
                const int32_t a = pos[r], b = pos[colind[q]];
                const int32_t row = std::max(a, b), col = std::min(a, b);
                const int64_t u = __atomic_fetch_add(&fill[row], 1, __ATOMIC_RELAXED);
                ent[u] = col;
                src[u] = (int32_t)q;
            }
    });
    // order each new row by column and map old slots to new ones
    std::atomic<bool> dup{false};
    parallel_range(dim, [&](int64_t lo, int64_t hi) {
        std::vector<std::pair<int32_t, int32_t>> tmp;
        bool local_dup = false;
        for (int64_t i = lo; i < hi; i++) {
            const int64_t b = rowptr2[i], e = rowptr2[i + 1];
            tmp.clear();
            for (int64_t u = b; u < e; u++) tmp.emplace_back(ent[u], src[u]);
            std::sort(tmp.begin(), tmp.end());
            for (int64_t u = b; u < e; u++) {
                colind2[u] = tmp[u - b].first;
                map[tmp[u - b].second] = (int32_t)u;
                if (u > b && tmp[u - b].first == tmp[u - b - 1].first) local_dup = true;
            }
        }
        if (local_dup) dup = true;
    });
    if (dup) return fail(OCP_ERR_ARG, "ocp_kkt_permute: duplicate entry in the input CSR");
    std::atomic<bool> bad{false};
    parallel_range(std::max(nnzj, nnzh), [&](int64_t lo, int64_t hi) {
        bool local_bad = false;
        for (int64_t e = lo; e < hi; e++) {
            if (perm_j2 && e < nnzj) {
                const int32_t q = perm_j[e];
                if (q < 0 || q >= nnzk) local_bad = true;
                else perm_j2[e] = map[q];
            }
            if (perm_h2 && e < nnzh) {
                const int32_t q = perm_h[e];
                if (q < 0 || q >= nnzk) local_bad = true;
                else perm_h2[e] = map[q];
            }
        }
        if (local_bad) bad = true;
    });
    if (bad) return fail(OCP_ERR_ARG, "ocp_kkt_permute: a slot map points outside the KKT");
    if (diag2)
        parallel_range(dim, [&](int64_t lo, int64_t hi) {
            for (int64_t dd = lo; dd < hi; dd++) diag2[dd] = map[rowptr[dd + 1] - 1];
        });
    return OCP_OK;
}

}  // extern "C"
