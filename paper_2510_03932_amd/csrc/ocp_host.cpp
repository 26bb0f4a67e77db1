// Host index layer: problem sizes, the Jacobian / Hessian COO patterns and the
// lower-triangular CSR structure of the KKT matrix with the COO -> CSR slot
// maps.  Everything is generated in closed form from (N, n, m) -- the one-time
// host symbolic step that precedes device-side assembly in an interior-point
// iteration (paper Sec. 6).  No HIP call is made here.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

#include "ocp_internal.h"

namespace ocp {

static thread_local std::string g_err;

// OCP_VERBOSE (environment, read once): set to anything but "" or "0", every
// error the library records is also printed to stderr with its code.
static bool verbose()
{
    static const bool v = [] {
        const char *e = std::getenv("OCP_VERBOSE");
        return e && *e && std::strcmp(e, "0") != 0;
    }();
    return v;
}

int fail(int code, const std::string &msg)
{
    g_err = msg;
    if (verbose()) std::fprintf(stderr, "[ocp] error %d: %s\n", code, msg.c_str());
    return code;
}

void clear_error() { g_err.clear(); }

int make_dims_ex(int64_t N, int32_t n, int32_t m, int32_t scheme, int32_t bnd, Dims *d)
{
    if (!d) return fail(OCP_ERR_ARG, "null output pointer");
    if (N < 1) return fail(OCP_ERR_ARG, "N must be >= 1 (got " + std::to_string(N) + ")");
    if (n < 1 || n > OCP_MAX_DIM)
        return fail(OCP_ERR_ARG, "n must be in [1, " + std::to_string(OCP_MAX_DIM) + "] (got " +
                                     std::to_string(n) + ")");
    if (m < 0 || m > OCP_MAX_DIM)
        return fail(OCP_ERR_ARG, "m must be in [0, " + std::to_string(OCP_MAX_DIM) + "] (got " +
                                     std::to_string(m) + ")");
    if (scheme != OCP_SCHEME_TRAPEZOIDAL && scheme != OCP_SCHEME_EULER)
        return fail(OCP_ERR_ARG, "unknown scheme " + std::to_string(scheme));
    if (bnd < OCP_BOUNDARY_NONE || bnd > OCP_BOUNDARY_INITIAL_FINAL)
        return fail(OCP_ERR_ARG, "unknown boundary option " + std::to_string(bnd));
    // n, m <= 32 so T, S <= 128: every product below fits easily in int64
    // once N is bounded; bound N first so nothing overflows int64 either.
    if (N > INT32_MAX) return fail(OCP_ERR_OVERFLOW, "N does not fit in int32");
    Dims r;
    r.N = N;
    r.n = n;
    r.m = m;
    r.scheme = scheme;
    r.bnd = bnd;
    r.npair = n >= 3 ? n : (n == 2 ? 1 : 0);
    r.T = scheme == OCP_SCHEME_TRAPEZOIDAL ? 2 * n + 2 * m : n + 1 + m;
    r.S = n + r.npair + m;
    r.N1 = N + 1;
    r.NU = scheme == OCP_SCHEME_TRAPEZOIDAL ? N + 1 : N;
    r.nvar = (int64_t)n * r.N1 + (int64_t)m * r.NU;
    r.ndef = (int64_t)n * N;
    r.nb = (int64_t)bnd * n;
    r.ncon = r.ndef + r.nb;
    r.nnzj_def = r.ndef * r.T;
    r.nnzj = r.nnzj_def + r.nb;
    r.nnzh = (int64_t)(n + r.npair) * r.N1 + (int64_t)m * r.NU;
    r.nnzk = r.nnzh + r.nnzj + r.ncon;
    r.dim = r.nvar + r.ncon;
    // The largest index ever formed is below nnzk (CSR slots) or dim+1
    // (rowptr entries); COO positions are below nnzj, nnzh.
    if (r.nnzk > INT32_MAX || r.dim + 1 > INT32_MAX)
        return fail(OCP_ERR_OVERFLOW, "KKT size " + std::to_string(r.nnzk) + " entries / " +
                                          std::to_string(r.dim) + " rows does not fit in int32");
    *d = r;
    return OCP_OK;
}

int make_dims(int64_t N, int32_t n, int32_t m, Dims *d)
{
    return make_dims_ex(N, n, m, OCP_SCHEME_TRAPEZOIDAL, OCP_BOUNDARY_NONE, d);
}

void to_public(const Dims &d, ocp_sizes_t *out)
{
    out->nvar = d.nvar;
    out->ncon = d.ncon;
    out->nnzj = d.nnzj;
    out->nnzh = d.nnzh;
    out->nnzk = d.nnzk;
    out->dim = d.dim;
    out->npair = d.npair;
    out->T = d.T;
    out->S = d.S;
}

// Run body(lo, hi) over [0, count) split across host threads.
template <class F>
static void parallel_range(int64_t count, F body)
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

// ---- KKT row structure, closed form ---------------------------------------
//
// Rows are ordered: state rows vx(j,k) (j-major, k-minor), control rows
// vu(l,k), then constraint rows nvar + i N + k.  Within a row columns ascend
// and the diagonal comes last.
//
// State row vx(a,k) holds the bilinear Hessian entries whose larger index is a
// (pair i couples states i and p(i) = (i+1) mod n at the same node):
//   n >= 3: a = 0 has none; 1 <= a <= n-2 has pair a-1 (column a-1);
//           a = n-1 has pair n-1 (column 0) and pair n-2 (column n-2).
//   n = 2:  a = 1 has the merged pair (column 0).
//   n = 1:  none.
// Control rows hold the diagonal only; constraint row (i,k) holds its T
// Jacobian entries in slot order (already ascending) and the diagonal.

static int pairs_in_row(const Dims &d, int a)
{
    if (d.n >= 3) return a == 0 ? 0 : (a == d.n - 1 ? 2 : 1);
    if (d.n == 2) return a == 1 ? 1 : 0;
    return 0;
}

// Index of the first CSR slot of state row block a (row vx(a,0)).
static int64_t state_block_start(const Dims &d, int a)
{
    int64_t s = 0;
    for (int b = 0; b < a; b++) s += (int64_t)(pairs_in_row(d, b) + 1) * d.N1;
    return s;
}

}  // namespace ocp

using namespace ocp;

// Column (variable index) of Jacobian slot t of defect row (i, k), and the
// constraint rows' closed forms.  Trapezoidal: X_j at k, k+1 (slots 2j, 2j+1),
// then U_l at k, k+1.  Euler: X_0..X_i at k, X_i at k+1, X_{i+1}.. at k, then
// U_l at k.  Either way the slots are in ascending column order.
static int64_t jac_col(const Dims &d, int64_t i, int64_t t, int64_t k)
{
    const int64_t NX = (int64_t)d.n * d.N1;
    if (d.scheme == OCP_SCHEME_TRAPEZOIDAL) {
        if (t < 2 * d.n) return (t / 2) * d.N1 + k + (t % 2);
        return NX + ((t - 2 * d.n) / 2) * d.NU + k + ((t - 2 * d.n) % 2);
    }
    if (t <= i) return t * d.N1 + k;
    if (t == i + 1) return i * d.N1 + k + 1;
    if (t <= d.n) return (t - 1) * d.N1 + k;
    return NX + (t - d.n - 1) * d.NU + k;
}

// Column of boundary row b (X_i0 for b < n, X_iN after).
static int64_t bnd_col(const Dims &d, int64_t b)
{
    return (b % d.n) * d.N1 + (b < d.n ? 0 : d.N);
}

static int options_of(const ocp_options *opt, int32_t *scheme, int32_t *bnd)
{
    *scheme = opt ? opt->scheme : OCP_SCHEME_TRAPEZOIDAL;
    *bnd = opt ? opt->boundary : OCP_BOUNDARY_NONE;
    return OCP_OK;
}

extern "C" {

int ocp_sizes_ex(int64_t N, int32_t n, int32_t m, const ocp_options *opt, ocp_sizes_t *out)
{
    clear_error();
    if (!out) return fail(OCP_ERR_ARG, "ocp_sizes: out is NULL");
    int32_t scheme, bnd;
    options_of(opt, &scheme, &bnd);
    Dims d;
    int rc = make_dims_ex(N, n, m, scheme, bnd, &d);
    if (rc) return rc;
    to_public(d, out);
    return OCP_OK;
}

int ocp_sizes(int64_t N, int32_t n, int32_t m, ocp_sizes_t *out)
{
    return ocp_sizes_ex(N, n, m, nullptr, out);
}

int ocp_build_pattern_ex(int64_t N, int32_t n, int32_t m, const ocp_options *opt, int32_t *jrow,
                         int32_t *jcol, int32_t *hrow, int32_t *hcol)
{
    clear_error();
    int32_t scheme, bnd;
    options_of(opt, &scheme, &bnd);
    Dims d;
    int rc = make_dims_ex(N, n, m, scheme, bnd, &d);
    if (rc) return rc;
    if ((jrow == nullptr) != (jcol == nullptr) || (hrow == nullptr) != (hcol == nullptr))
        return fail(OCP_ERR_ARG, "ocp_build_pattern: row and column arrays must both be given or both NULL");
    const int64_t NX = (int64_t)d.n * d.N1;
    if (jrow) {
        // defect entry e = (i T + t) N + k; parallel over (i, t) slot rows
        parallel_range((int64_t)d.n * d.T, [&](int64_t lo, int64_t hi) {
            for (int64_t it = lo; it < hi; it++) {
                int64_t i = it / d.T, t = it % d.T;
                const int64_t colbase = jac_col(d, i, t, 0);  // column at k = 0; +k after
                int32_t *rr = jrow + it * d.N;
                int32_t *cc = jcol + it * d.N;
                for (int64_t k = 0; k < d.N; k++) {
                    rr[k] = (int32_t)(i * d.N + k);
                    cc[k] = (int32_t)(colbase + k);
                }
            }
        });
        for (int64_t b = 0; b < d.nb; b++) {
            jrow[d.nnzj_def + b] = (int32_t)(d.ndef + b);
            jcol[d.nnzj_def + b] = (int32_t)bnd_col(d, b);
        }
    }
    if (hrow) {
        parallel_range((int64_t)d.S, [&](int64_t lo, int64_t hi) {
            for (int64_t s = lo; s < hi; s++) {
                int64_t rb, cb, base, cnt;  // row / column of node 0, COO start, nodes
                if (s < d.n) {
                    rb = cb = s * d.N1;
                    base = s * d.N1;
                    cnt = d.N1;
                } else if (s < d.n + d.npair) {
                    int64_t i = s - d.n;
                    int64_t a = (d.n == 2) ? 0 : i, b = (d.n == 2) ? 1 : (i + 1) % d.n;
                    rb = std::max(a, b) * d.N1;
                    cb = std::min(a, b) * d.N1;
                    base = s * d.N1;
                    cnt = d.N1;
                } else {
                    const int64_t l = s - d.n - d.npair;
                    rb = cb = NX + l * d.NU;
                    base = (int64_t)(d.n + d.npair) * d.N1 + l * d.NU;
                    cnt = d.NU;
                }
                int32_t *rr = hrow + base;
                int32_t *cc = hcol + base;
                for (int64_t k = 0; k < cnt; k++) {
                    rr[k] = (int32_t)(rb + k);
                    cc[k] = (int32_t)(cb + k);
                }
            }
        });
    }
    return OCP_OK;
}

int ocp_build_pattern(int64_t N, int32_t n, int32_t m, int32_t *jrow, int32_t *jcol,
                      int32_t *hrow, int32_t *hcol)
{
    return ocp_build_pattern_ex(N, n, m, nullptr, jrow, jcol, hrow, hcol);
}

int ocp_build_kkt_ex(int64_t N, int32_t n, int32_t m, const ocp_options *opt, int32_t *rowptr,
                     int32_t *colind, int32_t *perm_j, int32_t *perm_h)
{
    clear_error();
    int32_t scheme, bnd;
    options_of(opt, &scheme, &bnd);
    Dims d;
    int rc = make_dims_ex(N, n, m, scheme, bnd, &d);
    if (rc) return rc;
    const int64_t N1 = d.N1, NU = d.NU, NX = (int64_t)d.n * N1;
    const int64_t ctrl_start = state_block_start(d, d.n);      // = (n + npair) (N+1)
    const int64_t cons_start = ctrl_start + (int64_t)d.m * NU;  // = nnzh
    const int64_t T1 = d.T + 1;
    const int64_t bnd_start = cons_start + d.ndef * T1;         // boundary rows: 2 entries each

    if (rowptr) {
        // state rows
        for (int a = 0; a < d.n; a++) {
            int64_t base = state_block_start(d, a), len = pairs_in_row(d, a) + 1;
            int32_t *rp = rowptr + (int64_t)a * N1;
            parallel_range(N1, [&](int64_t lo, int64_t hi) {
                for (int64_t k = lo; k < hi; k++) rp[k] = (int32_t)(base + k * len);
            });
        }
        // control rows
        parallel_range((int64_t)d.m * NU, [&](int64_t lo, int64_t hi) {
            for (int64_t x = lo; x < hi; x++) rowptr[NX + x] = (int32_t)(ctrl_start + x);
        });
        // defect rows
        parallel_range(d.ndef, [&](int64_t lo, int64_t hi) {
            for (int64_t x = lo; x < hi; x++) rowptr[d.nvar + x] = (int32_t)(cons_start + x * T1);
        });
        // boundary rows and the end
        for (int64_t b = 0; b <= d.nb; b++) rowptr[d.nvar + d.ndef + b] = (int32_t)(bnd_start + 2 * b);
    }
    if (colind) {
        for (int a = 0; a < d.n; a++) {
            int64_t base = state_block_start(d, a);
            int np = pairs_in_row(d, a);
            int c0 = 0, c1 = 0;  // pair columns (state indices), ascending
            if (d.n >= 3 && a == d.n - 1) { c0 = 0; c1 = d.n - 2; }
            else if (d.n >= 3 && a >= 1) { c0 = a - 1; }
            else if (d.n == 2 && a == 1) { c0 = 0; }
            parallel_range(N1, [&](int64_t lo, int64_t hi) {
                for (int64_t k = lo; k < hi; k++) {
                    int32_t *out = colind + base + k * (np + 1);
                    int x = 0;
                    if (np >= 1) out[x++] = (int32_t)(c0 * N1 + k);
                    if (np >= 2) out[x++] = (int32_t)(c1 * N1 + k);
                    out[x] = (int32_t)(a * N1 + k);
                }
            });
        }
        parallel_range((int64_t)d.m * NU, [&](int64_t lo, int64_t hi) {
            for (int64_t x = lo; x < hi; x++) colind[ctrl_start + x] = (int32_t)(NX + x);
        });
        parallel_range(d.ndef, [&](int64_t lo, int64_t hi) {
            for (int64_t r = lo; r < hi; r++) {
                const int64_t i = r / d.N, k = r % d.N;
                int32_t *out = colind + cons_start + r * T1;
                for (int64_t t = 0; t < d.T; t++) out[t] = (int32_t)jac_col(d, i, t, k);
                out[d.T] = (int32_t)(d.nvar + r);
            }
        });
        for (int64_t b = 0; b < d.nb; b++) {
            colind[bnd_start + 2 * b] = (int32_t)bnd_col(d, b);
            colind[bnd_start + 2 * b + 1] = (int32_t)(d.nvar + d.ndef + b);
        }
    }
    if (perm_j) {
        // defect entry (i T + t) N + k -> slot cons_start + (i N + k)(T+1) + t
        parallel_range((int64_t)d.n * d.T, [&](int64_t lo, int64_t hi) {
            for (int64_t it = lo; it < hi; it++) {
                int64_t i = it / d.T, t = it % d.T;
                int32_t *out = perm_j + it * d.N;
                int64_t base = cons_start + i * d.N * T1 + t;
                for (int64_t k = 0; k < d.N; k++) out[k] = (int32_t)(base + k * T1);
            }
        });
        for (int64_t b = 0; b < d.nb; b++) perm_j[d.nnzj_def + b] = (int32_t)(bnd_start + 2 * b);
    }
    if (perm_h) {
        for (int64_t s = 0; s < d.S; s++) {
            int64_t base, stride, hbase, cnt;  // slot of node 0, per-node stride, COO start, nodes
            if (s < d.n) {
                int a = (int)s;
                int np = pairs_in_row(d, a);
                base = state_block_start(d, a) + np;  // diagonal is last
                stride = np + 1;
                hbase = s * N1;
                cnt = N1;
            } else if (s < d.n + d.npair) {
                int i = (int)(s - d.n);
                int a;        // row (larger state index)
                int off;      // position within the row
                if (d.n == 2) { a = 1; off = 0; }
                else if (i == d.n - 1) { a = d.n - 1; off = 0; }          // column 0
                else { a = i + 1; off = (a == d.n - 1) ? 1 : 0; }          // column i
                base = state_block_start(d, a) + off;
                stride = pairs_in_row(d, a) + 1;
                hbase = s * N1;
                cnt = N1;
            } else {
                const int64_t l = s - d.n - d.npair;
                base = ctrl_start + l * NU;
                stride = 1;
                hbase = (int64_t)(d.n + d.npair) * N1 + l * NU;
                cnt = NU;
            }
            int32_t *out = perm_h + hbase;
            parallel_range(cnt, [&](int64_t lo, int64_t hi) {
                for (int64_t k = lo; k < hi; k++) out[k] = (int32_t)(base + k * stride);
            });
        }
    }
    return OCP_OK;
}

int ocp_build_kkt(int64_t N, int32_t n, int32_t m, int32_t *rowptr, int32_t *colind,
                  int32_t *perm_j, int32_t *perm_h)
{
    return ocp_build_kkt_ex(N, n, m, nullptr, rowptr, colind, perm_j, perm_h);
}

const char *ocp_last_error(void) { return g_err.c_str(); }

}  // extern "C"
