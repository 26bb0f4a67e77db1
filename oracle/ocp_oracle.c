/*
 * ocp_oracle.c -- CPU oracle for the trapezoidal direct-transcription NLP.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header
 * or generated table with the GPU library, and the GPU library never calls it.
 *
 * Everything here is the plain definition, evaluated with plain loops in
 * IEEE double precision (built with -ffp-contract=off, no fast-math):
 *
 *   Transcription (paper, Sec. 3 and the trapezoidal generated code of Sec. 5):
 *     grid t_k = k h, h = 1/N, k = 0..N; hh = h/2; state X_{jk}, control U_{lk}
 *     on every node k = 0..N; one constraint generator per state component,
 *       c_{ik} = (X_{i,k+1} - X_{ik}) - hh (F_i(k) + F_i(k+1)),  k = 0..N-1
 *     and the Lagrange cost summed with the trapezoidal rule (two objective
 *     generators: end nodes weighted dt/2, interior nodes dt).
 *   Dynamics of the workload family:
 *     F_i(k) = sum_j A_ij sin X_jk + sum_l B_il U_lk + gamma_i X_ik X_{p(i)k},
 *     p(i) = (i+1) mod n.
 *   Cost: f = sum_k w_k (sum_j q_j X_jk^2 + sum_l r_l U_lk^2).
 *   Derivatives (the evaluations an interior-point iteration requests, Sec. 6):
 *     gradient of f, Jacobian of c, Hessian of L = sigma f + y^T c,
 *     and the KKT matrix [[H, J^T], [J, 0]] in lower-triangular CSR.
 *
 * Index conventions (component-major unknowns):
 *   vx(j,k) = j (N+1) + k,   vu(l,k) = n (N+1) + l (N+1) + k,
 *   constraint row r(i,k) = i N + k,  y indexed like c.
 *   Jacobian COO position of slot t in row r(i,k):  (i T + t) N + k,  T = 2n + 2m.
 *   Hessian COO position of slot s at node k:       s (N+1) + k.
 *
 * Node-range functions take [k0, k1) and write a compact block whose slot
 * stride is K = k1 - k0; the full range reproduces the full-size layout.
 * Each value function also writes a magnitude mu: the sum of the absolute
 * values of the terms the value is made of (the scale for a rounding bound).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_OK 0
#define ORC_BAD 1

static int npair_of(int n) { return n >= 3 ? n : (n == 2 ? 1 : 0); }

static int bad_sizes(int64_t N, int n, int m)
{
    return N < 1 || n < 1 || m < 0;
}

/* Cost weight of node k: trapezoidal rule on a uniform grid. */
static double weight(int64_t N, int64_t k)
{
    double h = 1.0 / (double)N;
    double hh = 0.5 * h;
    return (k == 0 || k == N) ? hh : h;
}

/* out = {nvar, ncon, nnzj, nnzh, dim, npair, T, S} */
int orc_sizes(int64_t N, int n, int m, int64_t *out)
{
    if (bad_sizes(N, n, m) || !out) return ORC_BAD;
    int64_t npair = npair_of(n);
    int64_t T = 2 * (int64_t)n + 2 * (int64_t)m;
    int64_t S = (int64_t)n + npair + (int64_t)m;
    out[0] = ((int64_t)n + m) * (N + 1);
    out[1] = (int64_t)n * N;
    out[2] = (int64_t)n * N * T;
    out[3] = S * (N + 1);
    out[4] = out[0] + out[1];
    out[5] = npair;
    out[6] = T;
    out[7] = S;
    return ORC_OK;
}

void orc_set_threads(int t) { if (t > 0) omp_set_num_threads(t); }
int orc_get_threads(void) { return omp_get_max_threads(); }

/* ---- dynamics at one node ------------------------------------------------ */

/* F_i(k) and |F|_i(k) (sum of |terms|), summed j ascending, l ascending, then
 * the bilinear term. */
static void dynamics(int64_t N, int n, int m, const double *A, const double *B,
                     const double *gam, const double *z, int64_t k,
                     double *F, double *Fabs)
{
    const double *X = z;
    const double *U = z + (int64_t)n * (N + 1);
    for (int i = 0; i < n; i++) {
        double s = 0.0, sa = 0.0, t;
        for (int j = 0; j < n; j++) {
            t = A[i * n + j] * sin(X[(int64_t)j * (N + 1) + k]);
            s += t; sa += fabs(t);
        }
        for (int l = 0; l < m; l++) {
            t = B[i * m + l] * U[(int64_t)l * (N + 1) + k];
            s += t; sa += fabs(t);
        }
        int p = (i + 1) % n;
        t = gam[i] * X[(int64_t)i * (N + 1) + k] * X[(int64_t)p * (N + 1) + k];
        s += t; sa += fabs(t);
        F[i] = s;
        if (Fabs) Fabs[i] = sa;
    }
}

/* ---- objective (o1) ------------------------------------------------------ */

/* Neumaier-compensated accumulator. */
typedef struct { double s, c; } acc_t;
static void acc_add(acc_t *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

#define OBJ_CHUNK 4096

/* out[0] = f, out[1] = mu(f).  Per-node terms are summed with Neumaier
 * compensation inside fixed chunks of OBJ_CHUNK nodes, then the chunk results
 * are summed with Neumaier in chunk order: the result does not depend on the
 * number of threads. */
int orc_obj(int64_t N, int n, int m, const double *q, const double *r,
            const double *z, double *out)
{
    if (bad_sizes(N, n, m) || !q || (m && !r) || !z || !out) return ORC_BAD;
    const double *X = z;
    const double *U = z + (int64_t)n * (N + 1);
    int64_t nodes = N + 1;
    int64_t nch = (nodes + OBJ_CHUNK - 1) / OBJ_CHUNK;
    double *cs = (double *)malloc(sizeof(double) * 2 * nch);
    double *ca = (double *)malloc(sizeof(double) * nch);
    if (!cs || !ca) { free(cs); free(ca); return ORC_BAD; }
    #pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nch; c++) {
        acc_t a = {0.0, 0.0};
        double mu = 0.0;
        int64_t kend = (c + 1) * OBJ_CHUNK < nodes ? (c + 1) * OBJ_CHUNK : nodes;
        for (int64_t k = c * OBJ_CHUNK; k < kend; k++) {
            double s = 0.0, sa = 0.0;
            for (int j = 0; j < n; j++) {
                double x = X[(int64_t)j * (N + 1) + k];
                double t = q[j] * x * x;
                s += t; sa += fabs(t);
            }
            for (int l = 0; l < m; l++) {
                double u = U[(int64_t)l * (N + 1) + k];
                double t = r[l] * u * u;
                s += t; sa += fabs(t);
            }
            double w = weight(N, k);
            acc_add(&a, w * s);
            mu += w * sa;
        }
        cs[2 * c] = a.s;
        cs[2 * c + 1] = a.c;
        ca[c] = mu;
    }
    acc_t tot = {0.0, 0.0};
    double mu = 0.0;
    for (int64_t c = 0; c < nch; c++) {
        acc_add(&tot, cs[2 * c]);
        acc_add(&tot, cs[2 * c + 1]);
        mu += ca[c];
    }
    out[0] = tot.s + tot.c;
    out[1] = mu;
    free(cs);
    free(ca);
    return ORC_OK;
}

/* ---- gradient (o2) ------------------------------------------------------- */

/* Nodes k in [k0, k1) of [0, N]; g[j K + k-k0] for states, g[(n+l) K + k-k0]
 * for controls. */
int orc_grad(int64_t N, int n, int m, const double *q, const double *r,
             const double *z, int64_t k0, int64_t k1, double *g, double *mu)
{
    if (bad_sizes(N, n, m) || k0 < 0 || k1 > N + 1 || k0 > k1 || !z || !g) return ORC_BAD;
    const double *X = z;
    const double *U = z + (int64_t)n * (N + 1);
    int64_t K = k1 - k0;
    #pragma omp parallel for schedule(static)
    for (int64_t k = k0; k < k1; k++) {
        double w = weight(N, k);
        for (int j = 0; j < n; j++) {
            double v = 2.0 * w * q[j] * X[(int64_t)j * (N + 1) + k];
            g[(int64_t)j * K + (k - k0)] = v;
            if (mu) mu[(int64_t)j * K + (k - k0)] = fabs(v);
        }
        for (int l = 0; l < m; l++) {
            double v = 2.0 * w * r[l] * U[(int64_t)l * (N + 1) + k];
            g[(int64_t)(n + l) * K + (k - k0)] = v;
            if (mu) mu[(int64_t)(n + l) * K + (k - k0)] = fabs(v);
        }
    }
    return ORC_OK;
}

/* ---- constraints (o3) ---------------------------------------------------- */

/* Intervals k in [k0, k1) of [0, N); c[i K + k-k0]. */
int orc_cons(int64_t N, int n, int m, const double *A, const double *B,
             const double *gam, const double *z, int64_t k0, int64_t k1,
             double *c, double *mu)
{
    if (bad_sizes(N, n, m) || k0 < 0 || k1 > N || k0 > k1 || !z || !c) return ORC_BAD;
    const double *X = z;
    double hh = 0.5 * (1.0 / (double)N);
    int64_t K = k1 - k0;
    #pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * 4 * n);
        double *F0 = buf, *F1 = buf + n, *A0 = buf + 2 * n, *A1 = buf + 3 * n;
        #pragma omp for schedule(static)
        for (int64_t k = k0; k < k1; k++) {
            dynamics(N, n, m, A, B, gam, z, k, F0, A0);
            dynamics(N, n, m, A, B, gam, z, k + 1, F1, A1);
            for (int i = 0; i < n; i++) {
                double x0 = X[(int64_t)i * (N + 1) + k];
                double x1 = X[(int64_t)i * (N + 1) + k + 1];
                c[(int64_t)i * K + (k - k0)] = (x1 - x0) - hh * (F0[i] + F1[i]);
                if (mu) mu[(int64_t)i * K + (k - k0)] = fabs(x1) + fabs(x0) + hh * (A0[i] + A1[i]);
            }
        }
        free(buf);
    }
    return ORC_OK;
}

/* ---- Jacobian values (o4) ------------------------------------------------ */

/* dF_i/dX_j at node k, and its magnitude. */
static void dF_dx(int64_t N, int n, const double *A, const double *gam,
                  const double *X, int i, int j, int64_t k, double *v, double *va)
{
    int p = (i + 1) % n;
    double a = A[i * n + j] * cos(X[(int64_t)j * (N + 1) + k]);
    double g = 0.0, ga = 0.0;
    if (j == i) { g += gam[i] * X[(int64_t)p * (N + 1) + k]; ga += fabs(gam[i] * X[(int64_t)p * (N + 1) + k]); }
    if (j == p) { g += gam[i] * X[(int64_t)i * (N + 1) + k]; ga += fabs(gam[i] * X[(int64_t)i * (N + 1) + k]); }
    *v = a + g;
    *va = fabs(a) + ga;
}

/* Intervals k in [k0, k1); value of slot t of row (i, k) at (i T + t) K + k-k0.
 * Slots in ascending column order: X_j at k, X_j at k+1 (j ascending), then
 * U_l at k, U_l at k+1 (l ascending). */
int orc_jac(int64_t N, int n, int m, const double *A, const double *B,
            const double *gam, const double *z, int64_t k0, int64_t k1,
            double *out, double *mu)
{
    if (bad_sizes(N, n, m) || k0 < 0 || k1 > N || k0 > k1 || !z || !out) return ORC_BAD;
    const double *X = z;
    double hh = 0.5 * (1.0 / (double)N);
    int64_t K = k1 - k0;
    int64_t T = 2 * (int64_t)n + 2 * (int64_t)m;
    #pragma omp parallel for schedule(static)
    for (int64_t k = k0; k < k1; k++) {
        for (int i = 0; i < n; i++) {
            for (int j = 0; j < n; j++) {
                double d = (i == j) ? 1.0 : 0.0;
                double g0, g0a, g1, g1a;
                dF_dx(N, n, A, gam, X, i, j, k, &g0, &g0a);
                dF_dx(N, n, A, gam, X, i, j, k + 1, &g1, &g1a);
                int64_t e0 = ((int64_t)i * T + 2 * j) * K + (k - k0);
                int64_t e1 = ((int64_t)i * T + 2 * j + 1) * K + (k - k0);
                out[e0] = -d - hh * g0;
                out[e1] = d - hh * g1;
                if (mu) { mu[e0] = d + hh * g0a; mu[e1] = d + hh * g1a; }
            }
            for (int l = 0; l < m; l++) {
                double v = -hh * B[i * m + l];
                int64_t e0 = ((int64_t)i * T + 2 * n + 2 * l) * K + (k - k0);
                int64_t e1 = e0 + K;
                out[e0] = v;
                out[e1] = v;
                if (mu) { mu[e0] = fabs(v); mu[e1] = fabs(v); }
            }
        }
    }
    return ORC_OK;
}

/* ---- Hessian of the Lagrangian values (o5) ------------------------------- */

/* Nodes k in [k0, k1) of [0, N]; slot s at s K + k-k0.
 * Slots: state diagonals (n), bilinear pairs (npair), control diagonals (m). */
int orc_hess(int64_t N, int n, int m, const double *A, const double *B,
             const double *gam, const double *q, const double *r,
             const double *z, const double *y, double sigma,
             int64_t k0, int64_t k1, double *out, double *mu)
{
    (void)B;
    if (bad_sizes(N, n, m) || k0 < 0 || k1 > N + 1 || k0 > k1 || !z || !y || !out) return ORC_BAD;
    const double *X = z;
    double h = 1.0 / (double)N;
    double hh = 0.5 * h;
    int np = npair_of(n);
    int64_t K = k1 - k0;
    #pragma omp parallel
    {
        double *yt = (double *)malloc(sizeof(double) * 2 * n);
        double *ya = yt + n;
        #pragma omp for schedule(static)
        for (int64_t k = k0; k < k1; k++) {
            double w = weight(N, k);
            /* Node-combined multiplier: node k appears in the defect of
             * interval k-1 (as its right end) and of interval k (left end). */
            for (int i = 0; i < n; i++) {
                double a = 0.0, aa = 0.0;
                if (k >= 1) { a += y[(int64_t)i * N + k - 1]; aa += fabs(y[(int64_t)i * N + k - 1]); }
                if (k <= N - 1) { a += y[(int64_t)i * N + k]; aa += fabs(y[(int64_t)i * N + k]); }
                yt[i] = a;
                ya[i] = aa;
            }
            for (int j = 0; j < n; j++) {
                double sx = sin(X[(int64_t)j * (N + 1) + k]);
                double s = 0.0, sa = 0.0;
                for (int i = 0; i < n; i++) {
                    s += yt[i] * A[i * n + j];
                    sa += ya[i] * fabs(A[i * n + j]);
                }
                double v = 2.0 * sigma * w * q[j] + hh * sx * s;
                double va = fabs(2.0 * sigma * w * q[j]) + hh * fabs(sx) * sa;
                if (n == 1) {
                    v += -h * yt[0] * gam[0];
                    va += h * ya[0] * fabs(gam[0]);
                }
                out[(int64_t)j * K + (k - k0)] = v;
                if (mu) mu[(int64_t)j * K + (k - k0)] = va;
            }
            if (n >= 3) {
                for (int i = 0; i < n; i++) {
                    int64_t e = (int64_t)(n + i) * K + (k - k0);
                    out[e] = -hh * yt[i] * gam[i];
                    if (mu) mu[e] = hh * ya[i] * fabs(gam[i]);
                }
            } else if (n == 2) {
                int64_t e = (int64_t)n * K + (k - k0);
                out[e] = -hh * (yt[0] * gam[0] + yt[1] * gam[1]);
                if (mu) mu[e] = hh * (ya[0] * fabs(gam[0]) + ya[1] * fabs(gam[1]));
            }
            for (int l = 0; l < m; l++) {
                int64_t e = (int64_t)(n + np + l) * K + (k - k0);
                double v = 2.0 * sigma * w * r[l];
                out[e] = v;
                if (mu) mu[e] = fabs(v);
            }
        }
        free(yt);
    }
    return ORC_OK;
}

/* ---- sparsity patterns (a1) ---------------------------------------------- */

int orc_pattern(int64_t N, int n, int m, int32_t *jrow, int32_t *jcol,
                int32_t *hrow, int32_t *hcol)
{
    if (bad_sizes(N, n, m)) return ORC_BAD;
    int64_t s[8];
    orc_sizes(N, n, m, s);
    if (s[4] > INT32_MAX || s[2] > INT32_MAX || s[3] > INT32_MAX) return ORC_BAD;
    int64_t T = s[6];
    int np = (int)s[5];
    int64_t NX = (int64_t)n * (N + 1);
    if (jrow && jcol) {
        for (int i = 0; i < n; i++)
            for (int64_t t = 0; t < T; t++)
                for (int64_t k = 0; k < N; k++) {
                    int64_t e = ((int64_t)i * T + t) * N + k;
                    int64_t col;
                    if (t < 2 * n) {
                        int64_t j = t / 2;
                        col = j * (N + 1) + k + (t % 2);
                    } else {
                        int64_t l = (t - 2 * n) / 2;
                        col = NX + l * (N + 1) + k + ((t - 2 * n) % 2);
                    }
                    jrow[e] = (int32_t)((int64_t)i * N + k);
                    jcol[e] = (int32_t)col;
                }
    }
    if (hrow && hcol) {
        for (int64_t k = 0; k <= N; k++) {
            for (int j = 0; j < n; j++) {
                int64_t e = (int64_t)j * (N + 1) + k;
                hrow[e] = hcol[e] = (int32_t)((int64_t)j * (N + 1) + k);
            }
            for (int i = 0; i < np; i++) {
                int a = i, b = (i + 1) % n;
                int hi = a > b ? a : b, lo = a < b ? a : b;
                int64_t e = (int64_t)(n + i) * (N + 1) + k;
                hrow[e] = (int32_t)((int64_t)hi * (N + 1) + k);
                hcol[e] = (int32_t)((int64_t)lo * (N + 1) + k);
            }
            for (int l = 0; l < m; l++) {
                int64_t e = (int64_t)(n + np + l) * (N + 1) + k;
                hrow[e] = hcol[e] = (int32_t)(NX + (int64_t)l * (N + 1) + k);
            }
        }
    }
    return ORC_OK;
}

/* ---- generic KKT build (a2) ---------------------------------------------- */

typedef struct { int64_t col; int64_t src; } ent_t;   /* src: -1 diag, 2e H, 2e+1 J */

static int ent_cmp(const void *a, const void *b)
{
    const ent_t *x = (const ent_t *)a, *y = (const ent_t *)b;
    if (x->col != y->col) return x->col < y->col ? -1 : 1;
    if (x->src != y->src) return x->src < y->src ? -1 : 1;
    return 0;
}

/* Lower-triangular CSR of K = [[H, J^T], [J, 0]] from the COO patterns, built
 * generically: triplets (H entries, J entries shifted down by nvar, and every
 * diagonal) -> counting sort by row -> sort columns within each row -> merge
 * duplicates -> map each COO entry to its CSR slot.  No structural shortcut.
 * rowptr has dim+1 entries; colind must hold nnzh + nnzj + dim entries (an
 * upper bound); *nnzk receives the true count.  Returns ORC_BAD if any entry
 * lies above the diagonal or a size exceeds int32. */
int orc_kkt(int64_t N, int n, int m, const int32_t *jrow, const int32_t *jcol,
            const int32_t *hrow, const int32_t *hcol, int32_t *rowptr,
            int32_t *colind, int32_t *perm_j, int32_t *perm_h, int64_t *nnzk)
{
    if (bad_sizes(N, n, m)) return ORC_BAD;
    int64_t s[8];
    orc_sizes(N, n, m, s);
    int64_t nvar = s[0], nnzj = s[2], nnzh = s[3], dim = s[4];
    int64_t ntrip = nnzh + nnzj + dim;
    if (dim > INT32_MAX || ntrip > INT32_MAX) return ORC_BAD;
    int64_t *cnt = (int64_t *)calloc((size_t)dim + 1, sizeof(int64_t));
    ent_t *ent = (ent_t *)malloc(sizeof(ent_t) * (size_t)ntrip);
    if (!cnt || !ent) { free(cnt); free(ent); return ORC_BAD; }
    int rc = ORC_OK;
    /* count per row */
    for (int64_t e = 0; e < nnzh; e++) cnt[hrow[e] + 1]++;
    for (int64_t e = 0; e < nnzj; e++) cnt[nvar + jrow[e] + 1]++;
    for (int64_t d = 0; d < dim; d++) cnt[d + 1]++;
    for (int64_t d = 0; d < dim; d++) cnt[d + 1] += cnt[d];
    /* place (stable) */
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)dim);
    if (!pos) { free(cnt); free(ent); return ORC_BAD; }
    memcpy(pos, cnt, sizeof(int64_t) * (size_t)dim);
    for (int64_t e = 0; e < nnzh; e++) {
        if (hcol[e] > hrow[e]) rc = ORC_BAD;
        ent_t t = { hcol[e], 2 * e };
        ent[pos[hrow[e]]++] = t;
    }
    for (int64_t e = 0; e < nnzj; e++) {
        int64_t row = nvar + jrow[e];
        if (jcol[e] > row) rc = ORC_BAD;
        ent_t t = { jcol[e], 2 * e + 1 };
        ent[pos[row]++] = t;
    }
    for (int64_t d = 0; d < dim; d++) {
        ent_t t = { d, -1 };
        ent[pos[d]++] = t;
    }
    free(pos);
    /* sort within rows, merge duplicates, assign slots */
    int64_t slot = -1;
    rowptr[0] = 0;
    for (int64_t d = 0; d < dim; d++) {
        int64_t b = cnt[d], en = cnt[d + 1];
        qsort(ent + b, (size_t)(en - b), sizeof(ent_t), ent_cmp);
        int64_t prev = -1;
        for (int64_t x = b; x < en; x++) {
            if (x == b || ent[x].col != prev) {
                slot++;
                colind[slot] = (int32_t)ent[x].col;
                prev = ent[x].col;
            }
            int64_t sr = ent[x].src;
            if (sr >= 0) {
                if (sr % 2 == 0) perm_h[sr / 2] = (int32_t)slot;
                else perm_j[sr / 2] = (int32_t)slot;
            }
        }
        rowptr[d + 1] = (int32_t)(slot + 1);
    }
    *nnzk = slot + 1;
    free(cnt);
    free(ent);
    return rc;
}

/* ---- KKT assembly (o7) --------------------------------------------------- */

/* kkt = 0; kkt[perm_h[e]] = hess[e]; kkt[perm_j[e]] = jac[e];
 * then, if reg is given, kkt[rowptr[d+1]-1] += reg[d] for every row d. */
int orc_assemble(int64_t nnzk, int64_t dim, const int32_t *rowptr,
                 int64_t nnzj, const int32_t *perm_j, const double *jac,
                 int64_t nnzh, const int32_t *perm_h, const double *hess,
                 const double *reg, double *kkt)
{
    if (!kkt || !rowptr || nnzk < 0) return ORC_BAD;
    for (int64_t x = 0; x < nnzk; x++) kkt[x] = 0.0;
    for (int64_t e = 0; e < nnzh; e++) kkt[perm_h[e]] = hess[e];
    for (int64_t e = 0; e < nnzj; e++) kkt[perm_j[e]] = jac[e];
    if (reg)
        for (int64_t d = 0; d < dim; d++) kkt[rowptr[d + 1] - 1] += reg[d];
    return ORC_OK;
}

/* ---- Lagrangian and its derivatives (differentiation workload) ----------- */
/*
 * L(z, y; A, B, gamma, sigma) = sigma f(z) + y^T c(z).  Each function below is
 * the plain definition written as a sum over the Jacobian / Hessian entries
 * defined above (no rearranged closed forms):
 *   orc_lagrangian  L and mu(L)
 *   orc_lag_grad    grad_z L = sigma grad f + J^T y            (node range)
 *   orc_hvp         (Hessian of L) v, block by block per node   (node range)
 *   orc_jvp         J v                                          (interval range)
 *   orc_coef_grad   dL/dA, dL/dB, dL/dgamma: sum over all defect rows of
 *                   y_ik dc_ik/dtheta (fixed-chunk Neumaier sums)
 */

/* L = sigma f + sum_r y_r c_r: f as orc_obj; the product sum compensated in
 * fixed chunks of OBJ_CHUNK intervals.  out = {L, mu}. */
int orc_lagrangian(int64_t N, int n, int m, const double *A, const double *B,
                   const double *gam, const double *q, const double *r,
                   const double *z, const double *y, double sigma, double *out)
{
    if (bad_sizes(N, n, m) || !z || !y || !out) return ORC_BAD;
    double fo[2];
    if (orc_obj(N, n, m, q, r, z, fo)) return ORC_BAD;
    double *c = (double *)malloc(sizeof(double) * (size_t)(n * N));
    double *cm = (double *)malloc(sizeof(double) * (size_t)(n * N));
    if (!c || !cm) { free(c); free(cm); return ORC_BAD; }
    orc_cons(N, n, m, A, B, gam, z, 0, N, c, cm);
    int64_t R = (int64_t)n * N;
    int64_t nch = (R + OBJ_CHUNK - 1) / OBJ_CHUNK;
    acc_t tot = {0.0, 0.0};
    double mu = 0.0;
    for (int64_t ch = 0; ch < nch; ch++) {
        acc_t a = {0.0, 0.0};
        int64_t e = (ch + 1) * OBJ_CHUNK < R ? (ch + 1) * OBJ_CHUNK : R;
        for (int64_t x = ch * OBJ_CHUNK; x < e; x++) {
            acc_add(&a, y[x] * c[x]);
            mu += fabs(y[x]) * cm[x];
        }
        acc_add(&tot, a.s);
        acc_add(&tot, a.c);
    }
    double yc = tot.s + tot.c;
    out[0] = sigma * fo[0] + yc;
    out[1] = fabs(sigma) * fo[1] + mu;
    free(c);
    free(cm);
    return ORC_OK;
}

/* Jacobian entry d c_{i,kk} / d X_{j,node} for node in {kk, kk+1}, and its
 * magnitude (the o4 table: -delta - hh G at the left node, delta - hh G at
 * the right node). */
static void jac_entry_x(int64_t N, int n, const double *A, const double *gam,
                        const double *X, int i, int j, int64_t kk, int right,
                        double *v, double *va)
{
    double hh = 0.5 * (1.0 / (double)N);
    double d = (i == j) ? 1.0 : 0.0;
    double g, ga;
    dF_dx(N, n, A, gam, X, i, j, kk + right, &g, &ga);
    *v = (right ? d : -d) - hh * g;
    *va = d + hh * ga;
}

/* grad_z L at nodes [k0, k1) of [0, N]; layout as orc_grad. */
int orc_lag_grad(int64_t N, int n, int m, const double *A, const double *B,
                 const double *gam, const double *q, const double *r,
                 const double *z, const double *y, double sigma,
                 int64_t k0, int64_t k1, double *out, double *mu)
{
    if (bad_sizes(N, n, m) || k0 < 0 || k1 > N + 1 || k0 > k1 || !z || !y || !out) return ORC_BAD;
    const double *X = z;
    const double *U = z + (int64_t)n * (N + 1);
    double hh = 0.5 * (1.0 / (double)N);
    int64_t K = k1 - k0;
    #pragma omp parallel for schedule(static)
    for (int64_t k = k0; k < k1; k++) {
        double w = weight(N, k);
        for (int j = 0; j < n; j++) {
            double s = 2.0 * sigma * w * q[j] * X[(int64_t)j * (N + 1) + k];
            double sa = fabs(s);
            for (int i = 0; i < n; i++) {
                double v, va;
                if (k >= 1) {  /* row (i, k-1): node k is its right node */
                    jac_entry_x(N, n, A, gam, X, i, j, k - 1, 1, &v, &va);
                    s += v * y[(int64_t)i * N + k - 1];
                    sa += va * fabs(y[(int64_t)i * N + k - 1]);
                }
                if (k <= N - 1) {  /* row (i, k): node k is its left node */
                    jac_entry_x(N, n, A, gam, X, i, j, k, 0, &v, &va);
                    s += v * y[(int64_t)i * N + k];
                    sa += va * fabs(y[(int64_t)i * N + k]);
                }
            }
            out[(int64_t)j * K + (k - k0)] = s;
            if (mu) mu[(int64_t)j * K + (k - k0)] = sa;
        }
        for (int l = 0; l < m; l++) {
            double s = 2.0 * sigma * w * r[l] * U[(int64_t)l * (N + 1) + k];
            double sa = fabs(s);
            for (int i = 0; i < n; i++) {
                double v = -hh * B[i * m + l];
                if (k >= 1) { s += v * y[(int64_t)i * N + k - 1]; sa += fabs(v * y[(int64_t)i * N + k - 1]); }
                if (k <= N - 1) { s += v * y[(int64_t)i * N + k]; sa += fabs(v * y[(int64_t)i * N + k]); }
            }
            out[(int64_t)(n + l) * K + (k - k0)] = s;
            if (mu) mu[(int64_t)(n + l) * K + (k - k0)] = sa;
        }
    }
    return ORC_OK;
}

/* (Hessian of L) v at nodes [k0, k1): the Hessian is block diagonal per node;
 * each block entry is the second derivative of sigma w_k running cost minus
 * hh sum_i yt_ik F_i(k), from the definitions
 *   d2F_i/dX_a dX_b = -A_ia sin X_a [a = b] + gamma_i ([a = i][b = p(i)] + [a = p(i)][b = i]),
 * controls enter F linearly. */
int orc_hvp(int64_t N, int n, int m, const double *A, const double *gam,
            const double *q, const double *r, const double *z, const double *y,
            double sigma, const double *v, int64_t k0, int64_t k1, double *out, double *mu)
{
    if (bad_sizes(N, n, m) || k0 < 0 || k1 > N + 1 || k0 > k1 || !z || !y || !v || !out) return ORC_BAD;
    const double *X = z;
    double hh = 0.5 * (1.0 / (double)N);
    int64_t K = k1 - k0;
    int nv = n + m;
    #pragma omp parallel
    {
        double *Hb = (double *)malloc(sizeof(double) * 2 * nv * nv + sizeof(double) * 2 * n);
        double *Ha = Hb + nv * nv;
        double *yt = Ha + nv * nv, *ya = yt + n;
        #pragma omp for schedule(static)
        for (int64_t k = k0; k < k1; k++) {
            double w = weight(N, k);
            for (int i = 0; i < n; i++) {
                double a = 0.0, aa = 0.0;
                if (k >= 1) { a += y[(int64_t)i * N + k - 1]; aa += fabs(y[(int64_t)i * N + k - 1]); }
                if (k <= N - 1) { a += y[(int64_t)i * N + k]; aa += fabs(y[(int64_t)i * N + k]); }
                yt[i] = a;
                ya[i] = aa;
            }
            for (int a = 0; a < nv; a++)
                for (int b = 0; b < nv; b++) { Hb[a * nv + b] = 0.0; Ha[a * nv + b] = 0.0; }
            for (int a = 0; a < n; a++) {
                Hb[a * nv + a] += 2.0 * sigma * w * q[a];
                Ha[a * nv + a] += fabs(2.0 * sigma * w * q[a]);
            }
            for (int l = 0; l < m; l++) {
                Hb[(n + l) * nv + n + l] += 2.0 * sigma * w * r[l];
                Ha[(n + l) * nv + n + l] += fabs(2.0 * sigma * w * r[l]);
            }
            for (int i = 0; i < n; i++) {
                int p = (i + 1) % n;
                for (int a = 0; a < n; a++) {
                    double sx = sin(X[(int64_t)a * (N + 1) + k]);
                    double t = -hh * yt[i] * (-A[i * n + a] * sx);
                    Hb[a * nv + a] += t;
                    Ha[a * nv + a] += hh * ya[i] * fabs(A[i * n + a] * sx);
                }
                /* gamma_i X_i X_p: d2/dX_i dX_p = d2/dX_p dX_i = gamma_i (both
                 * on the diagonal, 2 gamma_i, when p = i) */
                Hb[i * nv + p] += -hh * yt[i] * gam[i];
                Hb[p * nv + i] += -hh * yt[i] * gam[i];
                Ha[i * nv + p] += hh * ya[i] * fabs(gam[i]);
                Ha[p * nv + i] += hh * ya[i] * fabs(gam[i]);
            }
            for (int a = 0; a < nv; a++) {
                double s = 0.0, sa = 0.0;
                for (int b = 0; b < nv; b++) {
                    double vb = v[(int64_t)b * (N + 1) + k];
                    s += Hb[a * nv + b] * vb;
                    sa += Ha[a * nv + b] * fabs(vb);
                }
                out[(int64_t)a * K + (k - k0)] = s;
                if (mu) mu[(int64_t)a * K + (k - k0)] = sa;
            }
        }
        free(Hb);
    }
    return ORC_OK;
}

/* J v at intervals [k0, k1) of [0, N): (J v)_{ik} = sum over the row's slots
 * of the Jacobian entry times v at the slot's column; layout as orc_cons. */
int orc_jvp(int64_t N, int n, int m, const double *A, const double *B,
            const double *gam, const double *z, const double *v,
            int64_t k0, int64_t k1, double *out, double *mu)
{
    if (bad_sizes(N, n, m) || k0 < 0 || k1 > N || k0 > k1 || !z || !v || !out) return ORC_BAD;
    const double *X = z;
    const double *VU = v + (int64_t)n * (N + 1);
    double hh = 0.5 * (1.0 / (double)N);
    int64_t K = k1 - k0;
    #pragma omp parallel for schedule(static)
    for (int64_t k = k0; k < k1; k++) {
        for (int i = 0; i < n; i++) {
            double s = 0.0, sa = 0.0;
            for (int j = 0; j < n; j++) {
                for (int right = 0; right <= 1; right++) {
                    double e, ea;
                    jac_entry_x(N, n, A, gam, X, i, j, k, right, &e, &ea);
                    double vv = v[(int64_t)j * (N + 1) + k + right];
                    s += e * vv;
                    sa += ea * fabs(vv);
                }
            }
            for (int l = 0; l < m; l++) {
                for (int right = 0; right <= 1; right++) {
                    double e = -hh * B[i * m + l];
                    double vv = VU[(int64_t)l * (N + 1) + k + right];
                    s += e * vv;
                    sa += fabs(e * vv);
                }
            }
            out[(int64_t)i * K + (k - k0)] = s;
            if (mu) mu[(int64_t)i * K + (k - k0)] = sa;
        }
    }
    return ORC_OK;
}

/* dL/dA (n x n), dL/dB (n x m), dL/dgamma (n): sum over defect rows (i, k) of
 * y_ik dc_ik/dtheta, with
 *   dc_ik/dA_ij = -hh (sin X_jk + sin X_j,k+1),
 *   dc_ik/dB_il = -hh (U_lk + U_l,k+1),
 *   dc_ik/dgamma_i = -hh (X_ik X_pk + X_i,k+1 X_p,k+1).
 * Each sum runs over k in fixed chunks of OBJ_CHUNK with Neumaier
 * compensation, chunks summed in order (independent of the thread count).
 * mu arrays (nullable) get the sums of |terms|. */
int orc_coef_grad(int64_t N, int n, int m, const double *z, const double *y,
                  double *gA, double *gB, double *gg, double *muA, double *muB, double *mug)
{
    if (bad_sizes(N, n, m) || !z || !y || !gA || !gg || (m && !gB)) return ORC_BAD;
    const double *X = z;
    const double *U = z + (int64_t)n * (N + 1);
    double hh = 0.5 * (1.0 / (double)N);
    int nc = n * n + n * m + n;
    int64_t nch = (N + OBJ_CHUNK - 1) / OBJ_CHUNK;
    double *part = (double *)calloc((size_t)(nch * nc * 3), sizeof(double));
    if (!part) return ORC_BAD;
    #pragma omp parallel for schedule(static)
    for (int64_t ch = 0; ch < nch; ch++) {
        int64_t e = (ch + 1) * OBJ_CHUNK < N ? (ch + 1) * OBJ_CHUNK : N;
        for (int c = 0; c < nc; c++) {
            int i, kind, idx;
            if (c < n * n) { kind = 0; i = c / n; idx = c % n; }
            else if (c < n * n + n * m) { kind = 1; i = (c - n * n) / m; idx = (c - n * n) % m; }
            else { kind = 2; i = c - n * n - n * m; idx = 0; }
            int p = (i + 1) % n;
            acc_t a = {0.0, 0.0};
            double ma = 0.0;
            for (int64_t k = ch * OBJ_CHUNK; k < e; k++) {
                double d;
                if (kind == 0)
                    d = -hh * (sin(X[(int64_t)idx * (N + 1) + k]) + sin(X[(int64_t)idx * (N + 1) + k + 1]));
                else if (kind == 1)
                    d = -hh * (U[(int64_t)idx * (N + 1) + k] + U[(int64_t)idx * (N + 1) + k + 1]);
                else
                    d = -hh * (X[(int64_t)i * (N + 1) + k] * X[(int64_t)p * (N + 1) + k]
                               + X[(int64_t)i * (N + 1) + k + 1] * X[(int64_t)p * (N + 1) + k + 1]);
                double t = y[(int64_t)i * N + k] * d;
                acc_add(&a, t);
                ma += fabs(t);
            }
            part[(ch * nc + c) * 3 + 0] = a.s;
            part[(ch * nc + c) * 3 + 1] = a.c;
            part[(ch * nc + c) * 3 + 2] = ma;
        }
    }
    for (int c = 0; c < nc; c++) {
        acc_t a = {0.0, 0.0};
        double ma = 0.0;
        for (int64_t ch = 0; ch < nch; ch++) {
            acc_add(&a, part[(ch * nc + c) * 3 + 0]);
            acc_add(&a, part[(ch * nc + c) * 3 + 1]);
            ma += part[(ch * nc + c) * 3 + 2];
        }
        double val = a.s + a.c;
        if (c < n * n) { gA[c] = val; if (muA) muA[c] = ma; }
        else if (c < n * n + n * m) { gB[c - n * n] = val; if (muB) muB[c - n * n] = ma; }
        else { gg[c - n * n - n * m] = val; if (mug) mug[c - n * n - n * m] = ma; }
    }
    free(part);
    return ORC_OK;
}

/* ---- schemes and boundary rows (the _ex family) --------------------------- */
/*
 * scheme 0: trapezoidal (everything above);
 * scheme 1: forward Euler (paper Sec. 3): unknowns X_0..X_N and U_0..U_{N-1}
 *   (controls on N nodes), defects c_ik = X_{i,k+1} - X_ik - h F_i(k), and the
 *   Bolza-type cost sum_{k<N} h f0(X_k, U_k) (node N carries no cost).
 * bnd 0: no boundary rows; 1: initial rows X_i0 (i < n); 2: initial and final
 *   rows X_i0, X_iN.  As in the paper's generated code for x(0) == x0 (a
 *   constraint generator over the components with lcon = ucon), the row's
 *   value is the state itself; the target goes into the solver's bounds.
 * Layout: vx(j,k) = j (N+1) + k; vu(l,k) = n (N+1) + l NU + k with NU = N+1
 *   (trapezoidal) or N (Euler); defect rows i N + k, then the boundary rows.
 *   Jacobian COO: the defect entries slot-major as before with T slots per
 *   row (T = 2n+2m trapezoidal, n+1+m Euler, slots in ascending column
 *   order), then one entry per boundary row.  Hessian COO: state and pair
 *   slots s (N+1) + k as before, then control slots (n+npair)(N+1) + l NU + k.
 */

typedef struct {
    int64_t N, NU, nvar, ncon, ndef, nb, nnzj_def, nnzj, nnzh, dim;
    int n, m, npair, T, S, scheme, bnd;
} exdims_t;

static int ex_dims(int64_t N, int n, int m, int scheme, int bnd, exdims_t *d)
{
    if (bad_sizes(N, n, m) || scheme < 0 || scheme > 1 || bnd < 0 || bnd > 2) return ORC_BAD;
    d->N = N; d->n = n; d->m = m; d->scheme = scheme; d->bnd = bnd;
    d->NU = scheme == 0 ? N + 1 : N;
    d->npair = npair_of(n);
    d->T = scheme == 0 ? 2 * n + 2 * m : n + 1 + m;
    d->S = n + d->npair + m;
    d->nvar = (int64_t)n * (N + 1) + (int64_t)m * d->NU;
    d->ndef = (int64_t)n * N;
    d->nb = (int64_t)bnd * n;
    d->ncon = d->ndef + d->nb;
    d->nnzj_def = d->ndef * d->T;
    d->nnzj = d->nnzj_def + d->nb;
    d->nnzh = (int64_t)(n + d->npair) * (N + 1) + (int64_t)m * d->NU;
    d->dim = d->nvar + d->ncon;
    return ORC_OK;
}

/* out = {nvar, ncon, nnzj, nnzh, dim, npair, T, S, NU, nb} */
int orc_sizes_ex(int64_t N, int n, int m, int scheme, int bnd, int64_t *out)
{
    exdims_t d;
    if (ex_dims(N, n, m, scheme, bnd, &d) || !out) return ORC_BAD;
    out[0] = d.nvar; out[1] = d.ncon; out[2] = d.nnzj; out[3] = d.nnzh; out[4] = d.dim;
    out[5] = d.npair; out[6] = d.T; out[7] = d.S; out[8] = d.NU; out[9] = d.nb;
    return ORC_OK;
}

/* Cost weight of node k under the scheme. */
static double weight_ex(const exdims_t *d, int64_t k)
{
    double h = 1.0 / (double)d->N;
    if (d->scheme == 0) return (k == 0 || k == d->N) ? 0.5 * h : h;
    return k < d->N ? h : 0.0;
}

#define XV(z, d, j, k) ((z)[(int64_t)(j) * ((d)->N + 1) + (k)])
#define UV(z, d, l, k) ((z)[(int64_t)(d)->n * ((d)->N + 1) + (int64_t)(l) * (d)->NU + (k)])

/* F_i at node k with controls at node k (k < NU), and |F|. */
static void dyn_ex(const exdims_t *d, const double *A, const double *B, const double *gam,
                   const double *z, int64_t k, double *F, double *Fa)
{
    int n = d->n, m = d->m;
    for (int i = 0; i < n; i++) {
        double s = 0.0, sa = 0.0, t;
        for (int j = 0; j < n; j++) { t = A[i * n + j] * sin(XV(z, d, j, k)); s += t; sa += fabs(t); }
        for (int l = 0; l < m; l++) { t = B[i * m + l] * UV(z, d, l, k); s += t; sa += fabs(t); }
        int p = (i + 1) % n;
        t = gam[i] * XV(z, d, i, k) * XV(z, d, p, k);
        s += t; sa += fabs(t);
        F[i] = s;
        if (Fa) Fa[i] = sa;
    }
}

/* out = {f, mu}: sum over nodes of w_k (sum q X^2 + sum r U^2), U only where
 * it exists (k < NU); compensated as orc_obj. */
int orc_obj_ex(int64_t N, int n, int m, int scheme, int bnd, const double *q, const double *r,
               const double *z, double *out)
{
    exdims_t d;
    if (ex_dims(N, n, m, scheme, bnd, &d) || !z || !out) return ORC_BAD;
    acc_t tot = {0.0, 0.0};
    double mu = 0.0;
    for (int64_t k = 0; k <= N; k++) {
        double s = 0.0, sa = 0.0;
        for (int j = 0; j < n; j++) { double x = XV(z, &d, j, k); s += q[j] * x * x; sa += fabs(q[j] * x * x); }
        if (k < d.NU)
            for (int l = 0; l < m; l++) { double u = UV(z, &d, l, k); s += r[l] * u * u; sa += fabs(r[l] * u * u); }
        double w = weight_ex(&d, k);
        acc_add(&tot, w * s);
        mu += w * sa;
    }
    out[0] = tot.s + tot.c;
    out[1] = mu;
    return ORC_OK;
}

/* Full gradient of f (nvar entries, layout of z). */
int orc_grad_ex(int64_t N, int n, int m, int scheme, int bnd, const double *q, const double *r,
                const double *z, double *g, double *mu)
{
    exdims_t d;
    if (ex_dims(N, n, m, scheme, bnd, &d) || !z || !g) return ORC_BAD;
    for (int64_t k = 0; k <= N; k++) {
        double w = weight_ex(&d, k);
        for (int j = 0; j < n; j++) {
            int64_t e = (int64_t)j * (N + 1) + k;
            g[e] = 2.0 * w * q[j] * z[e];
            if (mu) mu[e] = fabs(g[e]);
        }
        if (k < d.NU)
            for (int l = 0; l < m; l++) {
                int64_t e = (int64_t)n * (N + 1) + (int64_t)l * d.NU + k;
                g[e] = 2.0 * w * r[l] * z[e];
                if (mu) mu[e] = fabs(g[e]);
            }
    }
    return ORC_OK;
}

/* All constraint rows (ncon): defects, then boundary rows. */
int orc_cons_ex(int64_t N, int n, int m, int scheme, int bnd, const double *A, const double *B,
                const double *gam, const double *z, double *c, double *mu)
{
    exdims_t d;
    if (ex_dims(N, n, m, scheme, bnd, &d) || !z || !c) return ORC_BAD;
    double h = 1.0 / (double)N, hh = 0.5 * h;
    #pragma omp parallel
    {
        double *F0 = (double *)malloc(sizeof(double) * 4 * n);
        double *F1 = F0 + n, *A0 = F0 + 2 * n, *A1 = F0 + 3 * n;
        #pragma omp for schedule(static)
        for (int64_t k = 0; k < N; k++) {
            dyn_ex(&d, A, B, gam, z, k, F0, A0);
            if (scheme == 0) dyn_ex(&d, A, B, gam, z, k + 1, F1, A1);
            for (int i = 0; i < n; i++) {
                double x0 = XV(z, &d, i, k), x1 = XV(z, &d, i, k + 1);
                int64_t r0 = (int64_t)i * N + k;
                if (scheme == 0) {
                    c[r0] = (x1 - x0) - hh * (F0[i] + F1[i]);
                    if (mu) mu[r0] = fabs(x1) + fabs(x0) + hh * (A0[i] + A1[i]);
                } else {
                    c[r0] = (x1 - x0) - h * F0[i];
                    if (mu) mu[r0] = fabs(x1) + fabs(x0) + h * A0[i];
                }
            }
        }
        free(F0);
    }
    for (int64_t b = 0; b < d.nb; b++) {
        int i = (int)(b % n);
        int64_t node = b < n ? 0 : N;
        c[d.ndef + b] = XV(z, &d, i, node);
        if (mu) mu[d.ndef + b] = fabs(c[d.ndef + b]);
    }
    return ORC_OK;
}

/* Column (variable index) of Jacobian slot t of defect row (i, k). */
static int64_t jac_col_ex(const exdims_t *d, int i, int t, int64_t k)
{
    int n = d->n;
    int64_t NX = (int64_t)n * (d->N + 1);
    if (d->scheme == 0) {
        if (t < 2 * n) return (int64_t)(t / 2) * (d->N + 1) + k + (t % 2);
        return NX + (int64_t)((t - 2 * n) / 2) * d->NU + k + ((t - 2 * n) % 2);
    }
    if (t <= i) return (int64_t)t * (d->N + 1) + k;               /* X_t at k */
    if (t == i + 1) return (int64_t)i * (d->N + 1) + k + 1;      /* X_i at k+1 */
    if (t <= n) return (int64_t)(t - 1) * (d->N + 1) + k;        /* X_{t-1} at k */
    return NX + (int64_t)(t - n - 1) * d->NU + k;                /* U_{t-n-1} at k */
}

int orc_pattern_ex(int64_t N, int n, int m, int scheme, int bnd, int32_t *jrow, int32_t *jcol,
                   int32_t *hrow, int32_t *hcol)
{
    exdims_t d;
    if (ex_dims(N, n, m, scheme, bnd, &d)) return ORC_BAD;
    if (d.dim + 1 > INT32_MAX || d.nnzj > INT32_MAX || d.nnzh > INT32_MAX) return ORC_BAD;
    int64_t NX = (int64_t)n * (N + 1);
    if (jrow && jcol) {
        for (int i = 0; i < n; i++)
            for (int t = 0; t < d.T; t++)
                for (int64_t k = 0; k < N; k++) {
                    int64_t e = ((int64_t)i * d.T + t) * N + k;
                    jrow[e] = (int32_t)((int64_t)i * N + k);
                    jcol[e] = (int32_t)jac_col_ex(&d, i, t, k);
                }
        for (int64_t b = 0; b < d.nb; b++) {
            int64_t e = d.nnzj_def + b;
            jrow[e] = (int32_t)(d.ndef + b);
            jcol[e] = (int32_t)((int64_t)(b % n) * (N + 1) + (b < n ? 0 : N));
        }
    }
    if (hrow && hcol) {
        for (int64_t k = 0; k <= N; k++) {
            for (int j = 0; j < n; j++) {
                int64_t e = (int64_t)j * (N + 1) + k;
                hrow[e] = hcol[e] = (int32_t)e;
            }
            for (int i = 0; i < d.npair; i++) {
                int a = i, b = (i + 1) % n;
                int hi = a > b ? a : b, lo = a < b ? a : b;
                int64_t e = (int64_t)(n + i) * (N + 1) + k;
                hrow[e] = (int32_t)((int64_t)hi * (N + 1) + k);
                hcol[e] = (int32_t)((int64_t)lo * (N + 1) + k);
            }
        }
        for (int l = 0; l < m; l++)
            for (int64_t k = 0; k < d.NU; k++) {
                int64_t e = (int64_t)(n + d.npair) * (N + 1) + (int64_t)l * d.NU + k;
                hrow[e] = hcol[e] = (int32_t)(NX + (int64_t)l * d.NU + k);
            }
    }
    return ORC_OK;
}

/* Jacobian values: defect entries (as orc_jac for the trapezoidal scheme; for
 * Euler the slots of the o4-style table X_t at k: -delta - h G, X_i at k+1:
 * +1, U_l at k: -h B), then 1.0 for every boundary row. */
int orc_jac_ex(int64_t N, int n, int m, int scheme, int bnd, const double *A, const double *B,
               const double *gam, const double *z, double *out, double *mu)
{
    exdims_t d;
    if (ex_dims(N, n, m, scheme, bnd, &d) || !z || !out) return ORC_BAD;
    double h = 1.0 / (double)N, hh = 0.5 * h;
    const double *X = z;
    #pragma omp parallel for collapse(2) schedule(static)
    for (int i = 0; i < n; i++)
        for (int t = 0; t < d.T; t++)
            for (int64_t k = 0; k < N; k++) {
                int64_t e = ((int64_t)i * d.T + t) * N + k;
                double v, va;
                if (scheme == 0) {
                    if (t < 2 * n) {
                        int j = t / 2, right = t % 2;
                        double dd = (i == j) ? 1.0 : 0.0, g, ga;
                        dF_dx(N, n, A, gam, X, i, j, k + right, &g, &ga);
                        v = (right ? dd : -dd) - hh * g;
                        va = dd + hh * ga;
                    } else {
                        v = -hh * B[i * m + (t - 2 * n) / 2];
                        va = fabs(v);
                    }
                } else {
                    if (t == i + 1) {
                        v = 1.0; va = 1.0;
                    } else if (t <= n) {
                        int j = t <= i ? t : t - 1;
                        double dd = (i == j) ? 1.0 : 0.0, g, ga;
                        dF_dx(N, n, A, gam, X, i, j, k, &g, &ga);
                        v = -dd - h * g;
                        va = dd + h * ga;
                    } else {
                        v = -h * B[i * m + (t - n - 1)];
                        va = fabs(v);
                    }
                }
                out[e] = v;
                if (mu) mu[e] = va;
            }
    for (int64_t b = 0; b < d.nb; b++) {
        out[d.nnzj_def + b] = 1.0;
        if (mu) mu[d.nnzj_def + b] = 1.0;
    }
    return ORC_OK;
}

/* Hessian of L = sigma f + y^T c (boundary rows are linear and add nothing).
 * Node multiplier and factor: trapezoidal yt = y_{k-1} + y_k, factor hh;
 * Euler yt = y_k (k < N), factor h.  Layout as orc_pattern_ex. */
int orc_hess_ex(int64_t N, int n, int m, int scheme, int bnd, const double *A, const double *gam,
                const double *q, const double *r, const double *z, const double *y, double sigma,
                double *out, double *mu)
{
    exdims_t d;
    if (ex_dims(N, n, m, scheme, bnd, &d) || !z || !y || !out) return ORC_BAD;
    double h = 1.0 / (double)N;
    double fac = scheme == 0 ? 0.5 * h : h;
    double *yt = (double *)malloc(sizeof(double) * 2 * n), *ya = yt + n;
    for (int64_t k = 0; k <= N; k++) {
        double w = weight_ex(&d, k);
        for (int i = 0; i < n; i++) {
            double a = 0.0, aa = 0.0;
            if (scheme == 0 && k >= 1) { a += y[(int64_t)i * N + k - 1]; aa += fabs(y[(int64_t)i * N + k - 1]); }
            if (k <= N - 1) { a += y[(int64_t)i * N + k]; aa += fabs(y[(int64_t)i * N + k]); }
            yt[i] = a; ya[i] = aa;
        }
        for (int j = 0; j < n; j++) {
            double sx = sin(XV(z, &d, j, k)), s = 0.0, sa = 0.0;
            for (int i = 0; i < n; i++) { s += yt[i] * A[i * n + j]; sa += ya[i] * fabs(A[i * n + j]); }
            double v = 2.0 * sigma * w * q[j] + fac * sx * s;
            double va = fabs(2.0 * sigma * w * q[j]) + fac * fabs(sx) * sa;
            if (n == 1) { v += -2.0 * fac * yt[0] * gam[0]; va += 2.0 * fac * ya[0] * fabs(gam[0]); }
            int64_t e = (int64_t)j * (N + 1) + k;
            out[e] = v;
            if (mu) mu[e] = va;
        }
        if (n >= 3) {
            for (int i = 0; i < n; i++) {
                int64_t e = (int64_t)(n + i) * (N + 1) + k;
                out[e] = -fac * yt[i] * gam[i];
                if (mu) mu[e] = fac * ya[i] * fabs(gam[i]);
            }
        } else if (n == 2) {
            int64_t e = (int64_t)n * (N + 1) + k;
            out[e] = -fac * (yt[0] * gam[0] + yt[1] * gam[1]);
            if (mu) mu[e] = fac * (ya[0] * fabs(gam[0]) + ya[1] * fabs(gam[1]));
        }
        if (k < d.NU)
            for (int l = 0; l < m; l++) {
                int64_t e = (int64_t)(n + d.npair) * (N + 1) + (int64_t)l * d.NU + k;
                out[e] = 2.0 * sigma * w * r[l];
                if (mu) mu[e] = fabs(out[e]);
            }
    }
    free(yt);
    return ORC_OK;
}

/* Generic KKT build from explicit sizes and COO patterns (see orc_kkt). */
int orc_kkt_generic(int64_t nvar, int64_t ncon, int64_t nnzj, int64_t nnzh,
                    const int32_t *jrow, const int32_t *jcol, const int32_t *hrow,
                    const int32_t *hcol, int32_t *rowptr, int32_t *colind, int32_t *perm_j,
                    int32_t *perm_h, int64_t *nnzk)
{
    int64_t dim = nvar + ncon;
    int64_t ntrip = nnzh + nnzj + dim;
    if (dim + 1 > INT32_MAX || ntrip > INT32_MAX) return ORC_BAD;
    int64_t *cnt = (int64_t *)calloc((size_t)dim + 1, sizeof(int64_t));
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)dim);
    ent_t *ent = (ent_t *)malloc(sizeof(ent_t) * (size_t)ntrip);
    if (!cnt || !pos || !ent) { free(cnt); free(pos); free(ent); return ORC_BAD; }
    int rc = ORC_OK;
    for (int64_t e = 0; e < nnzh; e++) cnt[hrow[e] + 1]++;
    for (int64_t e = 0; e < nnzj; e++) cnt[nvar + jrow[e] + 1]++;
    for (int64_t x = 0; x < dim; x++) cnt[x + 1]++;
    for (int64_t x = 0; x < dim; x++) cnt[x + 1] += cnt[x];
    memcpy(pos, cnt, sizeof(int64_t) * (size_t)dim);
    for (int64_t e = 0; e < nnzh; e++) {
        if (hcol[e] > hrow[e]) rc = ORC_BAD;
        ent_t t = { hcol[e], 2 * e };
        ent[pos[hrow[e]]++] = t;
    }
    for (int64_t e = 0; e < nnzj; e++) {
        int64_t row = nvar + jrow[e];
        if (jcol[e] > row) rc = ORC_BAD;
        ent_t t = { jcol[e], 2 * e + 1 };
        ent[pos[row]++] = t;
    }
    for (int64_t x = 0; x < dim; x++) {
        ent_t t = { x, -1 };
        ent[pos[x]++] = t;
    }
    free(pos);
    int64_t slot = -1;
    rowptr[0] = 0;
    for (int64_t x = 0; x < dim; x++) {
        int64_t b = cnt[x], en = cnt[x + 1];
        qsort(ent + b, (size_t)(en - b), sizeof(ent_t), ent_cmp);
        int64_t prev = -1;
        for (int64_t u = b; u < en; u++) {
            if (u == b || ent[u].col != prev) {
                slot++;
                colind[slot] = (int32_t)ent[u].col;
                prev = ent[u].col;
            }
            int64_t sr = ent[u].src;
            if (sr >= 0) {
                if (sr % 2 == 0) perm_h[sr / 2] = (int32_t)slot;
                else perm_j[sr / 2] = (int32_t)slot;
            }
        }
        rowptr[x + 1] = (int32_t)(slot + 1);
    }
    *nnzk = slot + 1;
    free(cnt);
    free(ent);
    return rc;
}

/* ===========================================================================
 * The quadrotor model (paper Appendix A), trapezoidal transcription (Sec. 5).
 *
 * Node-local variables v = 0..12: states x1..x9 are v = 0..8, controls
 * u1..u4 are v = 9..12; every variable lives on the N+1 nodes, so the global
 * index of v at node k is v (N+1) + k.  Defect row (i, k) is i N + k; the
 * boundary rows X_i0 (bnd >= 1) and X_iN (bnd == 2) follow the 9 N defects.
 *
 * Dynamics, as the paper writes them (phi = x7, theta = x8, psi = x9):
 *   F1 = x2, F3 = x4, F5 = x6,
 *   F2 = u1 c7 s8 c9 + u1 s7 s9,      F4 = u1 c7 s8 s9 - u1 s7 c9,
 *   F6 = u1 c7 c8 - g,
 *   F7 = u2 c7 / c8 + u3 s7 / c8,     F8 = -u2 s7 + u3 c7,
 *   F9 = u2 c7 t8 + u3 s7 t8 + u4.
 * Cost: 1/2 integral of (x1 - sin 2 pi t)^2 + (x3 - 2 sin 4 pi t)^2
 *   + (x5 - 2t)^2 + x7^2 + x8^2 + x9^2 + r (u1^2 + u2^2 + u3^2 + u4^2),
 *   with the trapezoidal weights w_k and t_k = k h.
 *
 * Patterns (structural support of the model):
 *   Jacobian row i holds, in ascending column order, for each variable v of
 *   its support (x_i itself and the variables F_i depends on) the two
 *   entries (v at node k, v at node k+1).  COO position of entry
 *   (i, p-th support variable, side s) of interval k: (off_i + 2p + s) N + k,
 *   off_i = 2 (support sizes of rows 0..i-1).  Boundary entries follow.
 *   Hessian: 23 lower-triangle entries per node, in (row, col) order, at
 *   COO position s (N+1) + k.  Every variable diagonal is listed (the KKT
 *   needs it), including those of x2, x4, x6, whose value is zero.
 * ======================================================================== */

#define QN 9
#define QV 13

static const int q_sup_len[QN] = { 2, 5, 2, 5, 2, 4, 4, 4, 6 };
static const int q_sup[QN][6] = {
    { 0, 1 },                /* F1 = x2 */
    { 1, 6, 7, 8, 9 },       /* F2(x7, x8, x9, u1) */
    { 2, 3 },                /* F3 = x4 */
    { 3, 6, 7, 8, 9 },       /* F4(x7, x8, x9, u1) */
    { 4, 5 },                /* F5 = x6 */
    { 5, 6, 7, 9 },          /* F6(x7, x8, u1) */
    { 6, 7, 10, 11 },        /* F7(x7, x8, u2, u3) */
    { 6, 7, 10, 11 },        /* F8(x7, u2, u3); x8 is the row's own state */
    { 6, 7, 8, 10, 11, 12 }, /* F9(x7, x8, u2, u3, u4); x9 own state */
};
#define Q_NNZH_NODE 23
static const int q_hpat[Q_NNZH_NODE][2] = {
    { 0, 0 }, { 1, 1 }, { 2, 2 }, { 3, 3 }, { 4, 4 }, { 5, 5 }, { 6, 6 },
    { 7, 6 }, { 7, 7 }, { 8, 6 }, { 8, 7 }, { 8, 8 },
    { 9, 6 }, { 9, 7 }, { 9, 8 }, { 9, 9 },
    { 10, 6 }, { 10, 7 }, { 10, 10 },
    { 11, 6 }, { 11, 7 }, { 11, 11 },
    { 12, 12 },
};

static int q_slots_per_interval(void)
{
    int t = 0;
    for (int i = 0; i < QN; i++) t += 2 * q_sup_len[i];
    return t;
}

/* out = {nvar, ncon, nnzj, nnzh, dim} */
int orc_quad_sizes(int64_t N, int bnd, int64_t *out)
{
    if (N < 1 || bnd < 0 || bnd > 2 || !out) return ORC_BAD;
    out[0] = (int64_t)QV * (N + 1);
    out[1] = (int64_t)QN * N + (int64_t)QN * bnd;
    out[2] = (int64_t)q_slots_per_interval() * N + (int64_t)QN * bnd;
    out[3] = (int64_t)Q_NNZH_NODE * (N + 1);
    out[4] = out[0] + out[1];
    return ORC_OK;
}

int orc_quad_pattern(int64_t N, int bnd, int32_t *jrow, int32_t *jcol, int32_t *hrow, int32_t *hcol)
{
    if (N < 1 || bnd < 0 || bnd > 2) return ORC_BAD;
    int64_t N1 = N + 1;
    if (jrow && jcol) {
        int64_t off = 0;
        for (int i = 0; i < QN; i++) {
            for (int p = 0; p < q_sup_len[i]; p++)
                for (int s = 0; s < 2; s++) {
                    int64_t slot = off + 2 * p + s;
                    for (int64_t k = 0; k < N; k++) {
                        jrow[slot * N + k] = (int32_t)((int64_t)i * N + k);
                        jcol[slot * N + k] = (int32_t)((int64_t)q_sup[i][p] * N1 + k + s);
                    }
                }
            off += 2 * q_sup_len[i];
        }
        int64_t e0 = off * N;
        for (int b = 0; b < QN * bnd; b++) {
            jrow[e0 + b] = (int32_t)((int64_t)QN * N + b);
            jcol[e0 + b] = (int32_t)((int64_t)(b % QN) * N1 + (b < QN ? 0 : N));
        }
    }
    if (hrow && hcol)
        for (int s = 0; s < Q_NNZH_NODE; s++)
            for (int64_t k = 0; k < N1; k++) {
                hrow[s * N1 + k] = (int32_t)((int64_t)q_hpat[s][0] * N1 + k);
                hcol[s * N1 + k] = (int32_t)((int64_t)q_hpat[s][1] * N1 + k);
            }
    return ORC_OK;
}

static void q_node(int64_t N, const double *z, int64_t k, double *x, double *u)
{
    for (int j = 0; j < 9; j++) x[j] = z[(int64_t)j * (N + 1) + k];
    for (int l = 0; l < 4; l++) u[l] = z[(int64_t)(9 + l) * (N + 1) + k];
}

typedef struct { double s7, c7, s8, c8, t8, s9, c9; } qtrig_t;

static qtrig_t q_trig(const double *x)
{
    qtrig_t t = { sin(x[6]), cos(x[6]), sin(x[7]), cos(x[7]), tan(x[7]), sin(x[8]), cos(x[8]) };
    return t;
}

/* F (9 values) and the magnitude of each (sum of |terms|). */
static void q_rhs(const double *x, const double *u, double g, double *F, double *Fa)
{
    qtrig_t t = q_trig(x);
    double a, b;
    F[0] = x[1];
    Fa[0] = fabs(x[1]);
    a = u[0] * t.c7 * t.s8 * t.c9; b = u[0] * t.s7 * t.s9;
    F[1] = a + b; Fa[1] = fabs(a) + fabs(b);
    F[2] = x[3];
    Fa[2] = fabs(x[3]);
    a = u[0] * t.c7 * t.s8 * t.s9; b = u[0] * t.s7 * t.c9;
    F[3] = a - b; Fa[3] = fabs(a) + fabs(b);
    F[4] = x[5];
    Fa[4] = fabs(x[5]);
    a = u[0] * t.c7 * t.c8;
    F[5] = a - g; Fa[5] = fabs(a) + fabs(g);
    a = u[1] * t.c7 / t.c8; b = u[2] * t.s7 / t.c8;
    F[6] = a + b; Fa[6] = fabs(a) + fabs(b);
    a = -u[1] * t.s7; b = u[2] * t.c7;
    F[7] = a + b; Fa[7] = fabs(a) + fabs(b);
    double c;
    a = u[1] * t.c7 * t.t8; b = u[2] * t.s7 * t.t8; c = u[3];
    F[8] = a + b + c; Fa[8] = fabs(a) + fabs(b) + fabs(c);
}

/* Dense first partials D[i][v] = dF_i/dv, each differentiated term by term
 * from the expressions above, and their magnitudes. */
static void q_d1(const double *x, const double *u, double D[QN][QV], double Da[QN][QV])
{
    qtrig_t t = q_trig(x);
    double sec2 = 1.0 / (t.c8 * t.c8);
    memset(D, 0, sizeof(double) * QN * QV);
    memset(Da, 0, sizeof(double) * QN * QV);
#define SET1(i, v, A) do { D[i][v] = (A); Da[i][v] = fabs(A); } while (0)
#define SET2(i, v, A, B) do { double a_ = (A), b_ = (B); D[i][v] = a_ + b_; Da[i][v] = fabs(a_) + fabs(b_); } while (0)
    SET1(0, 1, 1.0);
    /* F2 = u1 c7 s8 c9 + u1 s7 s9 */
    SET2(1, 6, -u[0] * t.s7 * t.s8 * t.c9, u[0] * t.c7 * t.s9);
    SET1(1, 7, u[0] * t.c7 * t.c8 * t.c9);
    SET2(1, 8, -u[0] * t.c7 * t.s8 * t.s9, u[0] * t.s7 * t.c9);
    SET2(1, 9, t.c7 * t.s8 * t.c9, t.s7 * t.s9);
    SET1(2, 3, 1.0);
    /* F4 = u1 c7 s8 s9 - u1 s7 c9 */
    SET2(3, 6, -u[0] * t.s7 * t.s8 * t.s9, -u[0] * t.c7 * t.c9);
    SET1(3, 7, u[0] * t.c7 * t.c8 * t.s9);
    SET2(3, 8, u[0] * t.c7 * t.s8 * t.c9, u[0] * t.s7 * t.s9);
    SET2(3, 9, t.c7 * t.s8 * t.s9, -t.s7 * t.c9);
    SET1(4, 5, 1.0);
    /* F6 = u1 c7 c8 - g */
    SET1(5, 6, -u[0] * t.s7 * t.c8);
    SET1(5, 7, -u[0] * t.c7 * t.s8);
    SET1(5, 9, t.c7 * t.c8);
    /* F7 = u2 c7 / c8 + u3 s7 / c8;  d(1/c8)/dx8 = s8 / c8^2 */
    SET2(6, 6, -u[1] * t.s7 / t.c8, u[2] * t.c7 / t.c8);
    SET2(6, 7, u[1] * t.c7 * t.s8 * sec2, u[2] * t.s7 * t.s8 * sec2);
    SET1(6, 10, t.c7 / t.c8);
    SET1(6, 11, t.s7 / t.c8);
    /* F8 = -u2 s7 + u3 c7 */
    SET2(7, 6, -u[1] * t.c7, -u[2] * t.s7);
    SET1(7, 10, -t.s7);
    SET1(7, 11, t.c7);
    /* F9 = u2 c7 t8 + u3 s7 t8 + u4;  d(t8)/dx8 = 1 / c8^2 */
    SET2(8, 6, -u[1] * t.s7 * t.t8, u[2] * t.c7 * t.t8);
    SET2(8, 7, u[1] * t.c7 * sec2, u[2] * t.s7 * sec2);
    SET1(8, 10, t.c7 * t.t8);
    SET1(8, 11, t.s7 * t.t8);
    SET1(8, 12, 1.0);
#undef SET1
#undef SET2
}

/* Dense second partials W[i][a][b] (both triangles) and magnitudes. */
static void q_d2(const double *x, const double *u, double W[QN][QV][QV], double Wa[QN][QV][QV])
{
    qtrig_t t = q_trig(x);
    double c8 = t.c8, s8 = t.s8;
    double sec2 = 1.0 / (c8 * c8);
    /* d^2(1/c8)/dx8^2 = (1 + s8^2) / c8^3,  d^2(t8)/dx8^2 = 2 s8 / c8^3 */
    double dsec2 = (1.0 + s8 * s8) / (c8 * c8 * c8);
    double dtan2 = 2.0 * s8 / (c8 * c8 * c8);
    memset(W, 0, sizeof(double) * QN * QV * QV);
    memset(Wa, 0, sizeof(double) * QN * QV * QV);
#define S1(i, a, b, A) do { double v_ = (A); W[i][a][b] = v_; W[i][b][a] = v_; \
        Wa[i][a][b] = fabs(v_); Wa[i][b][a] = fabs(v_); } while (0)
#define S2(i, a, b, A, B) do { double a_ = (A), b_ = (B); W[i][a][b] = a_ + b_; W[i][b][a] = a_ + b_; \
        Wa[i][a][b] = fabs(a_) + fabs(b_); Wa[i][b][a] = fabs(a_) + fabs(b_); } while (0)
    /* F2 = u1 c7 s8 c9 + u1 s7 s9 */
    S2(1, 6, 6, -u[0] * t.c7 * t.s8 * t.c9, -u[0] * t.s7 * t.s9);
    S1(1, 6, 7, -u[0] * t.s7 * t.c8 * t.c9);
    S2(1, 6, 8, u[0] * t.s7 * t.s8 * t.s9, u[0] * t.c7 * t.c9);
    S1(1, 7, 7, -u[0] * t.c7 * t.s8 * t.c9);
    S1(1, 7, 8, -u[0] * t.c7 * t.c8 * t.s9);
    S2(1, 8, 8, -u[0] * t.c7 * t.s8 * t.c9, -u[0] * t.s7 * t.s9);
    S2(1, 9, 6, -t.s7 * t.s8 * t.c9, t.c7 * t.s9);
    S1(1, 9, 7, t.c7 * t.c8 * t.c9);
    S2(1, 9, 8, -t.c7 * t.s8 * t.s9, t.s7 * t.c9);
    /* F4 = u1 c7 s8 s9 - u1 s7 c9 */
    S2(3, 6, 6, -u[0] * t.c7 * t.s8 * t.s9, u[0] * t.s7 * t.c9);
    S1(3, 6, 7, -u[0] * t.s7 * t.c8 * t.s9);
    S2(3, 6, 8, -u[0] * t.s7 * t.s8 * t.c9, u[0] * t.c7 * t.s9);
    S1(3, 7, 7, -u[0] * t.c7 * t.s8 * t.s9);
    S1(3, 7, 8, u[0] * t.c7 * t.c8 * t.c9);
    S2(3, 8, 8, -u[0] * t.c7 * t.s8 * t.s9, u[0] * t.s7 * t.c9);
    S2(3, 9, 6, -t.s7 * t.s8 * t.s9, -t.c7 * t.c9);
    S1(3, 9, 7, t.c7 * t.c8 * t.s9);
    S2(3, 9, 8, t.c7 * t.s8 * t.c9, t.s7 * t.s9);
    /* F6 = u1 c7 c8 - g */
    S1(5, 6, 6, -u[0] * t.c7 * t.c8);
    S1(5, 6, 7, u[0] * t.s7 * t.s8);
    S1(5, 7, 7, -u[0] * t.c7 * t.c8);
    S1(5, 9, 6, -t.s7 * t.c8);
    S1(5, 9, 7, -t.c7 * t.s8);
    /* F7 = u2 c7 / c8 + u3 s7 / c8 */
    S2(6, 6, 6, -u[1] * t.c7 / c8, -u[2] * t.s7 / c8);
    S2(6, 6, 7, -u[1] * t.s7 * s8 * sec2, u[2] * t.c7 * s8 * sec2);
    S2(6, 7, 7, u[1] * t.c7 * dsec2, u[2] * t.s7 * dsec2);
    S1(6, 10, 6, -t.s7 / c8);
    S1(6, 10, 7, t.c7 * s8 * sec2);
    S1(6, 11, 6, t.c7 / c8);
    S1(6, 11, 7, t.s7 * s8 * sec2);
    /* F8 = -u2 s7 + u3 c7 */
    S2(7, 6, 6, u[1] * t.s7, -u[2] * t.c7);
    S1(7, 10, 6, -t.c7);
    S1(7, 11, 6, -t.s7);
    /* F9 = u2 c7 t8 + u3 s7 t8 + u4 */
    S2(8, 6, 6, -u[1] * t.c7 * t.t8, -u[2] * t.s7 * t.t8);
    S2(8, 6, 7, -u[1] * t.s7 * sec2, u[2] * t.c7 * sec2);
    S2(8, 7, 7, u[1] * t.c7 * dtan2, u[2] * t.s7 * dtan2);
    S1(8, 10, 6, -t.s7 * t.t8);
    S1(8, 10, 7, t.c7 * sec2);
    S1(8, 11, 6, t.c7 * t.t8);
    S1(8, 11, 7, t.s7 * sec2);
#undef S1
#undef S2
}

/* Reference trajectory of the tracked states at time t: (x1, x3, x5) targets. */
#define Q_PI 3.14159265358979323846

static void q_refs(double t, double *d)
{
    d[0] = sin(2.0 * Q_PI * t);
    d[1] = 2.0 * sin(4.0 * Q_PI * t);
    d[2] = 2.0 * t;
}

/* out[0] = f, out[1] = mu(f); compensated sums in fixed chunks (as orc_obj). */
int orc_quad_obj(int64_t N, double r, const double *z, double *out)
{
    if (N < 1 || !z || !out) return ORC_BAD;
    int64_t N1 = N + 1;
    double h = 1.0 / (double)N;
    int64_t nch = (N1 + OBJ_CHUNK - 1) / OBJ_CHUNK;
    acc_t *part = (acc_t *)calloc((size_t)nch, sizeof(acc_t));
    double *pmu = (double *)calloc((size_t)nch, sizeof(double));
    if (!part || !pmu) { free(part); free(pmu); return ORC_BAD; }
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nch; c++) {
        acc_t a = { 0.0, 0.0 };
        double mu = 0.0;
        int64_t k1 = (c + 1) * OBJ_CHUNK < N1 ? (c + 1) * OBJ_CHUNK : N1;
        for (int64_t k = c * OBJ_CHUNK; k < k1; k++) {
            double x[9], u[4], d[3];
            q_node(N, z, k, x, u);
            q_refs((double)k * h, d);
            double e0 = x[0] - d[0], e2 = x[2] - d[1], e4 = x[4] - d[2];
            double L = e0 * e0 + e2 * e2 + e4 * e4 + x[6] * x[6] + x[7] * x[7] + x[8] * x[8]
                       + r * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2] + u[3] * u[3]);
            double La = (fabs(x[0]) + fabs(d[0])) * (fabs(x[0]) + fabs(d[0]))
                        + (fabs(x[2]) + fabs(d[1])) * (fabs(x[2]) + fabs(d[1]))
                        + (fabs(x[4]) + fabs(d[2])) * (fabs(x[4]) + fabs(d[2]))
                        + x[6] * x[6] + x[7] * x[7] + x[8] * x[8]
                        + fabs(r) * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2] + u[3] * u[3]);
            double w = weight(N, k);
            acc_add(&a, w * (0.5 * L));
            mu += w * 0.5 * La;
        }
        part[c] = a;
        pmu[c] = mu;
    }
    acc_t tot = { 0.0, 0.0 };
    double mu = 0.0;
    for (int64_t c = 0; c < nch; c++) {
        acc_add(&tot, part[c].s);
        acc_add(&tot, part[c].c);
        mu += pmu[c];
    }
    out[0] = tot.s + tot.c;
    out[1] = mu;
    free(part);
    free(pmu);
    return ORC_OK;
}

/* Gradient of the cost: w_k (x - target) for x1, x3, x5; w_k x for x7..x9;
 * w_k r u for the controls; zero for x2, x4, x6. */
int orc_quad_grad(int64_t N, double r, const double *z, double *g, double *mu)
{
    if (N < 1 || !z || !g || !mu) return ORC_BAD;
    int64_t N1 = N + 1;
    double h = 1.0 / (double)N;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < N1; k++) {
        double x[9], u[4], d[3];
        q_node(N, z, k, x, u);
        q_refs((double)k * h, d);
        double w = weight(N, k);
        for (int v = 0; v < QV; v++) { g[v * N1 + k] = 0.0; mu[v * N1 + k] = 0.0; }
        for (int q = 0; q < 3; q++) {
            int v = 2 * q;
            g[v * N1 + k] = w * (x[v] - d[q]);
            mu[v * N1 + k] = w * (fabs(x[v]) + fabs(d[q]));
        }
        for (int v = 6; v < 9; v++) {
            g[v * N1 + k] = w * x[v];
            mu[v * N1 + k] = fabs(w * x[v]);
        }
        for (int l = 0; l < 4; l++) {
            g[(9 + l) * N1 + k] = w * r * u[l];
            mu[(9 + l) * N1 + k] = fabs(w * r * u[l]);
        }
    }
    return ORC_OK;
}

int orc_quad_cons(int64_t N, int bnd, double g, const double *z, double *c, double *mu)
{
    if (N < 1 || bnd < 0 || bnd > 2 || !z || !c || !mu) return ORC_BAD;
    double hh = 0.5 * (1.0 / (double)N);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < N; k++) {
        double x0[9], u0[4], x1[9], u1[4], F0[9], Fa0[9], F1[9], Fa1[9];
        q_node(N, z, k, x0, u0);
        q_node(N, z, k + 1, x1, u1);
        q_rhs(x0, u0, g, F0, Fa0);
        q_rhs(x1, u1, g, F1, Fa1);
        for (int i = 0; i < QN; i++) {
            c[(int64_t)i * N + k] = (x1[i] - x0[i]) - hh * (F0[i] + F1[i]);
            mu[(int64_t)i * N + k] = fabs(x1[i]) + fabs(x0[i]) + hh * (Fa0[i] + Fa1[i]);
        }
    }
    for (int b = 0; b < QN * bnd; b++) {
        double v = z[(int64_t)(b % QN) * (N + 1) + (b < QN ? 0 : N)];
        c[(int64_t)QN * N + b] = v;
        mu[(int64_t)QN * N + b] = fabs(v);
    }
    return ORC_OK;
}

int orc_quad_jac(int64_t N, int bnd, const double *z, double *jac, double *mu)
{
    if (N < 1 || bnd < 0 || bnd > 2 || !z || !jac || !mu) return ORC_BAD;
    double hh = 0.5 * (1.0 / (double)N);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < N; k++) {
        double x[2][9], u[2][4];
        double D[2][QN][QV], Da[2][QN][QV];
        for (int s = 0; s < 2; s++) {
            q_node(N, z, k + s, x[s], u[s]);
            q_d1(x[s], u[s], D[s], Da[s]);
        }
        int64_t off = 0;
        for (int i = 0; i < QN; i++) {
            for (int p = 0; p < q_sup_len[i]; p++) {
                int v = q_sup[i][p];
                for (int s = 0; s < 2; s++) {
                    double id = v == i ? (s ? 1.0 : -1.0) : 0.0;
                    int64_t e = (off + 2 * p + s) * N + k;
                    jac[e] = id - hh * D[s][i][v];
                    mu[e] = fabs(id) + hh * Da[s][i][v];
                }
            }
            off += 2 * q_sup_len[i];
        }
    }
    int64_t e0 = (int64_t)q_slots_per_interval() * N;
    for (int b = 0; b < QN * bnd; b++) {
        jac[e0 + b] = 1.0;
        mu[e0 + b] = 1.0;
    }
    return ORC_OK;
}

/* Hessian of L = sigma f + y^T c on the 23-entry node pattern:
 * sigma w_k C_ab - hh sum_i ytilde_ik d2F_i/(da db), where C is the cost's
 * constant second derivative (1 for x1, x3, x5, x7, x8, x9; r for controls)
 * and ytilde_ik = y_{i,k-1} [k >= 1] + y_{ik} [k < N].  Boundary rows are
 * linear and add nothing. */
int orc_quad_hess(int64_t N, double r, const double *z, const double *y, double sigma,
                  double *hess, double *mu)
{
    if (N < 1 || !z || !y || !hess || !mu) return ORC_BAD;
    int64_t N1 = N + 1;
    double hh = 0.5 * (1.0 / (double)N);
    static const int tracked[QV] = { 1, 0, 1, 0, 1, 0, 1, 1, 1, 0, 0, 0, 0 };
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < N1; k++) {
        double x[9], u[4], yt[QN];
        double (*W)[QV][QV] = malloc(sizeof(double) * QN * QV * QV);
        double (*Wa)[QV][QV] = malloc(sizeof(double) * QN * QV * QV);
        q_node(N, z, k, x, u);
        q_d2(x, u, W, Wa);
        for (int i = 0; i < QN; i++) {
            yt[i] = 0.0;
            if (k >= 1) yt[i] += y[(int64_t)i * N + k - 1];
            if (k < N) yt[i] += y[(int64_t)i * N + k];
        }
        double w = weight(N, k);
        for (int s = 0; s < Q_NNZH_NODE; s++) {
            int a = q_hpat[s][0], b = q_hpat[s][1];
            double cst = 0.0;
            if (a == b) cst = a < 9 ? (tracked[a] ? 1.0 : 0.0) : r;
            double v = sigma * w * cst, m = fabs(sigma * w * cst);
            for (int i = 0; i < QN; i++) {
                v += -hh * yt[i] * W[i][a][b];
                m += hh * fabs(yt[i]) * Wa[i][a][b];
            }
            hess[s * N1 + k] = v;
            mu[s * N1 + k] = m;
        }
        free(W);
        free(Wa);
    }
    return ORC_OK;
}

/* ===========================================================================
 * Symmetric reordering of the KKT matrix (paper Sec. 6: the one-time host
 * analysis reorders the matrix to reduce fill before LDL^T).
 *
 * Given the lower CSR of K (any of the builds above) and an ordering
 * order[new] = old, the lower CSR of P K P^T (entry (pos[r], pos[c]) for each
 * stored (r, c), pos = order^-1, mirrored into the lower triangle) is built
 * generically -- triplets -> counting sort by new row -> sort by new column --
 * and every old slot is mapped to its new slot: perm_j2 = map o perm_j,
 * perm_h2 = map o perm_h, and diag2[d] = map(diagonal slot of old row d).
 * ======================================================================== */
int orc_kkt_permute(int64_t dim, const int32_t *rowptr, const int32_t *colind,
                    int64_t nnzj, const int32_t *perm_j, int64_t nnzh, const int32_t *perm_h,
                    const int32_t *order, int32_t *rowptr2, int32_t *colind2, int32_t *perm_j2,
                    int32_t *perm_h2, int32_t *diag2)
{
    if (dim < 1 || !rowptr || !colind || !order || !rowptr2 || !colind2) return ORC_BAD;
    int64_t nnzk = rowptr[dim];
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)dim);
    int64_t *cnt = (int64_t *)calloc((size_t)dim + 1, sizeof(int64_t));
    int64_t *map = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnzk ? nnzk : 1));
    ent_t *ent = (ent_t *)malloc(sizeof(ent_t) * (size_t)(nnzk ? nnzk : 1));
    int64_t *fillp = (int64_t *)malloc(sizeof(int64_t) * (size_t)dim);
    int rc = ORC_OK;
    if (!pos || !cnt || !map || !ent || !fillp) { rc = ORC_BAD; goto done; }
    for (int64_t i = 0; i < dim; i++) pos[i] = -1;
    for (int64_t i = 0; i < dim; i++) {
        int64_t o = order[i];
        if (o < 0 || o >= dim || pos[o] >= 0) { rc = ORC_BAD; goto done; }
        pos[o] = i;
    }
    /* new row of every stored entry */
    for (int64_t r = 0; r < dim; r++)
        for (int64_t q = rowptr[r]; q < rowptr[r + 1]; q++) {
            int64_t a = pos[r], b = pos[colind[q]];
            cnt[(a > b ? a : b) + 1]++;
        }
    for (int64_t i = 0; i < dim; i++) cnt[i + 1] += cnt[i];
    memcpy(fillp, cnt, sizeof(int64_t) * (size_t)dim);
    for (int64_t r = 0; r < dim; r++)
        for (int64_t q = rowptr[r]; q < rowptr[r + 1]; q++) {
            int64_t a = pos[r], b = pos[colind[q]];
            int64_t row = a > b ? a : b, col = a > b ? b : a;
            ent_t t = { col, q };
            ent[fillp[row]++] = t;
        }
    for (int64_t i = 0; i < dim; i++) {
        qsort(ent + cnt[i], (size_t)(cnt[i + 1] - cnt[i]), sizeof(ent_t), ent_cmp);
        rowptr2[i] = (int32_t)cnt[i];
        for (int64_t u = cnt[i]; u < cnt[i + 1]; u++) {
            if (u > cnt[i] && ent[u].col == ent[u - 1].col) rc = ORC_BAD;  /* duplicate */
            colind2[u] = (int32_t)ent[u].col;
            map[ent[u].src] = u;
        }
    }
    rowptr2[dim] = (int32_t)nnzk;
    if (perm_j2) for (int64_t e = 0; e < nnzj; e++) perm_j2[e] = (int32_t)map[perm_j[e]];
    if (perm_h2) for (int64_t e = 0; e < nnzh; e++) perm_h2[e] = (int32_t)map[perm_h[e]];
    if (diag2) for (int64_t d = 0; d < dim; d++) diag2[d] = (int32_t)map[rowptr[d + 1] - 1];
done:
    free(pos); free(cnt); free(map); free(ent); free(fillp);
    return rc;
}

/* Assembly through slot maps alone: kkt = 0; kkt[perm_h[e]] = hess[e];
 * kkt[perm_j[e]] = jac[e]; then kkt[diag[d]] += reg[d] for every row d. */
int orc_assemble_mapped(int64_t nnzk, int64_t dim, const int32_t *diag,
                        int64_t nnzj, const int32_t *perm_j, const double *jac,
                        int64_t nnzh, const int32_t *perm_h, const double *hess,
                        const double *reg, double *kkt)
{
    if (!kkt || !diag || nnzk < 0) return ORC_BAD;
    for (int64_t x = 0; x < nnzk; x++) kkt[x] = 0.0;
    for (int64_t e = 0; e < nnzh; e++) kkt[perm_h[e]] = hess[e];
    for (int64_t e = 0; e < nnzj; e++) kkt[perm_j[e]] = jac[e];
    if (reg)
        for (int64_t d = 0; d < dim; d++) kkt[diag[d]] += reg[d];
    return ORC_OK;
}
