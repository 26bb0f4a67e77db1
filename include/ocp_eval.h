/*
 * ocp_eval.h -- C ABI of the MI355X (gfx950) evaluation library for the
 * trapezoidal direct-transcription NLP of an optimal control problem.
 *
 * What it evaluates (paper Sec. 3: direct transcription; Sec. 5: the
 * trapezoidal constraint and objective generators; Sec. 6: the evaluations an
 * interior-point iteration requests on the device and the KKT assembly):
 *
 *   unknowns   z = [X | U], X_{jk} (n states), U_{lk} (m controls) on the
 *              nodes k = 0..N of the uniform grid t_k = k h, h = 1/N
 *   dynamics   F_i(k) = sum_j A_ij sin X_jk + sum_l B_il U_lk
 *                       + gamma_i X_ik X_{p(i)k},   p(i) = (i+1) mod n
 *   defects    c_{ik} = (X_{i,k+1} - X_ik) - (h/2) (F_i(k) + F_i(k+1)),  k < N
 *   cost       f = sum_k w_k (sum_j q_j X_jk^2 + sum_l r_l U_lk^2),
 *              w_0 = w_N = h/2, w_k = h otherwise (trapezoidal rule)
 *   Lagrangian L = sigma f + y^T c
 *   KKT        K = [[H, J^T], [J, 0]], H = Hessian of L, J = Jacobian of c
 *
 * Layouts (all structure-of-arrays, node index fastest):
 *   z          index vx(j,k) = j (N+1) + k, vu(l,k) = n (N+1) + l (N+1) + k;
 *              nvar = (n+m)(N+1) doubles
 *   c, y       row r(i,k) = i N + k; ncon = n N doubles
 *   Jacobian   T = 2n + 2m slots per row, in ascending column order:
 *              slot 2j: X_j at k, 2j+1: X_j at k+1, 2n+2l: U_l at k,
 *              2n+2l+1: U_l at k+1.  COO entry e = (i T + t) N + k.
 *              nnzj = n N T.  Structural: every slot is stored even if zero.
 *   Hessian    lower triangle, block-diagonal per node; S = n + npair + m
 *              slots per node, npair = n (n >= 3), 1 (n = 2), 0 (n = 1):
 *              slot j < n: (vx(j,k), vx(j,k)); slot n+i (n >= 3):
 *              (vx(max(i,p(i)),k), vx(min(i,p(i)),k)); slot n (n = 2):
 *              (vx(1,k), vx(0,k)) with both bilinear terms merged; slot
 *              n+npair+l: (vu(l,k), vu(l,k)).  For n = 1 the bilinear term
 *              folds into the state diagonal.  COO entry e = s (N+1) + k.
 *   KKT        lower-triangular CSR of K, dim = nvar + ncon rows, columns
 *              ascending within a row, every diagonal present and last in its
 *              row; nnzk = nnzh + nnzj + ncon.  perm_j[e] / perm_h[e] give the
 *              CSR slot of Jacobian / Hessian COO entry e.
 *
 * Precision: IEEE binary64 throughout.  Indices are int32; every size and
 * index must fit in int32 or the call fails with OCP_ERR_OVERFLOW.
 *
 * Ownership: the caller owns every array.  Arrays passed to ocp_eval_* and
 * ocp_assemble_kkt are device pointers (HBM), contiguous; the index builders
 * fill host arrays.  The problem handle owns device copies of the dynamics and
 * cost coefficients and two device workspaces, both fixed at create time: the
 * per-workgroup partial sums of the objective and Lagrangian (at most 4096
 * doubles) and of the coefficient gradient (n (n+m+1) G doubles, G =
 * min(1024, ceil((N+1) / 64)) workgroups); the library never hands out
 * memory for the caller to free.
 *
 * Streams: every device call is asynchronous on the given HIP stream (0 = the
 * null stream) and never synchronizes; the objective lands in a device double.
 * Each call fully overwrites its output array.  Errors found on the host
 * (arguments, sizes) are returned before any HIP call; a launch failure is
 * reported as OCP_ERR_HIP; faults inside a kernel surface at the caller's next
 * synchronization.  No C++ exception crosses this interface.
 *
 * Reentrancy: evaluations on one handle may run concurrently on different
 * streams, except calls that share one of the handle's two workspaces:
 * ocp_eval_obj and ocp_eval_lagrangian (the reduction workspace), and
 * ocp_eval_coef_grad, ocp_eval_coef_mixed and ocp_eval_lagrangian_backward
 * with coefficient outputs (the coefficient-gradient workspace); two
 * overlapping calls on one workspace race.  ocp_set_coefficients changes what
 * the other calls read, so the caller orders it against them.  Create and
 * destroy are not thread-safe for the same handle.
 */
#ifndef OCP_EVAL_H
#define OCP_EVAL_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define OCP_OK 0
#define OCP_ERR_ARG 1       /* null pointer, N < 1, n < 1, m < 0, n or m above OCP_MAX_DIM */
#define OCP_ERR_OVERFLOW 2  /* a size or index does not fit in int32 */
#define OCP_ERR_HIP 3       /* a HIP runtime call or kernel launch failed */
#define OCP_ERR_ALLOC 4     /* host or device allocation failed */

/* Largest supported state or control dimension. */
#define OCP_MAX_DIM 32

typedef struct ocp_sizes_t {
    int64_t nvar;   /* (n+m)(N+1)                unknowns */
    int64_t ncon;   /* n N                       defect rows */
    int64_t nnzj;   /* n N (2n+2m)               Jacobian entries */
    int64_t nnzh;   /* (n + npair + m)(N+1)      Hessian (lower) entries */
    int64_t nnzk;   /* nnzh + nnzj + ncon        KKT (lower CSR) entries */
    int64_t dim;    /* nvar + ncon               KKT rows */
    int32_t npair;  /* bilinear Hessian slots per node */
    int32_t T;      /* Jacobian slots per row */
    int32_t S;      /* Hessian slots per node */
} ocp_sizes_t;

typedef struct ocp_problem ocp_problem;

/* Transcription options (the *_ex entry points; NULL means the defaults). */
#define OCP_SCHEME_TRAPEZOIDAL 0   /* default: the trapezoidal scheme above */
#define OCP_SCHEME_EULER 1         /* forward Euler (paper Sec. 3), see below */
#define OCP_BOUNDARY_NONE 0        /* default: defect rows only */
#define OCP_BOUNDARY_INITIAL 1     /* n rows X_i0 after the defects */
#define OCP_BOUNDARY_INITIAL_FINAL 2  /* n rows X_i0, then n rows X_iN */

/* Forward Euler (paper Sec. 3): controls on the N nodes 0..N-1 (vu(l,k) =
 * n (N+1) + l N + k, nvar = n (N+1) + m N); defects c_ik = X_{i,k+1} - X_ik
 * - h F_i(k); cost sum_{k<N} h (sum q X_k^2 + sum r U_k^2).  Jacobian rows
 * have T = n + 1 + m slots in ascending column order: X_0..X_i at k, X_i at
 * k+1, X_{i+1}..X_{n-1} at k, then U_0..U_{m-1} at k.  Hessian: state and
 * pair slots as above (node N carries zeros), control slots
 * (n+npair)(N+1) + l N + k.
 * Boundary rows (either scheme), after the n N defect rows: their value is
 * the state itself (X_i0, then X_iN), as in the paper's generated code for
 * x(0) == x0 (Sec. 5), whose target enters the solver as lcon = ucon.  Each
 * adds one Jacobian entry (1.0) after the defect entries and no Hessian
 * entry. */
typedef struct ocp_options {
    int32_t scheme;    /* OCP_SCHEME_* */
    int32_t boundary;  /* OCP_BOUNDARY_* */
} ocp_options;

/* Sizes of the transcribed NLP (paper Sec. 3, trapezoidal scheme of Sec. 5).
 * Host only; no HIP call.  Errors: OCP_ERR_ARG, OCP_ERR_OVERFLOW. */
int ocp_sizes(int64_t N, int32_t n, int32_t m, ocp_sizes_t *out);

/* Sparsity patterns (the fixed structure the derivative evaluations fill;
 * paper Sec. 4 and 6: sparsity-preserving derivatives, one-time host
 * analysis).  Host buffers, caller-owned: jrow, jcol hold nnzj int32 each;
 * hrow, hcol hold nnzh int32 each.  Either pair may be NULL to skip it.
 * Entries are written in COO order e as documented above.  Host only.
 * Errors: OCP_ERR_ARG, OCP_ERR_OVERFLOW. */
int ocp_build_pattern(int64_t N, int32_t n, int32_t m, int32_t *jrow, int32_t *jcol,
                      int32_t *hrow, int32_t *hcol);

/* Lower-triangular CSR structure of the KKT matrix and the slot maps of the
 * Jacobian and Hessian COO entries into it (paper Sec. 6: the one-time host
 * symbolic step before device-side assembly).  Host buffers, caller-owned:
 * rowptr dim+1, colind nnzk, perm_j nnzj, perm_h nnzh int32.  Any of them may
 * be NULL to skip it.  Closed form; uses several host threads.
 * Errors: OCP_ERR_ARG, OCP_ERR_OVERFLOW. */
int ocp_build_kkt(int64_t N, int32_t n, int32_t m, int32_t *rowptr, int32_t *colind,
                  int32_t *perm_j, int32_t *perm_h);

/* ocp_sizes with transcription options (NULL = defaults).  Errors: as
 * ocp_sizes, plus OCP_ERR_ARG for an unknown scheme or boundary value. */
int ocp_sizes_ex(int64_t N, int32_t n, int32_t m, const ocp_options *opt, ocp_sizes_t *out);

/* ocp_build_pattern with transcription options (NULL = defaults). */
int ocp_build_pattern_ex(int64_t N, int32_t n, int32_t m, const ocp_options *opt, int32_t *jrow,
                         int32_t *jcol, int32_t *hrow, int32_t *hcol);

/* ocp_build_kkt with transcription options (NULL = defaults). */
int ocp_build_kkt_ex(int64_t N, int32_t n, int32_t m, const ocp_options *opt, int32_t *rowptr,
                     int32_t *colind, int32_t *perm_j, int32_t *perm_h);

/* Create a problem handle on the current HIP device.  A: n x n row-major,
 * B: n x m row-major, gamma: n, q: n, r: m (host pointers; B and r may be
 * NULL when m = 0).  Copies them to the device.
 * Errors: OCP_ERR_ARG, OCP_ERR_OVERFLOW (checked before any HIP call),
 * OCP_ERR_ALLOC, OCP_ERR_HIP. */
int ocp_create(int64_t N, int32_t n, int32_t m, const double *A, const double *B,
               const double *gamma, const double *q, const double *r, ocp_problem **out);

/* ocp_create with transcription options (NULL = defaults).  Every evaluation,
 * the assembly, the fused ocp_eval_kkt and the Lagrangian derivatives follow
 * the handle's options; the batched entry points accept only the defaults. */
int ocp_create_ex(int64_t N, int32_t n, int32_t m, const ocp_options *opt, const double *A,
                  const double *B, const double *gamma, const double *q, const double *r,
                  ocp_problem **out);

/* Release a handle and its device memory.  NULL-safe.  The caller must make
 * sure no work using the handle is still in flight. */
void ocp_destroy(ocp_problem *p);

/* Sizes of a handle's problem. */
int ocp_problem_sizes(const ocp_problem *p, ocp_sizes_t *out);

/* Objective f(z) (trapezoidal Lagrange cost, Sec. 5) into obj[0] (device).
 * z: nvar doubles (device).  Deterministic: fixed reduction order for a
 * given N.  Uses the handle's workspace. */
int ocp_eval_obj(const ocp_problem *p, const double *z, double *obj, hipStream_t stream);

/* Gradient of f (the trapezoidal cost of Sec. 5, differentiated per node:
 * 2 w_k q_j X_jk, 2 w_k r_l U_lk; Sec. 6 lists the objective gradient among
 * the derivative evaluations of each interior-point iteration) into g (nvar
 * doubles, device, the layout of z). */
int ocp_eval_grad(const ocp_problem *p, const double *z, double *g, hipStream_t stream);

/* Defects c(z) (Sec. 5, one generator per state component) into c (ncon
 * doubles, device). */
int ocp_eval_cons(const ocp_problem *p, const double *z, double *c, hipStream_t stream);

/* Jacobian values of the defects at the fixed pattern (Sec. 4: derivatives
 * that preserve the sparsity of the transcription; Sec. 6: the Jacobian an
 * interior-point iteration evaluates on the device) into jvals (nnzj doubles,
 * device, COO order e = (i T + t) N + k).  Reads only the state block of z. */
int ocp_eval_jac(const ocp_problem *p, const double *z, double *jvals, hipStream_t stream);

/* Hessian-of-Lagrangian values of L = sigma f + y^T c (Sec. 4 and Sec. 6:
 * second derivatives on the sparse pattern, block-diagonal per node because
 * every generator of Sec. 5 couples one interval) at the fixed lower pattern
 * into hvals (nnzh doubles, device, COO order e = s (N+1) + k).  y: ncon
 * doubles (device). */
int ocp_eval_hess(const ocp_problem *p, const double *z, const double *y, double sigma,
                  double *hvals, hipStream_t stream);

/* KKT assembly (Sec. 6: the KKT system is assembled in device buffers):
 *   kkt[perm_h[e]] = hvals[e], kkt[perm_j[e]] = jvals[e],
 *   every constraint-row diagonal = reg[d] (0 when reg is NULL), and every
 *   variable-row diagonal = hvals[e] + reg[d] in one IEEE add.
 * perm_j (nnzj), perm_h (nnzh), rowptr (dim+1), jvals, hvals, reg (dim,
 * nullable) and kkt (nnzk) are device arrays.  perm_j / perm_h must be
 * injective into [0, nnzk) and together with the constraint diagonals cover
 * every slot (as produced by ocp_build_kkt); rowptr locates the diagonal of
 * row d at rowptr[d+1] - 1.  Fully overwrites kkt.  No atomics. */
int ocp_assemble_kkt(const ocp_problem *p, const int32_t *perm_j, const int32_t *perm_h,
                     const int32_t *rowptr, const double *jvals, const double *hvals,
                     const double *reg, double *kkt, hipStream_t stream);

/* Fused evaluation into the KKT matrix: the values ocp_eval_jac,
 * ocp_eval_hess(z, y, sigma) and ocp_assemble_kkt (with the slot maps of
 * ocp_build_kkt and the same reg) would produce, written straight into kkt
 * (nnzk doubles, device, the layout of ocp_build_kkt), without the COO value
 * arrays.  This is what an interior-point iteration factorizes (Sec. 6); the
 * matrix is written once.  Same expressions as the separate calls.  Supports
 * the synthetic family under either scheme and any boundary option, and the
 * quadrotor model (the layout of ocp_quad_kkt). */
int ocp_eval_kkt(const ocp_problem *p, const double *z, const double *y, double sigma, const double *reg,
                 double *kkt, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Symmetric reordering of the KKT matrix (Sec. 6: the one-time host analysis
 * reorders the matrix for the sparse LDL^T factorization).  Folding the
 * ordering into the slot maps lets the device assemble P K P^T directly.
 * An ordering is given as order[new] = old, a permutation of [0, dim).
 * ------------------------------------------------------------------------- */

/* A fill-reducing ordering in closed form for the problem of (N, n, m, opt):
 * unknowns and rows grouped by grid node -- node k's block holds its states,
 * its controls (when it has any), the boundary rows fixed at it, then the
 * defect rows of interval k.  The reordered KKT matrix is banded with a
 * bandwidth independent of N, so the LDL^T fill grows linearly in N.
 * order: dim int32 (host, caller-owned).  Host only.
 * Errors: as ocp_sizes_ex, OCP_ERR_ARG for a NULL order. */
int ocp_stage_order(int64_t N, int32_t n, int32_t m, const ocp_options *opt, int32_t *order);

/* The same ordering for the quadrotor NLP (ocp_quad_sizes). */
int ocp_quad_stage_order(int64_t N, int32_t boundary, int32_t *order);

/* Lower CSR of P K P^T from the lower CSR (rowptr, colind) of K and an
 * ordering, with the slot maps carried over: perm_j2[e] and perm_h2[e] are
 * the new slots of the entries perm_j[e], perm_h[e] point at, and diag2[d]
 * the new slot of old row d's diagonal.  An entry (r, c) of K moves to
 * (pos r, pos c), mirrored into the lower triangle, where pos inverts order.
 * All host arrays, caller-owned: rowptr2 dim+1, colind2 nnzk, perm_j2 nnzj,
 * perm_h2 nnzh, diag2 dim (perm_j/perm_j2, perm_h/perm_h2 and diag2 may be
 * NULL to skip them).  Generic in the structure: any lower CSR with every
 * diagonal last in its row.  Host only, several threads.
 * Errors: OCP_ERR_ARG (not a permutation, malformed CSR, a slot map outside
 * [0, nnzk)), OCP_ERR_ALLOC. */
int ocp_kkt_permute(int64_t dim, const int32_t *rowptr, const int32_t *colind, int64_t nnzj,
                    const int32_t *perm_j, int64_t nnzh, const int32_t *perm_h, const int32_t *order,
                    int32_t *rowptr2, int32_t *colind2, int32_t *perm_j2, int32_t *perm_h2,
                    int32_t *diag2);

/* KKT assembly through slot maps alone, for any ordering:
 *   kkt[perm_h[e]] = hvals[e] (+ reg[d] when entry e is row d's diagonal),
 *   kkt[perm_j[e]] = jvals[e], and kkt[diag[d]] = reg[d] (0 when reg is
 *   NULL) for every constraint row d.
 * perm_j (nnzj), perm_h (nnzh), diag (dim: the slot of every row's
 * diagonal, as from ocp_kkt_permute), jvals, hvals, reg (dim, nullable,
 * indexed by the original rows) and kkt (nnzk) are device arrays; the slot
 * maps must be injective and together cover [0, nnzk).  plan is the output
 * of ocp_mapped_plan for these maps; it saves a pass over the maps on every
 * call.  With plan = NULL the handle keeps a plan of its own for the maps of
 * its last unplanned call (keyed by the three addresses): the first such call
 * allocates it on the device (so it cannot be captured in a graph; later
 * ones can) and fills it on `stream`, later calls with the same addresses
 * reuse it.  Calls that build it must not overlap other mapped assemblies on
 * the handle.  A plan made from other maps (a stale cached plan included) is
 * detected tile by tile (the staged slots must cover the tile's range
 * exactly) and those tiles store their values one by one: always the right
 * values, never an access outside the arrays.  Works for every handle (both
 * models and schemes).  Fastest for node-grouped orderings such as
 * ocp_stage_order, whose rows of a run of nodes form one contiguous range of
 * the CSR.  Fully overwrites kkt.  No atomics in global memory. */
int ocp_assemble_kkt_mapped(const ocp_problem *p, const int32_t *perm_j, const int32_t *perm_h,
                            const int32_t *diag, const int32_t *plan, const double *jvals,
                            const double *hvals, const double *reg, double *kkt, hipStream_t stream);

/* Number of int32 entries of a plan for ocp_assemble_kkt_mapped on this
 * handle (two per tile of grid nodes).  Host only. */
int ocp_mapped_plan_size(const ocp_problem *p, int64_t *entries);

/* Record, for slot maps (perm_j, perm_h, diag as for
 * ocp_assemble_kkt_mapped), the CSR range each node tile fills: plan
 * (device, ocp_mapped_plan_size entries) receives per tile the first slot
 * (or -1 when the tile's slots are not one contiguous range) and the
 * number of slots.  One launch; the maps are fixed across an
 * interior-point solve, so this runs once. */
int ocp_mapped_plan(const ocp_problem *p, const int32_t *perm_j, const int32_t *perm_h,
                    const int32_t *diag, int32_t *plan, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Lagrangian derivatives for differentiable programming (the paper names
 * tighter integration with differentiable programming workflows as future
 * work, Sec. 8).  L(z, y) = sigma f(z) + y^T c(z); the dynamics coefficients
 * (A, B, gamma) are parameters of c.  Either scheme and any boundary option
 * of the handle: y has ncon doubles (defect rows, then boundary rows), and z,
 * v and the gradients use the handle's layout (controls on NU nodes).  The
 * boundary rows are linear in z and do not involve the coefficients.  All
 * arrays are device pointers; every sum over nodes uses a fixed reduction
 * order (bitwise reproducible).  A quadrotor handle is accepted by
 * ocp_eval_lagrangian, ocp_eval_lag_grad, ocp_eval_hvp and ocp_eval_jvp (its
 * own layouts); the model has no coefficient arrays, so ocp_set_coefficients,
 * ocp_eval_coef_grad and ocp_eval_coef_mixed reject it (OCP_ERR_ARG).
 * ------------------------------------------------------------------------- */

/* Replace the handle's A (n x n), B (n x m; NULL when m = 0) and gamma (n)
 * with device arrays: one kernel on `stream` copies them and rebuilds the
 * handle's column-major copies of A and B (stream-ordered, asynchronous).
 * Evaluations queued on other streams must be ordered by the caller.
 * Errors: OCP_ERR_ARG, OCP_ERR_HIP. */
int ocp_set_coefficients(ocp_problem *p, const double *A, const double *B, const double *gamma,
                         hipStream_t stream);

/* L(z, y) into L[0] (device).  Uses the handle's reduction workspace, like
 * ocp_eval_obj (concurrent calls on one handle race). */
int ocp_eval_lagrangian(const ocp_problem *p, const double *z, const double *y, double sigma,
                        double *L, hipStream_t stream);

/* grad_z L = sigma grad f + J^T y into g (nvar doubles). */
int ocp_eval_lag_grad(const ocp_problem *p, const double *z, const double *y, double sigma,
                      double *g, hipStream_t stream);

/* Hessian-vector product (Hessian of L in z) v into out (nvar doubles); v has
 * nvar doubles in the layout of z. */
int ocp_eval_hvp(const ocp_problem *p, const double *z, const double *y, double sigma,
                 const double *v, double *out, hipStream_t stream);

/* Jacobian-vector product J v into out (ncon doubles); v has nvar doubles. */
int ocp_eval_jvp(const ocp_problem *p, const double *z, const double *v, double *out,
                 hipStream_t stream);

/* Gradient of L with respect to the dynamics coefficients: gA (n x n
 * row-major), gB (n x m; may be NULL when m = 0), ggamma (n), each a sum over
 * all nodes.  Uses the handle's coefficient-gradient workspace (concurrent
 * calls on one handle race). */
int ocp_eval_coef_grad(const ocp_problem *p, const double *z, const double *y, double *gA,
                       double *gB, double *ggamma, hipStream_t stream);

/* The derivative of the coefficient gradient along a direction v of z (nvar
 * doubles, the layout of z): the mixed second derivatives of L contracted
 * with v, d/dtheta (v^T grad_z L) for theta = (A, B, gamma), into gA (n x n
 * row-major), gB (n x m; may be NULL when m = 0) and ggamma (n).  With
 * C = cos X * v_X and Q_i = v_X,i X_p(i) + X_i v_X,p(i) (p(i) = (i+1) mod n)
 * these are the sums of ocp_eval_coef_grad with sin X, U and X_i X_p(i)
 * replaced by C, v_U and Q -- what a Hessian-vector product through the
 * Lagrangian gradient returns for the coefficients (differentiable
 * programming, named as future work in Sec. 8; the defects of Sec. 3).
 * Same workspace and reduction order rules as ocp_eval_coef_grad.
 * Errors: OCP_ERR_ARG (null array, quadrotor handle), OCP_ERR_HIP. */
int ocp_eval_coef_mixed(const ocp_problem *p, const double *z, const double *y, const double *v, double *gA,
                        double *gB, double *ggamma, hipStream_t stream);

/* The adjoint of the coefficient gradient: for cotangents tA (n x n
 * row-major), tB (n x m; may be NULL when m = 0) and tgamma (n) of
 * (dL/dA, dL/dB, dL/dgamma), the gradients of
 *   t . dL/dtheta = sum tA_ij dL/dA_ij + sum tB_il dL/dB_il + sum tgamma_i dL/dgamma_i
 * in z, into gz (nvar doubles, the layout of z), and in y, into gy (ncon
 * doubles, the layout of c) -- what the backward of ocp_eval_coef_grad needs.
 * The defects are linear in theta = (A, B, gamma), so this is the
 * coefficient part of J^T y and of c with theta replaced by t: gy holds the
 * defects' theta part under t (zero on the boundary rows), and gz the part of
 * grad_z L (sigma = 0) that the coefficients contribute (differentiable
 * programming, named as future work in Sec. 8; the defects of Sec. 3, either
 * scheme, any boundary option).  gz or gy may be NULL to skip that output,
 * not both.  The call reads t from the caller's arrays and leaves the
 * handle's coefficients and workspaces untouched; it may run concurrently
 * with any other call on the handle.  Errors: OCP_ERR_ARG (null array, no
 * output, quadrotor handle), OCP_ERR_HIP. */
int ocp_eval_coef_adjoint(const ocp_problem *p, const double *z, const double *y, const double *tA,
                          const double *tB, const double *tgamma, double *gz, double *gy, hipStream_t stream);

/* One backward pass of L(z, y) = sigma f + y^T c, what a reverse-mode
 * wrapper needs from one call (differentiable programming, named as future
 * work in Sec. 8): with gL the incoming gradient (one device double),
 * gz = gL grad_z L (nvar doubles), gy = gL c(z) (ncon doubles, the gradient
 * in y) and gA, gB, ggamma = gL dL/d(A, B, gamma) (the layouts of
 * ocp_eval_coef_grad).  The same kernels as ocp_eval_lag_grad,
 * ocp_eval_cons and ocp_eval_coef_grad, then one kernel that multiplies
 * every output by gL, so each value is bit for bit that call's value times
 * gL.  Any output may be NULL to skip it, not all; gA, gB and ggamma go
 * together (gB NULL when m = 0), use the coefficient-gradient workspace as
 * ocp_eval_coef_grad does, and are rejected on a quadrotor handle.
 * Errors: OCP_ERR_ARG (null input, no output, incomplete coefficient
 * outputs, quadrotor handle with coefficient outputs, non-finite sigma),
 * OCP_ERR_HIP. */
int ocp_eval_lagrangian_backward(const ocp_problem *p, const double *z, const double *y, double sigma,
                                 const double *gL, double *gz, double *gy, double *gA, double *gB,
                                 double *ggamma, hipStream_t stream);

/* Allocation-free ocp_eval_coef_grad, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same kernels, same arguments and bitwise the same
 * results as ocp_eval_coef_grad, but the per-workgroup partial sums live in a
 * fixed device array of the library (OCP_NOALLOC_SCRATCH doubles = 4 MiB;
 * each device holds its own copy until the process ends) instead of the
 * handle's workspace.  The call allocates nothing and calls no allocating
 * routine.  Limit: n (n+m+1) G <= OCP_NOALLOC_SCRATCH, G = min(1024,
 * ceil((N+1) / 64)) workgroups (every N at n <= 16, m <= 8); a larger
 * problem returns OCP_ERR_ARG before any HIP call.  The current device must
 * be the handle's (OCP_ERR_ARG otherwise).  Every call on one device shares
 * that device's array, which keeps the last call's contents: calls that
 * overlap on one device race (serialize them, e.g. on one stream).  Each call
 * writes every partial it reads before reading it, so nothing needs clearing.
 * The array's device address is looked up when a handle is created on the
 * device (OCP_ERR_HIP if that lookup failed). */
#define OCP_NOALLOC_SCRATCH 524288
int ocp_eval_coef_grad_noalloc(const ocp_problem *p, const double *z, const double *y, double *gA,
                               double *gB, double *ggamma, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * The quadrotor model of the paper's benchmark set (Appendix A), transcribed
 * with the trapezoidal scheme (Sec. 5) on t in [0, 1], h = 1/N.
 *
 * States x1..x9 (node-local v = 0..8: positions x1, x3, x5, velocities x2,
 * x4, x6, Euler angles x7, x8, x9) and controls u1..u4 (v = 9..12) all live
 * on the N+1 nodes: z[v (N+1) + k], nvar = 13 (N+1).  Dynamics:
 *   x1' = x2, x3' = x4, x5' = x6,
 *   x2' = u1 (c7 s8 c9 + s7 s9), x4' = u1 (c7 s8 s9 - s7 c9), x6' = u1 c7 c8 - g,
 *   x7' = (u2 c7 + u3 s7) / c8, x8' = -u2 s7 + u3 c7, x9' = (u2 c7 + u3 s7) t8 + u4
 * (cj, sj, tj: cos, sin, tan of xj).  Cost: the trapezoidal sum of one half
 * of (x1 - sin 2 pi t)^2 + (x3 - 2 sin 4 pi t)^2 + (x5 - 2t)^2 + x7^2 + x8^2
 * + x9^2 + r |u|^2 at t_k = k h.  Defect rows i N + k as above; with
 * `boundary` = OCP_BOUNDARY_INITIAL the 9 rows X_i0 follow (the paper fixes
 * x(0) = 0; the target enters the solver as lcon = ucon), with
 * OCP_BOUNDARY_INITIAL_FINAL also the 9 rows X_iN.
 *
 * Patterns (the structural support of the model, not a dense block):
 *   Jacobian: row i holds two entries (node k, node k+1) per variable of its
 *   support -- its own state and the variables its right-hand side depends
 *   on -- in ascending column order; 68 entries per interval, slot-major:
 *   entry t of the interval's 68 (rows 0..8 in order) sits at t N + k.
 *   Supports: x1:{x1,x2}  x2:{x2,x7,x8,x9,u1}  x3:{x3,x4}  x4:{x4,x7,x8,x9,u1}
 *   x5:{x5,x6}  x6:{x6,x7,x8,u1}  x7,x8:{x7,x8,u2,u3}  x9:{x7,x8,x9,u2,u3,u4}.
 *   Boundary entries (1.0) follow at 68 N + b.
 *   Hessian: 23 lower entries per node, sorted by (row, col) in node-local
 *   numbering, at s (N+1) + k: the 13 diagonals (those of x2, x4, x6 are
 *   zero, kept so every KKT diagonal is a Hessian entry), (x8,x7), (x9,x7),
 *   (x9,x8), (u1,x7), (u1,x8), (u1,x9), (u2,x7), (u2,x8), (u3,x7), (u3,x8).
 *   ocp_sizes_t reports T = 68 (entries per interval), S = 23, npair = 0.
 *
 * A handle from ocp_quad_create works with ocp_problem_sizes, ocp_eval_obj,
 * ocp_eval_grad, ocp_eval_cons, ocp_eval_jac, ocp_eval_hess,
 * ocp_assemble_kkt, ocp_eval_kkt, ocp_eval_lagrangian, ocp_eval_lag_grad,
 * ocp_eval_hvp, ocp_eval_jvp and ocp_destroy, with the arrays and layouts
 * above.  ocp_set_coefficients and ocp_eval_coef_grad reject it
 * (OCP_ERR_ARG).
 * ------------------------------------------------------------------------- */

/* Sizes of the quadrotor NLP.  Host only.  Errors: OCP_ERR_ARG (N < 1,
 * unknown boundary), OCP_ERR_OVERFLOW. */
int ocp_quad_sizes(int64_t N, int32_t boundary, ocp_sizes_t *out);

/* Jacobian and Hessian COO patterns of the quadrotor NLP into caller-owned
 * host arrays (nnzj, nnzh int32 each; any may be NULL to skip it). */
int ocp_quad_pattern(int64_t N, int32_t boundary, int32_t *jrow, int32_t *jcol, int32_t *hrow,
                     int32_t *hcol);

/* Lower CSR of the quadrotor KKT matrix and the slot maps (Sec. 6 one-time
 * host step), into caller-owned host arrays: rowptr dim+1, colind nnzk,
 * perm_j nnzj, perm_h nnzh (any may be NULL). */
int ocp_quad_kkt(int64_t N, int32_t boundary, int32_t *rowptr, int32_t *colind, int32_t *perm_j,
                 int32_t *perm_h);

/* Create a quadrotor handle on the current HIP device with gravity g and
 * control weight r (the paper uses g = 9.8, r = 0.1).  Allocates only the
 * objective's reduction workspace.  Errors: OCP_ERR_ARG (also for non-finite
 * g or r), OCP_ERR_OVERFLOW, OCP_ERR_ALLOC, OCP_ERR_HIP. */
int ocp_quad_create(int64_t N, int32_t boundary, double g, double r, ocp_problem **out);

/* ---------------------------------------------------------------------------
 * Batches: many independent instances with their own N_b and coefficients
 * (shared n, m), evaluated together.  The paper motivates data parallelism
 * across grid nodes (Sec. 3) and real-time use; a batch extends the same
 * node-parallel evaluation across instances.
 *
 * Packed layout: instance b's z, y/c, gradient, Jacobian, Hessian and KKT
 * values and its regularization are the single-instance arrays of that
 * instance (same layouts as above, with its own N_b, under the batch's
 * scheme and boundary option), stored back to back in instance order;
 * objectives are one double per instance.  ocp_batch_offsets and
 * ocp_batch_offsets_ex give the int64 start of each instance in each packed
 * array.  An interior-point step over the batch (Sec. 6: derivative
 * evaluations and the KKT assembly, every iteration, on the device) is one
 * ocp_batch_eval_io call.
 * ------------------------------------------------------------------------- */

typedef struct ocp_batch ocp_batch;
typedef struct ocp_graph ocp_graph;

/* What a batched evaluation computes (bit mask). */
#define OCP_EVAL_JAC 1    /* Jacobian values (COO order of each instance) */
#define OCP_EVAL_HESS 2   /* Hessian-of-Lagrangian values (COO order) */
#define OCP_EVAL_OBJ 4    /* objective of each instance */
#define OCP_EVAL_GRAD 8   /* objective gradient */
#define OCP_EVAL_CONS 16  /* defects and boundary rows */
#define OCP_EVAL_KKT 32   /* fused KKT values (ocp_eval_kkt of each instance) */
#define OCP_EVAL_ALL 63

/* How a batched evaluation runs. */
#define OCP_BATCH_PERSISTENT 0    /* one persistent launch over a static tile list */
#define OCP_BATCH_PER_INSTANCE 1  /* one single-instance launch per instance and evaluation */

/* Tile shape of the persistent launch. */
typedef struct ocp_batch_config {
    int32_t block;        /* threads per workgroup: 128 or 256 */
    int32_t pair;         /* 1: Jacobian lanes take two intervals (16-byte stores) where the
                             instance allows it (N_b even, output 16-byte aligned); 0: one */
    int32_t wgs_per_cu;   /* persistent workgroups per compute unit, 1..32; 0: one
                             workgroup per tile (the loop over tiles runs once) */
    int32_t order;        /* tile order within an instance: 0 node range major (all columns
                             of a node range together), 1 column major (a column's node
                             ranges together) */
} ocp_batch_config;

/* Create a batch of `count` instances on the current HIP device.  Ns: count
 * interval counts (host int64, each >= 1).  A: count x n x n, B: count x n x m,
 * gamma: count x n, q: count x n, r: count x m, all host, instance-major and
 * row-major within an instance (B and r may be NULL when m = 0).  Copies the
 * coefficients to the device, builds the offset table and the tile list of
 * the default configuration {256, 1, 8}.
 * Errors: OCP_ERR_ARG (count < 1, bad N_b, n, m or pointers), OCP_ERR_OVERFLOW
 * (an instance's sizes do not fit int32), OCP_ERR_ALLOC, OCP_ERR_HIP. */
int ocp_batch_create(int32_t count, const int64_t *Ns, int32_t n, int32_t m, const double *A,
                     const double *B, const double *gamma, const double *q, const double *r,
                     ocp_batch **out);

/* ocp_batch_create with options: every instance uses opt's scheme and
 * boundary option (NULL: the defaults), as ocp_create_ex does for one
 * instance. */
int ocp_batch_create_ex(int32_t count, const int64_t *Ns, int32_t n, int32_t m, const ocp_options *opt,
                        const double *A, const double *B, const double *gamma, const double *q,
                        const double *r, ocp_batch **out);

/* Release a batch.  NULL-safe.  No work using it may be in flight. */
void ocp_batch_destroy(ocp_batch *b);

/* Packed offsets (host int64 arrays of count+1 entries each, any may be NULL):
 * z_off (nvar_b), c_off (ncon_b; also y), jac_off (nnzj_b), hess_off (nnzh_b).
 * Entry `count` holds the total length of the packed array. */
int ocp_batch_offsets(const ocp_batch *b, int64_t *z_off, int64_t *c_off, int64_t *jac_off,
                      int64_t *hess_off);

/* Packed offsets of the KKT values (kkt_off, nnzk_b per instance) and of the
 * regularization (dim_off, dim_b), count+1 host int64 entries each (either
 * may be NULL); entry `count` is the total. */
int ocp_batch_offsets_ex(const ocp_batch *b, int64_t *kkt_off, int64_t *dim_off);

/* Current tile shape, and setting a new one.  Setting rebuilds the tile list
 * and synchronizes the device first (no evaluation with the batch may be in
 * flight on another thread).  Graphs captured earlier keep their own copy of
 * the tile list and are unaffected.  Errors: OCP_ERR_ARG for a shape outside
 * the documented ranges. */
int ocp_batch_get_config(const ocp_batch *b, ocp_batch_config *cfg);
int ocp_batch_set_config(ocp_batch *b, const ocp_batch_config *cfg);

/* Evaluate Jacobian and/or Hessian values (`what`) of every instance into the
 * packed device arrays jac / hess (NULL when not requested), from packed z and
 * y (y may be NULL without OCP_EVAL_HESS).  `mode` selects the single
 * persistent launch or the per-instance launches; both give bitwise the same
 * values, independent of the tile shape.  Asynchronous on `stream`. */
int ocp_batch_eval(const ocp_batch *b, int32_t what, int32_t mode, const double *z,
                   const double *y, double sigma, double *jac, double *hess, hipStream_t stream);

/* Arrays of one batched evaluation (all device pointers into packed arrays;
 * an output not requested by `what` may be NULL and is not touched). */
typedef struct ocp_batch_io {
    const double *z;    /* packed z (always read) */
    const double *y;    /* packed multipliers (OCP_EVAL_HESS, OCP_EVAL_KKT) */
    const double *reg;  /* packed KKT regularization, dim_b per instance (OCP_EVAL_KKT; NULL: none) */
    double sigma;       /* objective weight of the Lagrangian (OCP_EVAL_HESS, OCP_EVAL_KKT) */
    double *obj;        /* count doubles: instance b's objective at obj[b] (OCP_EVAL_OBJ) */
    double *grad;       /* packed, nvar_b per instance, offsets z_off (OCP_EVAL_GRAD) */
    double *cons;       /* packed, ncon_b, offsets c_off (OCP_EVAL_CONS) */
    double *jac;        /* packed, nnzj_b, offsets jac_off (OCP_EVAL_JAC) */
    double *hess;       /* packed, nnzh_b, offsets hess_off (OCP_EVAL_HESS) */
    double *kkt;        /* packed, nnzk_b, offsets kkt_off: each instance's lower CSR KKT values in
                           the layout of ocp_build_kkt_ex, as ocp_eval_kkt writes them (OCP_EVAL_KKT) */
} ocp_batch_io;

/* Evaluate the requested parts (`what`, any non-empty mask of OCP_EVAL_*) of
 * every instance: in persistent mode one launch walks the tile list of that
 * mask; in per-instance mode the single-instance kernels run instance after
 * instance.  Both give bitwise the same values, independent of the tile
 * shape; the objective is bitwise the per-instance (ocp_eval_obj) value for
 * N_b < 2^20 (beyond that the single-instance reduction takes several nodes
 * per lane and the two agree to rounding).  The values are those of the
 * single-instance entry points (Sec. 5 formulas; the KKT values those of
 * ocp_eval_kkt with the instance's part of reg).  The first evaluation with a
 * mask builds that mask's tile list (a device allocation and a copy; see
 * ocp_batch_prepare).  Objective evaluations on one batch share its per-
 * instance partial sums and counters: evaluations with OCP_EVAL_OBJ must not
 * overlap (serialize them, e.g. on one stream).  Asynchronous on `stream`.
 * Errors: OCP_ERR_ARG (NULL batch or io, empty or unknown mask, a requested
 * array NULL, sigma not finite when used), OCP_ERR_ALLOC, OCP_ERR_HIP. */
int ocp_batch_eval_io(const ocp_batch *b, int32_t what, int32_t mode, const ocp_batch_io *io,
                      hipStream_t stream);

/* Build and keep the persistent tile list of mask `what` for the current
 * tile shape now (a device allocation and a host-to-device copy), so that a
 * later evaluation or capture with that mask allocates nothing.  Lists are
 * rebuilt when the shape changes.  Not thread-safe with a concurrent
 * ocp_batch_set_config on the same batch. */
int ocp_batch_prepare(const ocp_batch *b, int32_t what);

/* Capture one ocp_batch_eval (same arguments, pointers bound at capture) into
 * a HIP graph on a private stream and instantiate it.  The graph owns a copy of
 * the tile list, so later configuration changes do not affect it.  It still
 * reads the batch's coefficients and offset table and the arrays bound at
 * capture: the batch and those arrays must outlive every launch of the graph.
 * Errors: as ocp_batch_eval, plus OCP_ERR_HIP when capture or instantiation
 * fails. */
int ocp_batch_graph_create(const ocp_batch *b, int32_t what, int32_t mode, const double *z,
                           const double *y, double sigma, double *jac, double *hess,
                           ocp_graph **out);

/* Capture one ocp_batch_eval_io (same arguments; the arrays of io are bound
 * at capture) into a HIP graph, as ocp_batch_graph_create does. */
int ocp_batch_graph_create_io(const ocp_batch *b, int32_t what, int32_t mode, const ocp_batch_io *io,
                              ocp_graph **out);

/* Replay a captured evaluation on `stream` (asynchronous).  The arrays bound
 * at capture must still be alive. */
int ocp_graph_launch(const ocp_graph *g, hipStream_t stream);

/* Release a graph and its tile list.  NULL-safe; no replay may be in flight. */
void ocp_graph_destroy(ocp_graph *g);

/* Autotuner: time every tile shape in {128, 256} x {pair 0, 1} x
 * {1, 2, 4, 8, 16, 32, 0 = one per tile} workgroups per CU x {order 0, 1}
 * (56 shapes, in that nesting order, order fastest) with `reps` persistent
 * evaluations each (HIP events on `stream`, after one untimed run), keep the
 * fastest as the batch's config and return it with its mean time in
 * milliseconds.  `all_ms` (nullable, OCP_AUTOTUNE_SHAPES floats) receives
 * every shape's mean time.  Synchronizes the device.  Outputs are overwritten
 * by the trial runs. */
#define OCP_AUTOTUNE_SHAPES 56
int ocp_batch_autotune(ocp_batch *b, int32_t what, const double *z, const double *y, double sigma,
                       double *jac, double *hess, int32_t reps, hipStream_t stream,
                       ocp_batch_config *best, float *best_ms, float *all_ms);

/* The autotuner over a whole-step mask: as ocp_batch_autotune, timing
 * ocp_batch_eval_io(b, what, OCP_BATCH_PERSISTENT, io). */
int ocp_batch_autotune_io(ocp_batch *b, int32_t what, const ocp_batch_io *io, int32_t reps,
                          hipStream_t stream, ocp_batch_config *best, float *best_ms, float *all_ms);

/* Message describing the last error on the calling thread ("" if none).
 * With the environment variable OCP_VERBOSE set (to anything but "" or "0")
 * when the library first records an error, every error is also printed to
 * stderr as "[ocp] error <code>: <message>". */
const char *ocp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* OCP_EVAL_H */
