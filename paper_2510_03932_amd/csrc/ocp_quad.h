// Internal interface of the quadrotor model's evaluations (ocp_quad.hip) and
// its sizes (ocp_quad_host.cpp).  The public entry points dispatch here for a
// handle made by ocp_quad_create.
#pragma once

#include <hip/hip_runtime.h>

#include "ocp_internal.h"

struct ocp_problem;

namespace ocp {
namespace quad {

constexpr int kModel = 1;  // ocp_problem::model of a quadrotor handle

// Sizes of the quadrotor NLP with `bnd` boundary row groups (0, 1, 2).
// Returns OCP_OK, OCP_ERR_ARG or OCP_ERR_OVERFLOW with the message set.
int make_dims(int64_t N, int32_t bnd, Dims *d);

int eval_obj(const ocp_problem *p, const double *z, double *obj, hipStream_t stream);
int eval_grad(const ocp_problem *p, const double *z, double *g, hipStream_t stream);
int eval_cons(const ocp_problem *p, const double *z, double *c, hipStream_t stream);
int eval_jac(const ocp_problem *p, const double *z, double *jvals, hipStream_t stream);
int eval_hess(const ocp_problem *p, const double *z, const double *y, double sigma, double *hvals,
              hipStream_t stream);
// Fused evaluation of the Jacobian and Hessian values (+ reg) into the KKT
// values of ocp_quad_kkt's layout.
int eval_kkt(const ocp_problem *p, const double *z, const double *y, double sigma, const double *reg,
             double *kkt, hipStream_t stream);
// Lagrangian derivatives (no coefficient gradient: the model has no
// coefficient arrays).
int eval_lagrangian(const ocp_problem *p, const double *z, const double *y, double sigma, double *L,
                    hipStream_t stream);
int eval_lag_grad(const ocp_problem *p, const double *z, const double *y, double sigma, double *g,
                  hipStream_t stream);
int eval_hvp(const ocp_problem *p, const double *z, const double *y, double sigma, const double *v,
             double *out, hipStream_t stream);
int eval_jvp(const ocp_problem *p, const double *z, const double *v, double *out, hipStream_t stream);
int assemble_kkt(const ocp_problem *p, const int32_t *perm_j, const int32_t *perm_h,
                 const int32_t *rowptr, const double *jvals, const double *hvals, const double *reg,
                 double *kkt, hipStream_t stream);

}  // namespace quad
}  // namespace ocp
