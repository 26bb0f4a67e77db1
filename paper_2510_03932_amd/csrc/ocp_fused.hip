// Fused evaluation into the KKT matrix (ocp_eval_kkt): the Jacobian and the
// Hessian of the Lagrangian are evaluated straight into their slots of the
// lower CSR KKT matrix of ocp_build_kkt, with the regularization on the
// diagonal, skipping the COO value arrays.  An interior-point iteration that
// only needs the assembled matrix (paper Sec. 6) then moves the matrix once:
// the state rows, y and reg in, the KKT values out (about 7 GB at N = 1e6,
// n = 16, m = 8, against 23 GB for eval_jac + eval_hess + assemble_kkt).
//
// The values are computed with the same expressions, in the same order, as
// the COO kernels and the assembly.  The tile bodies (ocp_step_device.h) are
// shared with the batched evaluation.
//
// Defect rows: workgroup b owns intervals [b KT, b KT + KT), KT = 16, 32 or
// 64 so that one row block (KT rows of T+1 entries) holds 500 to 1000 values.
// It stages the states and their cosines at the KT+1 nodes, the rows'
// regularization and the scaled coefficients -hh A, -hh B, -hh gamma in LDS
// (a wavefront spans several slots of a row, so coefficient reads from global
// memory would be per-lane loads, each waited for); then, for each state
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
#include "ocp_step_device.h"

using namespace ocp;
using namespace ocp::dev;

namespace {

__global__ __launch_bounds__(kBlock) void kkt_defect_kernel(KP P, KKTLayout Lo, int LG, const double *__restrict__ z,
                                                            const double *__restrict__ reg,
                                                            double *__restrict__ kkt)
{
    extern __shared__ double lds[];
    kkt_defect_tile<kBlock>(P, Lo, z, reg, kkt, (int64_t)blockIdx.x << LG, LG, lds);
}

template <int NB>
__global__ __launch_bounds__(kBlock) void kkt_var_kernel(KP P, KKTLayout Lo, const double *__restrict__ z,
                                                         const double *__restrict__ y, double sigma,
                                                         const double *__restrict__ reg,
                                                         double *__restrict__ kkt)
{
    __shared__ double buf[3 * kBlock];  // one state block's rows of this workgroup (<= 3 entries each)
    kkt_var_tile<NB, kBlock>(P, Lo, z, y, sigma, reg, kkt, (int64_t)blockIdx.x * kBlock, buf);
}

// Boundary rows: their state entry (1) and their diagonal.
__global__ __launch_bounds__(kBlock) void kkt_bnd_kernel(KP P, KKTLayout Lo, const double *__restrict__ reg,
                                                         double *__restrict__ kkt)
{
    const int b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= P.nb) return;
    kkt_bnd_row(P, Lo, reg, kkt, b);
}

}  // namespace

namespace ocp {
namespace dev {

hipError_t launch_eval_kkt(const KP &P, const double *z, const double *y, double sigma, const double *reg,
                           double *kkt, hipStream_t stream)
{
    const KKTLayout Lo = kkt_layout(P.n);
    // defect-row tiles of KT = 2^LG intervals; LDS holds the tile's states,
    // their cosines, the rows' regularization, the scaled coefficients and the
    // output row block
    const int KT = kkt_defect_kt(P.n, P.m, P.T);
    const int LG = __builtin_ctz((unsigned)KT);
    const size_t lds = kkt_defect_lds(P.n, P.m, P.T, KT) * sizeof(double);
    hipLaunchKernelGGL(kkt_defect_kernel, dim3(blocks_for(P.N, KT)), dim3(kBlock), lds, stream, P, Lo, LG, z, reg,
                       kkt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 g(blocks_for(P.N1, kBlock));
    if (P.n <= 4) hipLaunchKernelGGL(kkt_var_kernel<4>, g, dim3(kBlock), 0, stream, P, Lo, z, y, sigma, reg, kkt);
    else if (P.n <= 8) hipLaunchKernelGGL(kkt_var_kernel<8>, g, dim3(kBlock), 0, stream, P, Lo, z, y, sigma, reg, kkt);
    else if (P.n <= 16) hipLaunchKernelGGL(kkt_var_kernel<16>, g, dim3(kBlock), 0, stream, P, Lo, z, y, sigma, reg, kkt);
    else hipLaunchKernelGGL(kkt_var_kernel<32>, g, dim3(kBlock), 0, stream, P, Lo, z, y, sigma, reg, kkt);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (P.nb > 0)
        hipLaunchKernelGGL(kkt_bnd_kernel, dim3(blocks_for(P.nb, kBlock)), dim3(kBlock), 0, stream, P, Lo, reg,
                           kkt);
    return hipGetLastError();
}

}  // namespace dev
}  // namespace ocp

extern "C" {

int ocp_eval_kkt(const ocp_problem *p, const double *z, const double *y, double sigma, const double *reg,
                 double *kkt, hipStream_t stream)
{
    clear_error();
    if (int rc = check_handle(p, "ocp_eval_kkt")) return rc;
    if (!z || !y || !kkt) return fail(OCP_ERR_ARG, "ocp_eval_kkt: null array");
    if (!std::isfinite(sigma)) return fail(OCP_ERR_ARG, "ocp_eval_kkt: sigma is not finite");
    if (p->model == quad::kModel) return quad::eval_kkt(p, z, y, sigma, reg, kkt, stream);
    const hipError_t e = launch_eval_kkt(p->kp, z, y, sigma, reg, kkt, stream);
    if (e != hipSuccess) return hip_fail("ocp_eval_kkt", e);
    return OCP_OK;
}

}  // extern "C"
