// Internal declarations shared by the host index layer and the device layer of
// the evaluation library.  Not part of the public interface.
#pragma once

#include <cstdint>
#include <string>

#include "ocp_eval.h"

namespace ocp {

// Record a message for ocp_last_error() on this thread and return `code`.
int fail(int code, const std::string &msg);
void clear_error();

// Validated sizes of one problem; every field fits in int32 when ok.
struct Dims {
    int64_t N;
    int32_t n, m, npair, T, S;
    int32_t scheme;  // OCP_SCHEME_TRAPEZOIDAL or OCP_SCHEME_EULER
    int32_t bnd;     // OCP_BOUNDARY_*: number of boundary row groups (0, 1, 2)
    int64_t N1;      // N + 1 state nodes
    int64_t NU;      // control nodes: N + 1 (trapezoidal) or N (Euler)
    int64_t nvar, ncon, nnzj, nnzh, nnzk, dim;
    int64_t ndef;      // defect rows n N (the boundary rows follow them)
    int64_t nb;        // boundary rows bnd * n
    int64_t nnzj_def;  // Jacobian entries of the defect rows (the boundary entries follow)
};

// Validate (N, n, m, options) and compute every size.  Returns OCP_OK,
// OCP_ERR_ARG or OCP_ERR_OVERFLOW (with the message set).
int make_dims(int64_t N, int32_t n, int32_t m, Dims *d);
int make_dims_ex(int64_t N, int32_t n, int32_t m, int32_t scheme, int32_t bnd, Dims *d);

void to_public(const Dims &d, ocp_sizes_t *out);

}  // namespace ocp
