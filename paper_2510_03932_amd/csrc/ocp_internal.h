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
    int64_t N1;      // N + 1 nodes
    int64_t nvar, ncon, nnzj, nnzh, nnzk, dim;
};

// Validate (N, n, m) and compute every size.  Returns OCP_OK, OCP_ERR_ARG or
// OCP_ERR_OVERFLOW (with the message set).
int make_dims(int64_t N, int32_t n, int32_t m, Dims *d);

void to_public(const Dims &d, ocp_sizes_t *out);

}  // namespace ocp
