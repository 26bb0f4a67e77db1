// The single-instance problem handle and host helpers shared by the
// translation units that implement its entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "ocp_device.h"
#include "ocp_internal.h"

// Most partial sums of the one-pass-per-workgroup reductions (objective,
// Lagrangian value), and workgroups per row of the coefficient-gradient sum.
constexpr int kObjBlocks = 4096;
constexpr int kCoefBlocks = 1024;

// Nodes per chunk of the coefficient-gradient sum, and its workgroups over
// N1 nodes: one per chunk, at most kCoefBlocks.
constexpr int kCoefChunk = 64;
inline int coef_blocks(int64_t N1)
{
    const int64_t chunks = (N1 + kCoefChunk - 1) / kCoefChunk;
    return (int)(chunks < kCoefBlocks ? chunks : kCoefBlocks);
}

// Device address of the allocation-free entry point's fixed scratch array on
// `device` (which must be the current device on the first call for it), looked
// up once per device and kept; null if the lookup fails.
double *noalloc_scratch(int device);

struct ocp_problem {
    ocp::Dims d;
    int device;
    double *coef;       // device: A | B | gamma | q | r | AT | BT (padded columns, kLd each)
    double *partials;   // device: kObjBlocks doubles (objective and Lagrangian sums)
    double *cpart;      // device: n (n+m+1) coef_blocks(N1) doubles (coefficient-gradient sums)
    ocp::dev::KP kp;
    int model = 0;        // 0: the synthetic dynamics family; ocp::quad::kModel: the quadrotor
    double quad_g = 0.0;  // quadrotor gravity and control weight
    double quad_r = 0.0;
    // plan of the slot maps of the last unplanned ocp_assemble_kkt_mapped
    // (device, allocated on first use), keyed by the maps' addresses
    mutable std::mutex mplan_mu;
    mutable int32_t *mplan = nullptr;
    mutable const void *mplan_key[3] = {nullptr, nullptr, nullptr};
};

static inline int hip_fail(const char *what, hipError_t e)
{
    return ocp::fail(OCP_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

static inline int check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(what, e);
    return OCP_OK;
}

static inline int check_handle(const ocp_problem *p, const char *what)
{
    if (!p) return ocp::fail(OCP_ERR_ARG, std::string(what) + ": problem handle is NULL");
    return OCP_OK;
}

static inline unsigned blocks_for(int64_t count, int per_block)
{
    return (unsigned)((count + per_block - 1) / per_block);
}
