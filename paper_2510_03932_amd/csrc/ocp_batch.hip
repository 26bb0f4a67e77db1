// Batched evaluation: many independent instances (own N_b and coefficients,
// shared n and m) in one persistent launch, the per-instance launches it
// replaces, HIP-graph capture of either, and an autotuner for the tile shape.
//
// The persistent kernel walks a static tile list: workgroup w takes tiles
// w, w + G, w + 2G, ... (G = grid size), so every wave reaches the end of the
// list and exits, and the assignment is fixed (no atomics, no queue).  A tile
// is (instance, first node, kind): a Jacobian tile covers `block * npt`
// intervals of one column (state or control) of one instance, a Hessian tile
// covers `block` nodes.  Tiles are ordered instance-major, node-range next,
// column last, so the workgroups in flight share the state rows they read.
// The per-lane arithmetic is the single-instance path's (ocp_device.h): the
// values are bitwise those of per-instance evaluation, for any tile shape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ocp_device.h"
#include "ocp_internal.h"

using namespace ocp;
using namespace ocp::dev;

namespace {

// One instance's place in the packed arrays (device copy of the offset table).
struct InstDesc {
    int64_t z_off, c_off, jac_off, hess_off;
    int32_t N, pad;
    double h, hh;
};

// One unit of work of the persistent kernel.
struct TileDesc {
    int32_t b;     // instance
    int32_t k0;    // first interval (Jacobian) or node (Hessian)
    int32_t col;   // Jacobian column 0 .. n+m-1, or -1 for a Hessian tile
    int32_t npt;   // intervals per lane of a Jacobian tile (1 or 2)
};

// Coefficients of the whole batch (device), instance-major.
struct BP {
    int n, m, npair, T, S;
    const double *A, *B, *gam, *q, *r;
    const double *AT, *BT;  // padded columns: n kLd and m kLd doubles per instance
};

template <int NB, int BS>
__global__ __launch_bounds__(BS) void batch_kernel(BP bp, const InstDesc *__restrict__ inst,
                                                   const TileDesc *__restrict__ tiles, int ntiles,
                                                   int what, bool pair_ok,
                                                   const double *__restrict__ z,
                                                   const double *__restrict__ y, double sigma,
                                                   double *__restrict__ jac, double *__restrict__ hess)
{
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const TileDesc td = tiles[t];
        const bool is_jac = td.col >= 0;
        if (is_jac ? !(what & OCP_EVAL_JAC) : !(what & OCP_EVAL_HESS)) continue;
        const InstDesc id = inst[td.b];
        KP P;
        P.N = id.N;
        P.N1 = id.N + 1;
        P.n = bp.n;
        P.m = bp.m;
        P.npair = bp.npair;
        P.T = bp.T;
        P.S = bp.S;
        P.nnzk = 0;
        P.NU = id.N + 1;
        P.scheme = 0;
        P.nb = 0;
        P.h = id.h;
        P.hh = id.hh;
        P.A = bp.A + (int64_t)td.b * bp.n * bp.n;
        P.B = bp.B + (int64_t)td.b * bp.n * bp.m;
        P.gam = bp.gam + (int64_t)td.b * bp.n;
        P.q = bp.q + (int64_t)td.b * bp.n;
        P.r = bp.r + (int64_t)td.b * bp.m;
        P.AT = bp.AT + (int64_t)td.b * bp.n * kLd;
        P.BT = bp.BT + (int64_t)td.b * bp.m * kLd;
        const double *zb = z + id.z_off;
        if (is_jac) {
            if (td.npt == 2) {
                // the tile spans two intervals per lane; paired stores need a
                // 16-byte aligned output, else the lane stores them one by one
                const int64_t k = td.k0 + 2 * (int64_t)threadIdx.x;
                if (k < P.N) {
                    if (pair_ok) {
                        jac_column<2>(P, zb, jac + id.jac_off, k, td.col);
                    } else {
                        jac_column<1>(P, zb, jac + id.jac_off, k, td.col);
                        jac_column<1>(P, zb, jac + id.jac_off, k + 1, td.col);
                    }
                }
            } else {
                const int64_t k = td.k0 + (int64_t)threadIdx.x;
                if (k < P.N) jac_column<1>(P, zb, jac + id.jac_off, k, td.col);
            }
        } else {
            const int k = td.k0 + (int)threadIdx.x;
            if (k <= P.N) hess_node<NB>(P, zb, y + id.c_off, sigma, hess + id.hess_off, k);
        }
    }
}

}  // namespace

struct ocp_batch {
    int32_t count, n, m;
    Dims shape;                    // sizes of a one-interval instance (for T, S, npair)
    std::vector<int64_t> Ns;
    std::vector<int64_t> z_off, c_off, jac_off, hess_off;  // count + 1 each
    int device = 0;
    int cus = 0;
    double *coef = nullptr;        // device: A | B | gamma | q | r | AT | BT (instance-major blocks)
    InstDesc *inst = nullptr;      // device offset table
    TileDesc *tiles = nullptr;     // device tile list of the current config
    int ntiles = 0;
    ocp_batch_config cfg{256, 1, 0, 1};
    BP bp{};
};

struct ocp_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    TileDesc *tiles = nullptr;     // the graph's own tile list
};

static int hip_fail_b(const char *what, hipError_t e)
{
    return fail(OCP_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

static bool valid_config(const ocp_batch_config &c)
{
    return (c.block == 128 || c.block == 256) && (c.pair == 0 || c.pair == 1) &&
           c.wgs_per_cu >= 0 && c.wgs_per_cu <= 32 && (c.order == 0 || c.order == 1);
}

// Tile list of a config, instance-major.  Jacobian tiles use paired lanes only
// for instances with an even N (every slot row of the instance then starts on
// a 16-byte boundary, since its packed offset is even).
static std::vector<TileDesc> build_tiles(const ocp_batch &b, const ocp_batch_config &c)
{
    std::vector<TileDesc> t;
    const int cols = b.n + b.m;
    for (int32_t i = 0; i < b.count; i++) {
        const int64_t N = b.Ns[i];
        const int npt = (c.pair && N % 2 == 0) ? 2 : 1;
        const int64_t span = (int64_t)c.block * npt;
        if (c.order == 0) {
            for (int64_t k0 = 0; k0 < N; k0 += span)
                for (int col = 0; col < cols; col++) t.push_back({i, (int32_t)k0, col, npt});
        } else {
            for (int col = 0; col < cols; col++)
                for (int64_t k0 = 0; k0 < N; k0 += span) t.push_back({i, (int32_t)k0, col, npt});
        }
        for (int64_t k0 = 0; k0 <= N; k0 += c.block) t.push_back({i, (int32_t)k0, -1, 1});
    }
    return t;
}

static int upload_tiles(ocp_batch *b, const ocp_batch_config &c)
{
    std::vector<TileDesc> t = build_tiles(*b, c);
    if (t.size() > (size_t)INT32_MAX) return fail(OCP_ERR_OVERFLOW, "ocp_batch: too many tiles");
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail_b("ocp_batch: hipDeviceSynchronize", e);
    if (b->tiles) (void)hipFree(b->tiles);
    b->tiles = nullptr;
    e = hipMalloc(&b->tiles, t.size() * sizeof(TileDesc));
    if (e != hipSuccess) return fail(OCP_ERR_ALLOC, std::string("ocp_batch: hipMalloc: ") + hipGetErrorString(e));
    e = hipMemcpy(b->tiles, t.data(), t.size() * sizeof(TileDesc), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail_b("ocp_batch: hipMemcpy", e);
    b->ntiles = (int)t.size();
    b->cfg = c;
    return OCP_OK;
}

template <int BS>
static void launch_batch_bs(const ocp_batch *b, const TileDesc *tiles, int ntiles, int what,
                            const double *z, const double *y, double sigma, double *jac,
                            double *hess, hipStream_t s)
{
    const int cap = b->cfg.wgs_per_cu > 0 ? b->cus * b->cfg.wgs_per_cu : ntiles;
    const unsigned grid = (unsigned)std::max(1, std::min(ntiles, cap));
    const int n = b->n;
    const bool pair_ok = ((uintptr_t)jac % 16 == 0);
    if (n <= 4)
        hipLaunchKernelGGL((batch_kernel<4, BS>), dim3(grid), dim3(BS), 0, s, b->bp, b->inst, tiles, ntiles, what, pair_ok, z, y, sigma, jac, hess);
    else if (n <= 8)
        hipLaunchKernelGGL((batch_kernel<8, BS>), dim3(grid), dim3(BS), 0, s, b->bp, b->inst, tiles, ntiles, what, pair_ok, z, y, sigma, jac, hess);
    else if (n <= 16)
        hipLaunchKernelGGL((batch_kernel<16, BS>), dim3(grid), dim3(BS), 0, s, b->bp, b->inst, tiles, ntiles, what, pair_ok, z, y, sigma, jac, hess);
    else
        hipLaunchKernelGGL((batch_kernel<32, BS>), dim3(grid), dim3(BS), 0, s, b->bp, b->inst, tiles, ntiles, what, pair_ok, z, y, sigma, jac, hess);
}

static int check_eval_args(const ocp_batch *b, int32_t what, int32_t mode, const double *z,
                           const double *y, double sigma, const double *jac, const double *hess,
                           const char *fn)
{
    if (!b) return fail(OCP_ERR_ARG, std::string(fn) + ": batch is NULL");
    if (what <= 0 || what > (OCP_EVAL_JAC | OCP_EVAL_HESS))
        return fail(OCP_ERR_ARG, std::string(fn) + ": `what` must be a non-empty mask of OCP_EVAL_JAC, OCP_EVAL_HESS");
    if (mode != OCP_BATCH_PERSISTENT && mode != OCP_BATCH_PER_INSTANCE)
        return fail(OCP_ERR_ARG, std::string(fn) + ": unknown mode");
    if (!z) return fail(OCP_ERR_ARG, std::string(fn) + ": z is NULL");
    if ((what & OCP_EVAL_JAC) && !jac) return fail(OCP_ERR_ARG, std::string(fn) + ": jac is NULL");
    if ((what & OCP_EVAL_HESS) && (!hess || !y))
        return fail(OCP_ERR_ARG, std::string(fn) + ": hess and y are required for OCP_EVAL_HESS");
    if ((what & OCP_EVAL_HESS) && !std::isfinite(sigma))
        return fail(OCP_ERR_ARG, std::string(fn) + ": sigma is not finite");
    return OCP_OK;
}

// Launch one evaluation on `s` (no argument checks; tiles = the list to use).
static int batch_launch(const ocp_batch *b, const TileDesc *tiles, int32_t what, int32_t mode,
                        const double *z, const double *y, double sigma, double *jac, double *hess,
                        hipStream_t s)
{
    if (mode == OCP_BATCH_PERSISTENT) {
        if (b->cfg.block == 128)
            launch_batch_bs<128>(b, tiles, b->ntiles, what, z, y, sigma, jac, hess, s);
        else
            launch_batch_bs<256>(b, tiles, b->ntiles, what, z, y, sigma, jac, hess, s);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail_b("ocp_batch_eval", e);
        return OCP_OK;
    }
    const bool pair_ok = ((uintptr_t)jac % 16 == 0);
    for (int32_t i = 0; i < b->count; i++) {
        KP P;
        P.N = (int)b->Ns[i];
        P.N1 = P.N + 1;
        P.n = b->n;
        P.m = b->m;
        P.npair = b->bp.npair;
        P.T = b->bp.T;
        P.S = b->bp.S;
        P.nnzk = 0;
        P.NU = P.N1;
        P.scheme = 0;
        P.nb = 0;
        P.h = 1.0 / (double)P.N;
        P.hh = 0.5 * P.h;
        P.A = b->bp.A + (int64_t)i * b->n * b->n;
        P.B = b->bp.B + (int64_t)i * b->n * b->m;
        P.gam = b->bp.gam + (int64_t)i * b->n;
        P.q = b->bp.q + (int64_t)i * b->n;
        P.r = b->bp.r + (int64_t)i * b->m;
        P.AT = b->bp.AT + (int64_t)i * b->n * kLd;
        P.BT = b->bp.BT + (int64_t)i * b->m * kLd;
        const double *zb = z + b->z_off[i];
        hipError_t e = hipSuccess;
        if (what & OCP_EVAL_JAC) e = launch_jac(P, zb, jac + b->jac_off[i], pair_ok, s);
        if (e == hipSuccess && (what & OCP_EVAL_HESS))
            e = launch_hess(P, zb, y + b->c_off[i], sigma, hess + b->hess_off[i], s);
        if (e != hipSuccess) return hip_fail_b("ocp_batch_eval (per instance)", e);
    }
    return OCP_OK;
}

extern "C" {

int ocp_batch_create(int32_t count, const int64_t *Ns, int32_t n, int32_t m, const double *A,
                     const double *B, const double *gamma, const double *q, const double *r,
                     ocp_batch **out)
{
    clear_error();
    if (!out) return fail(OCP_ERR_ARG, "ocp_batch_create: out is NULL");
    *out = nullptr;
    if (count < 1) return fail(OCP_ERR_ARG, "ocp_batch_create: count must be >= 1");
    if (!Ns || !A || !gamma || !q || (m > 0 && (!B || !r)))
        return fail(OCP_ERR_ARG, "ocp_batch_create: NULL input array");
    Dims shape;
    int rc = make_dims(1, n, m, &shape);
    if (rc) return rc;
    ocp_batch *b = new (std::nothrow) ocp_batch();
    if (!b) return fail(OCP_ERR_ALLOC, "ocp_batch_create: out of host memory");
    b->count = count;
    b->n = n;
    b->m = m;
    b->shape = shape;
    b->Ns.assign(Ns, Ns + count);
    b->z_off.assign(count + 1, 0);
    b->c_off.assign(count + 1, 0);
    b->jac_off.assign(count + 1, 0);
    b->hess_off.assign(count + 1, 0);
    for (int32_t i = 0; i < count; i++) {
        Dims d;
        rc = make_dims(b->Ns[i], n, m, &d);
        if (rc) {
            delete b;
            return fail(rc, "ocp_batch_create: instance " + std::to_string(i) + ": " + ocp_last_error());
        }
        b->z_off[i + 1] = b->z_off[i] + d.nvar;
        b->c_off[i + 1] = b->c_off[i] + d.ncon;
        b->jac_off[i + 1] = b->jac_off[i] + d.nnzj;
        b->hess_off[i + 1] = b->hess_off[i] + d.nnzh;
    }
    const size_t nA = (size_t)count * n * n, nB = (size_t)count * n * m, nV = (size_t)count * n,
                 nR = (size_t)count * m;
    for (size_t x = 0; x < nA; x++)
        if (!std::isfinite(A[x])) {
            delete b;
            return fail(OCP_ERR_ARG, "ocp_batch_create: A has a non-finite entry");
        }
    hipError_t e = hipGetDevice(&b->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, b->device);
    if (e != hipSuccess) {
        delete b;
        return hip_fail_b("ocp_batch_create", e);
    }
    const size_t nplain = nA + nB + 2 * nV + nR;
    const size_t nAT = (size_t)count * n * kLd, nBT = (size_t)count * m * kLd;
    const size_t ncoef = nplain + nAT + nBT;
    e = hipMalloc(&b->coef, ncoef * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&b->inst, (size_t)count * sizeof(InstDesc));
    if (e != hipSuccess) {
        ocp_batch_destroy(b);
        return fail(OCP_ERR_ALLOC, std::string("ocp_batch_create: hipMalloc: ") + hipGetErrorString(e));
    }
    std::vector<double> host(ncoef);
    size_t o = 0;
    std::memcpy(host.data() + o, A, nA * sizeof(double)); o += nA;
    if (nB) std::memcpy(host.data() + o, B, nB * sizeof(double)); o += nB;
    std::memcpy(host.data() + o, gamma, nV * sizeof(double)); o += nV;
    std::memcpy(host.data() + o, q, nV * sizeof(double)); o += nV;
    if (nR) std::memcpy(host.data() + o, r, nR * sizeof(double));
    for (int32_t i = 0; i < count; i++)
        pack_columns(n, m, A + (size_t)i * n * n, B ? B + (size_t)i * n * m : nullptr,
                     host.data() + nplain + (size_t)i * n * kLd,
                     host.data() + nplain + nAT + (size_t)i * m * kLd);
    std::vector<InstDesc> inst(count);
    for (int32_t i = 0; i < count; i++) {
        inst[i].z_off = b->z_off[i];
        inst[i].c_off = b->c_off[i];
        inst[i].jac_off = b->jac_off[i];
        inst[i].hess_off = b->hess_off[i];
        inst[i].N = (int32_t)b->Ns[i];
        inst[i].pad = 0;
        inst[i].h = 1.0 / (double)b->Ns[i];
        inst[i].hh = 0.5 * inst[i].h;
    }
    e = hipMemcpy(b->coef, host.data(), ncoef * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->inst, inst.data(), inst.size() * sizeof(InstDesc), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        ocp_batch_destroy(b);
        return hip_fail_b("ocp_batch_create: hipMemcpy", e);
    }
    b->bp.n = n;
    b->bp.m = m;
    b->bp.npair = shape.npair;
    b->bp.T = shape.T;
    b->bp.S = shape.S;
    b->bp.A = b->coef;
    b->bp.B = b->coef + nA;
    b->bp.gam = b->bp.B + nB;
    b->bp.q = b->bp.gam + nV;
    b->bp.r = b->bp.q + nV;
    b->bp.AT = b->coef + nplain;
    b->bp.BT = b->bp.AT + nAT;
    rc = upload_tiles(b, b->cfg);
    if (rc) {
        std::string msg = ocp_last_error();
        ocp_batch_destroy(b);
        return fail(rc, msg);
    }
    *out = b;
    return OCP_OK;
}

void ocp_batch_destroy(ocp_batch *b)
{
    if (!b) return;
    if (b->coef) (void)hipFree(b->coef);
    if (b->inst) (void)hipFree(b->inst);
    if (b->tiles) (void)hipFree(b->tiles);
    delete b;
}

int ocp_batch_offsets(const ocp_batch *b, int64_t *z_off, int64_t *c_off, int64_t *jac_off,
                      int64_t *hess_off)
{
    clear_error();
    if (!b) return fail(OCP_ERR_ARG, "ocp_batch_offsets: batch is NULL");
    const size_t n = (size_t)b->count + 1;
    if (z_off) std::memcpy(z_off, b->z_off.data(), n * sizeof(int64_t));
    if (c_off) std::memcpy(c_off, b->c_off.data(), n * sizeof(int64_t));
    if (jac_off) std::memcpy(jac_off, b->jac_off.data(), n * sizeof(int64_t));
    if (hess_off) std::memcpy(hess_off, b->hess_off.data(), n * sizeof(int64_t));
    return OCP_OK;
}

int ocp_batch_get_config(const ocp_batch *b, ocp_batch_config *cfg)
{
    clear_error();
    if (!b || !cfg) return fail(OCP_ERR_ARG, "ocp_batch_get_config: NULL argument");
    *cfg = b->cfg;
    return OCP_OK;
}

int ocp_batch_set_config(ocp_batch *b, const ocp_batch_config *cfg)
{
    clear_error();
    if (!b || !cfg) return fail(OCP_ERR_ARG, "ocp_batch_set_config: NULL argument");
    if (!valid_config(*cfg))
        return fail(OCP_ERR_ARG, "ocp_batch_set_config: block must be 128 or 256, pair 0 or 1, "
                                 "wgs_per_cu in [0, 32], order 0 or 1");
    return upload_tiles(b, *cfg);
}

int ocp_batch_eval(const ocp_batch *b, int32_t what, int32_t mode, const double *z,
                   const double *y, double sigma, double *jac, double *hess, hipStream_t stream)
{
    clear_error();
    if (int rc = check_eval_args(b, what, mode, z, y, sigma, jac, hess, "ocp_batch_eval")) return rc;
    return batch_launch(b, b->tiles, what, mode, z, y, sigma, jac, hess, stream);
}

int ocp_batch_graph_create(const ocp_batch *b, int32_t what, int32_t mode, const double *z,
                           const double *y, double sigma, double *jac, double *hess,
                           ocp_graph **out)
{
    clear_error();
    if (!out) return fail(OCP_ERR_ARG, "ocp_batch_graph_create: out is NULL");
    *out = nullptr;
    if (int rc = check_eval_args(b, what, mode, z, y, sigma, jac, hess, "ocp_batch_graph_create"))
        return rc;
    ocp_graph *g = new (std::nothrow) ocp_graph();
    if (!g) return fail(OCP_ERR_ALLOC, "ocp_batch_graph_create: out of host memory");
    hipError_t e = hipSuccess;
    if (mode == OCP_BATCH_PERSISTENT) {
        e = hipMalloc(&g->tiles, (size_t)b->ntiles * sizeof(TileDesc));
        if (e == hipSuccess)
            e = hipMemcpy(g->tiles, b->tiles, (size_t)b->ntiles * sizeof(TileDesc), hipMemcpyDeviceToDevice);
        if (e != hipSuccess) {
            ocp_graph_destroy(g);
            return hip_fail_b("ocp_batch_graph_create: tile list copy", e);
        }
    }
    hipStream_t s = nullptr;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) {
        ocp_graph_destroy(g);
        return hip_fail_b("ocp_batch_graph_create: hipStreamCreate", e);
    }
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    int rc = OCP_OK;
    if (e == hipSuccess) {
        rc = batch_launch(b, g->tiles, what, mode, z, y, sigma, jac, hess, s);
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(s, &graph);
        g->graph = graph;
        if (rc == OCP_OK && e2 != hipSuccess) rc = hip_fail_b("ocp_batch_graph_create: hipStreamEndCapture", e2);
    } else {
        rc = hip_fail_b("ocp_batch_graph_create: hipStreamBeginCapture", e);
    }
    (void)hipStreamDestroy(s);
    if (rc == OCP_OK) {
        e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = hip_fail_b("ocp_batch_graph_create: hipGraphInstantiate", e);
    }
    if (rc != OCP_OK) {
        std::string msg = ocp_last_error();
        ocp_graph_destroy(g);
        return fail(rc, msg);
    }
    *out = g;
    return OCP_OK;
}

int ocp_graph_launch(const ocp_graph *g, hipStream_t stream)
{
    clear_error();
    if (!g || !g->exec) return fail(OCP_ERR_ARG, "ocp_graph_launch: graph is NULL");
    hipError_t e = hipGraphLaunch(g->exec, stream);
    if (e != hipSuccess) return hip_fail_b("ocp_graph_launch", e);
    return OCP_OK;
}

void ocp_graph_destroy(ocp_graph *g)
{
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->tiles) (void)hipFree(g->tiles);
    delete g;
}

int ocp_batch_autotune(ocp_batch *b, int32_t what, const double *z, const double *y, double sigma,
                       double *jac, double *hess, int32_t reps, hipStream_t stream,
                       ocp_batch_config *best, float *best_ms, float *all_ms)
{
    clear_error();
    if (int rc = check_eval_args(b, what, OCP_BATCH_PERSISTENT, z, y, sigma, jac, hess,
                                 "ocp_batch_autotune"))
        return rc;
    if (reps < 1) return fail(OCP_ERR_ARG, "ocp_batch_autotune: reps must be >= 1");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return hip_fail_b("ocp_batch_autotune: hipEventCreate", e);
    ocp_batch_config win = b->cfg;
    float win_ms = 1e30f;
    int rc = OCP_OK;
    int shape = 0;
    for (int block : {128, 256})
        for (int pair : {0, 1})
            for (int wpc : {1, 2, 4, 8, 16, 32, 0})
                for (int order : {0, 1}) {
                ocp_batch_config c{block, pair, wpc, order};
                rc = upload_tiles(b, c);
                if (rc) break;
                rc = batch_launch(b, b->tiles, what, OCP_BATCH_PERSISTENT, z, y, sigma, jac, hess, stream);
                if (rc) break;
                e = hipEventRecord(e0, stream);
                for (int r = 0; r < reps && rc == OCP_OK; r++)
                    rc = batch_launch(b, b->tiles, what, OCP_BATCH_PERSISTENT, z, y, sigma, jac, hess, stream);
                if (rc) break;
                if (e == hipSuccess) e = hipEventRecord(e1, stream);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) {
                    rc = hip_fail_b("ocp_batch_autotune: timing", e);
                    break;
                }
                ms /= (float)reps;
                if (all_ms && shape < OCP_AUTOTUNE_SHAPES) all_ms[shape] = ms;
                shape++;
                if (ms < win_ms) {
                    win_ms = ms;
                    win = c;
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    rc = upload_tiles(b, win);
    if (rc) return rc;
    if (best) *best = win;
    if (best_ms) *best_ms = win_ms;
    return OCP_OK;
}

}  // extern "C"
