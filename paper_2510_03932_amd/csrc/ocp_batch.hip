// Batched evaluation: many independent instances (own N_b and coefficients,
// shared n, m, scheme and boundary option) evaluated together -- every
// evaluation of an interior-point step (objective, gradient, defects,
// Jacobian, Hessian of the Lagrangian, and the fused KKT values) in one
// persistent launch, the per-instance launches it replaces, HIP-graph capture
// of either, and an autotuner for the tile shape.
//
// The persistent kernel walks a static tile list: workgroup w takes tiles
// w, w + G, w + 2G, ... (G = grid size), so every wave reaches the end of the
// list and exits, and the assignment is fixed (no queue).  A tile is
// (instance, first interval or node, kind): a Jacobian column over
// `block * npt` intervals, a Hessian, gradient or variable-row KKT run of
// `block` nodes, a defect run of 63 intervals per wavefront, an objective
// group of 256 nodes, a defect-row KKT run of 16 intervals, or an instance's
// boundary rows.  One list per evaluation mask, instance-major (an instance's
// tiles together, so the workgroups in flight share the state rows they read).
// The per-lane arithmetic is the single-instance path's (ocp_device.h,
// ocp_step_device.h): the values are bitwise those of per-instance
// evaluation, for any tile shape.
//
// The evaluations fall into three groups, each with a kernel instantiation of
// its own register footprint: Jacobian and Hessian values; objective,
// gradient and defects; the fused KKT values.  A mask that spans several
// groups is one persistent launch per group, back to back on the stream.
//
// The objective of instance b is a fixed-order sum: each objective tile sums
// its 256 nodes in the order of the single-instance reduction, and a small
// second launch (one workgroup per instance) sums the instance's partials in
// the order of the single-instance second pass.  (A last-workgroup-finishes
// scheme would save that launch, but its device-scope release fence writes
// back the L2 of every tile that takes it: on this GPU a one-pass objective
// measured 3x slower than two passes.)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ocp_device.h"
#include "ocp_internal.h"
#include "ocp_step_device.h"

using namespace ocp;
using namespace ocp::dev;

namespace {

constexpr int kObjTile = 256;  // nodes per objective tile (the single-instance workgroup)
constexpr int kMasks = 256;    // tile-list keys: evaluation masks 1 .. OCP_EVAL_ALL and the two KKT keys below
// Tile-list keys of the two KKT groups (outside the OCP_EVAL_* bits): the
// defect-row tiles (with the boundary rows), and the variable-row tiles.
constexpr int kListKktDef = 64, kListKktVar = 128;

// One instance's place in the packed arrays (device copy of the offset table).
struct InstDesc {
    int64_t z_off, c_off, jac_off, hess_off, kkt_off, dim_off;
    int64_t part0;   // first objective partial of the instance
    int32_t N;       // intervals
    int32_t nparts;  // objective tiles: ceil((N+1) / 256)
    double h, hh;
};

enum TileKind : int16_t { kJac = 0, kHess, kCons, kGrad, kObj, kKktDef, kKktVar, kBnd };

// One unit of work of the persistent kernel.
struct TileDesc {
    int32_t b;     // instance
    int32_t k0;    // first interval or node
    int16_t kind;  // TileKind
    int16_t npt;   // intervals per lane of a Jacobian tile (1 or 2)
    int32_t col;   // Jacobian column 0 .. n+m-1
};

// Coefficients of the whole batch (device), instance-major, and the shared shape.
struct BP {
    int n, m, npair, T, S, scheme, nb;
    int defect_lg;  // defect-row KKT tiles of 2^defect_lg intervals
    const double *A, *B, *gam, *q, *r;
    const double *AT, *BT;  // padded columns: n kLd and m kLd doubles per instance
};

// Device arguments of one evaluation.
struct BIO {
    const double *z, *y, *reg;
    double sigma;
    double *obj, *grad, *cons, *jac, *hess, *kkt;
    double *parts;    // objective partials (sum of nparts)
};

template <int SCHEME>
__device__ __forceinline__ KP make_kp(const BP &bp, const InstDesc &id, int b)
{
    KP P;
    P.N = id.N;
    P.N1 = id.N + 1;
    P.n = bp.n;
    P.m = bp.m;
    P.npair = bp.npair;
    P.T = bp.T;
    P.S = bp.S;
    P.nnzk = 0;
    P.NU = SCHEME ? id.N : id.N + 1;
    P.scheme = SCHEME;  // a compile-time constant, so the other scheme's code folds away
    P.nb = bp.nb;
    P.h = id.h;
    P.hh = id.hh;
    P.A = bp.A + (int64_t)b * bp.n * bp.n;
    P.B = bp.B + (int64_t)b * bp.n * bp.m;
    P.gam = bp.gam + (int64_t)b * bp.n;
    P.q = bp.q + (int64_t)b * bp.n;
    P.r = bp.r + (int64_t)b * bp.m;
    P.AT = bp.AT + (int64_t)b * bp.n * kLd;
    P.BT = bp.BT + (int64_t)b * bp.m * kLd;
    return P;
}

template <int NPT, int SCHEME>
__device__ __forceinline__ void jac_cols(const KP &P, const double *z, double *jac, int64_t k, int col)
{
    if constexpr (SCHEME != 0) jac_column_euler<NPT>(P, z, jac, k, col);
    else jac_column<NPT>(P, z, jac, k, col);
}

// KINDS: the evaluation bits this instantiation handles (tiles of other kinds
// are not in its lists); fewer kinds keep the register footprint of the
// Jacobian/Hessian-only launch small.  SCHEME: the batch's scheme, fixed at
// compile time so that each instantiation holds one scheme's code.
// Every array is its own __restrict__ parameter: with the outputs inside a
// struct the compiler cannot tell that the tile list, the offset table and
// the coefficients are never written, and loads them per lane instead of
// through the scalar cache (14 % slower on the Jacobian/Hessian tiles).
template <int NB, int BS, int KINDS, int SCHEME>
__global__ __launch_bounds__(BS) void batch_kernel(BP bp, KKTLayout Lo, const InstDesc *__restrict__ inst,
                                                   const TileDesc *__restrict__ tiles, int ntiles, int what,
                                                   bool pair_ok, const double *__restrict__ z_,
                                                   const double *__restrict__ y_, const double *__restrict__ reg_,
                                                   double sigma, double *__restrict__ grad_,
                                                   double *__restrict__ cons_, double *__restrict__ jac_,
                                                   double *__restrict__ hess_, double *__restrict__ kkt_,
                                                   double *__restrict__ parts_)
{
    extern __shared__ double lds[];   // defect-row KKT tile (dynamic, only with OCP_EVAL_KKT)
    __shared__ double vbuf[3 * BS];   // variable-row KKT tile
    __shared__ double ws[4];          // objective sums
    const int tid = threadIdx.x;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const TileDesc td = tiles[t];
        const InstDesc id = inst[td.b];
        const KP P = make_kp<SCHEME>(bp, id, td.b);
        const double *zb = z_ + id.z_off;
        switch (td.kind) {
        case kJac: {
            if (!(KINDS & OCP_EVAL_JAC)) break;
            double *jb = jac_ + id.jac_off;
            if (td.npt == 2) {
                // two intervals per lane; paired stores need a 16-byte
                // aligned output, else the lane stores them one by one
                const int64_t k = td.k0 + 2 * (int64_t)tid;
                if (k < P.N) {
                    if (pair_ok) {
                        jac_cols<2, SCHEME>(P, zb, jb, k, td.col);
                    } else {
                        jac_cols<1, SCHEME>(P, zb, jb, k, td.col);
                        jac_cols<1, SCHEME>(P, zb, jb, k + 1, td.col);
                    }
                }
            } else {
                const int64_t k = td.k0 + (int64_t)tid;
                if (k < P.N) jac_cols<1, SCHEME>(P, zb, jb, k, td.col);
            }
            break;
        }
        case kHess: {
            if (!(KINDS & OCP_EVAL_HESS)) break;
            const int k = td.k0 + tid;
            if (k <= P.N) {
                if constexpr (SCHEME != 0)
                    hess_node_euler<NB, true>(P, zb, y_ + id.c_off, sigma, hess_ + id.hess_off, k);
                else hess_node<NB, true>(P, zb, y_ + id.c_off, sigma, hess_ + id.hess_off, k);
            }
            break;
        }
        case kCons: {
            if (!(KINDS & OCP_EVAL_CONS)) break;
            double *cb = cons_ + id.c_off;
            if constexpr (SCHEME != 0) {
                const int64_t k = td.k0 + (int64_t)tid;
                if (k < P.N) cons_euler_interval<NB>(P, zb, cb, k);
            } else {
                cons_wave<NB>(P, zb, cb, td.k0 + 63 * (int64_t)(tid >> 6));
            }
            break;
        }
        case kGrad: {
            if (!(KINDS & OCP_EVAL_GRAD)) break;
            const int64_t k = td.k0 + (int64_t)tid;
            if (k <= P.N) {
                double *gb = grad_ + id.z_off;
                for (int c = 0; c < P.n + P.m; c++)
                    if (c < P.n || k < P.NU) grad_entry(P, zb, gb, c, k);
            }
            break;
        }
        case kObj: {
            if (!(KINDS & OCP_EVAL_OBJ)) break;
            double v[256 / BS];
#pragma unroll
            for (int r = 0; r < 256 / BS; r++) {
                const int64_t k = td.k0 + tid + r * BS;
                v[r] = k < P.N1 ? obj_node<NB>(P, zb, k) : 0.0;
            }
            const double s = sum256<BS>(v, ws);
            if (tid == 0) parts_[id.part0 + td.k0 / kObjTile] = s;
            __syncthreads();  // ws is reused by the next tile
            break;
        }
        case kKktDef:
            if (!(KINDS & (OCP_EVAL_KKT | kListKktDef))) break;
            kkt_defect_tile<BS>(P, Lo, zb, reg_ ? reg_ + id.dim_off : nullptr, kkt_ + id.kkt_off, td.k0,
                                bp.defect_lg, lds);
            break;
        case kKktVar:
            if (!(KINDS & (OCP_EVAL_KKT | kListKktVar))) break;
            kkt_var_tile<NB, BS>(P, Lo, zb, y_ + id.c_off, sigma, reg_ ? reg_ + id.dim_off : nullptr,
                                 kkt_ + id.kkt_off, td.k0, vbuf);
            break;
        case kBnd: {
            const int b = tid;
            if ((KINDS & (OCP_EVAL_CONS | OCP_EVAL_JAC | OCP_EVAL_KKT | kListKktDef)) && b < P.nb) {
                if ((KINDS & OCP_EVAL_CONS) && (what & OCP_EVAL_CONS))
                    cons_[id.c_off + (int64_t)P.n * P.N + b] = bnd_value(P, zb, b);
                if ((KINDS & OCP_EVAL_JAC) && (what & OCP_EVAL_JAC)) jac_[id.jac_off + (int64_t)P.n * P.N * P.T + b] = 1.0;
                if ((KINDS & (OCP_EVAL_KKT | kListKktDef)) && (what & OCP_EVAL_KKT))
                    kkt_bnd_row(P, Lo, reg_ ? reg_ + id.dim_off : nullptr, kkt_ + id.kkt_off, b);
            }
            break;
        }
        default:
            break;
        }
    }
}

// Objective, second pass: workgroup b sums instance b's tile partials as the
// single-instance second pass does (lane t takes partials t, t + 256, ... in
// order, then the fixed tree).
__global__ __launch_bounds__(kBlock) void batch_obj_final_kernel(const InstDesc *__restrict__ inst,
                                                                 const double *__restrict__ parts,
                                                                 double *__restrict__ obj)
{
    const InstDesc id = inst[blockIdx.x];
    double acc = 0.0;
    for (int i = threadIdx.x; i < id.nparts; i += kBlock) acc += parts[id.part0 + i];
    const double t = block_sum<kBlock>(acc);
    if (threadIdx.x == 0) obj[blockIdx.x] = t;
}

struct TileList {
    TileDesc *d = nullptr;  // device
    int n = 0;
};

}  // namespace

struct ocp_batch {
    int32_t count, n, m, scheme, bnd;
    Dims shape;                    // sizes of a one-interval instance (for T, S, npair, nb)
    std::vector<int64_t> Ns;
    std::vector<int64_t> z_off, c_off, jac_off, hess_off, kkt_off, dim_off, part_off;  // count + 1 each
    int device = 0;
    int cus = 0;
    double *coef = nullptr;        // device: A | B | gamma | q | r | AT | BT (instance-major blocks)
    InstDesc *inst = nullptr;      // device offset table
    double *parts = nullptr;       // device objective partials (part_off[count] doubles)
    mutable std::mutex mu;         // guards the tile-list cache
    mutable TileList lists[kMasks];  // per evaluation mask, for cfg
    ocp_batch_config cfg{256, 1, 0, 1};
    BP bp{};
    KKTLayout Lo{};
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

// Tile list of a config and evaluation mask, instance-major.  Jacobian tiles
// use paired lanes only for instances with an even N and an even packed
// Jacobian offset (every slot row of the instance then starts on a 16-byte
// boundary of a 16-byte aligned packed array; forward-Euler rows or boundary
// rows can make an offset odd).
static std::vector<TileDesc> build_tiles(const ocp_batch &b, const ocp_batch_config &c, int what)
{
    std::vector<TileDesc> t;
    const int cols = b.n + b.m;
    const bool euler = b.scheme != OCP_SCHEME_TRAPEZOIDAL;
    for (int32_t i = 0; i < b.count; i++) {
        const int64_t N = b.Ns[i];
        auto put = [&](int64_t k0, TileKind kind, int npt, int col) {
            t.push_back({i, (int32_t)k0, (int16_t)kind, (int16_t)npt, (int32_t)col});
        };
        if (what & OCP_EVAL_JAC) {
            const int npt = (c.pair && N % 2 == 0 && b.jac_off[i] % 2 == 0) ? 2 : 1;
            const int64_t span = (int64_t)c.block * npt;
            if (c.order == 0) {
                for (int64_t k0 = 0; k0 < N; k0 += span)
                    for (int col = 0; col < cols; col++) put(k0, kJac, npt, col);
            } else {
                for (int col = 0; col < cols; col++)
                    for (int64_t k0 = 0; k0 < N; k0 += span) put(k0, kJac, npt, col);
            }
        }
        if (what & OCP_EVAL_HESS)
            for (int64_t k0 = 0; k0 <= N; k0 += c.block) put(k0, kHess, 1, 0);
        if (what & OCP_EVAL_CONS) {
            const int64_t span = euler ? c.block : 63 * (c.block / 64);  // 63 intervals per wavefront
            for (int64_t k0 = 0; k0 < N; k0 += span) put(k0, kCons, 1, 0);
        }
        if (what & OCP_EVAL_GRAD)
            for (int64_t k0 = 0; k0 <= N; k0 += c.block) put(k0, kGrad, 1, 0);
        if (what & OCP_EVAL_OBJ)
            for (int64_t k0 = 0; k0 <= N; k0 += kObjTile) put(k0, kObj, 1, 0);
        if (what & (OCP_EVAL_KKT | kListKktDef))
            for (int64_t k0 = 0; k0 < N; k0 += (int64_t)1 << b.bp.defect_lg) put(k0, kKktDef, 1, 0);
        if (what & (OCP_EVAL_KKT | kListKktVar))
            for (int64_t k0 = 0; k0 <= N; k0 += c.block) put(k0, kKktVar, 1, 0);
        if (b.shape.nb > 0 && (what & (OCP_EVAL_CONS | OCP_EVAL_JAC | OCP_EVAL_KKT | kListKktDef)))
            put(0, kBnd, 1, 0);
    }
    return t;
}

static void free_lists(const ocp_batch *b)
{
    for (TileList &l : b->lists) {
        if (l.d) (void)hipFree(l.d);
        l = TileList{};
    }
}

// The device tile list of `what` under the current config, built on first use
// (allocates and copies; no device-wide synchronization).
static int tile_list(const ocp_batch *b, int what, TileList *out)
{
    std::lock_guard<std::mutex> lock(b->mu);
    TileList &l = b->lists[what];
    if (!l.d) {
        std::vector<TileDesc> t = build_tiles(*b, b->cfg, what);
        if (t.size() > (size_t)INT32_MAX) return fail(OCP_ERR_OVERFLOW, "ocp_batch: too many tiles");
        if (t.empty()) t.push_back({0, 0, (int16_t)-1, 1, 0});  // keeps the pointer non-null
        TileDesc *d = nullptr;
        hipError_t e = hipMalloc(&d, t.size() * sizeof(TileDesc));
        if (e != hipSuccess)
            return fail(OCP_ERR_ALLOC, std::string("ocp_batch: hipMalloc: ") + hipGetErrorString(e));
        e = hipMemcpy(d, t.data(), t.size() * sizeof(TileDesc), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(d);
            return hip_fail_b("ocp_batch: hipMemcpy", e);
        }
        l.d = d;
        l.n = (int)t.size();
    }
    *out = l;
    return OCP_OK;
}

// Switch to a new config: every cached tile list is dropped (after the device
// has finished any work that may read them) and the Jacobian and Hessian
// lists rebuilt.
static int set_cfg(ocp_batch *b, const ocp_batch_config &c)
{
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail_b("ocp_batch: hipDeviceSynchronize", e);
    {
        std::lock_guard<std::mutex> lock(b->mu);
        free_lists(b);
        b->cfg = c;
    }
    TileList l;
    if (int rc = tile_list(b, OCP_EVAL_JAC, &l)) return rc;
    return tile_list(b, OCP_EVAL_HESS, &l);
}

static BIO to_bio(const ocp_batch *b, const ocp_batch_io &io)
{
    BIO d;
    d.z = io.z;
    d.y = io.y;
    d.reg = io.reg;
    d.sigma = io.sigma;
    d.obj = io.obj;
    d.grad = io.grad;
    d.cons = io.cons;
    d.jac = io.jac;
    d.hess = io.hess;
    d.kkt = io.kkt;
    d.parts = b->parts;
    return d;
}

// The kernel groups, one launch each: Jacobian values; Hessian values;
// objective and gradient; defects; the defect rows of the fused KKT values;
// their variable rows.  Each group is its own kernel, so it gets the
// registers of its own tile bodies: in one kernel, tile kinds take the
// registers of the heaviest (at n <= 8 the two KKT kinds together 127 VGPRs
// against 73 and 110 apart, the defects 111 against 39 for the objective
// and gradient), and the light tiles run at that residency.  kGroupKinds
// holds each group's tile kinds, kGroupBits the evaluation bits it serves.
constexpr int kNumGroups = 6;
constexpr int kGroupKinds[kNumGroups] = {OCP_EVAL_JAC, OCP_EVAL_HESS, OCP_EVAL_OBJ | OCP_EVAL_GRAD,
                                         OCP_EVAL_CONS, kListKktDef, kListKktVar};
constexpr int kGroupBits[kNumGroups] = {OCP_EVAL_JAC, OCP_EVAL_HESS, OCP_EVAL_OBJ | OCP_EVAL_GRAD,
                                        OCP_EVAL_CONS, OCP_EVAL_KKT, OCP_EVAL_KKT};

// The tile-list key of group g for the evaluation mask `what`: the bits it
// serves, or its own key for the two KKT groups.
static int group_key(int g, int what)
{
    return kGroupKinds[g] & (kListKktDef | kListKktVar) ? kGroupKinds[g] : (what & kGroupBits[g]);
}

template <int BS, int KINDS, int SCHEME>
static void launch_batch_scheme(const ocp_batch *b, const TileDesc *tiles, int ntiles, int what, const BIO &io,
                                hipStream_t s)
{
    const int cap = b->cfg.wgs_per_cu > 0 ? b->cus * b->cfg.wgs_per_cu : ntiles;
    const unsigned grid = (unsigned)std::max(1, std::min(ntiles, cap));
    const bool pair_ok = ((uintptr_t)io.jac % 16 == 0);
    const size_t lds = ((KINDS & kListKktDef) && (what & OCP_EVAL_KKT))
                           ? kkt_defect_lds(b->n, b->m, b->shape.T, 1 << b->bp.defect_lg) * sizeof(double)
                           : 0;
    const int n = b->n;
    if (n <= 4)
        hipLaunchKernelGGL((batch_kernel<4, BS, KINDS, SCHEME>), dim3(grid), dim3(BS), lds, s, b->bp, b->Lo, b->inst, tiles, ntiles, what, pair_ok, io.z, io.y, io.reg, io.sigma, io.grad, io.cons, io.jac, io.hess, io.kkt, io.parts);
    else if (n <= 8)
        hipLaunchKernelGGL((batch_kernel<8, BS, KINDS, SCHEME>), dim3(grid), dim3(BS), lds, s, b->bp, b->Lo, b->inst, tiles, ntiles, what, pair_ok, io.z, io.y, io.reg, io.sigma, io.grad, io.cons, io.jac, io.hess, io.kkt, io.parts);
    else if (n <= 16)
        hipLaunchKernelGGL((batch_kernel<16, BS, KINDS, SCHEME>), dim3(grid), dim3(BS), lds, s, b->bp, b->Lo, b->inst, tiles, ntiles, what, pair_ok, io.z, io.y, io.reg, io.sigma, io.grad, io.cons, io.jac, io.hess, io.kkt, io.parts);
    else
        hipLaunchKernelGGL((batch_kernel<32, BS, KINDS, SCHEME>), dim3(grid), dim3(BS), lds, s, b->bp, b->Lo, b->inst, tiles, ntiles, what, pair_ok, io.z, io.y, io.reg, io.sigma, io.grad, io.cons, io.jac, io.hess, io.kkt, io.parts);
}

template <int BS, int KINDS>
static void launch_batch_kinds(const ocp_batch *b, const TileDesc *tiles, int ntiles, int what, const BIO &io,
                               hipStream_t s)
{
    if (b->scheme == OCP_SCHEME_TRAPEZOIDAL) launch_batch_scheme<BS, KINDS, 0>(b, tiles, ntiles, what, io, s);
    else launch_batch_scheme<BS, KINDS, 1>(b, tiles, ntiles, what, io, s);
}

// One group's launch: `what` lies within group g.
template <int BS>
static void launch_batch_bs(const ocp_batch *b, int g, const TileDesc *tiles, int ntiles, int what,
                            const BIO &io, hipStream_t s)
{
    switch (g) {
    case 0: launch_batch_kinds<BS, kGroupKinds[0]>(b, tiles, ntiles, what, io, s); break;
    case 1: launch_batch_kinds<BS, kGroupKinds[1]>(b, tiles, ntiles, what, io, s); break;
    case 2: launch_batch_kinds<BS, kGroupKinds[2]>(b, tiles, ntiles, what, io, s); break;
    case 3: launch_batch_kinds<BS, kGroupKinds[3]>(b, tiles, ntiles, what, io, s); break;
    case 4: launch_batch_kinds<BS, kGroupKinds[4]>(b, tiles, ntiles, what, io, s); break;
    default: launch_batch_kinds<BS, kGroupKinds[5]>(b, tiles, ntiles, what, io, s); break;
    }
}

static int check_eval_args(const ocp_batch *b, int32_t what, int32_t mode, const ocp_batch_io *io,
                           const char *fn)
{
    if (!b) return fail(OCP_ERR_ARG, std::string(fn) + ": batch is NULL");
    if (!io) return fail(OCP_ERR_ARG, std::string(fn) + ": io is NULL");
    if (what <= 0 || what > OCP_EVAL_ALL)
        return fail(OCP_ERR_ARG, std::string(fn) + ": `what` must be a non-empty mask of the OCP_EVAL_* bits");
    if (mode != OCP_BATCH_PERSISTENT && mode != OCP_BATCH_PER_INSTANCE)
        return fail(OCP_ERR_ARG, std::string(fn) + ": unknown mode");
    if (!io->z) return fail(OCP_ERR_ARG, std::string(fn) + ": z is NULL");
    struct Need { int bit; const void *p; const char *name; };
    const Need need[] = {{OCP_EVAL_JAC, io->jac, "jac"},   {OCP_EVAL_HESS, io->hess, "hess"},
                         {OCP_EVAL_HESS, io->y, "y"},      {OCP_EVAL_OBJ, io->obj, "obj"},
                         {OCP_EVAL_GRAD, io->grad, "grad"}, {OCP_EVAL_CONS, io->cons, "cons"},
                         {OCP_EVAL_KKT, io->kkt, "kkt"},   {OCP_EVAL_KKT, io->y, "y"}};
    for (const Need &x : need)
        if ((what & x.bit) && !x.p)
            return fail(OCP_ERR_ARG, std::string(fn) + ": " + x.name + " is NULL but requested by `what`");
    if ((what & (OCP_EVAL_HESS | OCP_EVAL_KKT)) && !std::isfinite(io->sigma))
        return fail(OCP_ERR_ARG, std::string(fn) + ": sigma is not finite");
    return OCP_OK;
}

static KP host_kp(const ocp_batch *b, int32_t i)
{
    KP P;
    P.N = (int)b->Ns[i];
    P.N1 = P.N + 1;
    P.n = b->n;
    P.m = b->m;
    P.npair = b->bp.npair;
    P.T = b->bp.T;
    P.S = b->bp.S;
    P.nnzk = 0;
    P.NU = b->scheme ? P.N : P.N1;
    P.scheme = b->scheme;
    P.nb = b->bp.nb;
    P.h = 1.0 / (double)P.N;
    P.hh = 0.5 * P.h;
    P.A = b->bp.A + (int64_t)i * b->n * b->n;
    P.B = b->bp.B + (int64_t)i * b->n * b->m;
    P.gam = b->bp.gam + (int64_t)i * b->n;
    P.q = b->bp.q + (int64_t)i * b->n;
    P.r = b->bp.r + (int64_t)i * b->m;
    P.AT = b->bp.AT + (int64_t)i * b->n * kLd;
    P.BT = b->bp.BT + (int64_t)i * b->m * kLd;
    return P;
}

// The tile lists of one persistent evaluation: one per kernel group that
// `what` touches (an empty list where it touches none).
struct Plan {
    TileList g[kNumGroups];
};

static int plan_of(const ocp_batch *b, int32_t what, Plan *out)
{
    for (int g = 0; g < kNumGroups; g++) {
        out->g[g] = TileList{};
        if (what & kGroupBits[g])
            if (int rc = tile_list(b, group_key(g, what), &out->g[g])) return rc;
    }
    return OCP_OK;
}

// Launch one evaluation on `s` (no argument checks).  `plan` (persistent
// mode) holds the tile lists to walk.
static int batch_launch(const ocp_batch *b, const Plan &plan, int32_t what, int32_t mode,
                        const ocp_batch_io &io, hipStream_t s)
{
    if (mode == OCP_BATCH_PERSISTENT) {
        const BIO d = to_bio(b, io);
        for (int g = 0; g < kNumGroups; g++) {
            const int sub = what & kGroupBits[g];
            if (!sub) continue;
            const TileList &l = plan.g[g];
            if (b->cfg.block == 128) launch_batch_bs<128>(b, g, l.d, l.n, sub, d, s);
            else launch_batch_bs<256>(b, g, l.d, l.n, sub, d, s);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return hip_fail_b("ocp_batch_eval", e);
        }
        if (what & OCP_EVAL_OBJ) {
            hipLaunchKernelGGL(batch_obj_final_kernel, dim3(b->count), dim3(kBlock), 0, s, b->inst, b->parts,
                               io.obj);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return hip_fail_b("ocp_batch_eval", e);
        }
        return OCP_OK;
    }
    for (int32_t i = 0; i < b->count; i++) {
        const KP P = host_kp(b, i);
        const bool pair_ok = ((uintptr_t)(io.jac + b->jac_off[i]) % 16 == 0);
        const double *zb = io.z + b->z_off[i];
        hipError_t e = hipSuccess;
        if (what & OCP_EVAL_OBJ) e = launch_obj(P, zb, b->parts + b->part_off[i], io.obj + i, s);
        if (e == hipSuccess && (what & OCP_EVAL_GRAD)) e = launch_grad(P, zb, io.grad + b->z_off[i], s);
        if (e == hipSuccess && (what & OCP_EVAL_CONS)) e = launch_cons(P, zb, io.cons + b->c_off[i], s);
        if (e == hipSuccess && (what & OCP_EVAL_JAC)) e = launch_jac(P, zb, io.jac + b->jac_off[i], pair_ok, s);
        if (e == hipSuccess && (what & OCP_EVAL_HESS))
            e = launch_hess(P, zb, io.y + b->c_off[i], io.sigma, io.hess + b->hess_off[i], s);
        if (e == hipSuccess && (what & OCP_EVAL_KKT))
            e = launch_eval_kkt(P, zb, io.y + b->c_off[i], io.sigma, io.reg ? io.reg + b->dim_off[i] : nullptr,
                                io.kkt + b->kkt_off[i], s);
        if (e != hipSuccess) return hip_fail_b("ocp_batch_eval (per instance)", e);
    }
    return OCP_OK;
}

static ocp_batch_io io_of(const double *z, const double *y, double sigma, double *jac, double *hess)
{
    ocp_batch_io io{};
    io.z = z;
    io.y = y;
    io.sigma = sigma;
    io.jac = jac;
    io.hess = hess;
    return io;
}

extern "C" {

int ocp_batch_create(int32_t count, const int64_t *Ns, int32_t n, int32_t m, const double *A,
                     const double *B, const double *gamma, const double *q, const double *r,
                     ocp_batch **out)
{
    return ocp_batch_create_ex(count, Ns, n, m, nullptr, A, B, gamma, q, r, out);
}

int ocp_batch_create_ex(int32_t count, const int64_t *Ns, int32_t n, int32_t m, const ocp_options *opt,
                        const double *A, const double *B, const double *gamma, const double *q,
                        const double *r, ocp_batch **out)
{
    clear_error();
    if (!out) return fail(OCP_ERR_ARG, "ocp_batch_create: out is NULL");
    *out = nullptr;
    if (count < 1) return fail(OCP_ERR_ARG, "ocp_batch_create: count must be >= 1");
    if (!Ns || !A || !gamma || !q || (m > 0 && (!B || !r)))
        return fail(OCP_ERR_ARG, "ocp_batch_create: NULL input array");
    const int32_t scheme = opt ? opt->scheme : OCP_SCHEME_TRAPEZOIDAL;
    const int32_t bnd = opt ? opt->boundary : OCP_BOUNDARY_NONE;
    Dims shape;
    int rc = make_dims_ex(1, n, m, scheme, bnd, &shape);
    if (rc) return rc;
    ocp_batch *b = new (std::nothrow) ocp_batch();
    if (!b) return fail(OCP_ERR_ALLOC, "ocp_batch_create: out of host memory");
    b->count = count;
    b->n = n;
    b->m = m;
    b->scheme = scheme;
    b->bnd = bnd;
    b->shape = shape;
    b->Ns.assign(Ns, Ns + count);
    for (auto *v : {&b->z_off, &b->c_off, &b->jac_off, &b->hess_off, &b->kkt_off, &b->dim_off, &b->part_off})
        v->assign(count + 1, 0);
    for (int32_t i = 0; i < count; i++) {
        Dims d;
        rc = make_dims_ex(b->Ns[i], n, m, scheme, bnd, &d);
        if (rc) {
            delete b;
            return fail(rc, "ocp_batch_create: instance " + std::to_string(i) + ": " + ocp_last_error());
        }
        b->z_off[i + 1] = b->z_off[i] + d.nvar;
        b->c_off[i + 1] = b->c_off[i] + d.ncon;
        b->jac_off[i + 1] = b->jac_off[i] + d.nnzj;
        b->hess_off[i + 1] = b->hess_off[i] + d.nnzh;
        b->kkt_off[i + 1] = b->kkt_off[i] + d.nnzk;
        b->dim_off[i + 1] = b->dim_off[i] + d.dim;
        b->part_off[i + 1] = b->part_off[i] + (d.N1 + kObjTile - 1) / kObjTile;
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
    if (e == hipSuccess) e = hipMalloc(&b->parts, (size_t)b->part_off[count] * sizeof(double));
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
        inst[i].kkt_off = b->kkt_off[i];
        inst[i].dim_off = b->dim_off[i];
        inst[i].part0 = b->part_off[i];
        inst[i].N = (int32_t)b->Ns[i];
        inst[i].nparts = (int32_t)(b->part_off[i + 1] - b->part_off[i]);
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
    b->bp.scheme = scheme;
    b->bp.nb = (int)shape.nb;
    b->bp.defect_lg = __builtin_ctz((unsigned)kkt_defect_kt(n, m, shape.T));
    b->bp.A = b->coef;
    b->bp.B = b->coef + nA;
    b->bp.gam = b->bp.B + nB;
    b->bp.q = b->bp.gam + nV;
    b->bp.r = b->bp.q + nV;
    b->bp.AT = b->coef + nplain;
    b->bp.BT = b->bp.AT + nAT;
    b->Lo = kkt_layout(n);
    TileList l;
    rc = tile_list(b, OCP_EVAL_JAC, &l);
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
    if (b->parts) (void)hipFree(b->parts);
    free_lists(b);
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

int ocp_batch_offsets_ex(const ocp_batch *b, int64_t *kkt_off, int64_t *dim_off)
{
    clear_error();
    if (!b) return fail(OCP_ERR_ARG, "ocp_batch_offsets_ex: batch is NULL");
    const size_t n = (size_t)b->count + 1;
    if (kkt_off) std::memcpy(kkt_off, b->kkt_off.data(), n * sizeof(int64_t));
    if (dim_off) std::memcpy(dim_off, b->dim_off.data(), n * sizeof(int64_t));
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
    return set_cfg(b, *cfg);
}

int ocp_batch_prepare(const ocp_batch *b, int32_t what)
{
    clear_error();
    if (!b) return fail(OCP_ERR_ARG, "ocp_batch_prepare: batch is NULL");
    if (what <= 0 || what > OCP_EVAL_ALL)
        return fail(OCP_ERR_ARG, "ocp_batch_prepare: `what` must be a non-empty mask of the OCP_EVAL_* bits");
    Plan plan;
    return plan_of(b, what, &plan);
}

int ocp_batch_eval_io(const ocp_batch *b, int32_t what, int32_t mode, const ocp_batch_io *io,
                      hipStream_t stream)
{
    clear_error();
    if (int rc = check_eval_args(b, what, mode, io, "ocp_batch_eval")) return rc;
    Plan plan;
    if (mode == OCP_BATCH_PERSISTENT)
        if (int rc = plan_of(b, what, &plan)) return rc;
    return batch_launch(b, plan, what, mode, *io, stream);
}

int ocp_batch_eval(const ocp_batch *b, int32_t what, int32_t mode, const double *z,
                   const double *y, double sigma, double *jac, double *hess, hipStream_t stream)
{
    clear_error();
    if (what & ~(OCP_EVAL_JAC | OCP_EVAL_HESS))
        return fail(OCP_ERR_ARG, "ocp_batch_eval: `what` must be a non-empty mask of OCP_EVAL_JAC, "
                                 "OCP_EVAL_HESS (ocp_batch_eval_io takes the other evaluations)");
    const ocp_batch_io io = io_of(z, y, sigma, jac, hess);
    return ocp_batch_eval_io(b, what, mode, &io, stream);
}

int ocp_batch_graph_create_io(const ocp_batch *b, int32_t what, int32_t mode, const ocp_batch_io *io,
                              ocp_graph **out)
{
    clear_error();
    if (!out) return fail(OCP_ERR_ARG, "ocp_batch_graph_create: out is NULL");
    *out = nullptr;
    if (int rc = check_eval_args(b, what, mode, io, "ocp_batch_graph_create")) return rc;
    ocp_graph *g = new (std::nothrow) ocp_graph();
    if (!g) return fail(OCP_ERR_ALLOC, "ocp_batch_graph_create: out of host memory");
    Plan own;
    if (mode == OCP_BATCH_PERSISTENT) {
        Plan plan;
        if (int rc = plan_of(b, what, &plan)) {
            std::string msg = ocp_last_error();
            ocp_graph_destroy(g);
            return fail(rc, msg);
        }
        // one allocation holds the graph's copies of the group lists
        size_t total = 0;
        for (const TileList &l : plan.g) total += (size_t)l.n;
        hipError_t e = hipMalloc(&g->tiles, std::max<size_t>(total, 1) * sizeof(TileDesc));
        size_t at = 0;
        for (int k = 0; k < kNumGroups && e == hipSuccess; k++) {
            const TileList &l = plan.g[k];
            if (!l.n) continue;
            e = hipMemcpy(g->tiles + at, l.d, (size_t)l.n * sizeof(TileDesc), hipMemcpyDeviceToDevice);
            own.g[k].d = g->tiles + at;
            own.g[k].n = l.n;
            at += (size_t)l.n;
        }
        if (e != hipSuccess) {
            ocp_graph_destroy(g);
            return hip_fail_b("ocp_batch_graph_create: tile list copy", e);
        }
    }
    hipStream_t s = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) {
        ocp_graph_destroy(g);
        return hip_fail_b("ocp_batch_graph_create: hipStreamCreate", e);
    }
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    int rc = OCP_OK;
    if (e == hipSuccess) {
        rc = batch_launch(b, own, what, mode, *io, s);
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

int ocp_batch_graph_create(const ocp_batch *b, int32_t what, int32_t mode, const double *z,
                           const double *y, double sigma, double *jac, double *hess,
                           ocp_graph **out)
{
    clear_error();
    if (what & ~(OCP_EVAL_JAC | OCP_EVAL_HESS)) {
        if (out) *out = nullptr;
        return fail(OCP_ERR_ARG, "ocp_batch_graph_create: `what` must be a non-empty mask of OCP_EVAL_JAC, "
                                 "OCP_EVAL_HESS (ocp_batch_graph_create_io takes the other evaluations)");
    }
    const ocp_batch_io io = io_of(z, y, sigma, jac, hess);
    return ocp_batch_graph_create_io(b, what, mode, &io, out);
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

int ocp_batch_autotune_io(ocp_batch *b, int32_t what, const ocp_batch_io *io, int32_t reps,
                          hipStream_t stream, ocp_batch_config *best, float *best_ms, float *all_ms)
{
    clear_error();
    if (int rc = check_eval_args(b, what, OCP_BATCH_PERSISTENT, io, "ocp_batch_autotune")) return rc;
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
                    rc = set_cfg(b, c);
                    Plan plan;
                    if (rc == OCP_OK) rc = plan_of(b, what, &plan);
                    if (rc == OCP_OK) rc = batch_launch(b, plan, what, OCP_BATCH_PERSISTENT, *io, stream);
                    if (rc) break;
                    e = hipEventRecord(e0, stream);
                    for (int r = 0; r < reps && rc == OCP_OK; r++)
                        rc = batch_launch(b, plan, what, OCP_BATCH_PERSISTENT, *io, stream);
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
    rc = set_cfg(b, win);
    if (rc) return rc;
    Plan plan;
    rc = plan_of(b, what, &plan);
    if (rc) return rc;
    if (best) *best = win;
    if (best_ms) *best_ms = win_ms;
    return OCP_OK;
}

int ocp_batch_autotune(ocp_batch *b, int32_t what, const double *z, const double *y, double sigma,
                       double *jac, double *hess, int32_t reps, hipStream_t stream,
                       ocp_batch_config *best, float *best_ms, float *all_ms)
{
    clear_error();
    if (what & ~(OCP_EVAL_JAC | OCP_EVAL_HESS))
        return fail(OCP_ERR_ARG, "ocp_batch_autotune: `what` must be a non-empty mask of OCP_EVAL_JAC, "
                                 "OCP_EVAL_HESS (ocp_batch_autotune_io takes the other evaluations)");
    const ocp_batch_io io = io_of(z, y, sigma, jac, hess);
    return ocp_batch_autotune_io(b, what, &io, reps, stream, best, best_ms, all_ms);
}

}  // extern "C"
