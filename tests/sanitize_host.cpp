// Host-side sanitizer driver (test infrastructure): the library's host index
// layer (sizes, patterns, KKT structure, stage orderings, symmetric
// reordering, argument validation) and the C oracle are compiled by g++/gcc
// with -fsanitize=address,undefined and run here against each other.  Any
// out-of-bounds access, use after free, leak, signed overflow or misaligned
// access in either aborts the run with a sanitizer report; any mismatch
// between the closed-form builders and the oracle's generic sort-based ones
// prints a line and makes the exit status non-zero.
//
// Built and run by tests/test_sanitize_host.py; needs no GPU and makes no HIP
// call (the host layer calls none).
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "ocp_eval.h"

extern "C" {
int orc_sizes_ex(int64_t N, int n, int m, int scheme, int bnd, int64_t *out);
int orc_pattern_ex(int64_t N, int n, int m, int scheme, int bnd, int32_t *jrow, int32_t *jcol,
                   int32_t *hrow, int32_t *hcol);
int orc_kkt_generic(int64_t nvar, int64_t ncon, int64_t nnzj, int64_t nnzh, const int32_t *jrow,
                    const int32_t *jcol, const int32_t *hrow, const int32_t *hcol, int32_t *rowptr,
                    int32_t *colind, int32_t *perm_j, int32_t *perm_h, int64_t *nnzk);
int orc_kkt_permute(int64_t dim, const int32_t *rowptr, const int32_t *colind, int64_t nnzj,
                    const int32_t *perm_j, int64_t nnzh, const int32_t *perm_h, const int32_t *order,
                    int32_t *rowptr2, int32_t *colind2, int32_t *perm_j2, int32_t *perm_h2,
                    int32_t *diag2);
int orc_quad_sizes(int64_t N, int bnd, int64_t *out);
int orc_quad_pattern(int64_t N, int bnd, int32_t *jrow, int32_t *jcol, int32_t *hrow, int32_t *hcol);
int orc_obj_ex(int64_t N, int n, int m, int scheme, int bnd, const double *q, const double *r,
               const double *z, double *out);
int orc_grad_ex(int64_t N, int n, int m, int scheme, int bnd, const double *q, const double *r,
                const double *z, double *g, double *mu);
int orc_cons_ex(int64_t N, int n, int m, int scheme, int bnd, const double *A, const double *B,
                const double *gam, const double *z, double *c, double *mu);
int orc_jac_ex(int64_t N, int n, int m, int scheme, int bnd, const double *A, const double *B,
               const double *gam, const double *z, double *out, double *mu);
int orc_hess_ex(int64_t N, int n, int m, int scheme, int bnd, const double *A, const double *gam,
                const double *q, const double *r, const double *z, const double *y, double sigma,
                double *out, double *mu);
int orc_lagrangian(int64_t N, int n, int m, const double *A, const double *B, const double *gam,
                   const double *q, const double *r, const double *z, const double *y, double sigma,
                   double *out);
int orc_lag_grad(int64_t N, int n, int m, const double *A, const double *B, const double *gam,
                 const double *q, const double *r, const double *z, const double *y, double sigma,
                 int64_t k0, int64_t k1, double *out, double *mu);
int orc_hvp(int64_t N, int n, int m, const double *A, const double *gam, const double *q,
            const double *r, const double *z, const double *y, double sigma, const double *v,
            int64_t k0, int64_t k1, double *out, double *mu);
int orc_jvp(int64_t N, int n, int m, const double *A, const double *B, const double *gam,
            const double *z, const double *v, int64_t k0, int64_t k1, double *out, double *mu);
int orc_coef_grad(int64_t N, int n, int m, const double *z, const double *y, double *gA, double *gB,
                  double *gg, double *muA, double *muB, double *mug);
int orc_assemble(int64_t nnzk, int64_t dim, const int32_t *rowptr, int64_t nnzj,
                 const int32_t *perm_j, const double *jac, int64_t nnzh, const int32_t *perm_h,
                 const double *hess, const double *reg, double *kkt);
int orc_quad_obj(int64_t N, double r, const double *z, double *out);
int orc_quad_grad(int64_t N, double r, const double *z, double *g, double *mu);
int orc_quad_cons(int64_t N, int bnd, double g, const double *z, double *c, double *mu);
int orc_quad_jac(int64_t N, int bnd, const double *z, double *jac, double *mu);
int orc_quad_hess(int64_t N, double r, const double *z, const double *y, double sigma,
                  double *hess, double *mu);
}

static int g_fail = 0;

static void check(bool ok, const std::string &what)
{
    if (!ok) {
        std::printf("FAIL %s\n", what.c_str());
        g_fail = 1;
    }
}

typedef std::vector<int32_t> iv;
typedef std::vector<double> dv;

struct Kkt {
    iv rowptr, colind, perm_j, perm_h;
};

static std::string tag(int64_t N, int n, int m, int scheme, int bnd)
{
    return "N=" + std::to_string(N) + " n=" + std::to_string(n) + " m=" + std::to_string(m) +
           " scheme=" + std::to_string(scheme) + " bnd=" + std::to_string(bnd);
}

// The library's closed-form structure against the oracle's generic build for
// one shape and option set; also drives the reordering on both sides.
static void structure_case(int64_t N, int n, int m, int scheme, int bnd)
{
    const std::string t = tag(N, n, m, scheme, bnd);
    ocp_options opt{scheme, bnd};
    ocp_sizes_t s;
    int64_t o[10];
    check(ocp_sizes_ex(N, n, m, &opt, &s) == OCP_OK, "sizes " + t);
    check(orc_sizes_ex(N, n, m, scheme, bnd, o) == 0, "oracle sizes " + t);
    check(s.nvar == o[0] && s.ncon == o[1] && s.nnzj == o[2] && s.nnzh == o[3] && s.dim == o[4],
          "sizes agree " + t);
    iv jr(s.nnzj), jc(s.nnzj), hr(s.nnzh), hc(s.nnzh);
    iv ojr(s.nnzj), ojc(s.nnzj), ohr(s.nnzh), ohc(s.nnzh);
    check(ocp_build_pattern_ex(N, n, m, &opt, jr.data(), jc.data(), hr.data(), hc.data()) == OCP_OK,
          "pattern " + t);
    check(orc_pattern_ex(N, n, m, scheme, bnd, ojr.data(), ojc.data(), ohr.data(), ohc.data()) == 0,
          "oracle pattern " + t);
    check(jr == ojr && jc == ojc && hr == ohr && hc == ohc, "pattern bit-exact " + t);
    // one half of the pattern at a time (NULL pairs skipped)
    iv jr2(s.nnzj, -7), jc2(s.nnzj, -7);
    check(ocp_build_pattern_ex(N, n, m, &opt, jr2.data(), jc2.data(), nullptr, nullptr) == OCP_OK,
          "pattern J only " + t);
    check(jr2 == jr && jc2 == jc, "pattern J only equal " + t);

    Kkt L, O;
    L.rowptr.assign(s.dim + 1, -1);
    L.colind.assign(s.nnzk, -1);
    L.perm_j.assign(s.nnzj, -1);
    L.perm_h.assign(s.nnzh, -1);
    check(ocp_build_kkt_ex(N, n, m, &opt, L.rowptr.data(), L.colind.data(), L.perm_j.data(),
                           L.perm_h.data()) == OCP_OK,
          "kkt " + t);
    O.rowptr.assign(s.dim + 1, -1);
    O.colind.assign(s.nnzh + s.nnzj + s.dim, -1);
    O.perm_j.assign(s.nnzj, -1);
    O.perm_h.assign(s.nnzh, -1);
    int64_t nnzk = -1;
    check(orc_kkt_generic(s.nvar, s.ncon, s.nnzj, s.nnzh, ojr.data(), ojc.data(), ohr.data(),
                          ohc.data(), O.rowptr.data(), O.colind.data(), O.perm_j.data(),
                          O.perm_h.data(), &nnzk) == 0,
          "oracle kkt " + t);
    O.colind.resize(nnzk > 0 ? nnzk : 0);
    check(nnzk == s.nnzk, "nnzk " + t);
    check(L.rowptr == O.rowptr && L.colind == O.colind && L.perm_j == O.perm_j &&
              L.perm_h == O.perm_h,
          "kkt bit-exact " + t);
    // partial outputs: slot maps only
    iv pj(s.nnzj, -3), ph(s.nnzh, -3);
    check(ocp_build_kkt_ex(N, n, m, &opt, nullptr, nullptr, pj.data(), ph.data()) == OCP_OK,
          "kkt maps only " + t);
    check(pj == L.perm_j && ph == L.perm_h, "kkt maps only equal " + t);

    // the node-grouped ordering and the symmetric reordering, both sides
    iv order(s.dim, -1);
    check(ocp_stage_order(N, n, m, &opt, order.data()) == OCP_OK, "stage order " + t);
    iv r2(s.dim + 1), c2(s.nnzk), pj2(s.nnzj), ph2(s.nnzh), d2(s.dim);
    iv or2(s.dim + 1), oc2(s.nnzk), opj2(s.nnzj), oph2(s.nnzh), od2(s.dim);
    check(ocp_kkt_permute(s.dim, L.rowptr.data(), L.colind.data(), s.nnzj, L.perm_j.data(),
                          s.nnzh, L.perm_h.data(), order.data(), r2.data(), c2.data(), pj2.data(),
                          ph2.data(), d2.data()) == OCP_OK,
          "kkt permute " + t);
    check(orc_kkt_permute(s.dim, O.rowptr.data(), O.colind.data(), s.nnzj, O.perm_j.data(),
                          s.nnzh, O.perm_h.data(), order.data(), or2.data(), oc2.data(),
                          opj2.data(), oph2.data(), od2.data()) == 0,
          "oracle kkt permute " + t);
    check(r2 == or2 && c2 == oc2 && pj2 == opj2 && ph2 == oph2 && d2 == od2,
          "kkt permute bit-exact " + t);
}

static void quad_case(int64_t N, int bnd)
{
    const std::string t = "quad N=" + std::to_string(N) + " bnd=" + std::to_string(bnd);
    ocp_sizes_t s;
    int64_t o[10];
    check(ocp_quad_sizes(N, bnd, &s) == OCP_OK, "sizes " + t);
    check(orc_quad_sizes(N, bnd, o) == 0, "oracle sizes " + t);
    check(s.nvar == o[0] && s.ncon == o[1] && s.nnzj == o[2] && s.nnzh == o[3], "sizes agree " + t);
    iv jr(s.nnzj), jc(s.nnzj), hr(s.nnzh), hc(s.nnzh);
    iv ojr(s.nnzj), ojc(s.nnzj), ohr(s.nnzh), ohc(s.nnzh);
    check(ocp_quad_pattern(N, bnd, jr.data(), jc.data(), hr.data(), hc.data()) == OCP_OK,
          "pattern " + t);
    check(orc_quad_pattern(N, bnd, ojr.data(), ojc.data(), ohr.data(), ohc.data()) == 0,
          "oracle pattern " + t);
    check(jr == ojr && jc == ojc && hr == ohr && hc == ohc, "pattern bit-exact " + t);
    Kkt L, O;
    L.rowptr.resize(s.dim + 1);
    L.colind.resize(s.nnzk);
    L.perm_j.resize(s.nnzj);
    L.perm_h.resize(s.nnzh);
    check(ocp_quad_kkt(N, bnd, L.rowptr.data(), L.colind.data(), L.perm_j.data(),
                       L.perm_h.data()) == OCP_OK,
          "kkt " + t);
    O.rowptr.resize(s.dim + 1);
    O.colind.resize(s.nnzh + s.nnzj + s.dim);
    O.perm_j.resize(s.nnzj);
    O.perm_h.resize(s.nnzh);
    int64_t nnzk = -1;
    check(orc_kkt_generic(s.nvar, s.ncon, s.nnzj, s.nnzh, ojr.data(), ojc.data(), ohr.data(),
                          ohc.data(), O.rowptr.data(), O.colind.data(), O.perm_j.data(),
                          O.perm_h.data(), &nnzk) == 0,
          "oracle kkt " + t);
    O.colind.resize(nnzk > 0 ? nnzk : 0);
    check(L.rowptr == O.rowptr && L.colind == O.colind && L.perm_j == O.perm_j &&
              L.perm_h == O.perm_h,
          "kkt bit-exact " + t);
    iv order(s.dim);
    check(ocp_quad_stage_order(N, bnd, order.data()) == OCP_OK, "stage order " + t);
    iv r2(s.dim + 1), c2(s.nnzk), d2(s.dim), or2(s.dim + 1), oc2(s.nnzk), od2(s.dim);
    check(ocp_kkt_permute(s.dim, L.rowptr.data(), L.colind.data(), 0, nullptr, 0, nullptr,
                          order.data(), r2.data(), c2.data(), nullptr, nullptr, d2.data()) == OCP_OK,
          "permute " + t);
    iv pj2(s.nnzj), ph2(s.nnzh);
    check(orc_kkt_permute(s.dim, O.rowptr.data(), O.colind.data(), s.nnzj, O.perm_j.data(),
                          s.nnzh, O.perm_h.data(), order.data(), or2.data(), oc2.data(),
                          pj2.data(), ph2.data(), od2.data()) == 0,
          "oracle permute " + t);
    check(r2 == or2 && c2 == oc2 && d2 == od2, "permute bit-exact " + t);
}

// Argument validation: every rejection happens before any output is touched.
static void error_cases()
{
    ocp_sizes_t s;
    check(ocp_sizes(0, 4, 2, &s) == OCP_ERR_ARG, "N=0");
    check(ocp_sizes(10, 0, 2, &s) == OCP_ERR_ARG, "n=0");
    check(ocp_sizes(10, 33, 2, &s) == OCP_ERR_ARG, "n=33");
    check(ocp_sizes(10, 4, -1, &s) == OCP_ERR_ARG, "m=-1");
    check(ocp_sizes(10, 4, 2, nullptr) == OCP_ERR_ARG, "null sizes");
    check(std::strlen(ocp_last_error()) > 0, "message set");
    check(ocp_sizes((int64_t)1 << 31, 1, 0, &s) == OCP_ERR_OVERFLOW, "N=2^31");
    check(ocp_sizes(2700000, 16, 8, &s) == OCP_ERR_OVERFLOW, "int32 overflow");
    ocp_options bad{7, 0};
    check(ocp_sizes_ex(10, 4, 2, &bad, &s) == OCP_ERR_ARG, "bad scheme");
    ocp_options badb{0, 3};
    check(ocp_sizes_ex(10, 4, 2, &badb, &s) == OCP_ERR_ARG, "bad boundary");
    check(ocp_build_kkt(0, 4, 2, nullptr, nullptr, nullptr, nullptr) == OCP_ERR_ARG, "kkt N=0");
    check(ocp_build_pattern(10, 40, 2, nullptr, nullptr, nullptr, nullptr) == OCP_ERR_ARG,
          "pattern n=40");
    check(ocp_stage_order(10, 4, 2, nullptr, nullptr) == OCP_ERR_ARG, "order NULL");
    check(ocp_quad_sizes(0, 1, &s) == OCP_ERR_ARG, "quad N=0");
    check(ocp_quad_sizes(10, 5, &s) == OCP_ERR_ARG, "quad bnd=5");
    // a malformed ordering and a malformed CSR are rejected
    {
        const int64_t N = 6;
        const int n = 3, m = 1;
        check(ocp_sizes(N, n, m, &s) == OCP_OK, "sizes");
        iv rp(s.dim + 1), ci(s.nnzk), pj(s.nnzj), ph(s.nnzh);
        check(ocp_build_kkt(N, n, m, rp.data(), ci.data(), pj.data(), ph.data()) == OCP_OK, "kkt");
        iv order(s.dim);
        for (int64_t x = 0; x < s.dim; x++) order[x] = (int32_t)x;
        order[1] = 0;  // not a permutation
        iv r2(s.dim + 1), c2(s.nnzk);
        check(ocp_kkt_permute(s.dim, rp.data(), ci.data(), 0, nullptr, 0, nullptr, order.data(),
                              r2.data(), c2.data(), nullptr, nullptr, nullptr) == OCP_ERR_ARG,
              "not a permutation");
        order[1] = 1;
        iv rpb = rp;
        rpb[3] = rpb[4] + 1;  // rows out of order
        check(ocp_kkt_permute(s.dim, rpb.data(), ci.data(), 0, nullptr, 0, nullptr, order.data(),
                              r2.data(), c2.data(), nullptr, nullptr, nullptr) == OCP_ERR_ARG,
              "malformed rowptr");
        iv pjb = pj;
        pjb[0] = (int32_t)s.nnzk;  // a slot outside [0, nnzk)
        iv pj2(s.nnzj);
        check(ocp_kkt_permute(s.dim, rp.data(), ci.data(), s.nnzj, pjb.data(), 0, nullptr,
                              order.data(), r2.data(), c2.data(), pj2.data(), nullptr,
                              nullptr) == OCP_ERR_ARG,
              "slot map out of range");
    }
}

// The oracle's value functions on small instances (their values are pinned
// by the Python pin tests; here they only run under the sanitizers).
static void oracle_values(int64_t N, int n, int m, int scheme, int bnd, std::mt19937_64 &rng)
{
    const std::string t = tag(N, n, m, scheme, bnd);
    std::normal_distribution<double> nd(0.0, 1.0);
    int64_t o[10];
    check(orc_sizes_ex(N, n, m, scheme, bnd, o) == 0, "oracle sizes " + t);
    const int64_t nvar = o[0], ncon = o[1], nnzj = o[2], nnzh = o[3], dim = o[4];
    dv A(n * n), B(n * m), g(n), q(n, 1.0), r(m, 0.1), z(nvar), y(ncon), v(nvar);
    for (auto *a : {&A, &B, &g, &z, &y, &v})
        for (double &x : *a) x = nd(rng);
    double f[2];
    dv gr(nvar), gmu(nvar), c(ncon), cmu(ncon), jv(nnzj), jmu(nnzj), hv(nnzh), hmu(nnzh);
    check(orc_obj_ex(N, n, m, scheme, bnd, q.data(), r.data(), z.data(), f) == 0, "obj " + t);
    check(orc_grad_ex(N, n, m, scheme, bnd, q.data(), r.data(), z.data(), gr.data(), gmu.data()) == 0,
          "grad " + t);
    check(orc_cons_ex(N, n, m, scheme, bnd, A.data(), B.data(), g.data(), z.data(), c.data(),
                      cmu.data()) == 0,
          "cons " + t);
    check(orc_jac_ex(N, n, m, scheme, bnd, A.data(), B.data(), g.data(), z.data(), jv.data(),
                     jmu.data()) == 0,
          "jac " + t);
    check(orc_hess_ex(N, n, m, scheme, bnd, A.data(), g.data(), q.data(), r.data(), z.data(),
                      y.data(), 1.0, hv.data(), hmu.data()) == 0,
          "hess " + t);
    bool finite = std::isfinite(f[0]) && std::isfinite(f[1]);
    for (auto *a : {&gr, &c, &jv, &hv})
        for (double x : *a) finite = finite && std::isfinite(x);
    check(finite, "finite values " + t);
    // assembly into the oracle's own KKT structure
    iv jr(nnzj), jc(nnzj), hr(nnzh), hc(nnzh);
    check(orc_pattern_ex(N, n, m, scheme, bnd, jr.data(), jc.data(), hr.data(), hc.data()) == 0,
          "pattern " + t);
    iv rp(dim + 1), ci(nnzh + nnzj + dim), pj(nnzj), ph(nnzh);
    int64_t nnzk = 0;
    check(orc_kkt_generic(nvar, ncon, nnzj, nnzh, jr.data(), jc.data(), hr.data(), hc.data(),
                          rp.data(), ci.data(), pj.data(), ph.data(), &nnzk) == 0,
          "kkt " + t);
    dv reg(dim, 1e-8), kkt(nnzk);
    check(orc_assemble(nnzk, dim, rp.data(), nnzj, pj.data(), jv.data(), nnzh, ph.data(), hv.data(),
                       reg.data(), kkt.data()) == 0,
          "assemble " + t);
    if (scheme == 0 && bnd == 0) {
        double L[2];
        dv lg(nvar), lmu(nvar), hvp(nvar), hvmu(nvar), jvp(ncon), jvmu(ncon);
        dv gA(n * n), gB(n * m), gg(n), mA(n * n), mB(n * m), mg(n);
        check(orc_lagrangian(N, n, m, A.data(), B.data(), g.data(), q.data(), r.data(), z.data(),
                             y.data(), 1.0, L) == 0,
              "lagrangian " + t);
        check(orc_lag_grad(N, n, m, A.data(), B.data(), g.data(), q.data(), r.data(), z.data(),
                           y.data(), 1.0, 0, N + 1, lg.data(), lmu.data()) == 0,
              "lag_grad " + t);
        check(orc_hvp(N, n, m, A.data(), g.data(), q.data(), r.data(), z.data(), y.data(), 1.0,
                      v.data(), 0, N + 1, hvp.data(), hvmu.data()) == 0,
              "hvp " + t);
        check(orc_jvp(N, n, m, A.data(), B.data(), g.data(), z.data(), v.data(), 0, N, jvp.data(),
                      jvmu.data()) == 0,
              "jvp " + t);
        check(orc_coef_grad(N, n, m, z.data(), y.data(), gA.data(), m ? gB.data() : nullptr,
                            gg.data(), mA.data(), m ? mB.data() : nullptr, mg.data()) == 0,
              "coef_grad " + t);
    }
}

static void quad_values(int64_t N, int bnd, std::mt19937_64 &rng)
{
    const std::string t = "quad values N=" + std::to_string(N);
    std::normal_distribution<double> nd(0.0, 0.5);
    int64_t o[10];
    check(orc_quad_sizes(N, bnd, o) == 0, "sizes " + t);
    dv z(o[0]), y(o[1]);
    for (double &x : z) x = nd(rng);
    for (double &x : y) x = nd(rng);
    double f[2];
    dv g(o[0]), gm(o[0]), c(o[1]), cm(o[1]), j(o[2]), jm(o[2]), h(o[3]), hm(o[3]);
    check(orc_quad_obj(N, 0.1, z.data(), f) == 0, "obj " + t);
    check(orc_quad_grad(N, 0.1, z.data(), g.data(), gm.data()) == 0, "grad " + t);
    check(orc_quad_cons(N, bnd, 9.8, z.data(), c.data(), cm.data()) == 0, "cons " + t);
    check(orc_quad_jac(N, bnd, z.data(), j.data(), jm.data()) == 0, "jac " + t);
    check(orc_quad_hess(N, 0.1, z.data(), y.data(), 1.0, h.data(), hm.data()) == 0, "hess " + t);
}

int main()
{
    const int shapes[][3] = {{1, 1, 0}, {1, 1, 1}, {2, 1, 0}, {3, 2, 0}, {2, 2, 1}, {5, 3, 0},
                             {4, 3, 1}, {3, 4, 2}, {7, 5, 3}, {10, 6, 3}, {1, 16, 8}, {33, 16, 8},
                             {17, 32, 32}, {257, 4, 2}, {65, 8, 4}};
    int cases = 0;
    for (auto &sh : shapes)
        for (int scheme = 0; scheme < 2; scheme++)
            for (int bnd = 0; bnd < 3; bnd++) {
                structure_case(sh[0], sh[1], sh[2], scheme, bnd);
                cases++;
            }
    for (int64_t N : {1, 2, 7, 64})
        for (int bnd = 0; bnd < 3; bnd++) {
            quad_case(N, bnd);
            cases++;
        }
    error_cases();
    std::mt19937_64 rng(5);
    for (auto &sh : shapes)
        for (int scheme = 0; scheme < 2; scheme++)
            for (int bnd = 0; bnd < 3; bnd += 2) oracle_values(sh[0], sh[1], sh[2], scheme, bnd, rng);
    for (int64_t N : {1, 5, 40}) quad_values(N, 1, rng);
    std::printf("%s: %d structure cases\n", g_fail ? "FAILED" : "ok", cases);
    return g_fail;
}
