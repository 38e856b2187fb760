// Host-logic check of the engine (contexts, faults, recoveries, batches with
// armed Dirichlet-Dirichlet recoveries, graph bookkeeping) against the mock
// HIP runtime, under AddressSanitizer: the numerical kernels are skipped, so
// this checks control flow, table sizes and host memory use only.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/hhgr.h"

extern int g_mock_captures, g_mock_launches;
extern double g_mock_res2;
static int fails = 0;
static long long nd_vk(hhgr_ctx *c) {
    long long n = 0;
    hhgr_sizes(c, &n, nullptr, nullptr);
    return n;
}
#define CHECK(c, ...)                          \
    do {                                       \
        if (!(c)) {                            \
            std::printf("FAIL: " __VA_ARGS__); \
            std::printf("\n");                 \
            fails++;                           \
        }                                      \
    } while (0)

struct Ctx {
    hhgr_ctx *h = nullptr;
    void *ws = nullptr;
    long long ndof = 0;
    std::vector<double> vec;
};

static Ctx make(int n_sub, int level, int precision) {
    Ctx c;
    hhgr_desc d;
    hhgr_desc_default(&d);
    d.n_sub = n_sub;
    d.level = level;
    d.precision = precision;
    size_t bytes = 0;
    CHECK(hhgr_workspace_bytes(&d, &bytes) == HHGR_OK, "workspace bytes");
    c.ws = std::aligned_alloc(256, (bytes + 255) / 256 * 256);
    CHECK(hhgr_create(&d, c.ws, bytes, nullptr, &c.h) == HHGR_OK, "create: %s", hhgr_last_error());
    int nt = 0;
    long long ne = 0;
    hhgr_sizes(c.h, &c.ndof, &nt, &ne);
    c.vec.assign(c.ndof, 1.0);
    CHECK(hhgr_set_rhs(c.h, c.vec.data(), HHGR_RHS_LOAD) == HHGR_OK, "set_rhs");
    return c;
}

int main() {
    g_mock_res2 = 1.0;  // every residual norm is 1: members never converge
    std::vector<Ctx> cs;
    cs.push_back(make(2, 5, HHGR_FP64));
    cs.push_back(make(2, 4, HHGR_FP64));
    cs.push_back(make(1, 5, HHGR_FP64));
    cs.push_back(make(1, 4, HHGR_MIXED));
    double rr = 0;
    CHECK(hhgr_vcycle(cs[0].h, 2, &rr) == HHGR_OK, "vcycle");
    int t2[2] = {3, 17};
    for (int t : t2) CHECK(hhgr_inject_fault(cs[0].h, t) == HHGR_OK, "inject");
    CHECK(hhgr_recover_dd(cs[0].h, t2, 2, 2, 3) == HHGR_OK, "recover_dd: %s", hhgr_last_error());
    CHECK(hhgr_recover_local(cs[1].h, 5, 2, &rr) == HHGR_OK, "recover_local");
    for (int t : t2) hhgr_inject_fault(cs[0].h, t);
    CHECK(hhgr_recover_dn(cs[0].h, t2, 2, 3, 2) == HHGR_OK, "recover_dn: %s", hhgr_last_error());
    CHECK(hhgr_recover_dn(cs[0].h, t2, 2, -1, 2) == HHGR_EINVAL, "recover_dn bad count");
    CHECK(hhgr_vcycle(cs[0].h, 1, &rr) == HHGR_OK, "vcycle after dn");
    for (int t : t2) hhgr_inject_fault(cs[0].h, t);
    int t1 = 4;
    hhgr_inject_fault(cs[2].h, t1);
    std::vector<hhgr_ctx *> hs;
    for (auto &c : cs) hs.push_back(c.h);
    hhgr_batch *b = nullptr;
    CHECK(hhgr_batch_create(hs.data(), (int)hs.size(), nullptr, &b) == HHGR_OK, "batch create");
    CHECK(hhgr_batch_arm_dd(b, 0, t2, 2, 2, 4) == HHGR_OK, "arm 0: %s", hhgr_last_error());
    CHECK(hhgr_batch_arm_dd(b, 2, &t1, 1, 0, 3) == HHGR_OK, "arm 2: %s", hhgr_last_error());
    CHECK(hhgr_batch_arm_dd(b, 4, &t1, 1, 0, 3) == HHGR_EINVAL, "arm out of range");
    std::vector<std::vector<double>> hist(cs.size(), std::vector<double>(31));
    std::vector<hhgr_report> reps(cs.size());
    for (size_t q = 0; q < cs.size(); q++) reps[q] = hhgr_report{0, 0.0, hist[q].data(), 31};
    const int launches0 = g_mock_launches;
    // unit residuals: nobody converges, every member runs max_cycles = 5 cycles;
    // member 2 (local recovery only) has one extra step that is not a cycle
    int rc = hhgr_batch_run(b, 1e-10, 5, reps.data());
    CHECK(rc == HHGR_ENOCONV, "batch run: %d %s", rc, hhgr_last_error());
    for (int q = 0; q < 4; q++) CHECK(reps[q].cycles == 5, "member %d cycles %d", q, reps[q].cycles);
    CHECK(g_mock_launches - launches0 == 6, "graph launches %d", g_mock_launches - launches0);
    // zero residuals: the recovering members take their forced steps, the others none
    g_mock_res2 = 0.0;
    for (int t : t2) hhgr_inject_fault(cs[0].h, t);
    CHECK(hhgr_batch_arm_dd(b, 0, t2, 2, 2, 4) == HHGR_OK, "re-arm 0");
    rc = hhgr_batch_run(b, 1e-10, 30, reps.data());
    CHECK(rc == HHGR_OK, "batch run 2: %d %s", rc, hhgr_last_error());
    CHECK(reps[0].cycles == 2 && reps[1].cycles == 0 && reps[2].cycles == 0, "forced steps only");
    hhgr_batch_destroy(b);
    CHECK(hhgr_set_graph(cs[1].h, 1) == HHGR_OK, "graph on");
    CHECK(hhgr_vcycle(cs[1].h, 3, &rr) == HHGR_OK, "graph vcycle");
    CHECK(hhgr_set_tuning(cs[1].h, 0, 512, 0, 4) == HHGR_OK, "tuning");
    CHECK(hhgr_set_tuning(cs[1].h, 0, 100, 0, 4) == HHGR_EINVAL, "bad tuning");
    CHECK(hhgr_autotune(cs[1].h, nullptr) == HHGR_OK, "autotune");
    {
        // general macro mesh: stencils from moved vertices, cycles and recoveries
        g_mock_res2 = 1.0;
        hhgr_desc d;
        hhgr_desc_default(&d);
        d.n_sub = 2;
        d.level = 5;
        d.general_geometry = 1;
        hhgr_desc bad = d;
        bad.general_geometry = 2;
        size_t bytes = 0;
        CHECK(hhgr_workspace_bytes(&bad, &bytes) == HHGR_EINVAL, "general_geometry 2 rejected");
        bad = d;
        bad.precision = HHGR_MIXED;
        CHECK(hhgr_workspace_bytes(&bad, &bytes) == HHGR_OK, "general + mixed sized");
        CHECK(hhgr_workspace_bytes(&d, &bytes) == HHGR_OK, "general workspace");
        void *ws = std::aligned_alloc(256, (bytes + 255) / 256 * 256);
        hhgr_ctx *g = nullptr;
        CHECK(hhgr_create(&d, ws, bytes, nullptr, &g) == HHGR_OK, "general create: %s", hhgr_last_error());
        long long nd = 0;
        hhgr_sizes(g, &nd, nullptr, nullptr);
        std::vector<double> v(nd, 1.0), w(nd, 0.0);
        CHECK(hhgr_set_rhs(g, v.data(), HHGR_RHS_LOAD) == HHGR_OK, "general rhs");
        CHECK(hhgr_set_rhs(g, v.data(), HHGR_RHS_NODAL_F) == HHGR_ESTATE, "general nodal f needs geometry");
        CHECK(hhgr_vcycle(g, 1, &rr) == HHGR_ESTATE, "no geometry yet");
        std::vector<double> xyz;
        for (int z = 0; z <= 2; z++)
            for (int y = 0; y <= 2; y++)
                for (int x = 0; x <= 2; x++) {
                    const double j = 0.03 * std::sin(1.0 + x + 3.0 * y + 7.0 * z);
                    xyz.push_back(x / 2.0 + j);
                    xyz.push_back(y / 2.0 - j);
                    xyz.push_back(z / 2.0 + 0.5 * j);
                }
        CHECK(hhgr_set_geometry(cs[1].h, xyz.data()) == HHGR_ESTATE, "geometry needs a general context");
        CHECK(hhgr_set_geometry(g, xyz.data()) == HHGR_OK, "set geometry: %s", hhgr_last_error());
        CHECK(hhgr_vcycle(g, 2, &rr) == HHGR_OK, "general vcycle");
        CHECK(hhgr_set_graph(g, 1) == HHGR_OK, "general graph on");
        CHECK(hhgr_vcycle(g, 2, &rr) == HHGR_OK, "general graph vcycle");
        CHECK(hhgr_recover_local(g, 5, 2, &rr) == HHGR_OK, "general recover_local: %s", hhgr_last_error());
        CHECK(hhgr_recover_dd(g, t2, 2, 2, 3) == HHGR_OK, "general recover_dd: %s", hhgr_last_error());
        CHECK(hhgr_recover_dn(g, t2, 2, 2, 1) == HHGR_OK, "general dn: %s", hhgr_last_error());
        CHECK(hhgr_mass_apply(g, v.data(), w.data()) == HHGR_OK, "general mass: %s", hhgr_last_error());
        CHECK(hhgr_set_rhs(g, v.data(), HHGR_RHS_NODAL_F) == HHGR_OK, "general nodal f: %s", hhgr_last_error());
        CHECK(hhgr_autotune(g, nullptr) == HHGR_OK, "general autotune: %s", hhgr_last_error());
        CHECK(hhgr_debug_op(g, 0, 5, v.data(), v.data(), w.data()) == HHGR_OK, "general residual op");
        CHECK(hhgr_debug_op(g, 1, 5, v.data(), v.data(), w.data()) == HHGR_EINVAL, "general op 1 rejected");
        CHECK(hhgr_debug_op(g, 8 + 5, 5, v.data(), v.data(), w.data()) == HHGR_OK, "general class op");
        CHECK(hhgr_debug_op(g, 24, 5, v.data(), v.data(), w.data()) == HHGR_EINVAL, "op 24 rejected");
        CHECK(hhgr_debug_op(g, 6, 2, v.data(), v.data(), w.data()) == HHGR_OK, "general coarse op");
        xyz[3 * 13] = 5.0;  // centre vertex pulled far outside: inverted tetrahedra
        CHECK(hhgr_set_geometry(g, xyz.data()) == HHGR_EINVAL, "inverted mesh rejected");
        hhgr_ctx *pair[2] = {g, cs[1].h};
        hhgr_batch *gb = nullptr;
        CHECK(hhgr_batch_create(pair, 2, nullptr, &gb) == HHGR_OK, "general batch");
        rc = hhgr_batch_run(gb, 1e-10, 3, nullptr);
        CHECK(rc == HHGR_ENOCONV, "general batch run: %d %s", rc, hhgr_last_error());
        hhgr_batch_destroy(gb);
        hhgr_destroy(g);
        std::free(ws);
        {
            // mixed precision: FP32 copies of the stencil tables
            xyz[3 * 13] = 0.5;  // the centre vertex back inside
            hhgr_desc dm = d;
            dm.precision = HHGR_MIXED;
            size_t bm = 0;
            CHECK(hhgr_workspace_bytes(&dm, &bm) == HHGR_OK, "general mixed workspace");
            void *wm = std::aligned_alloc(256, (bm + 255) / 256 * 256);
            hhgr_ctx *gm = nullptr;
            CHECK(hhgr_create(&dm, wm, bm, nullptr, &gm) == HHGR_OK, "general mixed create: %s", hhgr_last_error());
            CHECK(hhgr_set_geometry(gm, xyz.data()) == HHGR_OK, "general mixed geometry");
            CHECK(hhgr_set_rhs(gm, v.data(), HHGR_RHS_LOAD) == HHGR_OK, "general mixed rhs");
            CHECK(hhgr_vcycle(gm, 2, &rr) == HHGR_OK, "general mixed vcycle: %s", hhgr_last_error());
            CHECK(hhgr_recover_dd(gm, t2, 2, 1, 2) == HHGR_OK, "general mixed dd: %s", hhgr_last_error());
            hhgr_destroy(gm);
            std::free(wm);
        }
        // variable coefficient: weights once both the geometry and k are set
        d.variable_coeff = 1;
        CHECK(hhgr_workspace_bytes(&d, &bytes) == HHGR_OK, "general vk workspace");
        ws = std::aligned_alloc(256, (bytes + 255) / 256 * 256);
        CHECK(hhgr_create(&d, ws, bytes, nullptr, &g) == HHGR_OK, "general vk create: %s", hhgr_last_error());
        long long ne = 0;
        hhgr_sizes(g, nullptr, nullptr, &ne);
        std::vector<double> k(ne, 1.5), gdat(33 * 33 * 33, 0.25);
        xyz[3 * 13] = 0.5;
        CHECK(hhgr_set_rhs(g, gdat.data(), HHGR_RHS_DIRICHLET) == HHGR_ESTATE, "vk Dirichlet needs k");
        CHECK(hhgr_set_coeff(g, k.data()) == HHGR_OK, "general vk coeff: %s", hhgr_last_error());
        CHECK(hhgr_set_rhs(g, gdat.data(), HHGR_RHS_DIRICHLET) == HHGR_ESTATE, "Dirichlet needs geometry");
        CHECK(hhgr_set_geometry(g, xyz.data()) == HHGR_OK, "general vk geometry: %s", hhgr_last_error());
        CHECK(hhgr_set_rhs(g, gdat.data(), HHGR_RHS_DIRICHLET) == HHGR_OK, "general Dirichlet: %s", hhgr_last_error());
        CHECK(hhgr_vcycle(g, 2, &rr) == HHGR_OK, "general vk vcycle");
        CHECK(hhgr_recover_local(g, 7, 2, &rr) == HHGR_OK, "general vk recover_local");
        CHECK(hhgr_recover_dd(g, t2, 2, 1, 2) == HHGR_OK, "general vk recover_dd: %s", hhgr_last_error());
        CHECK(hhgr_recover_dn(g, t2, 2, 2, 2) == HHGR_OK, "general vk recover_dn: %s", hhgr_last_error());
        {
            std::vector<double> gg(nd_vk(g), 0.5), dfv(nd_vk(g)), dkv(ne);
            CHECK(hhgr_adjoint_grad(g, gg.data(), 1e-10, 5, dfv.data(), dkv.data()) == HHGR_ENOCONV,
                  "general adjoint runs (mock residuals never converge): %s", hhgr_last_error());
        }
        CHECK(hhgr_set_coeff(g, k.data()) == HHGR_OK, "general vk coeff again");
        hhgr_destroy(g);
        std::free(ws);
    }
    {
        // the solve in the static scratch: two calls, the second smaller,
        // and a problem too large for the scratch
        hhgr_desc d;
        hhgr_desc_default(&d);
        d.n_sub = 2;
        d.level = 5;
        std::vector<double> rhs(31 * 31 * 31, 1.0), u(31 * 31 * 31, 7.0), hist(11);
        hhgr_report rep{0, 0.0, hist.data(), 11};
        // (mock residuals never converge)
        CHECK(hhgr_solve_static(&d, rhs.data(), HHGR_RHS_LOAD, 1e-8, 10, u.data(), &rep, nullptr) == HHGR_ENOCONV,
              "static solve: %s", hhgr_last_error());
        CHECK(rep.cycles == 10, "static solve report");
        d.n_sub = 1;
        d.level = 4;
        CHECK(hhgr_solve_static(&d, rhs.data(), HHGR_RHS_NODAL_F, 1e-8, 10, u.data(), &rep, nullptr) == HHGR_ENOCONV,
              "static solve, smaller: %s", hhgr_last_error());
        d.n_sub = 2;
        d.level = 7;
        CHECK(hhgr_solve_static(&d, rhs.data(), HHGR_RHS_LOAD, 1e-8, 10, u.data(), &rep, nullptr) == HHGR_EINVAL,
              "static solve too large rejected");
        d.level = 4;
        d.variable_coeff = 1;
        CHECK(hhgr_solve_static(&d, rhs.data(), HHGR_RHS_LOAD, 1e-8, 10, u.data(), &rep, nullptr) == HHGR_EINVAL,
              "static solve with variable k rejected");
    }
    {
        // unstructured macro mesh: the octahedron |x|+|y|+|z| <= 1 as 8
        // tetrahedra around its centre (colours: centre 0, poles 1, equator
        // vertices 2 and 3 alternately)
        const double vx[7][3] = {{0, 0, 0}, {0, 0, 1}, {0, 0, -1}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0}};
        std::vector<double> xyz;
        for (auto &p : vx)
            for (double c : p) xyz.push_back(c + 0.01 * c * c);
        std::vector<int> tv;
        for (int pole = 1; pole <= 2; pole++)
            for (int i = 0; i < 4; i++) {
                const int a = 3 + i, b = 3 + (i + 1) % 4;
                tv.insert(tv.end(), {0, pole, i % 2 ? b : a, i % 2 ? a : b});
            }
        hhgr_desc d;
        hhgr_desc_default(&d);
        d.level = 4;
        d.n_sub = 99;  // ignored for a mesh
        size_t bytes = 0;
        CHECK(hhgr_mesh_workspace_bytes(&d, 7, xyz.data(), 8, tv.data(), &bytes) == HHGR_OK, "mesh workspace: %s",
              hhgr_last_error());
        void *ws = std::aligned_alloc(256, (bytes + 255) / 256 * 256);
        hhgr_ctx *g = nullptr;
        CHECK(hhgr_create_mesh(&d, 7, xyz.data(), 8, tv.data(), ws, bytes, nullptr, &g) == HHGR_OK, "mesh create: %s",
              hhgr_last_error());
        long long nd = 0, ne = 0;
        int nt = 0;
        hhgr_sizes(g, &nd, &nt, &ne);
        // interior nodes at m = 16: the centre, 6 interior edges x 15,
        // 12 interior faces x 105, 8 x 455 tetrahedron interiors
        CHECK(nd == 1 + 6 * 15 + 12 * 105 + 8 * 455 && nt == 8 && ne == 8LL * 4096, "mesh sizes %lld %d %lld", nd, nt,
              ne);
        std::vector<double> v(nd, 1.0), w(nd, 0.0);
        double rr = 0;
        long long nb = 0;
        CHECK(hhgr_mesh_boundary(g, &nb, nullptr) == HHGR_OK && nb > 0, "mesh boundary count");
        std::vector<double> bx(3 * nb), gbv(nb, 1.0);
        CHECK(hhgr_mesh_boundary(g, &nb, bx.data()) == HHGR_OK, "mesh boundary positions");
        CHECK(hhgr_mesh_boundary(cs[1].h, &nb, nullptr) == HHGR_EINVAL, "cube has no mesh boundary list");
        CHECK(hhgr_set_rhs(g, gbv.data(), HHGR_RHS_DIRICHLET) == HHGR_OK, "mesh Dirichlet data: %s", hhgr_last_error());
        CHECK(hhgr_set_rhs(g, v.data(), HHGR_RHS_NODAL_F) == HHGR_OK, "mesh nodal f: %s", hhgr_last_error());
        CHECK(hhgr_set_rhs(g, v.data(), HHGR_RHS_LOAD) == HHGR_OK, "mesh rhs: %s", hhgr_last_error());
        CHECK(hhgr_set_solution(g, v.data()) == HHGR_OK, "mesh set solution");
        CHECK(hhgr_get_solution(g, w.data()) == HHGR_OK, "mesh get solution");
        CHECK(hhgr_vcycle(g, 2, &rr) == HHGR_OK, "mesh vcycle: %s", hhgr_last_error());
        CHECK(hhgr_set_graph(g, 1) == HHGR_OK, "mesh graph on");
        CHECK(hhgr_vcycle(g, 2, &rr) == HHGR_OK, "mesh graph vcycle");
        CHECK(hhgr_inject_fault(g, 3) == HHGR_OK, "mesh fault");
        CHECK(hhgr_recover_local(g, 3, 2, &rr) == HHGR_OK, "mesh recover_local: %s", hhgr_last_error());
        const int t2[2] = {1, 6};
        CHECK(hhgr_recover_dd(g, t2, 2, 2, 3) == HHGR_OK, "mesh dd: %s", hhgr_last_error());
        CHECK(hhgr_vcycle(g, 1, &rr) == HHGR_OK, "mesh vcycle after dd");
        CHECK(hhgr_recover_dn(g, t2, 2, 2, 1) == HHGR_OK, "mesh dn: %s", hhgr_last_error());
        CHECK(hhgr_vcycle(g, 1, &rr) == HHGR_OK, "mesh vcycle after dn");
        {
            // a coefficient per tetrahedron, with recoveries over it, then k = 1 again
            const double kt[8] = {1.0, 2.0, 0.5, 3.0, 1.5, 4.0, 0.25, 1.0};
            CHECK(hhgr_mesh_set_coeff(g, kt) == HHGR_OK, "mesh coeff: %s", hhgr_last_error());
            CHECK(hhgr_vcycle(g, 1, &rr) == HHGR_OK, "mesh vcycle with k");
            CHECK(hhgr_recover_dd(g, t2, 2, 1, 2) == HHGR_OK, "mesh dd with k: %s", hhgr_last_error());
            CHECK(hhgr_recover_dn(g, t2, 2, 1, 1) == HHGR_OK, "mesh dn with k: %s", hhgr_last_error());
            CHECK(hhgr_set_rhs(g, gbv.data(), HHGR_RHS_DIRICHLET) == HHGR_OK, "mesh Dirichlet with k");
            const double bad[8] = {1.0, 2.0, 0.0, 3.0, 1.5, 4.0, 0.25, 1.0};
            CHECK(hhgr_mesh_set_coeff(g, bad) == HHGR_EINVAL, "mesh coeff zero rejected");
            CHECK(hhgr_mesh_set_coeff(cs[0].h, kt) == HHGR_EINVAL, "cube takes no mesh coefficient");
            CHECK(hhgr_mesh_set_coeff(g, nullptr) == HHGR_OK, "mesh coeff reset: %s", hhgr_last_error());
        }
        {
            // a batch of the mesh member (armed DD) and a cube member
            hhgr_ctx *bm[2] = {g, cs[1].h};
            hhgr_batch *mb = nullptr;
            CHECK(hhgr_batch_create(bm, 2, nullptr, &mb) == HHGR_OK, "mesh batch: %s", hhgr_last_error());
            CHECK(hhgr_inject_fault(g, 1) == HHGR_OK && hhgr_inject_fault(g, 6) == HHGR_OK, "mesh batch faults");
            CHECK(hhgr_batch_arm_dd(mb, 0, t2, 2, 2, 3) == HHGR_OK, "mesh batch arm: %s", hhgr_last_error());
            std::vector<double> h0(8), h1(8);
            hhgr_report mr[2] = {{0, 0.0, h0.data(), 8}, {0, 0.0, h1.data(), 8}};
            const int mrc = hhgr_batch_run(mb, 1e-10, 4, mr);
            CHECK(mrc == HHGR_OK || mrc == HHGR_ENOCONV, "mesh batch run: %d %s", mrc, hhgr_last_error());
            hhgr_batch_destroy(mb);
        }
        CHECK(hhgr_mass_apply(g, v.data(), w.data()) == HHGR_OK, "mesh mass: %s", hhgr_last_error());
        CHECK(hhgr_adjoint_grad(g, v.data(), 1e-10, 5, w.data(), nullptr) == HHGR_ENOCONV, "mesh adjoint: %s",
              hhgr_last_error());
        {
            std::vector<double> gk(8);
            const int arc = hhgr_adjoint_grad(g, v.data(), 1e-10, 5, w.data(), gk.data());
            CHECK(arc == HHGR_OK || arc == HHGR_ENOCONV, "mesh dJ/dk per tetrahedron: %s", hhgr_last_error());
        }
        CHECK(hhgr_autotune(g, nullptr) == HHGR_OK, "mesh autotune: %s", hhgr_last_error());
        CHECK(hhgr_set_fused_sweeps(g, 4, 1) == HHGR_EINVAL, "mesh fused sweeps rejected");
        CHECK(hhgr_set_fused_sweeps(cs[0].h, 5, 1) == HHGR_OK, "cube fused sweeps: %s", hhgr_last_error());
        CHECK(hhgr_vcycle(cs[0].h, 1, &rr) == HHGR_OK, "cube fused vcycle");
        CHECK(hhgr_set_fused_sweeps(cs[0].h, 5, 0) == HHGR_OK, "cube fused sweeps off");
        CHECK(hhgr_set_fused_sweeps(cs[0].h, 2, 1) == HHGR_EINVAL, "fused sweeps on the coarsest level rejected");
        CHECK(hhgr_set_geometry(g, xyz.data()) == HHGR_EINVAL, "mesh geometry rejected");
        CHECK(hhgr_debug_op(g, 0, 4, v.data(), v.data(), w.data()) == HHGR_OK, "mesh residual op");
        CHECK(hhgr_debug_op(g, 8 + 6, 4, v.data(), v.data(), w.data()) == HHGR_OK, "mesh class op");
        CHECK(hhgr_debug_op(g, 4, 4, v.data(), v.data(), w.data()) == HHGR_OK, "mesh restrict op");
        CHECK(hhgr_debug_op(g, 5, 4, v.data(), v.data(), w.data()) == HHGR_OK, "mesh prolong op");
        CHECK(hhgr_debug_op(g, 7, 2, v.data(), v.data(), w.data()) == HHGR_OK, "mesh dense coarse op");
        CHECK(hhgr_debug_op(g, 6, 2, v.data(), v.data(), w.data()) == HHGR_EINVAL, "mesh pcg op rejected");
        hhgr_destroy(g);
        std::free(ws);
        d.precision = HHGR_MIXED;
        CHECK(hhgr_mesh_workspace_bytes(&d, 7, xyz.data(), 8, tv.data(), &bytes) == HHGR_OK, "mixed mesh workspace");
        ws = std::aligned_alloc(256, (bytes + 255) / 256 * 256);
        CHECK(hhgr_create_mesh(&d, 7, xyz.data(), 8, tv.data(), ws, bytes, nullptr, &g) == HHGR_OK,
              "mixed mesh create: %s", hhgr_last_error());
        CHECK(hhgr_set_rhs(g, v.data(), HHGR_RHS_LOAD) == HHGR_OK, "mixed mesh rhs");
        CHECK(hhgr_vcycle(g, 2, &rr) == HHGR_OK, "mixed mesh vcycle: %s", hhgr_last_error());
        CHECK(hhgr_recover_dd(g, t2, 2, 1, 2) == HHGR_OK, "mixed mesh dd: %s", hhgr_last_error());
        hhgr_destroy(g);
        std::free(ws);
        d.precision = HHGR_FP64;
        std::swap(tv[2], tv[3]);  // first tetrahedron's colours inconsistent
        CHECK(hhgr_mesh_workspace_bytes(&d, 7, xyz.data(), 8, tv.data(), &bytes) == HHGR_EINVAL, "bad colouring");
        std::swap(tv[2], tv[3]);
        d.variable_coeff = 1;
        CHECK(hhgr_mesh_workspace_bytes(&d, 7, xyz.data(), 8, tv.data(), &bytes) == HHGR_EINVAL, "mesh vk rejected");
    }
    for (auto &c : cs) {
        hhgr_destroy(c.h);
        std::free(c.ws);
    }
    std::printf("engine_host_check: %s (%d failures)\n", fails ? "FAILED" : "ok", fails);
    return fails ? 1 : 0;
}
