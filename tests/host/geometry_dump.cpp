// Writes the host-side 15-point stencils of a general macro mesh as raw
// files, for comparison with the oracle's assembled matrices (test use only).
//   geometry_dump n_sub level coarse_level vertices.f64 out_dir
// vertices.f64: (n+1)^3 x 3 doubles, x fastest.  Per level l:
//   l<l>_X.i32 (interface grid positions), l<l>_sid.i32, l<l>_wtab.f64,
//   l<l>_w15.f64, and the mass stencils l<l>_mwtab.f64, l<l>_mw15.f64;
//   coarse: c_pos.i32, c_col15.i32, c_val15.f64;
//   tets.i32 (V0 and axis order per macro tetrahedron).
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../paper_1506_06185_amd/csrc/geometry.hpp"
#include "../../paper_1506_06185_amd/csrc/topology.hpp"

using namespace hhgr;

template <typename T>
static bool put(const std::string &path, const T *p, size_t n) {
    FILE *f = std::fopen(path.c_str(), "wb");
    if (!f) return false;
    const bool ok = std::fwrite(p, sizeof(T), n, f) == n;
    std::fclose(f);
    return ok;
}

int main(int argc, char **argv) {
    if (argc != 6) {
        std::printf("usage: geometry_dump n_sub level coarse_level vertices.f64 out_dir\n");
        return 2;
    }
    const int n = std::atoi(argv[1]), L = std::atoi(argv[2]), Lc = std::atoi(argv[3]);
    const std::string out = argv[5];
    Topology tp;
    std::string e = tp.build(n, L, Lc);
    if (!e.empty()) {
        std::printf("topology: %s\n", e.c_str());
        return 1;
    }
    const size_t nv = 3 * (size_t)(n + 1) * (n + 1) * (n + 1);
    std::vector<double> xyz(nv);
    FILE *f = std::fopen(argv[4], "rb");
    if (!f || std::fread(xyz.data(), sizeof(double), nv, f) != nv) {
        std::printf("cannot read vertices\n");
        return 1;
    }
    std::fclose(f);
    e = check_macro_mesh(tp, xyz.data());
    if (!e.empty()) {
        std::printf("mesh: %s\n", e.c_str());
        return 1;
    }
    bool ok = true;
    for (int l = Lc; l <= L; l++) {
        LevelStencils G;
        e = level_stencils(tp, xyz.data(), l, 1 + 14 * tp.n_tets, G);
        if (!e.empty()) {
            std::printf("level %d: %s\n", l, e.c_str());
            return 1;
        }
        const TopoLevel &T = tp.lev[l];
        const std::string p = out + "/l" + std::to_string(l) + "_";
        ok = ok && put(p + "X.i32", &T.ifc_X[0][0], 3 * T.ifc_X.size());
        ok = ok && put(p + "sid.i32", G.sid.data(), G.sid.size());
        ok = ok && put(p + "wtab.f64", G.wtab.data(), G.wtab.size());
        ok = ok && put(p + "w15.f64", G.w15.data(), G.w15.size());
        ok = ok && put(p + "mwtab.f64", G.mwtab.data(), G.mwtab.size());
        ok = ok && put(p + "mw15.f64", G.mw15.data(), G.mw15.size());
        std::printf("level %d: %d interface masters, %zu distinct stencils\n", l, T.n_ifc, G.wtab.size() / 15);
    }
    std::vector<double> cval;
    coarse_stencils(tp, xyz.data(), cval);
    ok = ok && put(out + "/c_pos.i32", &tp.coarse.pos[0][0], 3 * tp.coarse.pos.size());
    ok = ok && put(out + "/c_col15.i32", tp.coarse.col15.data(), tp.coarse.col15.size());
    ok = ok && put(out + "/c_val15.f64", cval.data(), cval.size());
    std::vector<int> tets;
    for (int t = 0; t < tp.n_tets; t++)
        for (int a = 0; a < 3; a++) tets.push_back(tp.V0[t][a]);
    for (int t = 0; t < tp.n_tets; t++)
        for (int a = 0; a < 3; a++) tets.push_back(tp.perm[t][a]);
    ok = ok && put(out + "/tets.i32", tets.data(), tets.size());
    if (!ok) {
        std::printf("write failed\n");
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
