// Writes the dense inverse of the coarsest-level operator that the library
// factorises on the host for k = 1 (the cube's 7-point operator, or with a
// vertex file the 15-point operator of that general macro mesh), with the
// grid position of every coarse unknown, for comparison with the inverse of
// the oracle's own coarsest-level matrix (test use only).
//   coarse_inverse_dump n_sub out_dir [vertices.f64]
//     -> pos.i32 (n x 3), inv.f64 (n x n)
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../paper_1506_06185_amd/csrc/geometry.hpp"
#include "../../paper_1506_06185_amd/csrc/topology.hpp"

using namespace hhgr;

int main(int argc, char **argv) {
    if (argc != 3 && argc != 4) {
        std::printf("usage: coarse_inverse_dump n_sub out_dir [vertices.f64]\n");
        return 2;
    }
    const int n_sub = std::atoi(argv[1]);
    Topology tp;
    const std::string e = tp.build(n_sub, 3, 2);
    if (!e.empty()) {
        std::printf("topology: %s\n", e.c_str());
        return 1;
    }
    const CoarseSystem &cs = tp.coarse;
    std::vector<double> inv;
    bool ok = true;
    if (argc == 4) {
        const size_t nv = 3 * (size_t)(n_sub + 1) * (n_sub + 1) * (n_sub + 1);
        std::vector<double> xyz(nv);
        FILE *fv = std::fopen(argv[3], "rb");
        ok = fv && std::fread(xyz.data(), sizeof(double), nv, fv) == nv;
        if (fv) std::fclose(fv);
        if (!ok || !check_macro_mesh(tp, xyz.data()).empty()) {
            std::printf("bad vertices\n");
            return 1;
        }
        std::vector<double> cval;
        coarse_stencils(tp, xyz.data(), cval);
        ok = coarse_inverse(cs.n, 15, cs.col15, cval, inv);
    } else {
        ok = coarse_inverse(cs.n, 7, cs.col, cs.val, inv);
    }
    if (!ok) {
        std::printf("not positive definite\n");
        return 1;
    }
    const std::string out = argv[2];
    FILE *f = std::fopen((out + "/pos.i32").c_str(), "wb");
    ok = f && std::fwrite(&cs.pos[0][0], sizeof(int), 3 * (size_t)cs.n, f) == 3 * (size_t)cs.n;
    if (f) std::fclose(f);
    f = std::fopen((out + "/inv.f64").c_str(), "wb");
    ok = ok && f && std::fwrite(inv.data(), sizeof(double), inv.size(), f) == inv.size();
    if (f) std::fclose(f);
    std::printf(ok ? "n=%d ok\n" : "n=%d write failed\n", cs.n);
    return ok ? 0 : 1;
}
