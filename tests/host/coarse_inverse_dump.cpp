// Writes the dense inverse of the coarsest-level operator that hhgr_create
// factorises on the host (k = 1 on the cube), with the grid position of
// every coarse unknown, for comparison with the inverse of the oracle's own
// coarsest-level matrix (test use only).
//   coarse_inverse_dump n_sub out_dir  ->  pos.i32 (n x 3), inv.f64 (n x n)
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../paper_1506_06185_amd/csrc/topology.hpp"

using namespace hhgr;

int main(int argc, char **argv) {
    if (argc != 3) {
        std::printf("usage: coarse_inverse_dump n_sub out_dir\n");
        return 2;
    }
    Topology tp;
    const std::string e = tp.build(std::atoi(argv[1]), 3, 2);
    if (!e.empty()) {
        std::printf("topology: %s\n", e.c_str());
        return 1;
    }
    const CoarseSystem &cs = tp.coarse;
    std::vector<double> inv;
    if (!coarse_inverse(cs.n, cs.col, cs.val, inv)) {
        std::printf("not positive definite\n");
        return 1;
    }
    const std::string out = argv[2];
    FILE *f = std::fopen((out + "/pos.i32").c_str(), "wb");
    bool ok = f && std::fwrite(&cs.pos[0][0], sizeof(int), 3 * (size_t)cs.n, f) == 3 * (size_t)cs.n;
    if (f) std::fclose(f);
    f = std::fopen((out + "/inv.f64").c_str(), "wb");
    ok = ok && f && std::fwrite(inv.data(), sizeof(double), inv.size(), f) == inv.size();
    if (f) std::fclose(f);
    std::printf(ok ? "n=%d ok\n" : "n=%d write failed\n", cs.n);
    return ok ? 0 : 1;
}
