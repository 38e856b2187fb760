// CPU check of the fused red-black sweep kernels (fused.hip) compiled for the
// host against the device-code emulation in mockdev/ (a workgroup = host
// threads meeting at a barrier).  For several meshes, levels and tile shapes
// it runs one fused sweep of the volume interiors and compares every slot
// with a plain two-colour sweep written here from the closure layout
// (ClosureLayout::index, not the kernel's closed-form row bases): interior
// nodes must agree bitwise, every other slot must be left unchanged.  The
// zero-start variant runs with the source filled with NaN, so a read of it
// shows.  Built with AddressSanitizer: global buffers are exact-size
// vectors, and the LDS bytes beyond each launch's request are poisoned.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <random>
#include <vector>

#include "../../paper_1506_06185_amd/csrc/kernels.hpp"
#include "../../paper_1506_06185_amd/csrc/topology.hpp"

thread_local mockdev_idx threadIdx, blockIdx;
dim3 gridDim, blockDim;
std::barrier<> *mockdev_barrier = nullptr;
unsigned char fused_lds[kMockLds];

using namespace hhgr;

static int fails = 0;
#define CHECK(c, ...)                      \
    do {                                   \
        if (!(c)) {                        \
            std::printf("FAIL: " __VA_ARGS__); \
            std::printf("\n");             \
            fails++;                       \
        }                                  \
    } while (0)

struct Tables {
    std::vector<int> ps;
    std::vector<int4> tiles;
};

// plane starts and tiles as the engine builds them, for a given tile shape
static Tables tables(const TopoLevel &T, int TJ, int TK) {
    Tables t;
    const int m = T.m, M = T.M;
    const ClosureLayout &ly = T.lay;
    t.ps.assign(2 * (size_t)(m + 2), 0);
    for (int c = 0; c < 2; c++) {
        for (int k = 0; k <= m; k++)
            t.ps[c * (m + 2) + k] = ly.row0[2 * (size_t)row_id(M, 0, k) + c] - (c ? (int)ly.black0 : 0);
        t.ps[c * (m + 2) + m + 1] = (int)(c ? ly.n_black : ly.n_red);
    }
    const int ti = fused_tile_i();
    for (int k0 = 1; k0 <= m - 3; k0 += TK)
        for (int j0 = 1; j0 <= m - 3; j0 += TJ)
            for (int i0 = 1; i0 <= m - 3; i0 += ti)
                if (i0 + j0 + k0 <= m - 1) t.tiles.push_back(make_int4(i0, j0, k0, 0));
    return t;
}

static bool interior(int m, int i, int j, int k) { return i >= 1 && j >= 1 && k >= 1 && i + j + k <= m - 1; }

template <typename T>
static void run_case(int n_sub, int L, int TJ, int TK, bool zero, bool res) {
    Topology tp;
    const std::string e = tp.build(n_sub, L, 2);
    if (!e.empty()) {
        CHECK(false, "topology %s", e.c_str());
        return;
    }
    const TopoLevel &TL = tp.lev[L];
    const ClosureLayout &ly = TL.lay;
    const int m = TL.m;
    const Tables tb = tables(TL, TJ, TK);
    std::vector<VolDesc> vd(tp.n_tets);
    for (int t = 0; t < tp.n_tets; t++) vd[t] = VolDesc{(long long)t * TL.C_pad, (long long)t * TL.C_pad, t, 0};
    FusedGeom g;
    g.vd = vd.data();
    g.nvol = tp.n_tets;
    g.tiles = tb.tiles.data();
    g.ntiles = (int)tb.tiles.size();
    g.m = m;
    g.TJ = TJ;
    g.TK = TK;
    g.black0 = ly.black0;
    g.ps = tb.ps.data();
    g.remap = 1;
    if (!fused_shape_ok(g)) {
        CHECK(false, "shape rejected n=%d L=%d TJ=%d", n_sub, L, TJ);
        return;
    }
    std::mt19937_64 rng(1000 * n_sub + 10 * L + TJ + 7 * TK);
    std::uniform_real_distribution<double> U(-1.0, 1.0);
    const size_t ns = (size_t)TL.n_slots;
    std::vector<T> S(ns), D(ns), B(ns), R(ns);
    for (size_t q = 0; q < ns; q++) {
        S[q] = zero ? std::numeric_limits<T>::quiet_NaN() : (T)U(rng);
        D[q] = (T)U(rng);  // red boundary slots: the new interface values; the rest is overwritten or kept
        B[q] = (T)U(rng);
        R[q] = (T)U(rng);
    }
    const std::vector<T> D0 = D, R0 = R;
    const double hd = TL.h, omd = 1.25;
    const T h = (T)hd, om = (T)omd, om_d = (T)(omd / (6.0 * hd));
    // reference: red then black over every tetrahedron's interior
    std::vector<T> E = D0, ER = R0;
    auto sor = [&](T uo, T acc, T bb, T &rr) {
        rr = bb - h * (T(6) * uo - acc);
        return uo + om_d * rr;
    };
    static const int off[6][3] = {{1, 0, 0}, {-1, 0, 0}, {-1, 1, 0}, {1, -1, 0}, {0, -1, 1}, {0, 1, -1}};
    for (int t = 0; t < tp.n_tets; t++) {
        const size_t base = (size_t)t * TL.C_pad;
        for (int colour = 0; colour < 2; colour++)
            for (int k = 1; k <= m; k++)
                for (int j = 1; j <= m; j++)
                    for (int i = 1; i + j + k <= m - 1; i++) {
                        if (((i + k) & 1) != colour) continue;
                        T nb[6];
                        for (int d = 0; d < 6; d++) {
                            const int a = i + off[d][0], bq = j + off[d][1], c = k + off[d][2];
                            const size_t sl = base + (size_t)ly.index(a, bq, c);
                            // red pass: old black (zero when starting from zero);
                            // black pass: new red (interior from E, boundary given in D)
                            nb[d] = colour == 0 ? (zero ? T(0) : S[sl]) : E[sl];
                        }
                        const T acc = ((nb[0] + nb[1]) + (nb[2] + nb[3])) + (nb[4] + nb[5]);
                        const size_t sl = base + (size_t)ly.index(i, j, k);
                        T rr;
                        E[sl] = sor(zero ? T(0) : S[sl], acc, B[sl], rr);
                        if (colour == 1 && res) ER[sl] = (T(1) - om) * rr;
                    }
    }
    launch_sweep_fused_vol<T>(nullptr, g, S.data(), D.data(), B.data(), hd, omd, zero, res ? R.data() : nullptr);
    long long bad = 0, badr = 0;
    for (size_t q = 0; q < ns; q++) {
        const bool same = std::memcmp(&D[q], &E[q], sizeof(T)) == 0;
        if (!same) {
            if (bad < 3) std::printf("  slot %zu: got %.17g want %.17g\n", q, (double)D[q], (double)E[q]);
            bad++;
        }
        if (std::memcmp(&R[q], &ER[q], sizeof(T)) != 0) badr++;
    }
    CHECK(bad == 0, "fused sweep n=%d L=%d TJ=%d TK=%d zero=%d res=%d word=%zu: %lld slots differ", n_sub, L, TJ, TK,
          (int)zero, (int)res, sizeof(T), bad);
    CHECK(badr == 0, "residual tail n=%d L=%d TJ=%d TK=%d: %lld slots differ", n_sub, L, TJ, TK, badr);
}

int main(int argc, char **argv) {
    const bool all = argc > 1 && std::strcmp(argv[1], "all") == 0;
    std::printf("fused_check: tiles of %d i values\n", fused_tile_i());
    // engine-like shapes, then small and ragged ones ("all": also larger levels)
    run_case<double>(1, 4, 16, 16, false, true);
    run_case<double>(3, 3, 2, 3, false, true);
    run_case<float>(2, 4, 5, 4, true, false);
    if (all) {
        run_case<double>(1, 3, 8, 8, false, false);
        run_case<double>(2, 4, 16, 16, true, false);
        run_case<double>(1, 5, 7, 2, true, true);
        run_case<float>(1, 4, 3, 16, false, true);
        run_case<double>(1, 5, 28, 16, false, false);
        run_case<double>(1, 5, 28, 16, true, false);
        run_case<double>(1, 6, 28, 16, false, true);
        run_case<double>(1, 5, 1, 1, false, true);
        run_case<double>(1, 5, 3, 5, false, false);
        run_case<float>(1, 5, 28, 16, false, true);
    }
    std::printf("fused_check: %s (%d failures)\n", fails ? "FAILED" : "ok", fails);
    return fails ? 1 : 0;
}
