// Host-side checks of the HHG topology tables and of the closed-form index
// arithmetic that the volume kernels use (replicated here in plain C++):
// every table entry is in range, every neighbour/transfer offset computed in
// a kernel names the same slot as the topology's independent grid lookup.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>

#include "../../paper_1506_06185_amd/csrc/topology.hpp"

using namespace hhgr;

static int fails = 0;
#define CHECK(c, ...)                         \
    do {                                      \
        if (!(c)) {                           \
            if (fails < 20) {                 \
                std::printf("FAIL: " __VA_ARGS__); \
                std::printf("\n");            \
            }                                 \
            fails++;                          \
        }                                     \
    } while (0)

// --- replicas of the device index helpers (kernels.hip) ---
static int tetnum_d(int x) { return x * (x + 1) * (x + 2) / 6; }
static int pstart_d(int M, int k) { return tetnum_d(M) - tetnum_d(M - k); }
static int rstart_d(int s, int j) { return j * s - ((j * (j - 1)) >> 1); }
static int cidx_d(int M, int i, int j, int k) { return pstart_d(M, k) + rstart_d(M - k, j) + i; }
static int decode_row(int s, int o) {
    const float b = 2.0f * (float)s + 1.0f;
    const float disc = std::fmax(b * b - 8.0f * (float)o, 0.0f);
    int j = (int)((b - std::sqrt(disc)) * 0.5f);
    j = std::max(0, std::min(j, s - 1));
    while (j + 1 <= s - 1 && rstart_d(s, j + 1) <= o) ++j;
    while (j > 0 && rstart_d(s, j) > o) --j;
    return j;
}
static const int kD14[14][3] = {{1, 0, 0},  {-1, 0, 0}, {-1, 1, 0}, {1, -1, 0}, {0, -1, 1},  {0, 1, -1}, {0, 1, 0},
                                {0, -1, 0}, {-1, 0, 1}, {1, 0, -1}, {1, -1, 1}, {-1, 1, -1}, {0, 0, 1}, {0, 0, -1}};
static const int kParDir[8][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 1, 0}, {0, 0, 1}, {-1, 0, 1}, {0, -1, 1}, {1, -1, 1}};

static void grid_pos(const Topology &tp, int t, int m, int i, int j, int k, int X[3]) {
    for (int a = 0; a < 3; a++) X[a] = m * tp.V0[t][a] + k;
    X[tp.perm[t][0]] += i + j;
    X[tp.perm[t][1]] += j;
}

// replica of k_fused_sweep's index logic: every interior node written once,
// every LDS read backed by a phase-1 store of an existing node
static void check_fused(int m) {
    const int M = m + 1, FE = kTileRows + 2;
    std::vector<int> written((size_t)tetnum_d(M), 0);
    for (const auto &tl : fused_tile_list(m)) {
        const int j0 = tl[0], k0 = tl[1], i0 = tl[2];
        std::vector<char> have(FE * FE * 33, 0);
        for (int er = 0; er < FE * FE; er++)
            for (int t = 0; t < 32; t++) {
                const int j = j0 - 1 + er % FE, k = k0 - 1 + er / FE;
                const int prow = (k + i0 - 1) & 1, l = 2 * t + prow, i = i0 - 1 + l;
                if (l > 63 || j < 0 || k < 0 || i < 0 || i + j + k > m) continue;
                CHECK(((i + k) & 1) == 0, "phase-1 node is red");
                CHECK(cidx_d(M, i, j, k) >= 0 && cidx_d(M, i, j, k) < tetnum_d(M), "phase-1 index");
                have[er * 33 + t] = 1;
            }
        for (int tr = 0; tr < kTileRows * kTileRows; tr++) {
            const int jj = tr % kTileRows, kk = tr / kTileRows, j = j0 + jj, k = k0 + kk;
            if (j + k > m - 2) continue;
            const int er = (jj + 1) + FE * (kk + 1), prow = (k + i0 - 1) & 1;
            for (int l = 1; l <= kTileSeg; l++) {
                const int i = i0 - 1 + l;
                if (i + j + k > m - 1) continue;
                CHECK(i >= 1 && j >= 1 && k >= 1, "phase-2 node interior");
                written[cidx_d(M, i, j, k)]++;
                if (((l + prow) & 1) == 0) {
                    CHECK(have[er * 33 + (l >> 1)], "red value present");
                } else {
                    const int reads[6][2] = {{er, (l + 1) >> 1}, {er, (l - 1) >> 1}, {er + 1, (l - 1) >> 1},
                                             {er - 1, (l + 1) >> 1}, {er - 1 + FE, l >> 1}, {er + 1 - FE, l >> 1}};
                    for (auto &rd : reads) {
                        CHECK(rd[0] >= 0 && rd[0] < FE * FE && rd[1] >= 0 && rd[1] < 32, "LDS index in range");
                        CHECK(have[rd[0] * 33 + rd[1]], "black neighbour read a stored red value m=%d", m);
                    }
                }
            }
        }
    }
    for (int k = 0; k <= m; k++)
        for (int j = 0; j <= m - k; j++)
            for (int i = 0; i <= m - k - j; i++) {
                bool interior = i >= 1 && j >= 1 && k >= 1 && i + j + k <= m - 1;
                CHECK(written[cidx_d(M, i, j, k)] == (interior ? 1 : 0), "fused coverage m=%d (%d,%d,%d)", m, i, j, k);
            }
}

int main(int argc, char **argv) {
    for (int lv = 2; lv <= 9; lv++) check_fused(1 << lv);
    int n_sub = argc > 1 ? std::atoi(argv[1]) : 2;
    int L = argc > 2 ? std::atoi(argv[2]) : 5;
    // decode of every plane offset for the largest supported plane size
    for (int s = 1; s <= 513; s++)
        for (int o = 0; o < s * (s + 1) / 2; o++) {
            int j = decode_row(s, o);
            CHECK(rstart_d(s, j) <= o && o < rstart_d(s, j + 1), "decode s=%d o=%d", s, o);
        }
    Topology tp;
    std::string e = tp.build(n_sub, L, 2, 256);
    CHECK(e.empty(), "build: %s", e.c_str());
    if (!e.empty()) return 1;
    for (int l = tp.Lc; l <= L; l++) {
        const TopoLevel &T = tp.lev[l];
        const int m = T.m, M = T.M;
        // interface node count (closed forms for the n^3 x 6 Kuhn cube)
        if (n_sub == 2) {
            long long expect = 72LL * (m - 1) * (m - 2) / 2 + 26LL * (m - 1) + 1;
            CHECK(T.n_ifc == expect, "n_ifc l=%d %d vs %lld", l, T.n_ifc, expect);
        }
        auto in_slots = [&](long long s) { return s >= 0 && s < T.n_slots; };
        for (int v : T.nbr) CHECK(in_slots(v), "nbr range");
        for (int v : T.gidx) CHECK(v >= 0 && v < T.ifc_base, "ghost slot range");
        for (int v : T.nb15) CHECK(in_slots(v), "nb15 range");
        for (size_t q = 0; q < T.tg_dst.size(); q++) {
            CHECK(T.tg_dst[q] >= 0 && T.tg_dst[q] < T.ifc_base, "tg dst");
            CHECK(in_slots(T.tg_src[q]) && T.tg_src[q] >= T.ifc_base, "tg src");
        }
        CHECK(T.n_ifc_red > 0 && T.n_ifc_red < T.n_ifc, "colour split");
        for (int f = 0; f < T.n_ifc; f++) {
            const auto &X = T.ifc_X[f];
            CHECK(((X[0] + X[1] + X[2]) & 1) == (f >= T.n_ifc_red ? 1 : 0), "ifc colour order");
            int ng = T.gptr[f + 1] - T.gptr[f];
            CHECK(ng >= 2, "an interface node has >= 2 ghost copies");
        }
        if (l > tp.Lc) {
            const TopoLevel &Cl = tp.lev[l - 1];
            for (int v : T.prl) CHECK(v >= 0 && v < Cl.n_slots, "prl range");
        }
        if (l < L) {
            const TopoLevel &Fl = tp.lev[l + 1];
            for (int v : T.rst) CHECK(v >= 0 && v < Fl.n_slots, "rst range");
        }
        // chunk tables cover exactly the interior nodes / the whole closure
        long long covered = 0;
        for (auto &ch : T.chunks_full) {
            int s = M - ch.k;
            CHECK(ch.k >= 0 && ch.k <= m && ch.o0 < s * (s + 1) / 2, "full chunk");
            covered += std::min(256, s * (s + 1) / 2 - ch.o0);
        }
        CHECK(covered == T.C, "full chunks cover the closure");
        long long nint = 0;
        for (auto &ch : T.chunks_int)
            for (int q = 0; q < 256; q++) {
                int s = M - ch.k, o = ch.o0 + q;
                if (o >= s * (s + 1) / 2) break;
                int j = decode_row(s, o), i = o - rstart_d(s, j), k = ch.k;
                if (i >= 1 && j >= 1 && k >= 1 && i + j + k <= M - 2) nint++;
            }
        CHECK(nint == (long long)(m - 1) * (m - 2) * (m - 3) / 6, "interior chunks cover the interior l=%d", l);
        // node lists and row tables used by the list-mode kernels
        CHECK(T.ilist.size() == T.rlist.size() + T.blist.size(), "colour lists partition the interior");
        CHECK((long long)T.ilist.size() == (long long)(m - 1) * (m - 2) * (m - 3) / 6, "interior list size");
        for (unsigned wv : T.ilist) {
            const int i = wv & 1023, j = (wv >> 10) & 1023, k = (int)(wv >> 20);
            const auto &ra = T.rowA[row_id(M, j, k)];
            const auto &rb = T.rowB[row_id(M, j, k)];
            const int c0 = ra[0] + i, rj = ra[1];
            CHECK(c0 == closure_index(M, i, j, k), "rowA slot");
            const int offs[14] = {c0 + 1, c0 - 1, c0 + rj - 1, c0 - rj, c0 + ra[2], c0 + ra[3], c0 + rj,
                                  c0 - (rj + 1), c0 + rb[0] - 1, c0 + rb[1] + 1, c0 + ra[2] + 1, c0 + ra[3] - 1,
                                  c0 + rb[0], c0 + rb[1]};
            for (int e2 = 0; e2 < 14; e2++)
                CHECK(offs[e2] == cidx_d(M, i + kD14[e2][0], j + kD14[e2][1], k + kD14[e2][2]), "row offsets dir %d", e2);
        }
        for (unsigned wv : T.rlist) CHECK((((wv & 1023) + (wv >> 20)) & 1) == 0, "red list colour");
        for (unsigned wv : T.blist) CHECK((((wv & 1023) + (wv >> 20)) & 1) == 1, "black list colour");
        // volume neighbour arithmetic vs topology lookup, every tet, every interior node
        for (int t = 0; t < tp.n_tets; t++) {
            const long long base = (long long)t * T.C_pad;
            for (int k = 1; k <= m; k++)
                for (int j = 1; j <= m - k; j++)
                    for (int i = 1; i <= m - k - j; i++) {
                        if (i + j + k > m - 1) continue;
                        const int s = M - k, o = rstart_d(s, j) + i, ps = pstart_d(M, k), c0 = ps + o;
                        CHECK(c0 == closure_index(M, i, j, k), "closure index");
                        const int rj = s - j;
                        const int nb[6] = {c0 + 1, c0 - 1, c0 + rj - 1, c0 - rj,
                                           ps + s * (s + 1) / 2 + rstart_d(s - 1, j - 1) + i,
                                           ps - (s + 1) * (s + 2) / 2 + rstart_d(s + 1, j + 1) + i};
                        const int d[6][3] = {{1, 0, 0}, {-1, 0, 0}, {-1, 1, 0}, {1, -1, 0}, {0, -1, 1}, {0, 1, -1}};
                        int X[3];
                        grid_pos(tp, t, m, i, j, k, X);
                        CHECK(tp.slot_of(l, X[0], X[1], X[2]) == base + c0, "interior slot t=%d", t);
                        for (int e2 = 0; e2 < 6; e2++) {
                            CHECK(nb[e2] >= 0 && nb[e2] < T.C, "nb in closure");
                            CHECK(nb[e2] == cidx_d(M, i + d[e2][0], j + d[e2][1], k + d[e2][2]), "nb formula");
                            int Y[3];
                            grid_pos(tp, t, m, i + d[e2][0], j + d[e2][1], k + d[e2][2], Y);
                            int dist = std::abs(Y[0] - X[0]) + std::abs(Y[1] - X[1]) + std::abs(Y[2] - X[2]);
                            CHECK(dist == 1, "axis neighbour is one grid step");
                        }
                        // mass: 14 Freudenthal neighbours stay in the closure
                        for (int e2 = 0; e2 < 14; e2++) {
                            int a = i + kD14[e2][0], b = j + kD14[e2][1], c = k + kD14[e2][2];
                            CHECK(a >= 0 && b >= 0 && c >= 0 && a + b + c <= m, "d14 in closure");
                        }
                        // prolongation parents
                        if (l > tp.Lc) {
                            const TopoLevel &Cl = tp.lev[l - 1];
                            int code = (i & 1) | ((j & 1) << 1) | ((k & 1) << 2);
                            int p1[3] = {i - kParDir[code][0], j - kParDir[code][1], k - kParDir[code][2]};
                            int p2[3] = {i + kParDir[code][0], j + kParDir[code][1], k + kParDir[code][2]};
                            for (int a = 0; a < 3; a++) CHECK((p1[a] % 2) == 0 && (p2[a] % 2) == 0 && p1[a] >= 0, "parity");
                            int c1 = cidx_d(Cl.M, p1[0] / 2, p1[1] / 2, p1[2] / 2), c2 = cidx_d(Cl.M, p2[0] / 2, p2[1] / 2, p2[2] / 2);
                            CHECK(c1 >= 0 && c1 < Cl.C && c2 >= 0 && c2 < Cl.C, "parent in coarse closure");
                            int Y1[3], Y2[3];
                            grid_pos(tp, t, Cl.m, p1[0] / 2, p1[1] / 2, p1[2] / 2, Y1);
                            grid_pos(tp, t, Cl.m, p2[0] / 2, p2[1] / 2, p2[2] / 2, Y2);
                            for (int a = 0; a < 3; a++) CHECK(Y1[a] + Y2[a] == X[a], "fine node is the midpoint");
                        }
                        // restriction from the next finer level
                        if (l < L) {
                            const TopoLevel &Fl = tp.lev[l + 1];
                            for (int e2 = -1; e2 < 14; e2++) {
                                int a = 2 * i + (e2 >= 0 ? kD14[e2][0] : 0), b = 2 * j + (e2 >= 0 ? kD14[e2][1] : 0),
                                    c = 2 * k + (e2 >= 0 ? kD14[e2][2] : 0);
                                CHECK(a >= 1 && b >= 1 && c >= 1 && a + b + c <= Fl.m - 1, "restriction source interior");
                                int Y[3];
                                grid_pos(tp, t, Fl.m, a, b, c, Y);
                                int dist = 0;
                                for (int q = 0; q < 3; q++) dist += std::abs(Y[q] - 2 * X[q]);
                                CHECK(dist <= 3, "restriction source adjacent");
                            }
                        }
                    }
        }
        // interface neighbour tables agree with grid lookups
        for (int f = 0; f < T.n_ifc; f += 7) {
            const auto &X = T.ifc_X[f];
            const int d6[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
            for (int e2 = 0; e2 < 6; e2++)
                CHECK(T.nbr[(size_t)e2 * T.n_ifc + f] == tp.slot_of(l, X[0] + d6[e2][0], X[1] + d6[e2][1], X[2] + d6[e2][2]),
                      "ifc nbr");
        }
    }
    // coarse system
    const CoarseSystem &cs = tp.coarse;
    const TopoLevel &Tc = tp.lev[tp.Lc];
    long long Nc = Tc.N - 1;
    CHECK(cs.n == Nc * Nc * Nc, "coarse unknowns = interior nodes");
    for (int q = 0; q < cs.n; q++) {
        int nn = 0;
        for (int e2 = 1; e2 < 7; e2++) nn += cs.col[7 * q + e2] >= 0;
        CHECK(nn >= 3 && nn <= 6, "coarse neighbours");
        for (int c = cs.cptr[q]; c < cs.cptr[q + 1]; c++) CHECK(cs.cidx[c] >= 0 && cs.cidx[c] < Tc.n_slots, "coarse copies");
    }
    std::printf("topology_check n_sub=%d L=%d: %s (%d failures)\n", n_sub, L, fails ? "FAILED" : "ok", fails);
    return fails ? 1 : 0;
}
