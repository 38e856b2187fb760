// Host-side checks of the HHG topology tables and of the closed-form index
// arithmetic that the volume kernels use (replicated here in plain C++):
// every table entry is in range, every neighbour/transfer offset computed in
// a kernel names the same slot as the topology's independent grid lookup.
#include <algorithm>
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
static int row_of(int M, int j, int k) { return k * M - ((k * (k - 1)) >> 1) + j; }
static int lslot(const TopoLevel &T, int i, int j, int k) {
    const auto &r = T.rowC[row_of(T.M, j, k)];
    return (((i + k) & 1) ? r[1] : r[0]) + (i >> 1);
}
// nb7: own slot and the 6 axis neighbours (ap, am, bp, bm, cp, cm) from rowN
static void nb7(const TopoLevel &T, int i, int j, int k, int out[7]) {
    const int nrows = (int)T.rowC.size(), c = (i + k) & 1, t = i >> 1;
    const auto &e = T.rowN[(size_t)c * nrows + row_of(T.M, j, k)];
    out[0] = e[0] + t;
    out[1] = e[1] + t;
    out[2] = e[1] + t - 1;
    out[3] = e[2] + t;
    out[4] = e[3] + t;
    out[5] = e[4] + t;
    out[6] = e[5] + t;
}
// the 15 fine slots read by k_restrict for coarse node (i,j,k), in the order
// centre, then kD14
static void restrict_reads(const TopoLevel &F, int i, int j, int k, int out[15]) {
    const int Mf = F.M, I = 2 * i, J = 2 * j, K = 2 * k, t0 = I >> 1;
    auto R = [&](int jj, int kk) { return F.rowC[row_of(Mf, jj, kk)]; };
    const auto r0 = R(J, K), rjp = R(J + 1, K), rjm = R(J - 1, K), rcp = R(J - 1, K + 1), rcm = R(J + 1, K - 1),
               rkp = R(J, K + 1), rkm = R(J, K - 1);
    const int v[15] = {r0[0] + t0,      r0[1] + t0,      r0[1] + t0 - 1,  rjp[1] + t0 - 1, rjm[1] + t0,
                       rcp[1] + t0,     rcm[1] + t0,     rjp[0] + t0,     rjm[0] + t0,     rkp[0] + t0 - 1,
                       rkm[0] + t0,     rcp[0] + t0,     rcm[0] + t0 - 1, rkp[1] + t0,     rkm[1] + t0};
    for (int q = 0; q < 15; q++) out[q] = v[q];
}
static const int kD14[14][3] = {{1, 0, 0},  {-1, 0, 0}, {-1, 1, 0}, {1, -1, 0}, {0, -1, 1},  {0, 1, -1}, {0, 1, 0},
                                {0, -1, 0}, {-1, 0, 1}, {1, 0, -1}, {1, -1, 1}, {-1, 1, -1}, {0, 0, 1}, {0, 0, -1}};
static const int kParDir[8][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 1, 0}, {0, 0, 1}, {-1, 0, 1}, {0, -1, 1}, {1, -1, 1}};

static void grid_pos(const Topology &tp, int t, int m, int i, int j, int k, int X[3]) {
    for (int a = 0; a < 3; a++) X[a] = m * tp.V0[t][a] + k;
    X[tp.perm[t][0]] += i + j;
    X[tp.perm[t][1]] += j;
}

// the colour-split layout is a bijection of the closure nodes onto slots
// [0, span) that puts every red node before every black one, keeps plane/row/i
// order within a colour, and makes the nodes of one colour in a row consecutive
static void check_layout(int m) {
    const int M = m + 1;
    ClosureLayout ly;
    ly.build(M);
    CHECK(ly.C == tetnum(M), "node count m=%d", m);
    CHECK(ly.span % 64 == 0 && ly.black0 % 32 == 0 && ly.black0 >= ly.n_red, "padding m=%d", m);
    std::vector<int> hit((size_t)ly.span, 0);
    long long prev[2] = {-1, ly.black0 - 1};
    for (int k = 0; k <= m; k++)
        for (int j = 0; j <= m - k; j++)
            for (int i = 0; i <= m - k - j; i++) {
                const long long s = ly.index(i, j, k);
                const int c = (i + k) & 1;
                CHECK(s >= 0 && s < ly.span, "slot range m=%d", m);
                if (s < 0 || s >= ly.span) continue;
                hit[s]++;
                CHECK(c == 0 ? s < ly.n_red : (s >= ly.black0 && s < ly.black0 + ly.n_black), "colour part m=%d", m);
                CHECK(s == prev[c] + 1, "consecutive within a colour m=%d (%d,%d,%d)", m, i, j, k);
                prev[c] = s;
            }
    for (long long s = 0; s < ly.span; s++) {
        const bool used = s < ly.n_red || (s >= ly.black0 && s < ly.black0 + ly.n_black);
        CHECK(hit[s] == (used ? 1 : 0), "bijection m=%d slot %lld", m, s);
    }
}

// replica of the device mapping fine element (cell, permutation q) -> macro
// tetrahedron used by the Dirichlet-Neumann operators
static const int kPermH[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
static int perm_id_h(int a, int b) { return a == 0 ? (b == 1 ? 0 : 1) : a == 1 ? (b == 0 ? 2 : 3) : (b == 0 ? 4 : 5); }
static int macro_tet_of(int cx, int cy, int cz, int q, int m, int n_sub) {
    const int C[3] = {cx / m, cy / m, cz / m};
    int D[3] = {4 * (cx - m * C[0]), 4 * (cy - m * C[1]), 4 * (cz - m * C[2])};
    D[kPermH[q][0]] += 3;
    D[kPermH[q][1]] += 2;
    D[kPermH[q][2]] += 1;
    const int a0 = D[0] > D[1] ? (D[0] > D[2] ? 0 : 2) : (D[1] > D[2] ? 1 : 2);
    const int a2 = D[0] < D[1] ? (D[0] < D[2] ? 0 : 2) : (D[1] < D[2] ? 1 : 2);
    return 6 * (C[0] + n_sub * (C[1] + n_sub * C[2])) + perm_id_h(a0, 3 - a0 - a2);
}

// every vertex of every fine element lies in the closed macro tetrahedron the
// mapping names (grid position X of the vertex: X - m V0 sorted along the
// macro tet's axis order is a non-increasing sequence in [0, m])
static void check_element_macro(const Topology &tp, int l) {
    const int m = 1 << l, N = tp.n_sub * m;
    for (int cz = 0; cz < N; cz++)
        for (int cy = 0; cy < N; cy++)
            for (int cx = 0; cx < N; cx++)
                for (int q = 0; q < 6; q++) {
                    const int t = macro_tet_of(cx, cy, cz, q, m, tp.n_sub);
                    CHECK(t >= 0 && t < tp.n_tets, "macro tet range");
                    int X[3] = {cx, cy, cz};
                    for (int v = 0; v < 4; v++) {
                        if (v > 0) X[kPermH[q][v - 1]] += 1;
                        int D[3];
                        for (int a = 0; a < 3; a++) D[a] = X[a] - m * tp.V0[t][a];
                        const int d0 = D[tp.perm[t][0]], d1 = D[tp.perm[t][1]], d2 = D[tp.perm[t][2]];
                        CHECK(m >= d0 && d0 >= d1 && d1 >= d2 && d2 >= 0, "element vertex in macro tet l=%d", l);
                    }
                }
}

int main(int argc, char **argv) {
    for (int lv = 2; lv <= 8; lv++) check_layout(1 << lv);
    int n_sub = argc > 1 ? std::atoi(argv[1]) : 2;
    int L = argc > 2 ? std::atoi(argv[2]) : 5;
    Topology tp;
    std::string e = tp.build(n_sub, L, 2);
    CHECK(e.empty(), "build: %s", e.c_str());
    if (!e.empty()) return 1;
    for (int l = 0; l <= std::min(L, 4); l++) check_element_macro(tp, l);
    for (int l = tp.Lc; l <= L; l++) {
        const TopoLevel &T = tp.lev[l];
        const int m = T.m;
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
        // node lists: slot order, colours, coverage
        const long long nint = (long long)(m - 1) * (m - 2) * (m - 3) / 6;
        CHECK(T.ilist.size() == T.rlist.size() + T.blist.size(), "colour lists partition the interior");
        CHECK((long long)T.ilist.size() == nint, "interior list size");
        CHECK((long long)T.flist.size() == T.C, "full list size");
        {
            // ilist: the red and the black list merged row by row (a row's red
            // nodes, then its black ones, rows in slot order)
            std::vector<unsigned> want;
            size_t pr = 0, pb = 0;
            auto row = [](unsigned wv) { return wv >> 10; };  // (j, k)
            while (pr < T.rlist.size() || pb < T.blist.size()) {
                const unsigned r = pr < T.rlist.size() ? row(T.rlist[pr]) : ~0u;
                const unsigned b = pb < T.blist.size() ? row(T.blist[pb]) : ~0u;
                const unsigned k_r = r >> 10, k_b = b >> 10, j_r = r & 1023, j_b = b & 1023;
                const bool red_first = k_r < k_b || (k_r == k_b && j_r <= j_b);
                const unsigned cur = red_first ? r : b;
                while (pr < T.rlist.size() && row(T.rlist[pr]) == cur) want.push_back(T.rlist[pr++]);
                while (pb < T.blist.size() && row(T.blist[pb]) == cur) want.push_back(T.blist[pb++]);
            }
            CHECK(want == T.ilist, "ilist = rows of red then black nodes");
        }
        auto unpack = [](unsigned wv, int &i, int &j, int &k) {
            i = wv & 1023;
            j = (wv >> 10) & 1023;
            k = (int)(wv >> 20);
        };
        long long last = -1;
        for (unsigned wv : T.flist) {
            int i, j, k;
            unpack(wv, i, j, k);
            const int sl = lslot(T, i, j, k);
            CHECK(sl == T.lay.index(i, j, k), "lslot = layout index");
            CHECK(sl > last, "full list in slot order");
            last = sl;
        }
        for (unsigned wv : T.rlist) CHECK((((wv & 1023) + (wv >> 20)) & 1) == 0, "red list colour");
        for (unsigned wv : T.blist) CHECK((((wv & 1023) + (wv >> 20)) & 1) == 1, "black list colour");
        // 15-point tables of general macro meshes: class lists partition the
        // interior (and the masters), neighbours of a node are in other
        // classes, and the row bases give every neighbour's slot
        {
            size_t nq = 0, nf = 0;
            for (int q = 0; q < 4; q++) {
                nq += T.qlist[q].size();
                nf += T.ifcq[q].size();
                long long lastq = -1;
                for (unsigned wv : T.qlist[q]) {
                    const int i = wv & 1023, j = (wv >> 10) & 1023, k = (int)(wv >> 20);
                    CHECK(((i + 2 * j + 3 * k) & 3) == q, "class list membership");
                    const long long sl = T.lay.index(i, j, k);
                    const bool same_part = lastq < 0 || ((sl < T.lay.black0) == (lastq < T.lay.black0));
                    CHECK(!same_part || sl > lastq, "class list in slot order");
                    lastq = sl;
                    const auto &e = T.rowN15[(size_t)((i + k) & 1) * T.rowC.size() + row_of(T.M, j, k)];
                    for (int n = 0; n < 15; n++) {
                        const int a = i + kIdx15[n][0], b = j + kIdx15[n][1], c = k + kIdx15[n][2];
                        CHECK(a >= 0 && b >= 0 && c >= 0 && a + b + c <= m, "15-point neighbour in closure");
                        CHECK(e[n] + (i >> 1) == T.lay.index(a, b, c), "rowN15 slot n=%d", n);
                        if (n > 0) CHECK(((a + 2 * b + 3 * c) & 3) != q, "neighbour in another class");
                    }
                }
                for (int f : T.ifcq[q]) {
                    const auto &X = T.ifc_X[f];
                    CHECK(((X[0] + X[1] + X[2]) & 3) == q, "interface class");
                }
            }
            CHECK(nq == T.ilist.size() && nf == (size_t)T.n_ifc, "class lists partition");
            for (int t = 0; t < tp.n_tets; t++)
                for (int n = 1; n < 15; n++) {
                    int d[3] = {0, 0, 0};
                    const auto &P = tp.perm[t];
                    d[P[0]] += kIdx15[n][0] + kIdx15[n][1] + kIdx15[n][2];
                    d[P[1]] += kIdx15[n][1] + kIdx15[n][2];
                    d[P[2]] += kIdx15[n][2];
                    int hit = 0;
                    for (int e2 = 1; e2 < 15; e2++)
                        hit += d[0] == kGrid15[e2][0] && d[1] == kGrid15[e2][1] && d[2] == kGrid15[e2][2];
                    CHECK(hit == 1, "index offset %d of tet %d is one grid stencil offset", n, t);
                }
        }
        // every interior node of every tet: kernel slot arithmetic vs the
        // topology's independent grid lookup
        for (int t = 0; t < tp.n_tets; t++) {
            const long long base = (long long)t * T.C_pad;
            for (unsigned wv : T.ilist) {
                int i, j, k;
                unpack(wv, i, j, k);
                int X[3];
                grid_pos(tp, t, m, i, j, k, X);
                int nb[7];
                nb7(T, i, j, k, nb);
                CHECK(tp.slot_of(l, X[0], X[1], X[2]) == base + nb[0], "interior slot t=%d", t);
                CHECK(nb[0] == lslot(T, i, j, k), "nb7 own slot");
                const int d[6][3] = {{1, 0, 0}, {-1, 0, 0}, {-1, 1, 0}, {1, -1, 0}, {0, -1, 1}, {0, 1, -1}};
                for (int e2 = 0; e2 < 6; e2++) {
                    const int a = i + d[e2][0], b = j + d[e2][1], c = k + d[e2][2];
                    CHECK(nb[1 + e2] == T.lay.index(a, b, c), "nb7 dir %d (%d,%d,%d) l=%d", e2, i, j, k, l);
                    int Y[3];
                    grid_pos(tp, t, m, a, b, c, Y);
                    const int dist = std::abs(Y[0] - X[0]) + std::abs(Y[1] - X[1]) + std::abs(Y[2] - X[2]);
                    CHECK(dist == 1, "axis neighbour is one grid step");
                    // ghosts and interiors: the grid lookup names the same value
                    const long long g = tp.slot_of(l, Y[0], Y[1], Y[2]);
                    const bool interior = a >= 1 && b >= 1 && c >= 1 && a + b + c <= m - 1;
                    if (interior) CHECK(g == base + nb[1 + e2], "interior neighbour slot");
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
                    const int c1 = lslot(Cl, p1[0] >> 1, p1[1] >> 1, p1[2] >> 1),
                              c2 = lslot(Cl, p2[0] >> 1, p2[1] >> 1, p2[2] >> 1);
                    CHECK(c1 == Cl.lay.index(p1[0] / 2, p1[1] / 2, p1[2] / 2), "parent 1 slot");
                    CHECK(c2 == Cl.lay.index(p2[0] / 2, p2[1] / 2, p2[2] / 2), "parent 2 slot");
                    int Y1[3], Y2[3];
                    grid_pos(tp, t, Cl.m, p1[0] / 2, p1[1] / 2, p1[2] / 2, Y1);
                    grid_pos(tp, t, Cl.m, p2[0] / 2, p2[1] / 2, p2[2] / 2, Y2);
                    for (int a = 0; a < 3; a++) CHECK(Y1[a] + Y2[a] == X[a], "fine node is the midpoint");
                }
                // restriction from the next finer level: kernel's grouped row reads
                if (l < L) {
                    const TopoLevel &Fl = tp.lev[l + 1];
                    int rd[15];
                    restrict_reads(Fl, i, j, k, rd);
                    for (int e2 = -1; e2 < 14; e2++) {
                        int a = 2 * i + (e2 >= 0 ? kD14[e2][0] : 0), b = 2 * j + (e2 >= 0 ? kD14[e2][1] : 0),
                            c = 2 * k + (e2 >= 0 ? kD14[e2][2] : 0);
                        CHECK(a >= 1 && b >= 1 && c >= 1 && a + b + c <= Fl.m - 1, "restriction source interior");
                        CHECK(rd[e2 + 1] == Fl.lay.index(a, b, c), "restriction read %d", e2);
                        int Y[3];
                        grid_pos(tp, t, Fl.m, a, b, c, Y);
                        int dist = 0;
                        for (int q = 0; q < 3; q++) dist += std::abs(Y[q] - 2 * X[q]);
                        CHECK(dist <= 3, "restriction source adjacent");
                        CHECK(tp.slot_of(l + 1, Y[0], Y[1], Y[2]) == (long long)t * Fl.C_pad + rd[e2 + 1],
                              "restriction source slot");
                    }
                }
            }
        }
        // local coarsest level: the node (1,1,1) and its -a,-b,-c neighbours
        if (l == tp.Lc) CHECK(nint == 1, "one interior node per tet on the coarsest level");
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
