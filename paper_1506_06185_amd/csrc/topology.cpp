// Host-side HHG topology (see topology.hpp for the storage model).
#include "topology.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <tuple>

namespace hhgr {

namespace {

struct IfcRec {
    long long key;  // grid key x + (N+1)(y + (N+1) z)
    int colour;
    int dim;                 // 2 face, 1 edge, 0 vertex
    std::array<int, 3> prim; // macro vertex ids of the primitive, sorted, padded with -1
    std::array<int, 3> X;
};

inline long long gkey(int N, int x, int y, int z) { return x + (long long)(N + 1) * (y + (long long)(N + 1) * z); }

inline bool on_boundary(int N, int x, int y, int z) {
    return x == 0 || y == 0 || z == 0 || x == N || y == N || z == N;
}

constexpr int kAxis6[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};

}  // namespace

int Topology::ifc_index(int l, int x, int y, int z) const {
    const TopoLevel &Lv = lev[l];
    long long key = gkey(Lv.N, x, y, z);
    const auto &keys = ifc_key_[l];
    auto it = std::lower_bound(keys.begin(), keys.end(), key);
    if (it == keys.end() || *it != key) return -1;
    return ifc_key_idx_[l][it - keys.begin()];
}

bool Topology::locate_interior(int l, int x, int y, int z, int *tet, int *i, int *j, int *k) const {
    const TopoLevel &Lv = lev[l];
    const int m = Lv.m;
    int X[3] = {x, y, z}, c[3], D[3];
    for (int a = 0; a < 3; a++) {
        c[a] = X[a] / m;
        D[a] = X[a] - m * c[a];
        if (c[a] < 0 || c[a] >= n_sub || D[a] <= 0) return false;
    }
    int p[3] = {0, 1, 2};
    std::sort(p, p + 3, [&](int a, int b) { return D[a] > D[b]; });
    if (!(D[p[0]] > D[p[1]] && D[p[1]] > D[p[2]] && D[p[0]] < m)) return false;
    int q = -1;
    for (int s = 0; s < 6; s++)
        if (kPerm[s][0] == p[0] && kPerm[s][1] == p[1] && kPerm[s][2] == p[2]) q = s;
    *tet = 6 * (c[0] + n_sub * (c[1] + n_sub * c[2])) + q;
    *i = D[p[0]] - D[p[1]];
    *j = D[p[1]] - D[p[2]];
    *k = D[p[2]];
    return true;
}

long long Topology::slot_of(int l, int x, int y, int z) const {
    const TopoLevel &Lv = lev[l];
    if (x < 0 || y < 0 || z < 0 || x > Lv.N || y > Lv.N || z > Lv.N) return -1;
    if (on_boundary(Lv.N, x, y, z)) return Lv.zero_slot;
    int f = ifc_index(l, x, y, z);
    if (f >= 0) return Lv.ifc_base + f;
    int t, i, j, k;
    if (!locate_interior(l, x, y, z, &t, &i, &j, &k)) return -1;
    return (long long)t * Lv.C_pad + Lv.lay.index(i, j, k);
}

// Node lists and row tables of the colour-split closure layout of a level
// (the same for every tetrahedron and every macro mesh).
void build_closure_tables(TopoLevel &Lv) {
    const int m = Lv.m, M = Lv.M;
    // node lists and row tables (shared by all tetrahedra), in slot order
    Lv.rlist.clear();
    Lv.blist.clear();
    Lv.flist.clear();
    for (int c = 0; c < 2; c++)
        for (int k = 0; k <= m; k++)
            for (int j = 0; j <= m - k; j++)
                for (int i = (c + k) & 1; i <= m - k - j; i += 2) {
                    const unsigned w = pack_ijk(i, j, k);
                    Lv.flist.push_back(w);
                    if (i >= 1 && j >= 1 && k >= 1 && i + j + k <= m - 1) (c == 0 ? Lv.rlist : Lv.blist).push_back(w);
                }
    // all interior nodes row by row (plane k, row j; a row's red nodes, then
    // its black ones): a launch over both colours then reads each row's u and
    // b once while they are in cache, instead of once per colour half
    Lv.ilist.clear();
    for (int k = 1; k <= m - 3; k++)
        for (int j = 1; j <= m - 2 - k; j++)
            for (int c = 0; c < 2; c++)
                for (int i = 1 + ((1 + c + k) & 1); i <= m - 1 - k - j; i += 2) Lv.ilist.push_back(pack_ijk(i, j, k));
    for (int q = 0; q < 4; q++) Lv.qlist[q].clear();
    for (int c = 0; c < 2; c++)
        for (unsigned w : (c ? Lv.blist : Lv.rlist)) {
            const int i = (int)(w & 1023u), j = (int)((w >> 10) & 1023u), k = (int)(w >> 20);
            Lv.qlist[(i + 2 * j + 3 * k) & 3].push_back(w);
        }
    const int nrows = M * (M + 1) / 2;
    Lv.rowC.assign(nrows, {0, 0});
    for (int r = 0; r < nrows; r++) Lv.rowC[r] = {Lv.lay.row0[2 * (size_t)r], Lv.lay.row0[2 * (size_t)r + 1]};
    Lv.rowN.assign(2 * (size_t)nrows, {0, 0, 0, 0, 0, 0, 0, 0});
    for (int c = 0; c < 2; c++)
        for (int k = 1; k <= m - 3; k++)
            for (int j = 1; j + k <= m - 2; j++) {
                const int o = 1 - c, odd = (c + k) & 1;
                auto start = [&](int jj, int kk, int cc) { return Lv.lay.row0[2 * (size_t)row_id(M, jj, kk) + cc]; };
                Lv.rowN[(size_t)c * nrows + row_id(M, j, k)] = {start(j, k, c),          start(j, k, o) + odd,
                                                                start(j + 1, k, o) + odd - 1,
                                                                start(j - 1, k, o) + odd, start(j - 1, k + 1, o),
                                                                start(j + 1, k - 1, o),   0, 0};
            }
    // 15-point bases: node i = 2t + p (p = (c + k) & 1) of row (j, k); its
    // neighbour at index offset (di, dj, dk) has parity colour (c + di + dk) & 1
    // and storage index (i + di) >> 1 = t + ((p + di) >> 1)
    Lv.rowN15.assign(2 * (size_t)nrows, {});
    for (int c = 0; c < 2; c++)
        for (int k = 1; k <= m - 3; k++)
            for (int j = 1; j + k <= m - 2; j++) {
                const int p = (c + k) & 1;
                auto &e = Lv.rowN15[(size_t)c * nrows + row_id(M, j, k)];
                for (int n = 0; n < 15; n++) {
                    const int di = kIdx15[n][0], dj = kIdx15[n][1], dk = kIdx15[n][2];
                    const int cc = (c + di + dk) & 1;
                    e[n] = Lv.lay.row0[2 * (size_t)row_id(M, j + dj, k + dk) + cc] + ((p + di) >> 1);
                }
                e[15] = 0;
            }
}

void Topology::build_level(int l) {
    TopoLevel &Lv = lev[l];
    Lv.l = l;
    Lv.m = 1 << l;
    Lv.M = Lv.m + 1;
    Lv.N = n_sub * Lv.m;
    Lv.h = 1.0 / Lv.N;
    Lv.lay.build(Lv.M);
    Lv.C = Lv.lay.C;
    Lv.C_pad = Lv.lay.span;
    Lv.ifc_base = (long long)n_tets * Lv.C_pad;
    const int m = Lv.m, M = Lv.M, N = Lv.N;

    // macro vertex ids (level-0 grid) of tet t
    auto macro_vertex = [&](int t, int a) {
        int v[3] = {V0[t][0], V0[t][1], V0[t][2]};
        for (int s = 0; s < a; s++) v[perm[t][s]] += 1;
        return v[0] + (n_sub + 1) * (v[1] + (n_sub + 1) * v[2]);
    };
    auto grid_pos = [&](int t, int i, int j, int k, int X[3]) {
        for (int a = 0; a < 3; a++) X[a] = m * V0[t][a] + k;
        X[perm[t][0]] += i + j;
        X[perm[t][1]] += j;
    };

    // interface nodes from the boundary nodes of every closure
    std::vector<IfcRec> recs;
    for (int t = 0; t < n_tets; t++)
        for (int k = 0; k <= m; k++)
            for (int j = 0; j <= m - k; j++)
                for (int i = 0; i <= m - k - j; i++) {
                    bool bnd = i == 0 || j == 0 || k == 0 || i + j + k == m;
                    if (!bnd) continue;
                    int X[3];
                    grid_pos(t, i, j, k, X);
                    if (on_boundary(N, X[0], X[1], X[2])) continue;
                    IfcRec r;
                    r.key = gkey(N, X[0], X[1], X[2]);
                    r.colour = (X[0] + X[1] + X[2]) & 1;
                    int lam[4] = {m - i - j - k, i, j, k};
                    std::vector<int> pv;
                    for (int a = 0; a < 4; a++)
                        if (lam[a] > 0) pv.push_back(macro_vertex(t, a));
                    std::sort(pv.begin(), pv.end());
                    r.dim = (int)pv.size() - 1;
                    r.prim = {-1, -1, -1};
                    for (size_t s = 0; s < pv.size() && s < 3; s++) r.prim[s] = pv[s];
                    r.X = {X[0], X[1], X[2]};
                    recs.push_back(r);
                }
    std::sort(recs.begin(), recs.end(), [](const IfcRec &a, const IfcRec &b) { return a.key < b.key; });
    recs.erase(std::unique(recs.begin(), recs.end(), [](const IfcRec &a, const IfcRec &b) { return a.key == b.key; }),
               recs.end());
    // final order: colour (red first), faces, edges, vertices, primitive, then z, y, x
    std::sort(recs.begin(), recs.end(), [](const IfcRec &a, const IfcRec &b) {
        return std::make_tuple(a.colour, -a.dim, a.prim, a.X[2], a.X[1], a.X[0]) <
               std::make_tuple(b.colour, -b.dim, b.prim, b.X[2], b.X[1], b.X[0]);
    });
    Lv.n_ifc = (int)recs.size();
    Lv.n_ifc_red = 0;
    Lv.ifc_X.resize(Lv.n_ifc);
    Lv.ifc_dof.resize(Lv.n_ifc);
    std::vector<std::pair<long long, int>> keyidx(Lv.n_ifc);
    for (int f = 0; f < Lv.n_ifc; f++) {
        const IfcRec &r = recs[f];
        if (r.colour == 0) Lv.n_ifc_red++;
        Lv.ifc_X[f] = r.X;
        Lv.ifc_dof[f] = (r.X[0] - 1) + (N - 1) * ((r.X[1] - 1) + (N - 1) * (r.X[2] - 1));
        keyidx[f] = {r.key, f};
    }
    std::sort(keyidx.begin(), keyidx.end());
    ifc_key_[l].resize(Lv.n_ifc);
    ifc_key_idx_[l].resize(Lv.n_ifc);
    for (int f = 0; f < Lv.n_ifc; f++) {
        ifc_key_[l][f] = keyidx[f].first;
        ifc_key_idx_[l][f] = keyidx[f].second;
    }
    Lv.zero_slot = Lv.ifc_base + Lv.n_ifc;
    Lv.n_slots = round_up(Lv.zero_slot + 1, 64);

    // axis neighbours of interface nodes
    Lv.nbr.assign(6 * (size_t)Lv.n_ifc, -1);
    for (int f = 0; f < Lv.n_ifc; f++)
        for (int e = 0; e < 6; e++) {
            const auto &X = Lv.ifc_X[f];
            long long s = slot_of(l, X[0] + kAxis6[e][0], X[1] + kAxis6[e][1], X[2] + kAxis6[e][2]);
            Lv.nbr[(size_t)e * Lv.n_ifc + f] = (int)s;
        }
    // ghost copies of interface nodes, and per-tet ghost refresh lists
    std::vector<int> cnt(Lv.n_ifc + 1, 0);
    Lv.tg_ptr.assign(n_tets + 1, 0);
    Lv.tg_dst.clear();
    Lv.tg_src.clear();
    std::vector<std::pair<int, int>> ghost;  // (ifc, slot)
    for (int t = 0; t < n_tets; t++) {
        for (int k = 0; k <= m; k++)
            for (int j = 0; j <= m - k; j++)
                for (int i = 0; i <= m - k - j; i++) {
                    bool bnd = i == 0 || j == 0 || k == 0 || i + j + k == m;
                    if (!bnd) continue;
                    int X[3];
                    grid_pos(t, i, j, k, X);
                    long long dst = (long long)t * Lv.C_pad + Lv.lay.index(i, j, k);
                    long long src = slot_of(l, X[0], X[1], X[2]);
                    Lv.tg_dst.push_back((int)dst);
                    Lv.tg_src.push_back((int)src);
                    if (src != Lv.zero_slot) ghost.push_back({(int)(src - Lv.ifc_base), (int)dst});
                }
        Lv.tg_ptr[t + 1] = (int)Lv.tg_dst.size();
    }
    std::sort(ghost.begin(), ghost.end());
    Lv.gptr.assign(Lv.n_ifc + 1, 0);
    Lv.gidx.resize(ghost.size());
    for (size_t q = 0; q < ghost.size(); q++) {
        Lv.gptr[ghost[q].first + 1]++;
        Lv.gidx[q] = ghost[q].second;
    }
    for (int f = 0; f < Lv.n_ifc; f++) Lv.gptr[f + 1] += Lv.gptr[f];

    // same-level 15-point neighbourhoods (mass matrix on interface nodes)
    Lv.nb15.assign(15 * (size_t)Lv.n_ifc, -1);
    for (int f = 0; f < Lv.n_ifc; f++)
        for (int e = 0; e < 15; e++) {
            const auto &X = Lv.ifc_X[f];
            Lv.nb15[(size_t)e * Lv.n_ifc + f] = (int)slot_of(l, X[0] + kGrid15[e][0], X[1] + kGrid15[e][1], X[2] + kGrid15[e][2]);
        }

    for (int q = 0; q < 4; q++) Lv.ifcq[q].clear();
    for (int f = 0; f < Lv.n_ifc; f++) {
        const auto &X = Lv.ifc_X[f];
        Lv.ifcq[(X[0] + X[1] + X[2]) & 3].push_back(f);
    }
    build_closure_tables(Lv);
}

void Topology::build_transfer(int l) {
    TopoLevel &F = lev[l];
    TopoLevel &Cl = lev[l - 1];
    F.prl.assign(2 * (size_t)F.n_ifc, -1);
    for (int f = 0; f < F.n_ifc; f++) {
        const auto &X = F.ifc_X[f];
        int pi[3] = {X[0] & 1, X[1] & 1, X[2] & 1};
        long long s1 = slot_of(l - 1, (X[0] - pi[0]) / 2, (X[1] - pi[1]) / 2, (X[2] - pi[2]) / 2);
        long long s2 = slot_of(l - 1, (X[0] + pi[0]) / 2, (X[1] + pi[1]) / 2, (X[2] + pi[2]) / 2);
        F.prl[f] = (int)s1;
        F.prl[(size_t)F.n_ifc + f] = (int)s2;
    }
    Cl.rst.assign(15 * (size_t)Cl.n_ifc, -1);
    for (int f = 0; f < Cl.n_ifc; f++) {
        const auto &X = Cl.ifc_X[f];
        for (int e = 0; e < 15; e++)
            Cl.rst[(size_t)e * Cl.n_ifc + f] =
                (int)slot_of(l, 2 * X[0] + kGrid15[e][0], 2 * X[1] + kGrid15[e][1], 2 * X[2] + kGrid15[e][2]);
    }
}

void Topology::build_coarse() {
    const TopoLevel &Lv = lev[Lc];
    CoarseSystem &cs = coarse;
    cs = CoarseSystem();
    std::vector<std::array<int, 3>> pos;
    auto grid_pos = [&](int t, int i, int j, int k, int X[3]) {
        for (int a = 0; a < 3; a++) X[a] = Lv.m * V0[t][a] + k;
        X[perm[t][0]] += i + j;
        X[perm[t][1]] += j;
    };
    for (int t = 0; t < n_tets; t++)
        for (int k = 1; k <= Lv.m; k++)
            for (int j = 1; j <= Lv.m - k; j++)
                for (int i = 1; i <= Lv.m - k - j; i++) {
                    if (i + j + k > Lv.m - 1) continue;
                    int X[3];
                    grid_pos(t, i, j, k, X);
                    cs.slot.push_back((long long)t * Lv.C_pad + Lv.lay.index(i, j, k));
                    pos.push_back({X[0], X[1], X[2]});
                    cs.is_vol.push_back(1);
                    cs.tet.push_back(t);
                    cs.ifc.push_back(-1);
                }
    for (int f = 0; f < Lv.n_ifc; f++) {
        cs.slot.push_back(Lv.ifc_base + f);
        pos.push_back(Lv.ifc_X[f]);
        cs.is_vol.push_back(0);
        cs.tet.push_back(-1);
        cs.ifc.push_back(f);
    }
    cs.n = (int)cs.slot.size();
    cs.pos = pos;
    std::vector<std::pair<long long, int>> by_slot(cs.n);
    for (int q = 0; q < cs.n; q++) by_slot[q] = {cs.slot[q], q};
    std::sort(by_slot.begin(), by_slot.end());
    auto unknown_of_slot = [&](long long s) {
        auto it = std::lower_bound(by_slot.begin(), by_slot.end(), std::make_pair(s, -1));
        if (it == by_slot.end() || it->first != s) return -1;
        return it->second;
    };
    cs.col.assign(7 * (size_t)cs.n, -1);
    cs.val.assign(7 * (size_t)cs.n, 0.0);
    cs.grid_dir.assign(7 * (size_t)cs.n, 0);
    for (int q = 0; q < cs.n; q++) {
        cs.col[7 * q] = q;
        cs.val[7 * q] = 6.0 * Lv.h;
        for (int e = 0; e < 6; e++) {
            long long s = slot_of(Lc, pos[q][0] + kAxis6[e][0], pos[q][1] + kAxis6[e][1], pos[q][2] + kAxis6[e][2]);
            int c = s == Lv.zero_slot ? -1 : unknown_of_slot(s);
            cs.col[7 * q + 1 + e] = c;
            cs.val[7 * q + 1 + e] = c >= 0 ? -Lv.h : 0.0;
            cs.grid_dir[7 * q + 1 + e] = 1 + e;
        }
    }
    cs.col15.assign(15 * (size_t)cs.n, -1);
    for (int q = 0; q < cs.n; q++)
        for (int e = 0; e < 15; e++) {
            long long s = slot_of(Lc, pos[q][0] + kGrid15[e][0], pos[q][1] + kGrid15[e][1], pos[q][2] + kGrid15[e][2]);
            cs.col15[15 * (size_t)q + e] = s == Lv.zero_slot ? -1 : unknown_of_slot(s);
        }
    cs.cptr.assign(cs.n + 1, 0);
    cs.cidx.clear();
    for (int q = 0; q < cs.n; q++) {
        cs.cidx.push_back((int)cs.slot[q]);
        if (!cs.is_vol[q]) {
            int f = cs.ifc[q];
            for (int g = Lv.gptr[f]; g < Lv.gptr[f + 1]; g++) cs.cidx.push_back(Lv.gidx[g]);
        }
        cs.cptr[q + 1] = (int)cs.cidx.size();
    }
}

std::string Topology::build(int n, int L_, int Lc_) {
    if (n < 1 || n > 8) return "n_sub must be in 1..8";
    if (Lc_ < 2 || L_ <= Lc_ || L_ > 9) return "need 2 <= coarse_level < level <= 9";
    n_sub = n;
    L = L_;
    Lc = Lc_;
    n_tets = 6 * n * n * n;
    V0.resize(n_tets);
    perm.resize(n_tets);
    for (int cz = 0; cz < n; cz++)
        for (int cy = 0; cy < n; cy++)
            for (int cx = 0; cx < n; cx++)
                for (int p = 0; p < 6; p++) {
                    int t = 6 * (cx + n * (cy + n * cz)) + p;
                    V0[t] = {cx, cy, cz};
                    perm[t] = {kPerm[p][0], kPerm[p][1], kPerm[p][2]};
                }
    lev.assign(L + 1, TopoLevel());
    ifc_key_.assign(L + 1, {});
    ifc_key_idx_.assign(L + 1, {});
    for (int l = Lc; l <= L; l++) build_level(l);
    for (int l = Lc; l <= L; l++) {
        // every slot lookup must have succeeded
        const TopoLevel &Lv = lev[l];
        for (int v : Lv.nbr)
            if (v < 0) return "interface neighbour lookup failed";
        for (int v : Lv.nb15)
            if (v < 0) return "interface 15-point lookup failed";
        for (int v : Lv.tg_src)
            if (v < 0) return "ghost source lookup failed";
        if (Lv.n_slots >= (1LL << 31)) return "level too large for 32-bit slot indices";
    }
    for (int l = Lc + 1; l <= L; l++) {
        build_transfer(l);
        for (int v : lev[l].prl)
            if (v < 0) return "prolongation lookup failed";
        for (int v : lev[l - 1].rst)
            if (v < 0) return "restriction lookup failed";
    }
    build_coarse();
    if (coarse.n > 2048) return "coarsest level has more than 2048 unknowns";
    return "";
}

bool coarse_inverse(int n, int nb, const std::vector<int> &col, const std::vector<double> &val,
                    std::vector<double> &inv) {
    const size_t nn = (size_t)n;
    // lower triangle of A, overwritten by L
    std::vector<double> L(nn * nn, 0.0);
    for (int q = 0; q < n; q++)
        for (int e = 0; e < nb; e++) {
            const int c = col[(size_t)nb * q + e];
            if (c >= 0 && c <= q) L[q * nn + c] += val[(size_t)nb * q + e];
        }
    for (int j = 0; j < n; j++) {
        double *Lj = &L[j * nn];
        double s = Lj[j];
        for (int k = 0; k < j; k++) s -= Lj[k] * Lj[k];
        if (!(s > 0.0)) return false;
        const double d = std::sqrt(s);
        Lj[j] = d;
        for (int i = j + 1; i < n; i++) {
            double *Li = &L[i * nn];
            double t = Li[j];
            for (int k = 0; k < j; k++) t -= Li[k] * Lj[k];
            Li[j] = t / d;
        }
    }
    // U = L^T, row-major, for the backward substitution
    std::vector<double> U(nn * nn, 0.0);
    for (int i = 0; i < n; i++)
        for (int k = 0; k <= i; k++) U[k * nn + i] = L[i * nn + k];
    inv.assign(nn * nn, 0.0);
    std::vector<double> y(nn), x(nn);
    for (int j = 0; j < n; j++) {
        // L y = e_j (y_i = 0 for i < j)
        for (int i = 0; i < j; i++) y[i] = 0.0;
        for (int i = j; i < n; i++) {
            const double *Li = &L[i * nn];
            double t = i == j ? 1.0 : 0.0;
            for (int k = j; k < i; k++) t -= Li[k] * y[k];
            y[i] = t / Li[i];
        }
        // L^T x = y
        for (int i = n - 1; i >= 0; i--) {
            const double *Ui = &U[i * nn];
            double t = y[i];
            for (int k = i + 1; k < n; k++) t -= Ui[k] * x[k];
            x[i] = t / Ui[i];
        }
        for (int i = 0; i < n; i++) inv[i * nn + j] = x[i];
    }
    return true;
}

}  // namespace hhgr
