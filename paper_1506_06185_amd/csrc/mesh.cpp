// Host-side topology of unstructured macro meshes (Sec. 3.1): arbitrary
// tetrahedra, each refined regularly, with the storage model of topology.hpp.
// No HIP calls here.
//
// Every macro tetrahedron is refined the same way in its own index space:
// closure node (i, j, k) has weights (m - i - j - k, i, j, k) on the
// tetrahedron's vertices 0..3, so its position is the weighted mean of the
// corners, and the refined elements are the images of the Kuhn cells of the
// grid X = (i + j + k, j + k, k) (24 around every node).  A node shared by
// several tetrahedra is known by its (macro vertex, weight) pairs, which do
// not depend on the tetrahedron it is seen from.  With the vertices of every
// tetrahedron listed by a proper 4-colouring, the class
// (sum of colour x weight) mod 4 of a node is (i + 2j + 3k) mod 4 inside each
// closure, and no element edge joins two nodes of one class.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <map>
#include <set>
#include <tuple>
#include <unordered_map>

#include "topology.hpp"

namespace hhgr {
namespace {

// up to 3 (vertex, weight) pairs, vertex ascending (nodes on a tetrahedron's
// boundary): vertex < 2^21, weight < 2^10
struct NKey {
    uint64_t lo = 0, hi = 0;
    bool operator==(const NKey &o) const { return lo == o.lo && hi == o.hi; }
};
struct NKeyHash {
    size_t operator()(const NKey &k) const {
        return (size_t)((k.lo * 0x9E3779B97F4A7C15ULL) ^ (k.hi * 0xC2B2AE3D27D4EB4FULL) ^ (k.lo >> 29));
    }
};

struct Support {
    int n = 0;
    int v[4] = {-1, -1, -1, -1};
    int w[4] = {0, 0, 0, 0};
};

// pairs with nonzero weight, vertex ascending
Support support_of(const std::array<int, 4> &tv, const int lam[4]) {
    Support s;
    for (int a = 0; a < 4; a++)
        if (lam[a] > 0) {
            s.v[s.n] = tv[a];
            s.w[s.n] = lam[a];
            s.n++;
        }
    for (int a = 1; a < s.n; a++)
        for (int b = a; b > 0 && s.v[b] < s.v[b - 1]; b--) {
            std::swap(s.v[b], s.v[b - 1]);
            std::swap(s.w[b], s.w[b - 1]);
        }
    return s;
}

NKey key_of(const Support &s) {
    NKey k;
    for (int a = 0; a < s.n && a < 3; a++) {
        const uint64_t p = ((uint64_t)s.v[a] << 10) | (uint64_t)s.w[a];
        if (a < 2)
            k.lo |= p << (31 * a);
        else
            k.hi = p;
    }
    k.hi |= (uint64_t)s.n << 40;
    return k;
}

struct Master {
    NKey key;
    int cls = 0, dim = 0;
    std::array<int, 3> prim{-1, -1, -1};
    std::array<int, 3> w{0, 0, 0};
    long long dof = 0;
};

// the 24 refined elements around a node, as index-space offsets of their
// vertices (one of them the node itself, at self)
struct Around {
    int d[4][3];
    int self;
};

std::vector<Around> elements_around() {
    static const int P[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    std::vector<Around> out;
    for (int oz = -1; oz <= 0; oz++)
        for (int oy = -1; oy <= 0; oy++)
            for (int ox = -1; ox <= 0; ox++)
                for (int p = 0; p < 6; p++) {
                    int X[4][3];
                    const int o[3] = {ox, oy, oz};
                    for (int a = 0; a < 3; a++) {
                        X[0][a] = o[a];
                        X[3][a] = o[a] + 1;
                        X[1][a] = o[a] + (a == P[p][0]);
                        X[2][a] = o[a] + (a == P[p][0] || a == P[p][1]);
                    }
                    int self = -1;
                    for (int r = 0; r < 4; r++)
                        if (X[r][0] == 0 && X[r][1] == 0 && X[r][2] == 0) self = r;
                    if (self < 0) continue;
                    Around e;
                    e.self = self;
                    for (int r = 0; r < 4; r++) {
                        e.d[r][0] = X[r][0] - X[r][1];
                        e.d[r][1] = X[r][1] - X[r][2];
                        e.d[r][2] = X[r][2];
                    }
                    out.push_back(e);
                }
    return out;
}

int idx15_of(const int d[3]) {
    for (int n = 0; n < 15; n++)
        if (kIdx15[n][0] == d[0] && kIdx15[n][1] == d[1] && kIdx15[n][2] == d[2]) return n;
    return -1;
}

// P1 stiffness matrix of the tetrahedron with edge vectors e1, e2, e3 from
// its vertex 0: |det| / 6 times the products of the barycentric gradients
void stiffness(const double e[3][3], double K[4][4]) {
    const double det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                       e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                       e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
    // gradients of the barycentric coordinates 1..3: rows of the inverse of
    // the matrix with the edge vectors as columns (its cofactors / det)
    double g[4][3];
    for (int a = 0; a < 3; a++) {
        const double *p = e[(a + 1) % 3], *q = e[(a + 2) % 3];
        g[a + 1][0] = (p[1] * q[2] - p[2] * q[1]) / det;
        g[a + 1][1] = (p[2] * q[0] - p[0] * q[2]) / det;
        g[a + 1][2] = (p[0] * q[1] - p[1] * q[0]) / det;
    }
    for (int c = 0; c < 3; c++) g[0][c] = -(g[1][c] + g[2][c] + g[3][c]);
    const double vol = std::fabs(det) / 6.0;
    for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++) K[a][b] = vol * (g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2]);
}

// stiffness (K) and mass |e| / 20 (Mq) of the 24 elements around a node of a
// tetrahedron with corners tv refined to m intervals per edge (an element's
// shape depends only on the tetrahedron and its place in the star)
void star_matrices(const double *xyz, const int tv[4], int m, const std::vector<Around> &around, double K[24][4][4],
                   double Mq[24]) {
    double E[3][3];  // index-space unit steps in physical space
    for (int a = 0; a < 3; a++)
        for (int c = 0; c < 3; c++) E[a][c] = (xyz[3 * tv[a + 1] + c] - xyz[3 * tv[0] + c]) / m;
    for (int q = 0; q < 24; q++) {
        const Around &A = around[q];
        double x[4][3];
        for (int r = 0; r < 4; r++)
            for (int c = 0; c < 3; c++) x[r][c] = A.d[r][0] * E[0][c] + A.d[r][1] * E[1][c] + A.d[r][2] * E[2][c];
        double e[3][3];
        for (int r = 0; r < 3; r++)
            for (int c = 0; c < 3; c++) e[r][c] = x[r + 1][c] - x[0][c];
        stiffness(e, K[q]);
        const double det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                           e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                           e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
        Mq[q] = std::fabs(det) / 6.0 / 20.0;
    }
}

inline long long binom3(long long p) { return p >= 3 ? p * (p - 1) * (p - 2) / 6 : 0; }

// one entry of a master's row: slot, stiffness and mass value
struct Entry {
    int s;
    double k, m;
};

}  // namespace

std::string Topology::build_mesh(int nv_, const double *xyz, int nt, const int *tets, int L_, int Lc_) {
    if (nv_ < 4 || nt < 1 || !xyz || !tets) return "need at least 4 vertices and 1 tetrahedron";
    if (nv_ >= (1 << 21)) return "too many vertices";
    if (Lc_ < 2 || L_ <= Lc_ || L_ > 9) return "need 2 <= coarse_level < level <= 9";
    mesh = true;
    n_sub = 0;
    L = L_;
    Lc = Lc_;
    n_tets = nt;
    // vertex colours (positions) and validity of the macro mesh
    std::vector<int> col(nv_, -1);
    std::vector<std::array<int, 4>> tv(nt);
    for (int t = 0; t < nt; t++)
        for (int r = 0; r < 4; r++) {
            const int v = tets[4 * t + r];
            if (v < 0 || v >= nv_) return "vertex id out of range";
            if (col[v] >= 0 && col[v] != r)
                return "vertices must be listed by a 4-colouring (a vertex at the same position in every tetrahedron)";
            col[v] = r;
            tv[t][r] = v;
        }
    for (int v = 0; v < nv_; v++)
        if (col[v] < 0) return "a vertex belongs to no tetrahedron";
    for (int t = 0; t < nt; t++) {
        double e[3][3], lmax = 0.0;
        for (int a = 0; a < 3; a++)
            for (int c = 0; c < 3; c++) e[a][c] = xyz[3 * tv[t][a + 1] + c] - xyz[3 * tv[t][0] + c];
        for (int a = 0; a < 4; a++)
            for (int b = a + 1; b < 4; b++) {
                double d2 = 0.0;
                for (int c = 0; c < 3; c++) {
                    const double d = xyz[3 * tv[t][a] + c] - xyz[3 * tv[t][b] + c];
                    d2 += d * d;
                }
                lmax = std::max(lmax, std::sqrt(d2));
            }
        const double det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                           e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                           e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
        if (!(std::fabs(det) > 1e-8 * lmax * lmax * lmax)) return "a macro tetrahedron is flat";
    }
    // faces: boundary (one tetrahedron) or interior (two); edges and vertices
    // on a boundary face are boundary primitives
    std::map<std::array<int, 3>, int> faces;
    std::set<std::array<int, 2>> edges;
    for (int t = 0; t < nt; t++) {
        std::array<int, 4> s = tv[t];
        std::sort(s.begin(), s.end());
        if (s[0] == s[1] || s[1] == s[2] || s[2] == s[3]) return "a tetrahedron repeats a vertex";
        for (int o = 0; o < 4; o++) {
            std::array<int, 3> f;
            for (int r = 0, q = 0; r < 4; r++)
                if (r != o) f[q++] = s[r];
            if (++faces[f] > 2) return "a face belongs to more than two tetrahedra";
        }
        for (int a = 0; a < 4; a++)
            for (int b = a + 1; b < 4; b++) edges.insert({s[a], s[b]});
    }
    std::set<std::array<int, 3>> bface;
    std::set<std::array<int, 2>> bedge;
    std::vector<char> bvert(nv_, 0);
    for (const auto &f : faces)
        if (f.second == 1) {
            const auto &q = f.first;
            bface.insert(q);
            bedge.insert({q[0], q[1]});
            bedge.insert({q[0], q[2]});
            bedge.insert({q[1], q[2]});
            for (int v : q) bvert[v] = 1;
        }
    // ranks of the interior primitives in the user order
    std::vector<long long> vrank(nv_, -1);
    long long nvi = 0;
    for (int v = 0; v < nv_; v++)
        if (!bvert[v]) vrank[v] = nvi++;
    std::map<std::array<int, 2>, long long> erank;
    for (const auto &e : edges)
        if (!bedge.count(e)) erank.emplace(e, (long long)erank.size());
    std::map<std::array<int, 3>, long long> frank;
    for (const auto &f : faces)
        if (f.second == 2) frank.emplace(f.first, (long long)frank.size());
    auto dirichlet = [&](const Support &s) {
        if (s.n == 1) return bvert[s.v[0]] != 0;
        if (s.n == 2) return bedge.count({s.v[0], s.v[1]}) > 0;
        if (s.n == 3) return bface.count({s.v[0], s.v[1], s.v[2]}) > 0;
        return false;
    };

    mesh_xyz.assign(xyz, xyz + 3 * (size_t)nv_);
    mesh_tets.assign(tets, tets + 4 * (size_t)nt);
    lev.assign(L + 1, TopoLevel());
    std::vector<std::unordered_map<NKey, int, NKeyHash>> kmap(L + 1);
    std::vector<std::vector<Master>> mrec(L + 1);
    std::vector<std::vector<std::vector<Entry>>> rows(L + 1);
    const std::vector<Around> around = elements_around();
    if (around.size() != 24) return "internal: element star";
    int width = 1;
    for (int l = Lc; l <= L; l++) {
        TopoLevel &Lv = lev[l];
        Lv.l = l;
        Lv.m = 1 << l;
        Lv.M = Lv.m + 1;
        Lv.N = 0;
        Lv.h = 1.0 / Lv.m;
        Lv.lay.build(Lv.M);
        Lv.C = Lv.lay.C;
        Lv.C_pad = Lv.lay.span;
        Lv.ifc_base = (long long)nt * Lv.C_pad;
        const int m = Lv.m;
        const long long per_edge = m - 1, per_face = (long long)(m - 1) * (m - 2) / 2;
        Lv.nint = binom3(m - 1);
        Lv.vbase = nvi + (long long)erank.size() * per_edge + (long long)frank.size() * per_face;
        // interface masters: the non-Dirichlet nodes on closure boundaries
        auto &km = kmap[l];
        auto &recs = mrec[l];
        for (int t = 0; t < nt; t++)
            for (int k = 0; k <= m; k++)
                for (int j = 0; j <= m - k; j++)
                    for (int i = 0; i <= m - k - j; i++) {
                        if (!(i == 0 || j == 0 || k == 0 || i + j + k == m)) continue;
                        const int lam[4] = {m - i - j - k, i, j, k};
                        const Support s = support_of(tv[t], lam);
                        if (dirichlet(s)) continue;
                        const NKey key = key_of(s);
                        if (km.count(key)) continue;
                        km.emplace(key, (int)recs.size());
                        Master r;
                        r.key = key;
                        r.dim = s.n - 1;
                        int c = 0;
                        for (int a = 0; a < s.n; a++) {
                            r.prim[a] = s.v[a];
                            r.w[a] = s.w[a];
                            c += col[s.v[a]] * s.w[a];
                        }
                        r.cls = c & 3;
                        if (s.n == 1) {
                            r.dof = vrank[s.v[0]];
                        } else if (s.n == 2) {
                            r.dof = nvi + erank.at({s.v[0], s.v[1]}) * per_edge + (s.w[1] - 1);
                        } else {
                            const long long C = s.w[2], B = s.w[1];
                            r.dof = nvi + (long long)erank.size() * per_edge + frank.at({s.v[0], s.v[1], s.v[2]}) * per_face +
                                    (C - 1) * (m - 1) - (C - 1) * C / 2 + (B - 1);
                        }
                        recs.push_back(r);
                    }
        // masters ordered by class parity (even classes first), class,
        // primitive (faces, edges, vertices), then position
        std::sort(recs.begin(), recs.end(), [](const Master &a, const Master &b) {
            return std::make_tuple(a.cls & 1, a.cls, -a.dim, a.prim, a.w) <
                   std::make_tuple(b.cls & 1, b.cls, -b.dim, b.prim, b.w);
        });
        Lv.n_ifc = (int)recs.size();
        Lv.n_ifc_red = 0;
        Lv.ifc_X.assign(Lv.n_ifc, {0, 0, 0});
        Lv.ifc_dof.resize(Lv.n_ifc);
        for (int q = 0; q < 4; q++) Lv.ifcq[q].clear();
        for (int f = 0; f < Lv.n_ifc; f++) {
            km[recs[f].key] = f;
            if ((recs[f].cls & 1) == 0) Lv.n_ifc_red++;
            Lv.ifc_dof[f] = (int)recs[f].dof;
            Lv.ifcq[recs[f].cls].push_back(f);
        }
        Lv.zero_slot = Lv.ifc_base + Lv.n_ifc;
        Lv.n_slots = round_up(Lv.zero_slot + 1, 64);
        if (Lv.n_slots >= (1LL << 31)) return "level too large for 32-bit slot indices";
        if (Lv.vbase + (long long)nt * Lv.nint >= (1LL << 31)) return "too many unknowns for 32-bit user indices";
        // slot of closure node (i, j, k) of tetrahedron t (a closure
        // boundary node: its master's slot, or the zero slot)
        auto slot = [&](int t, int i, int j, int k) -> long long {
            if (i > 0 && j > 0 && k > 0 && i + j + k < m) return (long long)t * Lv.C_pad + Lv.lay.index(i, j, k);
            const int lam[4] = {m - i - j - k, i, j, k};
            const Support s = support_of(tv[t], lam);
            auto it = km.find(key_of(s));
            return it == km.end() ? Lv.zero_slot : Lv.ifc_base + it->second;
        };
        // the same for every node of one closure, looked up once per node;
        // on the finest level also the boundary index of Dirichlet nodes
        std::vector<int> cslot(Lv.C_pad), cbnd(Lv.C_pad, -1);
        std::unordered_map<NKey, int, NKeyHash> bmap;
        if (l == L) {
            // boundary nodes in the order of the interior ones: vertices by
            // id, edges (a < b) by the weight of b, faces (a < b < c) by the
            // weights of c then b
            std::vector<Master> br;
            for (int t = 0; t < nt; t++)
                for (int k = 0; k <= m; k++)
                    for (int j = 0; j <= m - k; j++)
                        for (int i = 0; i <= m - k - j; i++) {
                            if (!(i == 0 || j == 0 || k == 0 || i + j + k == m)) continue;
                            const int lam[4] = {m - i - j - k, i, j, k};
                            const Support s = support_of(tv[t], lam);
                            if (!dirichlet(s)) continue;
                            const NKey key = key_of(s);
                            if (bmap.count(key)) continue;
                            bmap.emplace(key, (int)br.size());
                            Master r;
                            r.key = key;
                            r.dim = s.n - 1;
                            for (int a = 0; a < s.n; a++) {
                                r.prim[a] = s.v[a];
                                r.w[a] = s.w[a];
                            }
                            br.push_back(r);
                        }
            auto order = [](const Master &r) {
                // (dim, primitive, weight of the last vertex, then of the middle one)
                const int wl = r.dim >= 1 ? r.w[r.dim] : 0, wm = r.dim == 2 ? r.w[1] : 0;
                return std::make_tuple(r.dim, r.prim, wl, wm);
            };
            std::sort(br.begin(), br.end(), [&](const Master &a, const Master &b) { return order(a) < order(b); });
            bnd_xyz.assign(3 * br.size(), 0.0);
            for (size_t q = 0; q < br.size(); q++) {
                bmap[br[q].key] = (int)q;
                for (int a = 0; a <= br[q].dim; a++)
                    for (int c = 0; c < 3; c++) bnd_xyz[3 * q + c] += br[q].w[a] * xyz[3 * br[q].prim[a] + c] / m;
            }
            n_bnd = (long long)br.size();
        }
        auto fill_cslot = [&](int t) {
            for (int k = 0; k <= m; k++)
                for (int j = 0; j <= m - k; j++)
                    for (int i = 0; i <= m - k - j; i++) {
                        const int q = Lv.lay.index(i, j, k);
                        cslot[q] = (int)slot(t, i, j, k);
                        if (l == L && cslot[q] == Lv.zero_slot) {
                            const int lam[4] = {m - i - j - k, i, j, k};
                            auto it = bmap.find(key_of(support_of(tv[t], lam)));
                            cbnd[q] = it == bmap.end() ? -1 : it->second;
                        } else {
                            cbnd[q] = -1;
                        }
                    }
        };
        // finest level: the couplings of interior nodes (slot, boundary
        // index, stiffness) to Dirichlet nodes, for eliminated boundary data
        std::map<std::pair<int, int>, double> dir;
        if (l == L) {
            dir_bnd_ptr.assign(nt + 1, 0);
            dir_bnd_pos.clear();
            dir_bnd_idx.clear();
        }
        // ghost copies
        Lv.nbr.assign(6 * (size_t)Lv.n_ifc, (int)Lv.zero_slot);
        Lv.tg_ptr.assign(nt + 1, 0);
        Lv.tg_dst.clear();
        Lv.tg_src.clear();
        std::vector<std::pair<int, int>> ghost;
        for (int t = 0; t < nt; t++) {
            for (int k = 0; k <= m; k++)
                for (int j = 0; j <= m - k; j++)
                    for (int i = 0; i <= m - k - j; i++) {
                        if (!(i == 0 || j == 0 || k == 0 || i + j + k == m)) continue;
                        const long long dst = (long long)t * Lv.C_pad + Lv.lay.index(i, j, k);
                        const long long src = slot(t, i, j, k);
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
        // stencils: the 24 element matrices of each tetrahedron at this level
        // (an element's shape depends only on its tetrahedron and its place
        // in the star), summed over the elements inside the closure
        Lv.mesh_w15.assign(15 * (size_t)nt, 0.0);
        Lv.mesh_mw15.assign(15 * (size_t)nt, 0.0);
        auto &R = rows[l];
        R.assign(Lv.n_ifc, {});
        for (int t = 0; t < nt; t++) {
            double K[24][4][4], Mq[24];  // stiffness; mass |e| / 20 (1 + delta)
            star_matrices(xyz, tv[t].data(), m, around, K, Mq);
            for (int q = 0; q < 24; q++) {
                const Around &A = around[q];
                for (int r = 0; r < 4; r++) {
                    int d[3] = {A.d[r][0] - A.d[A.self][0], A.d[r][1] - A.d[A.self][1], A.d[r][2] - A.d[A.self][2]};
                    const int n = idx15_of(d);
                    if (n < 0) return "internal: element star outside the 15-point stencil";
                    Lv.mesh_w15[15 * (size_t)t + n] += K[q][A.self][r];
                    Lv.mesh_mw15[15 * (size_t)t + n] += Mq[q] * (r == A.self ? 2.0 : 1.0);
                }
            }
            fill_cslot(t);
            if (l == L) {
                for (int q = 0; q < Lv.C_pad; q++)
                    if (cbnd[q] >= 0) {
                        dir_bnd_pos.push_back(q);
                        dir_bnd_idx.push_back(cbnd[q]);
                    }
                dir_bnd_ptr[t + 1] = (int)dir_bnd_pos.size();
            }
            if (l == L)
                for (int k = 1; k < m; k++)
                    for (int j = 1; j < m - k; j++)
                        for (int i = 1; i + j + k <= m - 1; i++) {
                            if (!(i == 1 || j == 1 || k == 1 || i + j + k == m - 1)) continue;
                            const int own = cslot[Lv.lay.index(i, j, k)];
                            for (int n = 1; n < 15; n++) {
                                const int q = Lv.lay.index(i + kIdx15[n][0], j + kIdx15[n][1], k + kIdx15[n][2]);
                                if (cbnd[q] >= 0) dir[{own, cbnd[q]}] += Lv.mesh_w15[15 * (size_t)t + n];
                            }
                        }
            for (int k = 0; k <= m; k++)
                for (int j = 0; j <= m - k; j++)
                    for (int i = 0; i <= m - k - j; i++) {
                        if (!(i == 0 || j == 0 || k == 0 || i + j + k == m)) continue;
                        const long long own = cslot[Lv.lay.index(i, j, k)];
                        if (own == Lv.zero_slot) continue;
                        auto &row = R[own - Lv.ifc_base];
                        if (row.empty()) row.push_back({(int)own, 0.0, 0.0});
                        for (int q = 0; q < 24; q++) {
                            const Around &A = around[q];
                            int p[4][3];
                            bool in = true;
                            for (int r = 0; r < 4 && in; r++) {
                                p[r][0] = i + A.d[r][0] - A.d[A.self][0];
                                p[r][1] = j + A.d[r][1] - A.d[A.self][1];
                                p[r][2] = k + A.d[r][2] - A.d[A.self][2];
                                in = p[r][0] >= 0 && p[r][1] >= 0 && p[r][2] >= 0 && p[r][0] + p[r][1] + p[r][2] <= m;
                            }
                            if (!in) continue;
                            for (int r = 0; r < 4; r++) {
                                const int pq = Lv.lay.index(p[r][0], p[r][1], p[r][2]);
                                if (cbnd[pq] >= 0) dir[{(int)own, cbnd[pq]}] += K[q][A.self][r];
                                const int s = cslot[pq];
                                size_t e = 0;
                                while (e < row.size() && row[e].s != s) e++;
                                if (e == row.size()) row.push_back({s, 0.0, 0.0});
                                row[e].k += K[q][A.self][r];
                                row[e].m += Mq[q] * (r == A.self ? 2.0 : 1.0);
                            }
                        }
                    }
        }
        for (const auto &row : R) width = std::max(width, (int)row.size());
        if (l == L) {
            // rows by slot, columns by boundary index (std::map order)
            dir_rows.clear();
            dir_ptr.assign(1, 0);
            dir_col.clear();
            dir_val.clear();
            for (const auto &e : dir) {
                if (dir_rows.empty() || dir_rows.back() != e.first.first) {
                    if (!dir_rows.empty()) dir_ptr.push_back((int)dir_col.size());
                    dir_rows.push_back(e.first.first);
                }
                dir_col.push_back(e.first.second);
                dir_val.push_back(e.second);
            }
            dir_ptr.push_back((int)dir_col.size());
        }
        build_closure_tables(Lv);
    }
    // stencil width of every level; neighbours after the diagonal by slot
    nbw = width;
    for (int l = Lc; l <= L; l++) {
        TopoLevel &Lv = lev[l];
        const size_t n = (size_t)Lv.n_ifc;
        Lv.nb15.assign((size_t)nbw * n, (int)Lv.zero_slot);
        Lv.mesh_wi.assign((size_t)nbw * n, 0.0);
        Lv.mesh_mwi.assign((size_t)nbw * n, 0.0);
        for (size_t f = 0; f < n; f++) {
            auto &row = rows[l][f];
            std::sort(row.begin() + 1, row.end(), [](const Entry &a, const Entry &b) { return a.s < b.s; });
            for (size_t e = 0; e < row.size(); e++) {
                Lv.nb15[e * n + f] = row[e].s;
                Lv.mesh_wi[e * n + f] = row[e].k;
                Lv.mesh_mwi[e * n + f] = row[e].m;
            }
        }
    }
    // transfers: a fine master is an old node (all weights even: one coarse
    // parent) or the midpoint of a coarse edge (two odd weights); the fine
    // nodes restricted into a coarse master are its fine twin and the twin's
    // neighbours, which are the midpoints of the coarse edges at the node
    for (int l = Lc + 1; l <= L; l++) {
        TopoLevel &F = lev[l], &Cl = lev[l - 1];
        const int nf = F.n_ifc, nc = Cl.n_ifc;
        auto coarse_slot = [&](const Support &s) -> long long {
            Support h;
            for (int a = 0; a < s.n; a++)
                if (s.w[a] > 0) {
                    h.v[h.n] = s.v[a];
                    h.w[h.n] = s.w[a];
                    h.n++;
                }
            auto it = kmap[l - 1].find(key_of(h));
            return it == kmap[l - 1].end() ? Cl.zero_slot : Cl.ifc_base + it->second;
        };
        F.prl.assign(2 * (size_t)nf, -1);
        for (int f = 0; f < nf; f++) {
            const Master &r = mrec[l][f];
            Support s;
            s.n = r.dim + 1;
            int odd[3], no = 0;
            for (int a = 0; a < s.n; a++) {
                s.v[a] = r.prim[a];
                s.w[a] = r.w[a];
                if (r.w[a] & 1) odd[no++] = a;
            }
            if (no != 0 && no != 2) return "internal: interface node is not an old node or an edge midpoint";
            Support p = s, q = s;
            if (no == 2) {
                p.w[odd[0]] -= 1;
                p.w[odd[1]] += 1;
                q.w[odd[0]] += 1;
                q.w[odd[1]] -= 1;
            }
            for (int a = 0; a < s.n; a++) {
                p.w[a] /= 2;
                q.w[a] /= 2;
            }
            F.prl[f] = (int)coarse_slot(p);
            F.prl[(size_t)nf + f] = (int)coarse_slot(q);
        }
        Cl.rst.assign((size_t)nbw * nc, (int)F.zero_slot);
        for (int f = 0; f < nc; f++) {
            const Master &r = mrec[l - 1][f];
            Support s;
            s.n = r.dim + 1;
            for (int a = 0; a < s.n; a++) {
                s.v[a] = r.prim[a];
                s.w[a] = 2 * r.w[a];
            }
            auto it = kmap[l].find(key_of(s));
            if (it == kmap[l].end()) return "internal: coarse master without a fine twin";
            for (int e = 0; e < nbw; e++) Cl.rst[(size_t)e * nc + f] = F.nb15[(size_t)e * nf + it->second];
        }
    }
    n_dofs = lev[L].vbase + (long long)nt * lev[L].nint;

    // coarsest level: the interior nodes of every closure, then the masters
    const TopoLevel &Lv = lev[Lc];
    CoarseSystem &cs = coarse;
    cs = CoarseSystem();
    std::vector<int> unk(Lv.n_slots, -1);
    for (int t = 0; t < nt; t++)
        for (int k = 1; k <= Lv.m; k++)
            for (int j = 1; j <= Lv.m - k; j++)
                for (int i = 1; i + j + k <= Lv.m - 1; i++) {
                    const long long sl = (long long)t * Lv.C_pad + Lv.lay.index(i, j, k);
                    unk[sl] = (int)cs.slot.size();
                    cs.slot.push_back(sl);
                    cs.is_vol.push_back(1);
                    cs.tet.push_back(t);
                    cs.ifc.push_back(-1);
                }
    for (int f = 0; f < Lv.n_ifc; f++) {
        unk[Lv.ifc_base + f] = (int)cs.slot.size();
        cs.slot.push_back(Lv.ifc_base + f);
        cs.is_vol.push_back(0);
        cs.tet.push_back(-1);
        cs.ifc.push_back(f);
    }
    for (size_t q = 0; q < Lv.tg_dst.size(); q++)
        if (Lv.tg_src[q] != Lv.zero_slot) unk[Lv.tg_dst[q]] = unk[Lv.tg_src[q]];
    cs.n = (int)cs.slot.size();
    cs.pos.assign(cs.n, {0, 0, 0});
    std::vector<std::vector<std::pair<int, double>>> crow(cs.n);
    auto add = [&](int q, long long s, double v) {
        const int c = s < 0 || s == Lv.zero_slot ? -1 : unk[s];
        if (c < 0) return;
        auto &row = crow[q];
        size_t e = 0;
        while (e < row.size() && row[e].first != c) e++;
        if (e == row.size()) row.push_back({c, 0.0});
        row[e].second += v;
    };
    for (int q = 0; q < cs.n; q++) {
        crow[q].push_back({q, 0.0});
        if (cs.is_vol[q]) {
            const int t = cs.tet[q];
            const long long sl = cs.slot[q] - (long long)t * Lv.C_pad;
            int ii = -1, jj = -1, kk = -1;
            for (int k = 1; k <= Lv.m && ii < 0; k++)
                for (int j = 1; j <= Lv.m - k && ii < 0; j++)
                    for (int i = 1; i + j + k <= Lv.m - 1; i++)
                        if (Lv.lay.index(i, j, k) == sl) {
                            ii = i;
                            jj = j;
                            kk = k;
                            break;
                        }
            for (int n = 0; n < 15; n++) {
                const int i = ii + kIdx15[n][0], j = jj + kIdx15[n][1], k = kk + kIdx15[n][2];
                add(q, (long long)t * Lv.C_pad + Lv.lay.index(i, j, k), Lv.mesh_w15[15 * (size_t)t + n]);
            }
        } else {
            const int f = cs.ifc[q];
            for (int e = 0; e < nbw; e++)
                add(q, Lv.nb15[(size_t)e * Lv.n_ifc + f], Lv.mesh_wi[(size_t)e * Lv.n_ifc + f]);
        }
    }
    cs.cw = 1;
    for (const auto &row : crow) cs.cw = std::max(cs.cw, (int)row.size());
    cs.colw.assign((size_t)cs.cw * cs.n, -1);
    cs.valw.assign((size_t)cs.cw * cs.n, 0.0);
    for (int q = 0; q < cs.n; q++)
        for (size_t e = 0; e < crow[q].size(); e++) {
            cs.colw[(size_t)cs.cw * q + e] = crow[q][e].first;
            cs.valw[(size_t)cs.cw * q + e] = crow[q][e].second;
        }
    // the cube's 7- and 15-column tables hold the diagonal only
    cs.col.assign(7 * (size_t)cs.n, -1);
    cs.val.assign(7 * (size_t)cs.n, 0.0);
    cs.grid_dir.assign(7 * (size_t)cs.n, 0);
    cs.col15.assign(15 * (size_t)cs.n, -1);
    for (int q = 0; q < cs.n; q++) {
        cs.col[7 * (size_t)q] = q;
        cs.val[7 * (size_t)q] = crow[q][0].second;
        cs.col15[15 * (size_t)q] = q;
    }
    cs.cptr.assign(cs.n + 1, 0);
    cs.cidx.clear();
    for (int q = 0; q < cs.n; q++) {
        cs.cidx.push_back((int)cs.slot[q]);
        if (!cs.is_vol[q]) {
            const int f = cs.ifc[q];
            for (int g = Lv.gptr[f]; g < Lv.gptr[f + 1]; g++) cs.cidx.push_back(Lv.gidx[g]);
        }
        cs.cptr[q + 1] = (int)cs.cidx.size();
    }
    return "";
}

void Topology::mesh_kuhn_matrices(int l, std::vector<double> &kel) const {
    static const int P[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    const int m = 1 << l;
    kel.assign(96 * (size_t)n_tets, 0.0);
    for (int t = 0; t < n_tets; t++) {
        const int *tv = &mesh_tets[4 * (size_t)t];
        double E[3][3];  // index-space unit steps (i, j, k) in physical space
        for (int a = 0; a < 3; a++)
            for (int c = 0; c < 3; c++) E[a][c] = (mesh_xyz[3 * tv[a + 1] + c] - mesh_xyz[3 * tv[0] + c]) / m;
        for (int p = 0; p < 6; p++) {
            int X[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {1, 1, 1}};
            X[1][P[p][0]] = 1;
            X[2][P[p][0]] = X[2][P[p][1]] = 1;
            double x[4][3];
            for (int r = 0; r < 4; r++) {
                const int ijk[3] = {X[r][0] - X[r][1], X[r][1] - X[r][2], X[r][2]};
                for (int c = 0; c < 3; c++) x[r][c] = ijk[0] * E[0][c] + ijk[1] * E[1][c] + ijk[2] * E[2][c];
            }
            double e[3][3], K[4][4];
            for (int r = 0; r < 3; r++)
                for (int c = 0; c < 3; c++) e[r][c] = x[r + 1][c] - x[0][c];
            stiffness(e, K);
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 4; b++) kel[96 * (size_t)t + 16 * p + 4 * a + b] = K[a][b];
        }
    }
}

std::string Topology::mesh_weighted_operators(const double *wt, const unsigned char *dirty,
                                              const std::vector<std::vector<double>> *base, MeshOps &out,
                                              bool with_dir) const {
    if (!mesh) return "not an unstructured macro mesh";
    const int nt = n_tets;
    const std::vector<Around> around = elements_around();
    if (around.size() != 24) return "internal: element star";
    out.w15.assign(L + 1, {});
    out.wi.assign(L + 1, {});
    std::vector<int> cslot;
    for (int l = Lc; l <= L; l++) {
        const TopoLevel &Lv = lev[l];
        const int m = Lv.m;
        const size_t n = (size_t)Lv.n_ifc;
        out.w15[l].resize(15 * (size_t)nt);
        for (int t = 0; t < nt; t++)
            for (int q = 0; q < 15; q++) out.w15[l][15 * (size_t)t + q] = wt[t] * Lv.mesh_w15[15 * (size_t)t + q];
        std::vector<double> &W = out.wi[l];
        W = base ? (*base)[l] : Lv.mesh_wi;
        if (W.size() != (size_t)nbw * n) return "internal: base rows of the wrong size";
        // masters with a copy in a flagged closure: their rows are summed
        // again, k times each element matrix, in the order of build_mesh
        std::vector<char> aff(n, 0);
        for (int t = 0; t < nt; t++)
            if (dirty[t])
                for (int q = Lv.tg_ptr[t]; q < Lv.tg_ptr[t + 1]; q++)
                    if (Lv.tg_src[q] != Lv.zero_slot) aff[Lv.tg_src[q] - Lv.ifc_base] = 1;
        for (size_t f = 0; f < n; f++)
            if (aff[f])
                for (int e = 0; e < nbw; e++) W[e * n + f] = 0.0;
        cslot.assign(Lv.C_pad, (int)Lv.zero_slot);
        for (int t = 0; t < nt; t++) {
            if (wt[t] == 0.0) continue;
            bool touch = false;
            for (int q = Lv.tg_ptr[t]; q < Lv.tg_ptr[t + 1] && !touch; q++)
                touch = Lv.tg_src[q] != Lv.zero_slot && aff[Lv.tg_src[q] - Lv.ifc_base];
            if (!touch) continue;
            // closure slots: interior nodes in the closure, boundary nodes
            // from the ghost list (built in the same plane, row, i order)
            int g = Lv.tg_ptr[t];
            for (int k = 0; k <= m; k++)
                for (int j = 0; j <= m - k; j++)
                    for (int i = 0; i <= m - k - j; i++) {
                        const int idx = Lv.lay.index(i, j, k);
                        if (i == 0 || j == 0 || k == 0 || i + j + k == m) {
                            if (g >= Lv.tg_ptr[t + 1] || Lv.tg_dst[g] != (long long)t * Lv.C_pad + idx)
                                return "internal: ghost list out of order";
                            cslot[idx] = Lv.tg_src[g++];
                        } else {
                            cslot[idx] = (int)((long long)t * Lv.C_pad + idx);
                        }
                    }
            double K[24][4][4], Mq[24];
            star_matrices(mesh_xyz.data(), &mesh_tets[4 * (size_t)t], m, around, K, Mq);
            for (int k = 0; k <= m; k++)
                for (int j = 0; j <= m - k; j++)
                    for (int i = 0; i <= m - k - j; i++) {
                        if (!(i == 0 || j == 0 || k == 0 || i + j + k == m)) continue;
                        const long long own = cslot[Lv.lay.index(i, j, k)];
                        if (own == Lv.zero_slot || !aff[own - Lv.ifc_base]) continue;
                        const size_t f = (size_t)(own - Lv.ifc_base);
                        for (int q = 0; q < 24; q++) {
                            const Around &A = around[q];
                            int p[4][3];
                            bool in = true;
                            for (int r = 0; r < 4 && in; r++) {
                                p[r][0] = i + A.d[r][0] - A.d[A.self][0];
                                p[r][1] = j + A.d[r][1] - A.d[A.self][1];
                                p[r][2] = k + A.d[r][2] - A.d[A.self][2];
                                in = p[r][0] >= 0 && p[r][1] >= 0 && p[r][2] >= 0 && p[r][0] + p[r][1] + p[r][2] <= m;
                            }
                            if (!in) continue;
                            for (int r = 0; r < 4; r++) {
                                const int s = cslot[Lv.lay.index(p[r][0], p[r][1], p[r][2])];
                                int e = 0;
                                while (e < nbw && Lv.nb15[e * n + f] != s) e++;
                                if (e == nbw) return "internal: weighted entry outside the master's row";
                                W[e * n + f] += wt[t] * K[q][A.self][r];
                            }
                        }
                    }
        }
    }
    // coarsest level: the rows of build_mesh from the weighted stencils
    const TopoLevel &Lv = lev[Lc];
    const CoarseSystem &cs = coarse;
    const size_t n = (size_t)Lv.n_ifc;
    std::vector<int> unk(Lv.n_slots, -1);
    for (int q = 0; q < cs.n; q++) unk[cs.slot[q]] = q;
    for (size_t q = 0; q < Lv.tg_dst.size(); q++)
        if (Lv.tg_src[q] != Lv.zero_slot) unk[Lv.tg_dst[q]] = unk[Lv.tg_src[q]];
    std::vector<std::array<int, 3>> ijk(Lv.C_pad, {-1, -1, -1});
    for (int k = 0; k <= Lv.m; k++)
        for (int j = 0; j <= Lv.m - k; j++)
            for (int i = 0; i <= Lv.m - k - j; i++) ijk[Lv.lay.index(i, j, k)] = {i, j, k};
    out.valw.assign(cs.valw.size(), 0.0);
    for (int q = 0; q < cs.n; q++) {
        double *row = &out.valw[(size_t)cs.cw * q];
        auto add = [&](long long s, double v) -> bool {
            const int c = s < 0 || s == Lv.zero_slot ? -1 : unk[s];
            if (c < 0) return true;
            int p = 0;
            while (p < cs.cw && cs.colw[(size_t)cs.cw * q + p] != c) p++;
            if (p == cs.cw) return false;
            row[p] += v;
            return true;
        };
        if (cs.is_vol[q]) {
            const int t = cs.tet[q];
            const std::array<int, 3> &x = ijk[cs.slot[q] - (long long)t * Lv.C_pad];
            for (int e = 0; e < 15; e++)
                if (!add((long long)t * Lv.C_pad + Lv.lay.index(x[0] + kIdx15[e][0], x[1] + kIdx15[e][1],
                                                                 x[2] + kIdx15[e][2]),
                         out.w15[Lc][15 * (size_t)t + e]))
                    return "internal: weighted coarse entry outside the row";
        } else {
            const size_t f = (size_t)cs.ifc[q];
            for (int e = 0; e < nbw; e++)
                if (!add(Lv.nb15[e * n + f], out.wi[Lc][e * n + f]))
                    return "internal: weighted coarse entry outside the row";
        }
    }
    // finest level: the couplings to the Dirichlet boundary nodes, summed
    // in the order of build_mesh (same keys, so the same entries)
    if (!with_dir) return "";
    const TopoLevel &F = lev[L];
    const int m = F.m;
    std::map<std::pair<int, int>, double> dir;
    std::vector<int> cbnd(F.C_pad, -1);
    cslot.assign(F.C_pad, (int)F.zero_slot);
    for (int t = 0; t < nt; t++) {
        if (dir_bnd_ptr[t] == dir_bnd_ptr[t + 1]) continue;
        int g = F.tg_ptr[t];
        for (int k = 0; k <= m; k++)
            for (int j = 0; j <= m - k; j++)
                for (int i = 0; i <= m - k - j; i++) {
                    const int idx = F.lay.index(i, j, k);
                    if (i == 0 || j == 0 || k == 0 || i + j + k == m) {
                        if (g >= F.tg_ptr[t + 1] || F.tg_dst[g] != (long long)t * F.C_pad + idx)
                            return "internal: ghost list out of order";
                        cslot[idx] = F.tg_src[g++];
                    } else {
                        cslot[idx] = (int)((long long)t * F.C_pad + idx);
                    }
                }
        for (int q = dir_bnd_ptr[t]; q < dir_bnd_ptr[t + 1]; q++) cbnd[dir_bnd_pos[q]] = dir_bnd_idx[q];
        for (int k = 1; k < m; k++)
            for (int j = 1; j < m - k; j++)
                for (int i = 1; i + j + k <= m - 1; i++) {
                    if (!(i == 1 || j == 1 || k == 1 || i + j + k == m - 1)) continue;
                    const int own = cslot[F.lay.index(i, j, k)];
                    for (int n = 1; n < 15; n++) {
                        const int q = F.lay.index(i + kIdx15[n][0], j + kIdx15[n][1], k + kIdx15[n][2]);
                        if (cbnd[q] >= 0) dir[{own, cbnd[q]}] += wt[t] * F.mesh_w15[15 * (size_t)t + n];
                    }
                }
        double K[24][4][4], Mq[24];
        star_matrices(mesh_xyz.data(), &mesh_tets[4 * (size_t)t], m, around, K, Mq);
        for (int k = 0; k <= m; k++)
            for (int j = 0; j <= m - k; j++)
                for (int i = 0; i <= m - k - j; i++) {
                    if (!(i == 0 || j == 0 || k == 0 || i + j + k == m)) continue;
                    const long long own = cslot[F.lay.index(i, j, k)];
                    if (own == F.zero_slot) continue;
                    for (int q = 0; q < 24; q++) {
                        const Around &A = around[q];
                        int p[4][3];
                        bool in = true;
                        for (int r = 0; r < 4 && in; r++) {
                            p[r][0] = i + A.d[r][0] - A.d[A.self][0];
                            p[r][1] = j + A.d[r][1] - A.d[A.self][1];
                            p[r][2] = k + A.d[r][2] - A.d[A.self][2];
                            in = p[r][0] >= 0 && p[r][1] >= 0 && p[r][2] >= 0 && p[r][0] + p[r][1] + p[r][2] <= m;
                        }
                        if (!in) continue;
                        for (int r = 0; r < 4; r++) {
                            const int pq = F.lay.index(p[r][0], p[r][1], p[r][2]);
                            if (cbnd[pq] >= 0) dir[{(int)own, cbnd[pq]}] += wt[t] * K[q][A.self][r];
                        }
                    }
                }
        for (int q = dir_bnd_ptr[t]; q < dir_bnd_ptr[t + 1]; q++) cbnd[dir_bnd_pos[q]] = -1;
    }
    if (dir.size() != dir_val.size()) return "internal: Dirichlet couplings of a different pattern";
    out.dir_val.clear();
    for (const auto &e : dir) out.dir_val.push_back(e.second);
    return "";
}

}  // namespace hhgr
