// Host-side stencils of the P1 stiffness matrix on a general macro mesh
// (see geometry.hpp).
#include "geometry.hpp"

#include <algorithm>
#include <cmath>
#include <thread>

namespace hhgr {

namespace {

// the 24 Kuhn elements around a grid node X: element of the unit cube with
// corner c = X - s and axis order kPerm[pi], X its vertex r; vertex r of
// such an element sits at c + o_r with o = {0, e_p0, e_p0 + e_p1, (1,1,1)}
struct Around {
    int pi, r;
    int o[4][3];
};

std::array<Around, 24> make_around() {
    std::array<Around, 24> a{};
    int q = 0;
    for (int pi = 0; pi < 6; pi++)
        for (int r = 0; r < 4; r++) {
            Around &e = a[q++];
            e.pi = pi;
            e.r = r;
            for (int v = 0; v < 4; v++)
                for (int d = 0; d < 3; d++) e.o[v][d] = 0;
            e.o[1][kPerm[pi][0]] = 1;
            e.o[2][kPerm[pi][0]] = 1;
            e.o[2][kPerm[pi][1]] = 1;
            for (int d = 0; d < 3; d++) e.o[3][d] = 1;
        }
    return a;
}

const std::array<Around, 24> &around() {
    static const std::array<Around, 24> a = make_around();
    return a;
}

inline void cross(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
inline double dot(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// P1 stiffness of the tetrahedron with edge vectors e1, e2, e3 from vertex 0:
// K_ab = |T| grad(phi_a) . grad(phi_b), the gradients being the rows of the
// inverse of [e1 e2 e3] (and minus their sum for vertex 0)
void p1_stiffness(const double *e1, const double *e2, const double *e3, double K[4][4]) {
    double g[4][3];
    cross(e2, e3, g[1]);
    cross(e3, e1, g[2]);
    cross(e1, e2, g[3]);
    const double det = dot(e1, g[1]);
    for (int v = 1; v < 4; v++)
        for (int d = 0; d < 3; d++) g[v][d] /= det;
    for (int d = 0; d < 3; d++) g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
    const double vol = std::fabs(det) / 6.0;
    for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++) K[a][b] = vol * dot(g[a], g[b]);
}

// consistent P1 mass matrix of the same tetrahedron: |T| / 20 (1 + delta_ab)
void p1_mass(const double *e1, const double *e2, const double *e3, double Mm[4][4]) {
    double c[3];
    cross(e2, e3, c);
    const double vol = std::fabs(dot(e1, c)) / 6.0;
    for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++) Mm[a][b] = vol / 20.0 * (a == b ? 2.0 : 1.0);
}

void corners(const Topology &tp, const double *xyz, int t, double P[4][3]) {
    const int n1 = tp.n_sub + 1;
    int v[3] = {tp.V0[t][0], tp.V0[t][1], tp.V0[t][2]};
    for (int s = 0; s < 4; s++) {
        if (s > 0) v[tp.perm[t][s - 1]] += 1;
        const long long id = v[0] + (long long)n1 * (v[1] + (long long)n1 * v[2]);
        for (int d = 0; d < 3; d++) P[s][d] = xyz[3 * id + d];
    }
}

}  // namespace

int grid15_index(int dx, int dy, int dz) {
    for (int e = 0; e < 15; e++)
        if (kGrid15[e][0] == dx && kGrid15[e][1] == dy && kGrid15[e][2] == dz) return e;
    return -1;
}

StencilBuilder::StencilBuilder(const Topology &tp, const double *xyz, int l) : tp_(tp), m_(1 << l) {
    E_.resize(tp.n_tets);
    for (int t = 0; t < tp.n_tets; t++) {
        double P[4][3];
        corners(tp, xyz, t, P);
        for (int s = 0; s < 3; s++)
            for (int d = 0; d < 3; d++) E_[t][3 * s + d] = (P[s + 1][d] - P[0][d]) / m_;
    }
}

// macro tetrahedron holding the element of the cube with corner c and axis
// order kPerm[pi]: 4 x its centroid is 4c + 3 e_p0 + 2 e_p1 + e_p2; the
// macro cube is that over 4m, the macro axis order sorts the remainders
int StencilBuilder::macro_tet(const int c[3], int pi) const {
    int C4[3] = {4 * c[0], 4 * c[1], 4 * c[2]};
    C4[kPerm[pi][0]] += 3;
    C4[kPerm[pi][1]] += 2;
    C4[kPerm[pi][2]] += 1;
    int cube[3], F[3];
    for (int d = 0; d < 3; d++) {
        cube[d] = C4[d] / (4 * m_);
        F[d] = C4[d] - 4 * m_ * cube[d];
    }
    int p[3] = {0, 1, 2};
    std::sort(p, p + 3, [&](int a, int b) { return F[a] > F[b]; });
    int q = 0;
    for (int s = 0; s < 6; s++)
        if (kPerm[s][0] == p[0] && kPerm[s][1] == p[1] && kPerm[s][2] == p[2]) q = s;
    const int n = tp_.n_sub;
    return 6 * (cube[0] + n * (cube[1] + n * cube[2])) + q;
}

void StencilBuilder::key(const int X[3], NodeKey &k) const {
    const auto &A = around();
    for (int q = 0; q < 24; q++) {
        const int *s = A[q].o[A[q].r];
        const int c[3] = {X[0] - s[0], X[1] - s[1], X[2] - s[2]};
        k[q] = macro_tet(c, A[q].pi);
    }
}

// sum of the element stiffness entries of the node (vertex r of each
// element) with itself and with the element's other vertices
void StencilBuilder::stencil(const NodeKey &k, double S[15], bool mass) const {
    const auto &A = around();
    for (int e = 0; e < 15; e++) S[e] = 0.0;
    for (int q = 0; q < 24; q++) {
        const Around &e = A[q];
        const int t = k[q];
        const int a = tp_.perm[t][0], b = tp_.perm[t][1], cc = tp_.perm[t][2];
        double ev[3][3];
        for (int v = 1; v < 4; v++) {
            const int *d = e.o[v];
            const double di = d[a] - d[b], dj = d[b] - d[cc], dk = d[cc];
            for (int x = 0; x < 3; x++) ev[v - 1][x] = di * E_[t][x] + dj * E_[t][3 + x] + dk * E_[t][6 + x];
        }
        double K[4][4];
        if (mass)
            p1_mass(ev[0], ev[1], ev[2], K);
        else
            p1_stiffness(ev[0], ev[1], ev[2], K);
        const int r = e.r;
        S[0] += K[r][r];
        for (int v = 0; v < 4; v++) {
            if (v == r) continue;
            S[grid15_index(e.o[v][0] - e.o[r][0], e.o[v][1] - e.o[r][1], e.o[v][2] - e.o[r][2])] += K[r][v];
        }
    }
}

void StencilBuilder::grid_stencil(const int X[3], double S[15], bool mass) {
    NodeKey k;
    key(X, k);
    auto &memo = mass ? memo_mass_ : memo_;
    auto it = memo.find(k);
    if (it == memo.end()) {
        std::array<double, 15> st;
        stencil(k, st.data(), mass);
        it = memo.emplace(k, st).first;
    }
    for (int e = 0; e < 15; e++) S[e] = it->second[e];
}

void StencilBuilder::volume_stencil(int t, double S[15], bool mass) {
    const int a = tp_.perm[t][0], b = tp_.perm[t][1], c = tp_.perm[t][2];
    int X[3] = {m_ * tp_.V0[t][0], m_ * tp_.V0[t][1], m_ * tp_.V0[t][2]};
    X[a] += 3;
    X[b] += 2;
    X[c] += 1;
    double G[15];
    grid_stencil(X, G, mass);
    for (int n = 0; n < 15; n++) {
        int g[3] = {0, 0, 0};
        g[a] += kIdx15[n][0] + kIdx15[n][1] + kIdx15[n][2];
        g[b] += kIdx15[n][1] + kIdx15[n][2];
        g[c] += kIdx15[n][2];
        S[n] = G[grid15_index(g[0], g[1], g[2])];
    }
}

// The masters' keys are found in parallel chunks, each numbering its own
// distinct keys, then numbered once over all chunks.
std::string level_stencils(const Topology &tp, const double *xyz, int l, int cap, LevelStencils &G) {
    const TopoLevel &T = tp.lev[l];
    StencilBuilder sb(tp, xyz, l);
    G.w15.assign(15 * (size_t)tp.n_tets, 0.0);
    G.mw15.assign(15 * (size_t)tp.n_tets, 0.0);
    for (int t = 0; t < tp.n_tets; t++) {
        sb.volume_stencil(t, &G.w15[15 * (size_t)t], false);
        sb.volume_stencil(t, &G.mw15[15 * (size_t)t], true);
    }
    const int n = T.n_ifc;
    const int nth = std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
    const int chunk = (n + nth - 1) / nth;
    std::vector<std::vector<NodeKey>> keys(nth);
    G.sid.assign(n, 0);
    auto work = [&](int w) {
        std::map<NodeKey, int> local;
        NodeKey k, last{};
        int last_id = -1;
        for (int f = w * chunk; f < std::min(n, (w + 1) * chunk); f++) {
            sb.key(T.ifc_X[f].data(), k);
            if (last_id < 0 || k != last) {
                auto it = local.find(k);
                if (it == local.end()) {
                    it = local.emplace(k, (int)keys[w].size()).first;
                    keys[w].push_back(k);
                }
                last = k;
                last_id = it->second;
            }
            G.sid[f] = last_id;
        }
    };
    std::vector<std::thread> th;
    for (int w = 1; w < nth; w++) th.emplace_back(work, w);
    work(0);
    for (auto &x : th) x.join();
    std::map<NodeKey, int> global;
    std::vector<NodeKey> all;
    std::vector<std::vector<int>> renum(nth);
    for (int w = 0; w < nth; w++)
        for (const NodeKey &k : keys[w]) {
            auto it = global.find(k);
            if (it == global.end()) {
                it = global.emplace(k, (int)all.size()).first;
                all.push_back(k);
            }
            renum[w].push_back(it->second);
        }
    if ((int)all.size() > cap) return "more distinct interface stencils than the table holds";
    for (int w = 0; w < nth; w++)
        for (int f = w * chunk; f < std::min(n, (w + 1) * chunk); f++) G.sid[f] = renum[w][G.sid[f]];
    G.wtab.assign(15 * all.size(), 0.0);
    G.mwtab.assign(15 * all.size(), 0.0);
    for (size_t q = 0; q < all.size(); q++) {
        sb.stencil(all[q], &G.wtab[15 * q], false);
        sb.stencil(all[q], &G.mwtab[15 * q], true);
    }
    return "";
}

void coarse_stencils(const Topology &tp, const double *xyz, std::vector<double> &val) {
    const CoarseSystem &cs = tp.coarse;
    StencilBuilder sb(tp, xyz, tp.Lc);
    val.assign(15 * (size_t)cs.n, 0.0);
    for (int q = 0; q < cs.n; q++) {
        double S[15];
        sb.grid_stencil(cs.pos[q].data(), S);
        for (int e = 0; e < 15; e++) val[15 * (size_t)q + e] = e == 0 || cs.col15[15 * (size_t)q + e] >= 0 ? S[e] : 0.0;
    }
}

void element_matrices(const Topology &tp, const double *xyz, std::vector<double> &kel) {
    kel.assign(96 * (size_t)tp.n_tets, 0.0);
    for (int t = 0; t < tp.n_tets; t++) {
        double P[4][3], E[3][3];
        corners(tp, xyz, t, P);
        for (int s = 0; s < 3; s++)
            for (int d = 0; d < 3; d++) E[s][d] = P[s + 1][d] - P[0][d];
        const int a = tp.perm[t][0], b = tp.perm[t][1], c = tp.perm[t][2];
        for (int q = 0; q < 6; q++) {
            int o[4][3] = {};
            for (int v = 1; v < 4; v++)
                for (int w = 0; w < v; w++) o[v][kPerm[q][w]] = 1;
            double ev[3][3];
            for (int v = 1; v < 4; v++) {
                const double di = o[v][a] - o[v][b], dj = o[v][b] - o[v][c], dk = o[v][c];
                for (int x = 0; x < 3; x++) ev[v - 1][x] = di * E[0][x] + dj * E[1][x] + dk * E[2][x];
            }
            double K[4][4];
            p1_stiffness(ev[0], ev[1], ev[2], K);
            for (int r = 0; r < 4; r++)
                for (int r2 = 0; r2 < 4; r2++) kel[(6 * (size_t)t + q) * 16 + 4 * r + r2] = K[r][r2];
        }
    }
}

std::string check_macro_mesh(const Topology &tp, const double *xyz) {
    const long long nv = (long long)(tp.n_sub + 1) * (tp.n_sub + 1) * (tp.n_sub + 1);
    for (long long q = 0; q < 3 * nv; q++)
        if (!std::isfinite(xyz[q])) return "macro vertex positions must be finite";
    for (int t = 0; t < tp.n_tets; t++) {
        double P[4][3], e[3][3], c[3];
        corners(tp, xyz, t, P);
        double lmax = 0.0;
        for (int s = 0; s < 3; s++)
            for (int d = 0; d < 3; d++) e[s][d] = P[s + 1][d] - P[0][d];
        for (int a = 0; a < 4; a++)
            for (int b = a + 1; b < 4; b++) {
                const double d[3] = {P[b][0] - P[a][0], P[b][1] - P[a][1], P[b][2] - P[a][2]};
                lmax = std::max(lmax, std::sqrt(dot(d, d)));
            }
        cross(e[1], e[2], c);
        const double det = dot(e[0], c);
        // undeformed: edges e_a, e_a + e_b, (1,1,1), determinant = sign of the axis order
        double u[3][3] = {{0, 0, 0}, {0, 0, 0}, {1, 1, 1}}, uc[3];
        u[0][tp.perm[t][0]] = 1;
        u[1][tp.perm[t][0]] = 1;
        u[1][tp.perm[t][1]] = 1;
        cross(u[1], u[2], uc);
        const double ref = dot(u[0], uc);
        if (!(det * ref > 1e-8 * lmax * lmax * lmax))
            return "macro tetrahedron " + std::to_string(t) + " is inverted or degenerate";
    }
    return "";
}

}  // namespace hhgr
