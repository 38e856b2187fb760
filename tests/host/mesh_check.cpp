// Host check of the unstructured-mesh topology (mesh.cpp): builds it from a
// mesh file and writes, per level, the operator that the tables define
// (volume stencils and master rows) and the interface rows of the transfers,
// as (row, column, value) triplets in the user order, for comparison with an
// independent assembly.  Also checks internal invariants and exits nonzero
// when one fails.
//
// usage: mesh_check <mesh file> <output file> [faulty tet ids, comma-separated, or -]
//                   [coefficient per tetrahedron, comma-separated]
// mesh file: "nv nt L Lc", then nv lines "x y z", then nt lines "a b c d"
// With the optional arguments it also writes the operators of a coefficient
// constant on each tetrahedron ("W", "WC", "WD") and the intact side of a
// Dirichlet-Neumann recovery over it: per level the operator of the intact
// volume stencils and the intact master rows ("I"), and the coarsest-level
// rows over the intact elements ("C").
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_1506_06185_amd/csrc/topology.hpp"

using namespace hhgr;

static int fails = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            fails++;                                                      \
        }                                                                 \
    } while (0)

// rank of interior node (i,j,k) in plane k, row j, i order, by enumeration
static long long rank_enum(int m, int i0, int j0, int k0) {
    long long r = 0;
    for (int k = 1; k < m; k++)
        for (int j = 1; j < m; j++)
            for (int i = 1; i + j + k <= m - 1; i++) {
                if (i == i0 && j == j0 && k == k0) return r;
                r++;
            }
    return -1;
}

int main(int argc, char **argv) {
    if (argc < 3 || argc > 5) return 2;
    FILE *f = std::fopen(argv[1], "r");
    if (!f) return 2;
    int nv, nt, L, Lc;
    if (std::fscanf(f, "%d %d %d %d", &nv, &nt, &L, &Lc) != 4) return 2;
    std::vector<double> xyz(3 * (size_t)nv);
    std::vector<int> tets(4 * (size_t)nt);
    for (auto &x : xyz)
        if (std::fscanf(f, "%lf", &x) != 1) return 2;
    for (auto &t : tets)
        if (std::fscanf(f, "%d", &t) != 1) return 2;
    std::fclose(f);
    Topology tp;
    std::string e = tp.build_mesh(nv, xyz.data(), nt, tets.data(), L, Lc);
    if (!e.empty()) {
        std::printf("error: %s\n", e.c_str());
        return 3;
    }
    FILE *o = std::fopen(argv[2], "w");
    std::fprintf(o, "nbw %d n_dofs %lld coarse %d cw %d\n", tp.nbw, tp.n_dofs, tp.coarse.n, tp.coarse.cw);
    std::vector<std::vector<long long>> user_of(L + 1);
    for (int l = Lc; l <= L; l++) {
        const TopoLevel &Lv = tp.lev[l];
        const int m = Lv.m;
        // slot -> user index (-1: zero slot or Dirichlet ghost)
        std::vector<long long> &U = user_of[l];
        U.assign(Lv.n_slots, -1);
        for (int t = 0; t < nt; t++)
            for (int k = 1; k < m; k++)
                for (int j = 1; j < m; j++)
                    for (int i = 1; i + j + k <= m - 1; i++)
                        U[(long long)t * Lv.C_pad + Lv.lay.index(i, j, k)] = Lv.vbase + (long long)t * Lv.nint +
                                                                            rank_enum(m, i, j, k);
        for (int q = 0; q < Lv.n_ifc; q++) U[Lv.ifc_base + q] = Lv.ifc_dof[q];
        for (size_t q = 0; q < Lv.tg_dst.size(); q++) {
            CHECK(U[Lv.tg_dst[q]] == -1);
            U[Lv.tg_dst[q]] = Lv.tg_src[q] == Lv.zero_slot ? -1 : U[Lv.tg_src[q]];
        }
        // every user index is taken exactly once
        const long long nd = Lv.vbase + (long long)nt * Lv.nint;
        std::vector<int> seen(nd, 0);
        for (int t = 0; t < nt; t++)
            for (int k = 1; k < m; k++)
                for (int j = 1; j < m; j++)
                    for (int i = 1; i + j + k <= m - 1; i++) seen[U[(long long)t * Lv.C_pad + Lv.lay.index(i, j, k)]]++;
        for (int q = 0; q < Lv.n_ifc; q++) seen[Lv.ifc_dof[q]]++;
        for (long long d = 0; d < nd; d++) CHECK(seen[d] == 1);
        // ghost lists agree with the per-master CSR
        long long ng = 0;
        for (size_t q = 0; q < Lv.tg_dst.size(); q++) ng += Lv.tg_src[q] != Lv.zero_slot;
        CHECK(ng == (long long)Lv.gidx.size());
        // classes: no stencil entry joins two nodes of one class
        std::vector<int> cls(Lv.n_slots, -1);
        for (int q = 0; q < 4; q++)
            for (int fq : Lv.ifcq[q]) cls[Lv.ifc_base + fq] = q;
        std::fprintf(o, "A %d %lld\n", l, nd);
        for (int t = 0; t < nt; t++)
            for (int k = 1; k < m; k++)
                for (int j = 1; j < m; j++)
                    for (int i = 1; i + j + k <= m - 1; i++) {
                        const long long r = U[(long long)t * Lv.C_pad + Lv.lay.index(i, j, k)];
                        const int c0 = (i + 2 * j + 3 * k) & 3;
                        for (int n = 0; n < 15; n++) {
                            const int ii = i + kIdx15[n][0], jj = j + kIdx15[n][1], kk = k + kIdx15[n][2];
                            const long long s = (long long)t * Lv.C_pad + Lv.lay.index(ii, jj, kk);
                            const long long c = U[s];
                            const double v = Lv.mesh_w15[15 * (size_t)t + n];
                            if (n > 0 && v != 0.0) {
                                const int cn = s >= Lv.ifc_base ? cls[s] : (ii + 2 * jj + 3 * kk) & 3;
                                const bool ghost = ii == 0 || jj == 0 || kk == 0 || ii + jj + kk == m;
                                if (!ghost) CHECK(cn != c0);
                            }
                            if (c >= 0) std::fprintf(o, "%lld %lld %.17g\n", r, c, v);
                        }
                    }
        for (int q = 0; q < Lv.n_ifc; q++) {
            const long long r = Lv.ifc_dof[q];
            for (int n = 0; n < tp.nbw; n++) {
                const int s = Lv.nb15[(size_t)n * Lv.n_ifc + q];
                const double v = Lv.mesh_wi[(size_t)n * Lv.n_ifc + q];
                if (n == 0) CHECK(s == Lv.ifc_base + q);
                const long long c = U[s];
                if (c >= 0) std::fprintf(o, "%lld %lld %.17g\n", r, c, v);
            }
        }
        std::fprintf(o, "end\n");
        if (l == L) {
            // the consistent mass matrix on the finest level, same layout
            std::fprintf(o, "M %d %lld\n", l, nd);
            for (int t = 0; t < nt; t++)
                for (int k = 1; k < m; k++)
                    for (int j = 1; j < m; j++)
                        for (int i = 1; i + j + k <= m - 1; i++) {
                            const long long r = U[(long long)t * Lv.C_pad + Lv.lay.index(i, j, k)];
                            for (int n = 0; n < 15; n++) {
                                const long long c = U[(long long)t * Lv.C_pad +
                                                      Lv.lay.index(i + kIdx15[n][0], j + kIdx15[n][1], k + kIdx15[n][2])];
                                if (c >= 0) std::fprintf(o, "%lld %lld %.17g\n", r, c, Lv.mesh_mw15[15 * (size_t)t + n]);
                            }
                        }
            for (int q = 0; q < Lv.n_ifc; q++)
                for (int n = 0; n < tp.nbw; n++) {
                    const long long c = U[Lv.nb15[(size_t)n * Lv.n_ifc + q]];
                    if (c >= 0)
                        std::fprintf(o, "%d %lld %.17g\n", Lv.ifc_dof[q], c, Lv.mesh_mwi[(size_t)n * Lv.n_ifc + q]);
                }
            std::fprintf(o, "end\n");
            // couplings to the Dirichlet boundary nodes, and their positions
            std::fprintf(o, "D %d %lld\n", l, tp.n_bnd);
            for (size_t q = 0; q < tp.dir_rows.size(); q++)
                for (int e = tp.dir_ptr[q]; e < tp.dir_ptr[q + 1]; e++)
                    std::fprintf(o, "%lld %d %.17g\n", U[tp.dir_rows[q]], tp.dir_col[e], tp.dir_val[e]);
            std::fprintf(o, "end\n");
            std::fprintf(o, "X %d\n", l);
            for (long long q = 0; q < tp.n_bnd; q++)
                for (int c = 0; c < 3; c++) std::fprintf(o, "%lld %d %.17g\n", q, c, tp.bnd_xyz[3 * q + c]);
            std::fprintf(o, "end\n");
        }
    }
    if (argc >= 4) {
        // optional: faulty tetrahedra ("-" for none) and a coefficient per
        // tetrahedron; the weighted operator of every level ("W"), its
        // coarsest rows ("WC") and Dirichlet couplings ("WD"), then with
        // faults the intact side over the same coefficient ("I", "C")
        std::vector<unsigned char> faulty(nt, 0);
        bool any_fault = false;
        for (const char *c = argv[3]; *c && std::string(argv[3]) != "-";) {
            char *end;
            const long t = std::strtol(c, &end, 10);
            if (end == c || t < 0 || t >= nt) return 2;
            faulty[t] = 1;
            any_fault = true;
            c = *end == ',' ? end + 1 : end;
        }
        std::vector<double> kt(nt, 1.0);
        if (argc == 5) {
            const char *c = argv[4];
            for (int t = 0; t < nt; t++) {
                char *end;
                kt[t] = std::strtod(c, &end);
                if (end == c) return 2;
                c = *end == ',' ? end + 1 : end;
            }
        }
        const std::vector<unsigned char> all(nt, 1);
        Topology::MeshOps K, I;
        e = tp.mesh_weighted_operators(kt.data(), all.data(), nullptr, K);
        if (e.empty() && any_fault) {
            std::vector<double> wi(nt);
            for (int t = 0; t < nt; t++) wi[t] = faulty[t] ? 0.0 : kt[t];
            e = tp.mesh_weighted_operators(wi.data(), faulty.data(), &K.wi, I, false);
        }
        if (!e.empty()) {
            std::printf("error: %s\n", e.c_str());
            return 4;
        }
        const CoarseSystem &cs = tp.coarse;
        auto write_ops = [&](const char *tag, const char *ctag, const Topology::MeshOps &W, bool skip_faulty) {
            for (int l = Lc; l <= L; l++) {
                const TopoLevel &Lv = tp.lev[l];
                const int m = Lv.m;
                const std::vector<long long> &U = user_of[l];
                std::fprintf(o, "%s %d\n", tag, l);
                for (int t = 0; t < nt; t++) {
                    if (skip_faulty && faulty[t]) continue;
                    for (int k = 1; k < m; k++)
                        for (int j = 1; j < m; j++)
                            for (int i = 1; i + j + k <= m - 1; i++) {
                                const long long r = U[(long long)t * Lv.C_pad + Lv.lay.index(i, j, k)];
                                for (int n = 0; n < 15; n++) {
                                    const long long c = U[(long long)t * Lv.C_pad + Lv.lay.index(i + kIdx15[n][0],
                                                                                                j + kIdx15[n][1],
                                                                                                k + kIdx15[n][2])];
                                    if (c >= 0) std::fprintf(o, "%lld %lld %.17g\n", r, c, W.w15[l][15 * (size_t)t + n]);
                                }
                            }
                }
                for (int q = 0; q < Lv.n_ifc; q++)
                    for (int n = 0; n < tp.nbw; n++) {
                        const size_t at = (size_t)n * Lv.n_ifc + q;
                        const long long c = U[Lv.nb15[at]];
                        if (c >= 0) std::fprintf(o, "%d %lld %.17g\n", Lv.ifc_dof[q], c, W.wi[l][at]);
                    }
                std::fprintf(o, "end\n");
            }
            std::fprintf(o, "%s %d\n", ctag, Lc);
            for (int q = 0; q < cs.n; q++)
                for (int e2 = 0; e2 < cs.cw; e2++) {
                    const int c = cs.colw[(size_t)cs.cw * q + e2];
                    if (c >= 0)
                        std::fprintf(o, "%lld %lld %.17g\n", user_of[Lc][cs.slot[q]], user_of[Lc][cs.slot[c]],
                                     W.valw[(size_t)cs.cw * q + e2]);
                }
            std::fprintf(o, "end\n");
        };
        write_ops("W", "WC", K, false);
        std::fprintf(o, "WD %d %lld\n", L, tp.n_bnd);
        for (size_t q = 0; q < tp.dir_rows.size(); q++)
            for (int e2 = tp.dir_ptr[q]; e2 < tp.dir_ptr[q + 1]; e2++)
                std::fprintf(o, "%lld %d %.17g\n", user_of[L][tp.dir_rows[q]], tp.dir_col[e2], K.dir_val[e2]);
        std::fprintf(o, "end\n");
        // with k = 1 the weighted tables are the plain ones, bit for bit
        if (argc == 4) {
            for (int l = Lc; l <= L; l++) {
                CHECK(K.wi[l] == tp.lev[l].mesh_wi);
                CHECK(K.w15[l] == tp.lev[l].mesh_w15);
            }
            CHECK(K.dir_val == tp.dir_val);
            CHECK(K.valw == tp.coarse.valw);
        }
        if (any_fault) {
            write_ops("I", "C", I, true);
            // masters that no faulty closure holds keep the weighted rows
            for (int l = Lc; l <= L; l++) {
                const TopoLevel &Lv = tp.lev[l];
                for (int q = 0; q < Lv.n_ifc; q++) {
                    bool touched = false;
                    for (int g = Lv.gptr[q]; g < Lv.gptr[q + 1]; g++) touched |= faulty[Lv.gidx[g] / Lv.C_pad] != 0;
                    for (int n = 0; n < tp.nbw && !touched; n++)
                        CHECK(I.wi[l][(size_t)n * Lv.n_ifc + q] == K.wi[l][(size_t)n * Lv.n_ifc + q]);
                }
            }
        }
    }
    // interface rows of the transfers: P (fine master <- coarse parents) and
    // R = P^T (coarse master <- its fine twin and the neighbours at 1/2)
    for (int l = Lc + 1; l <= L; l++) {
        const TopoLevel &F = tp.lev[l], &Cl = tp.lev[l - 1];
        std::fprintf(o, "P %d\n", l);
        for (int q = 0; q < F.n_ifc; q++) {
            const int s1 = F.prl[q], s2 = F.prl[(size_t)F.n_ifc + q];
            const long long c1 = user_of[l - 1][s1], c2 = user_of[l - 1][s2];
            if (c1 >= 0) std::fprintf(o, "%d %lld 0.5\n", F.ifc_dof[q], c1);
            if (c2 >= 0) std::fprintf(o, "%d %lld 0.5\n", F.ifc_dof[q], c2);
        }
        std::fprintf(o, "end\n");
        std::fprintf(o, "R %d\n", l);
        for (int q = 0; q < Cl.n_ifc; q++)
            for (int n = 0; n < tp.nbw; n++) {
                const int s = Cl.rst[(size_t)n * Cl.n_ifc + q];
                const long long c = user_of[l][s];
                if (c >= 0) std::fprintf(o, "%d %lld %s\n", Cl.ifc_dof[q], c, n == 0 ? "1" : "0.5");
            }
        std::fprintf(o, "end\n");
    }
    std::fclose(o);
    if (fails) return 1;
    std::printf("ok\n");
    return 0;
}
