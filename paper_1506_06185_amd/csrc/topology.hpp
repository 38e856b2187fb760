// Host-side HHG topology: macro mesh, primitive containers and the per-level
// index tables that the HIP kernels read.  No HIP calls here.
//
// Storage model (Sec. 3.1): every macro tetrahedron owns a volume container
// with the nodes of its closed tetrahedron at that level.  Its interior nodes
// are masters; its boundary nodes are ghost copies of face, edge and vertex
// masters (or Dirichlet zeros on the cube's boundary).  Face, edge and vertex
// masters of all levels live in one interface array per level, coloured red
// then black.  A level's vectors are one slot space:
//   [volume closures, each padded to a multiple of 64][interface masters][zero slot]
//
// Volume container of a tetrahedron refined to m = 2^l segments per edge:
// node (i,j,k), i,j,k >= 0, i+j+k <= m, grid position
//   X = m V0 + i a + j (a+b) + k (a+b+c),  a = e_p0, b = e_p1, c = e_p2.
// The grid axis neighbours of (i,j,k) are (i+-1,j,k), (i-+1,j+-1,k) and
// (i,j-+1,k+-1); the node colour parity(x+y+z) equals parity(i+k).
// Nodes are stored split by colour (ClosureLayout): all red nodes, then all
// black nodes, each in plane (k), row (j), i order, so a colour pass reads
// and writes whole cache lines of its own colour.
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <vector>

namespace hhgr {

constexpr int kPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

inline long long tetnum(long long x) { return x * (x + 1) * (x + 2) / 6; }
inline long long round_up(long long x, long long a) { return (x + a - 1) / a * a; }

// node (i,j,k) of a volume container packed into one word for the node lists
inline unsigned pack_ijk(int i, int j, int k) { return (unsigned)i | ((unsigned)j << 10) | ((unsigned)k << 20); }
// index of row (j,k) of a closure with M nodes per edge (plane k, row j order)
inline int row_id(int M, int j, int k) { return k * M - k * (k - 1) / 2 + j; }

// Colour-split closure layout, the same for every tetrahedron of a level.
// Red nodes (i+k even) come first, black nodes (i+k odd) start on a 256-byte
// boundary; within a colour the order is plane k, row j, then i.  The nodes
// of one colour in a row are every second i and sit consecutively, so node
// (i,j,k) of colour c = (i+k)&1 is at slot row0[2 row_id(j,k) + c] + (i >> 1).
struct ClosureLayout {
    int M = 0;
    long long n_red = 0, n_black = 0;
    long long black0 = 0;   // first black slot
    long long C = 0;        // nodes of the closure
    long long span = 0;     // slots of the closure (with padding), multiple of 64
    std::vector<int> row0;  // [2 * rows]
    void build(int M_) {
        M = M_;
        const int m = M - 1, nrows = M * (M + 1) / 2;
        row0.assign(2 * (size_t)nrows, 0);
        long long cnt[2] = {0, 0};
        std::vector<long long> start(2 * (size_t)nrows);
        for (int c = 0; c < 2; c++)
            for (int k = 0; k <= m; k++)
                for (int j = 0; j <= m - k; j++) {
                    const int rj = M - j - k, i0 = (c + k) & 1;
                    start[2 * (size_t)row_id(M, j, k) + c] = cnt[c];
                    cnt[c] += rj > i0 ? (rj - i0 + 1) / 2 : 0;
                }
        n_red = cnt[0];
        n_black = cnt[1];
        C = n_red + n_black;
        black0 = round_up(n_red, 32);
        span = round_up(black0 + n_black, 64);
        for (int r = 0; r < nrows; r++) {
            row0[2 * (size_t)r] = (int)start[2 * (size_t)r];
            row0[2 * (size_t)r + 1] = (int)(black0 + start[2 * (size_t)r + 1]);
        }
    }
    long long index(int i, int j, int k) const { return row0[2 * (size_t)row_id(M, j, k) + ((i + k) & 1)] + (i >> 1); }
};

struct TopoLevel {
    int l = 0, m = 0, M = 0, N = 0;
    double h = 0;
    ClosureLayout lay;
    long long C = 0, C_pad = 0;  // closure nodes, slot stride of the closures
    long long ifc_base = 0;      // first interface slot
    int n_ifc = 0, n_ifc_red = 0;
    long long zero_slot = 0;
    long long n_slots = 0;       // padded slot-space length
    std::vector<std::array<int, 3>> ifc_X;  // grid position of every interface node
    std::vector<int> ifc_dof;        // user vector index of every interface node
    std::vector<int> nbr;            // [6][n_ifc]: slots of +x,-x,+y,-y,+z,-z neighbours
    std::vector<int> gptr, gidx;     // interface node -> ghost slots (CSR)
    std::vector<int> rst;            // [15][n_ifc]: fine-level slots restricted into each node
    std::vector<int> prl;            // [2][n_ifc]: coarse-level slots interpolated into each node
    std::vector<int> nb15;           // [15][n_ifc]: same-level slots of centre + 14 Freudenthal nbrs
    // ghost refresh of one tetrahedron: pairs (ghost slot, master slot), per tet CSR
    std::vector<int> tg_ptr, tg_dst, tg_src;
    // nodes of a volume container (the same for every tetrahedron), in slot
    // order: interior red (even i+k), interior black, all interior (red then
    // black), every node of the closure
    std::vector<unsigned> rlist, blist, ilist, flist;
    // per row: first slot of its red and of its black nodes (ClosureLayout::row0)
    std::vector<std::array<int, 2>> rowC;
    // per colour c and row r, at [c * rows + r]: bases such that the node
    // (i,j,k) of colour c in row r and its axis neighbours are at base + (i >> 1):
    // {own, (i+1,j,k), (i-1,j+1,k), (i+1,j-1,k)}, {(i,j-1,k+1), (i,j+1,k-1), 0, 0};
    // (i-1,j,k) is the (i+1,j,k) base minus one.  Zero for rows without
    // interior nodes.
    std::vector<std::array<int, 8>> rowN;
    // general macro meshes (15-point stencils, 4-colour smoother): interior
    // nodes of each class (i + 2j + 3k) mod 4 = (x + y + z) mod 4, in slot order;
    // per parity colour c and row r at [c * rows + r], the 15 bases of the
    // node and of its neighbours at the index offsets kIdx15 (node at base +
    // (i >> 1)); interface masters of each class
    std::array<std::vector<unsigned>, 4> qlist;
    std::vector<std::array<int, 16>> rowN15;
    std::array<std::vector<int>, 4> ifcq;
    // unstructured macro meshes (Topology::build_mesh): user index of a
    // tetrahedron's first interior node is vbase + t nint (interior nodes in
    // plane k, row j, i order); the stiffness stencil of every tetrahedron's
    // interior nodes (kIdx15 order, [15 t + n]) and of every master
    // ([n n_ifc + f], n < Topology::nbw, entry 0 the diagonal, at the slots
    // nb15 of the same layout; unused entries 0 at the zero slot)
    long long vbase = 0, nint = 0;
    std::vector<double> mesh_w15, mesh_wi;
    std::vector<double> mesh_mw15, mesh_mwi;  // the consistent P1 mass matrix, same layout
};

// index-space offsets of the 15-point stencil (centre first); offset n
// of a tetrahedron with axis order (a, b, c) is the grid step
// di e_a + dj (e_a + e_b) + dk (e_a + e_b + e_c)
constexpr int kIdx15[15][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {-1, 1, 0}, {1, -1, 0},
                               {0, -1, 1}, {0, 1, -1}, {0, 1, 0},  {0, -1, 0}, {-1, 0, 1},
                               {1, 0, -1}, {1, -1, 1}, {-1, 1, -1}, {0, 0, 1}, {0, 0, -1}};
// grid offsets of the 15-point stencil (centre first), the order of nb15
constexpr int kGrid15[15][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                                {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {0, 1, 1},
                                {0, -1, -1}, {1, 0, 1}, {-1, 0, -1}, {1, 1, 1}, {-1, -1, -1}};

// coarsest-level direct data (Jacobi-PCG in one workgroup)
struct CoarseSystem {
    int n = 0;
    std::vector<long long> slot;     // master slot of every coarse unknown
    std::vector<int> col;            // [n][7], column 0 = self, -1 = none
    std::vector<double> val;         // [n][7] for k = 1
    std::vector<std::array<int, 3>> pos;  // grid position of every unknown
    std::vector<int> cptr, cidx;     // unknown -> all slots holding it (master + ghosts)
    std::vector<int> grid_dir;       // [n][7] grid direction code of each column (0 self, 1..6 +x,-x,+y,-y,+z,-z)
    std::vector<int> col15;          // [n][15] unknowns at the kGrid15 offsets, -1 = none
    std::vector<int> is_vol;         // 1 if volume-interior unknown
    std::vector<int> tet;            // tet of a volume unknown, -1 for interface
    std::vector<int> ifc;            // interface index, -1 for volume
    // unstructured macro meshes: rows of cw entries (column -1: none)
    int cw = 0;
    std::vector<int> colw;
    std::vector<double> valw;
};

struct Topology {
    int n_sub = 0, L = 0, Lc = 0, n_tets = 0;
    std::vector<std::array<int, 3>> V0;    // subcube corner (level-0 units) per tet
    std::vector<std::array<int, 3>> perm;  // axis order per tet
    std::vector<TopoLevel> lev;            // indexed by level, entries Lc..L filled
    CoarseSystem coarse;

    // Builds everything.  Returns an empty string on success, else the error.
    std::string build(int n_sub, int L, int Lc);

    // Unstructured macro mesh (mesh.cpp): nv vertices (xyz, 3 each) and nt
    // tetrahedra (tets, 4 vertex ids each, listed by a proper 4-colouring of
    // the vertices: a vertex has the same position in every tetrahedron that
    // contains it).  Closure node (i, j, k) of tetrahedron t is the node with
    // weights (m - i - j - k, i, j, k) on its vertices 0..3; a node is known
    // by its (macro vertex, weight) pairs.  Interface masters carry their own
    // stencils (nbw entries), and the user order is: interior macro vertices
    // by id, interior edges (a < b) by the weight of b, interior faces
    // (a < b < c) by the weights of c then b, tetrahedron interiors by tet id
    // in plane k, row j, i order.  Fills the stencils and the coarsest-level
    // rows too.  Returns an empty string on success, else the error.
    std::string build_mesh(int nv, const double *xyz, int nt, const int *tets, int L, int Lc);
    // Operators of a mesh whose elements in tetrahedron t carry the weight
    // wt[t] (eq. (2) with k constant on each macro tetrahedron; 0 drops the
    // tetrahedron's elements, as the intact side of a Dirichlet-Neumann
    // recovery does, Sec. 4.3, eq. (5)): per level the volume stencils
    // (15 per tetrahedron) and the master rows (the layout of mesh_wi), the
    // coarsest-level rows (the layout of coarse.valw) and, with with_dir, the
    // finest level's Dirichlet couplings (the layout of dir_val).  Master rows are summed
    // again only for masters with a copy in a closure flagged in dirty;
    // the others are taken from base (per level; null: the k = 1 rows), which
    // must hold them for the same weights.  Returns an empty string on
    // success, else the error.
    struct MeshOps {
        std::vector<std::vector<double>> w15, wi;
        std::vector<double> valw, dir_val;
    };
    std::string mesh_weighted_operators(const double *wt, const unsigned char *dirty,
                                        const std::vector<std::vector<double>> *base, MeshOps &out,
                                        bool with_dir = true) const;
    // Unit-k stiffness matrices of the 6 element types of a mesh level (kel,
    // 96 per tetrahedron: type p at 16 p, row-major): the element of type p
    // with lowest corner X has the index-space corners X, X + e_a, X + e_a +
    // e_b, X + (1, 1, 1) with (a, b) the first two axes of permutation p in
    // the order (0,1,2), (0,2,1), (1,0,2), (1,2,0), (2,0,1), (2,1,0), where
    // closure node (i, j, k) sits at X = (i + j + k, j + k, k).
    void mesh_kuhn_matrices(int l, std::vector<double> &kel) const;
    bool mesh = false;
    unsigned long long mesh_hash = 0;  // hash of the vertex and tetrahedron lists (set by the engine)
    std::vector<double> mesh_xyz;  // the mesh's vertices (3 each) and tetrahedra (4 vertex ids each)
    std::vector<int> mesh_tets;
    int nbw = 15;  // interface stencil and restriction width
    long long n_dofs = 0;
    // finest level of a mesh: the Dirichlet boundary nodes (their order: the
    // interior order's rule over boundary vertices, edges and faces) with
    // their positions, and the stiffness couplings of interior nodes to
    // them: rows dir_rows (slots) with entries dir_ptr[q] .. dir_ptr[q + 1]
    // of boundary index dir_col and value dir_val
    long long n_bnd = 0;
    std::vector<double> bnd_xyz;
    std::vector<int> dir_rows, dir_ptr, dir_col;
    std::vector<double> dir_val;
    // per tetrahedron (CSR over dir_bnd_ptr): the closure positions of its
    // Dirichlet boundary nodes and their boundary indices
    std::vector<int> dir_bnd_ptr, dir_bnd_pos, dir_bnd_idx;

    // slot of grid node X at level l (zero slot for boundary nodes)
    long long slot_of(int l, int x, int y, int z) const;
    // interface index lookup (or -1), tet-interior lookup
    int ifc_index(int l, int x, int y, int z) const;
    bool locate_interior(int l, int x, int y, int z, int *tet, int *i, int *j, int *k) const;

  private:
    std::vector<std::vector<long long>> ifc_key_;  // sorted keys per level
    std::vector<std::vector<int>> ifc_key_idx_;
    void build_level(int l);
    void build_transfer(int l);
    void build_coarse();
};

// node lists and row tables of the colour-split closure layout of a level
// (lay, m, M set)
void build_closure_tables(TopoLevel &Lv);

// Dense inverse (row-major n x n) of a symmetric coarsest-level operator
// given as [n][nb] columns and values (-1: no entry): Cholesky factorisation
// A = L L^T, then A^{-1} e_j by a forward and a backward substitution for
// every j.  Returns false if A is not numerically positive definite.
bool coarse_inverse(int n, int nb, const std::vector<int> &col, const std::vector<double> &val,
                    std::vector<double> &inv);

}  // namespace hhgr
