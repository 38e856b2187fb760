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
// Volume container layout for a tetrahedron refined to m = 2^l segments per
// edge: node (i,j,k), i,j,k >= 0, i+j+k <= m, grid position
//   X = m V0 + i a + j (a+b) + k (a+b+c),  a = e_p0, b = e_p1, c = e_p2,
// stored plane by plane (k), row by row (j), i fastest.  With M = m+1 and
// s = M-k the row-0 length of plane k:
//   idx(i,j,k) = T(k) + j s - j(j-1)/2 + i,   T(k) = tet(M) - tet(M-k),
//   tet(x) = x(x+1)(x+2)/6.
// The grid axis neighbours of (i,j,k) are (i+-1,j,k), (i-+1,j+-1,k) and
// (i,j-+1,k+-1); the node colour parity(x+y+z) equals parity(i+k).
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <vector>

namespace hhgr {

constexpr int kPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

inline long long tetnum(long long x) { return x * (x + 1) * (x + 2) / 6; }
inline long long plane_start(int M, int k) { return tetnum(M) - tetnum(M - k); }
inline long long row_start(int s, int j) { return (long long)j * s - (long long)j * (j - 1) / 2; }
inline long long closure_index(int M, int i, int j, int k) { return plane_start(M, k) + row_start(M - k, j) + i; }
inline long long round_up(long long x, long long a) { return (x + a - 1) / a * a; }

// tiles of the fused sweep over the interior rows (j,k) of a tetrahedron with
// m segments per edge: 8x8 blocks of rows (j0, k0) and 62-node segments along
// i starting at i0
constexpr int kTileRows = 8;
constexpr int kTileSeg = 62;
inline std::vector<std::array<int, 3>> fused_tile_list(int m) {
    std::vector<std::array<int, 3>> t;
    for (int j0 = 1; j0 <= m - 3; j0 += kTileRows)
        for (int k0 = 1; j0 + k0 <= m - 2; k0 += kTileRows)
            for (int i0 = 1; i0 <= m - 1 - j0 - k0; i0 += kTileSeg) t.push_back({j0, k0, i0});
    return t;
}

struct Chunk {
    int k;   // plane
    int o0;  // first offset within the plane
};

// node (i,j,k) of a volume container packed into one word for the node lists
inline unsigned pack_ijk(int i, int j, int k) { return (unsigned)i | ((unsigned)j << 10) | ((unsigned)k << 20); }
// index of row (j,k) of a closure with M nodes per edge, rows ordered like the slots
inline int row_id(int M, int j, int k) { return k * M - k * (k - 1) / 2 + j; }

struct TopoLevel {
    int l = 0, m = 0, M = 0, N = 0;
    double h = 0;
    long long C = 0, C_pad = 0;  // closure nodes, padded stride
    long long ifc_base = 0;      // first interface slot
    int n_ifc = 0, n_ifc_red = 0;
    long long zero_slot = 0;
    long long n_slots = 0;       // padded slot-space length
    std::vector<Chunk> chunks_int;   // chunks covering planes with interior nodes
    std::vector<Chunk> chunks_full;  // chunks covering the whole closure
    std::vector<std::array<int, 3>> ifc_X;  // grid position of every interface node
    std::vector<int> ifc_dof;        // user vector index of every interface node
    std::vector<int> nbr;            // [6][n_ifc]: slots of +x,-x,+y,-y,+z,-z neighbours
    std::vector<int> gptr, gidx;     // interface node -> ghost slots (CSR)
    std::vector<int> rst;            // [15][n_ifc]: fine-level slots restricted into each node
    std::vector<int> prl;            // [2][n_ifc]: coarse-level slots interpolated into each node
    std::vector<int> nb15;           // [15][n_ifc]: same-level slots of centre + 14 Freudenthal nbrs
    // ghost refresh of one tetrahedron: pairs (ghost slot, master slot), per tet CSR
    std::vector<int> tg_ptr, tg_dst, tg_src;
    // interior nodes of a volume container (the same for every tetrahedron), in
    // slot order: all, red (even i+k), black
    std::vector<unsigned> ilist, rlist, blist;
    // per row (j,k): rowA = (slot of (0,j,k), row length, offset to (i,j-1,k+1),
    // offset to (i,j+1,k-1)); rowB = (offset to (i,j,k+1), offset to (i,j,k-1), 0, 0)
    std::vector<std::array<int, 4>> rowA, rowB;
};

// coarsest-level direct data (Jacobi-PCG in one workgroup)
struct CoarseSystem {
    int n = 0;
    std::vector<long long> slot;     // master slot of every coarse unknown
    std::vector<int> col;            // [n][7], column 0 = self, -1 = none
    std::vector<double> val;         // [n][7] for k = 1
    std::vector<int> cptr, cidx;     // unknown -> all slots holding it (master + ghosts)
    std::vector<int> grid_dir;       // [n][7] grid direction code of each column (0 self, 1..6 +x,-x,+y,-y,+z,-z)
    std::vector<int> is_vol;         // 1 if volume-interior unknown
    std::vector<int> tet;            // tet of a volume unknown, -1 for interface
    std::vector<int> ifc;            // interface index, -1 for volume
};

struct Topology {
    int n_sub = 0, L = 0, Lc = 0, n_tets = 0;
    std::vector<std::array<int, 3>> V0;    // subcube corner (level-0 units) per tet
    std::vector<std::array<int, 3>> perm;  // axis order per tet
    std::vector<TopoLevel> lev;            // indexed by level, entries Lc..L filled
    CoarseSystem coarse;

    // Builds everything.  Returns an empty string on success, else the error.
    std::string build(int n_sub, int L, int Lc, int chunk);

    // slot of grid node X at level l (zero slot for boundary nodes)
    long long slot_of(int l, int x, int y, int z) const;
    // interface index lookup (or -1), tet-interior lookup
    int ifc_index(int l, int x, int y, int z) const;
    bool locate_interior(int l, int x, int y, int z, int *tet, int *i, int *j, int *k) const;

  private:
    std::vector<std::vector<long long>> ifc_key_;  // sorted keys per level
    std::vector<std::vector<int>> ifc_key_idx_;
    void build_level(int l, int chunk);
    void build_transfer(int l);
    void build_coarse();
};

}  // namespace hhgr
