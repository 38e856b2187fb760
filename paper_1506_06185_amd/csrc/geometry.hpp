// Host-side stencils of the P1 stiffness matrix on a general macro mesh: the
// Kuhn connectivity of the topology with moved macro vertices, every macro
// tetrahedron refined regularly and mapped affinely (Sec. 3.1: the refined
// mesh of a macro element is structured, so its stencil is the same at every
// node of one primitive).  No HIP calls here.
//
// A fine element of level l is a Kuhn tetrahedron of a unit grid cube; it lies
// in exactly one macro tetrahedron, found from its centroid.  Inside macro
// tetrahedron t with corners P0..P3 and axis order (a, b, c), the grid point
// with local coordinates x = X - m V0 has index coordinates
// (i, j, k) = (x_a - x_b, x_b - x_c, x_c) and position
// P0 + (i (P1 - P0) + j (P2 - P0) + k (P3 - P0)) / m,  m = 2^l,
// so an element's edge vectors depend only on t and on the element's shape.
#pragma once

#include <array>
#include <map>
#include <string>
#include <vector>

#include "topology.hpp"

namespace hhgr {

// the macro tetrahedra of the 24 fine elements around a grid node, in a
// fixed order; two nodes with the same key have the same stencil
using NodeKey = std::array<int, 24>;

class StencilBuilder {
  public:
    // xyz: (n_sub + 1)^3 macro vertex positions, x fastest
    StencilBuilder(const Topology &tp, const double *xyz, int l);
    // key of the interior grid node X
    void key(const int X[3], NodeKey &k) const;
    // stencil in kGrid15 order (entry 0 the diagonal) of a node with key k:
    // stiffness, or with mass the consistent P1 mass matrix
    void stencil(const NodeKey &k, double S[15], bool mass = false) const;
    // stencil of the interior grid node X in kGrid15 order (memoised by key)
    void grid_stencil(const int X[3], double S[15], bool mass = false);
    // volume stencil of tetrahedron t in kIdx15 order
    void volume_stencil(int t, double S[15], bool mass = false);

  private:
    const Topology &tp_;
    int m_;
    std::vector<std::array<double, 9>> E_;  // per macro tet: (P1-P0)/m, (P2-P0)/m, (P3-P0)/m
    std::map<NodeKey, std::array<double, 15>> memo_, memo_mass_;
    int macro_tet(const int c[3], int pi) const;
};

// Stencils of one level: the volume stencil of every tetrahedron (kIdx15
// order, [15 t + n]) and, per interface master, the index of its stencil in
// the table of the level's distinct stencils (kGrid15 order, [15 id + n]);
// the same for the mass matrix (mw15, mwtab, same indices).  cap bounds the
// table; returns an empty string or the error.
struct LevelStencils {
    std::vector<double> w15, wtab, mw15, mwtab;
    std::vector<int> sid;
};
std::string level_stencils(const Topology &tp, const double *xyz, int l, int cap, LevelStencils &G);

// Coarsest-level matrix rows in the kGrid15 order of CoarseSystem::col15
// ([15 q + e], zero where the column is a boundary node).
void coarse_stencils(const Topology &tp, const double *xyz, std::vector<double> &val);

// Unit-size element matrices of every macro tetrahedron: kel[(6 t + q) 16 +
// 4 r + r'] is the P1 stiffness entry of vertices r, r' of a fine element with
// axis order q (vertices at the cube corner offsets 0, e_q0, e_q0 + e_q1,
// (1,1,1)) inside macro tetrahedron t at m = 1; level m divides it by m.
void element_matrices(const Topology &tp, const double *xyz, std::vector<double> &kel);

// Orientation check of the macro mesh: every macro tetrahedron must keep the
// sign of its undeformed volume, and 6 |volume| must exceed 1e-8 times the
// cube of its longest edge.  Returns an empty string or the error.
std::string check_macro_mesh(const Topology &tp, const double *xyz);

// Index of the grid offset (dx, dy, dz) in kGrid15, or -1.
int grid15_index(int dx, int dy, int dz);

}  // namespace hhgr
