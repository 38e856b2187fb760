// Device data descriptors and kernel launchers of the HHG multigrid engine.
#pragma once

#include <hip/hip_runtime.h>

namespace hhgr {

// one volume container taking part in a launch: slot offset of its closure in
// the vector arrays and in the coefficient-weight arrays, and its tet id
struct VolDesc {
    long long vec;
    long long w;
    int tet;
    int pad;
};

// structured part of a launch: every listed volume x a list of nodes of its
// closure (packed (i,j,k), the same for every volume), with the row tables of
// the level's colour-split closure layout
struct VolGeom {
    const VolDesc *vd = nullptr;
    int nvol = 0;
    const unsigned *list = nullptr;
    int nlist = 0;
    const int2 *rowC = nullptr;  // per row: first slot of its red nodes, of its black nodes
    const int4 *rowN = nullptr;  // per (colour, row): two int4 of neighbour bases (see topology.hpp)
    int nrows = 0;
    int M = 0;        // nodes per macro edge at this level (2^l + 1)
    int bs = 256;
    int remap = 1;    // 1: contiguous block ranges per XCD, 0: hardware order
    int cpb = 1;      // nodes per thread (1 or 4), all loads issued before the stores
};

// table-driven part of a launch: interface nodes [i0, i1)
struct IfcGeom {
    int i0 = 0, i1 = 0;
    long long base = 0;                 // slot of interface node 0
    int stride = 0;                     // number of interface nodes (SoA stride of tables)
    const int *nbr = nullptr;           // [6][stride] axis neighbours (+x,-x,+y,-y,+z,-z)
    const int *gptr = nullptr;          // ghost copies (CSR) or nullptr
    const int *gidx = nullptr;
    const unsigned char *frozen = nullptr;  // Dirichlet-frozen nodes or nullptr
    int w = 15;  // entries per master of the 15-point (general mesh) stencil and restriction tables
};

// General macro meshes (moved macro vertices): 15-point stencils.  A volume
// node of tetrahedron t uses w15[15 t + n], n in the index-offset order of
// kIdx15 (entry 0 the diagonal), with slots rowN15[16 (c rows + r) + n] +
// (i >> 1) (c = parity colour, r = row); an interface master f uses the
// stencil wtab[15 sid[f] + n] at the slots nb15[n stride + f] (grid-offset
// order of kGrid15).  A class pass walks the masters listed in ifcq[0 .. nq).
// With a per-element coefficient (wv != nullptr) the stencils vary per node:
// a closure slot holds the weights of its 7 forward index offsets kIdx15[1],
// [3], ..., [13] at wv[e ws + slot] (e = 0..6, zero where the edge leaves the
// closure) and its diagonal at wv[7 ws + slot].  With wi15 != nullptr (per-
// element k, or the intact side of a Dirichlet-Neumann recovery) a master
// holds its own 15 entries at wi15[n stride + f] (kGrid15 order).
struct Gen15 {
    const int *rowN15 = nullptr;
    const double *w15 = nullptr;
    const int *sid = nullptr;
    const double *wtab = nullptr;
    const int *nb15 = nullptr;
    const int *ifcq = nullptr;
    int nq = 0;
    const double *wv = nullptr;
    long long ws = 0;
    const double *wi15 = nullptr;
    // FP32 copies of w15, wtab, wv, wi15 (mixed precision; nullptr otherwise)
    const float *w15f = nullptr, *wtabf = nullptr, *wvf = nullptr, *wi15f = nullptr;
};

// Per-element coefficient on a general macro mesh: k of the level's elements
// (element order), the unit-size element matrices kel[((6 t + q) 16 + 4 r + r']
// of macro tetrahedron t and axis order q, the level's cells per axis N and
// segments per macro edge m.
struct GenK {
    const double *k = nullptr;             // nullptr: k = 1
    const double *kel = nullptr;
    const unsigned char *faulty = nullptr;  // macro tetrahedra whose elements are left out, or nullptr
    int N = 0, m = 0, n_sub = 0;
};

template <typename T>
struct Weights {
    const T *w0 = nullptr, *w1 = nullptr, *w2 = nullptr;  // volume edge weights per slot, local dirs a,b,c
    const T *wi = nullptr;                                // [6][n_ifc] interface edge weights
};

// colour pass of red-black SOR: the volume nodes in vg's list and the
// interface nodes of ig (all of one colour).  own0: the nodes of this colour
// start from zero; nb0: all neighbours are zero.
template <typename T>
void launch_colour(hipStream_t s, const VolGeom &vg, const IfcGeom &ig, T *u, const T *b, const Weights<T> &w, bool vk,
                   double h, double omega, bool own0, bool nb0);

// Fused red-black sweep on the cube with k = 1 (fused.hip): the volume
// interiors of the listed tetrahedra, tile by tile.  A tile (i0, j0, k0, -)
// covers i0 .. i0 + fused_tile_i() - 1, rows j0 .. j0 + TJ - 1 and planes
// k0 .. k0 + TK - 1 of each tetrahedron's index space; m = segments per macro
// edge; ps holds the first slot of every plane's red nodes ([0][k]) and
// black nodes ([1][k], counted from black0), [2][m + 2].
struct FusedGeom {
    const VolDesc *vd = nullptr;
    int nvol = 0;
    const int4 *tiles = nullptr;
    int ntiles = 0;
    int m = 0;
    int TJ = 0, TK = 0;
    long long black0 = 0;
    const int *ps = nullptr;
    int remap = 1;
};
// LDS bytes of one workgroup (word = sizeof(T)), the i extent of a tile, and
// whether a shape fits the kernel
size_t fused_lds_bytes(const FusedGeom &g, size_t word);
int fused_tile_i();
bool fused_shape_ok(const FusedGeom &g);
// one sweep of the volume interiors from us to ud (us is not written; ud's
// red boundary copies must already hold the new red interface values);
// zero: the sweep starts from u = 0 (us is not read); rout (optional): the
// black nodes' residual after the sweep, (1 - omega) r
template <typename T>
void launch_sweep_fused_vol(hipStream_t s, const FusedGeom &g, const T *us, T *ud, const T *b, double h, double omega,
                            bool zero, T *rout);
// SOR update of the interface masters [ig.i0, ig.i1) of one colour with k = 1:
// own value from us (0 if own0), neighbours from un (0 if nb0), new value to
// ud at the master and its ghost copies; rout (optional) as above
template <typename T>
void launch_ifc_sor(hipStream_t s, const IfcGeom &ig, const T *us, const T *un, T *ud, const T *b, double h,
                    double omega, bool own0, bool nb0, T *rout);

// coarse-grid correction u += P e_c of the nodes of one colour, in the form
// launch_prolong takes it (coarse volume descriptors in the fine view's
// order, coarse row table and closure edge length, [2][n_ifc] coarse slots
// per interface master, the coarse correction)
template <typename T>
struct Prol {
    const VolDesc *vdc = nullptr;
    const int2 *cC = nullptr;
    int Mc = 0;
    const int *prl = nullptr;
    const T *ec = nullptr;
};

// colour pass that first adds the coarse-grid correction to each of its own
// nodes (bitwise the value launch_prolong would have stored) and then
// updates it.  Its neighbours are of the other colour and must already hold
// their corrected values.
template <typename T>
void launch_colour_prol(hipStream_t s, const VolGeom &vg, const IfcGeom &ig, T *u, const T *b, const Weights<T> &w,
                        bool vk, double h, double omega, const Prol<T> &p);

// number of workgroups of a colour pass (volume list and interface part)
int colour_blocks(const VolGeom &vg, const IfcGeom &ig);

// FP64 colour pass that also leaves, per workgroup, the sum of
// ((1 - omega) r)^2 over its nodes in partial (r = b - A u before each
// update: after the pass, the residual of each updated node is (1 - omega) r,
// since its neighbours are of the other colour).  Returns the number of
// workgroups, colour_blocks(vg, ig).
int launch_colour_norm(hipStream_t s, const VolGeom &vg, const IfcGeom &ig, double *u, const double *b,
                       const Weights<double> &w, bool vk, double h, double omega, double *partial);

// colour pass that also writes, at each updated node, its residual after the
// pass to r: (1 - omega) (b - A u) with A u taken before the update (the
// node's neighbours are of the other colour and do not change).  The other
// colour's entries of r are left as they are.
template <typename T>
void launch_colour_res(hipStream_t s, const VolGeom &vg, const IfcGeom &ig, T *u, const T *b, const Weights<T> &w,
                       bool vk, double h, double omega, T *r);

// r = b - A u on volume interiors and interface nodes; r (of type TO) may be
// nullptr; partial (one double per block) receives block sums of r^2 if not
// nullptr.  Returns the number of blocks launched.
template <typename T, typename TO>
int launch_residual(hipStream_t s, const VolGeom &vg, const IfcGeom &ig, const T *u, const T *b, const Weights<T> &w,
                    bool vk, double h, TO *r, double *partial);

// b_c = P^T r_f.  vc: coarse volumes (interior list of the coarse level),
// vdf: matching fine volumes, fC: row table of the fine level;
// rst: [15][n_ifc_c] fine slots per coarse interface node.
template <typename T>
void launch_restrict(hipStream_t s, const VolGeom &vc, const VolDesc *vdf, const int2 *fC, const IfcGeom &igc,
                     const int *rst, const T *rf, T *bc);

// u_f += P e_c in place.  vf: fine volumes (interior list), vdc: matching
// coarse volumes, cC and Mc: row table and nodes per edge of the coarse
// level; prl: [2][n_ifc_f] coarse slots per fine interface node (the
// interface part also updates the ghost copies).
template <typename T>
void launch_prolong(hipStream_t s, const VolGeom &vf, const VolDesc *vdc, const int2 *cC, int Mc, const IfcGeom &igf,
                    const int *prl, const T *ec, T *uf);

// coarsest level solved with a precomputed dense inverse inv (row-major
// n x n, FP64): x = inv b over the master slots, written to every slot that
// holds each unknown (cptr/cidx), in the value type of b and u
template <typename T>
void launch_coarse_dense(hipStream_t s, int n, const long long *slot, const double *inv, const T *b, T *u,
                         const int *cptr, const int *cidx);

// b = M f with the unit cube's k-independent P1 mass matrix, both in vector
// order ((N-1)^3 interior nodes, x fastest)
void launch_mass_grid(hipStream_t s, int N, double h, const double *f, double *b);

// per-block partial sums of v^2 over every interior node once (the volume
// nodes of vg's list, four per thread, and the masters of ig); returns the
// number of blocks (at most the block count of a one-node-per-thread list
// launch)
int launch_norm2(hipStream_t s, const VolGeom &vg, const IfcGeom &ig, const double *v, double *partial);

// Jacobi-PCG on the coarsest level in one workgroup
template <typename T>
void launch_coarse_pcg(hipStream_t s, int n, const long long *slot, const int *col, const double *val,
                       const unsigned char *frozen, const T *b, T *u, const int *cptr, const int *cidx, double rtol,
                       int maxit, int *iters);

// one-unknown coarsest level of local (single tetrahedron) hierarchies;
// sl = closure slots of the node (1,1,1) and of its -a, -b, -c neighbours
template <typename T>
void launch_local_coarse(hipStream_t s, const VolDesc *vd, int nvol, int4 sl, const T *b, T *u, const Weights<T> &w,
                         bool vk, double h);

void launch_reduce(hipStream_t s, const double *partial, int n, double *out);

template <typename T>
void launch_fill(hipStream_t s, T *p, long long n, T v);

// unstructured macro meshes: user vector <-> slot space for the interior
// nodes of the listed volumes (user index vbase + tet nint + the node's rank
// in plane k, row j, i order) and the masters of ig (ifc_dof); the ghost
// copies are set separately (launch_ghost_refresh)
template <typename T>
void launch_mesh_user_to_slots(hipStream_t s, const VolGeom &vint, long long vbase, long long nint, const IfcGeom &ig,
                               const int *ifc_dof, const double *user, T *vec);
template <typename T>
void launch_mesh_slots_to_user(hipStream_t s, const VolGeom &vint, long long vbase, long long nint, const IfcGeom &ig,
                               const int *ifc_dof, const T *vec, double *user);

// unstructured macro meshes, eliminated Dirichlet data: b[rows[q]] =
// -sum over ptr[q] .. ptr[q + 1] of val * g[col] (mesh_kernels.hip); the
// other slots of b are left as they are
void launch_dirichlet_rows(hipStream_t s, int nrows, const int *rows, const int *ptr, const int *col,
                           const double *val, const double *g, double *b);
// unstructured macro meshes, Dirichlet-Neumann Neumann data: at the masters
// flagged in gamma, b_out = sum over e < w of wi[e] u[nb[e]] (rows of width
// w, entry e of master t at e n_ifc + t; mesh_kernels.hip)
void launch_neumann_rhs_w(hipStream_t s, int n_ifc, long long base, const int *nb, const double *wi, int w,
                          const unsigned char *gamma, const double *u, double *b_out);
// unstructured macro meshes, dJ/dk_t = -lambda^T A_t u per tetrahedron (a
// coefficient constant on each): u and lam in slot space of the finest
// level (ghost copies current), kel the unit-k matrices of the 6 element
// types per tetrahedron (Topology::mesh_kuhn_matrices), partial scratch of
// nt m (m + 1) / 2 doubles, out nt values (mesh_kernels.hip)
void launch_mesh_grad_tet(hipStream_t s, int nt, int m, int M, const int2 *rowC, long long C_pad, const double *kel,
                          const double *u, const double *lam, double *partial, double *out);

// user vector (global lexicographic interior order) <-> slot space; vfull
// lists every closure node (ghosts receive the user value or the Dirichlet zero)
template <typename T>
void launch_user_to_slots(hipStream_t s, const VolGeom &vfull, const int *tetinfo, int m, int N, const IfcGeom &ig,
                          const int *ifc_dof, const double *user, T *vec);
template <typename T>
void launch_slots_to_user(hipStream_t s, const VolGeom &vint, const int *tetinfo, int m, int N, const IfcGeom &ig,
                          const int *ifc_dof, const T *vec, double *user);

// y = M x (consistent P1 mass matrix) at volume-interior and interface slots
void launch_mass(hipStream_t s, const VolGeom &vint, const IfcGeom &ig, const int *nb15, const double *x, double *y,
                 double h);

// u64 += e32 over the closure slots [0, span) of the listed volumes and the
// interface slots
void launch_update_add(hipStream_t s, const VolDesc *vd, int nvol, long long span, const IfcGeom &ig, double *u,
                       const float *e);

// u[dst[q]] = u[src[q]]
template <typename T>
void launch_ghost_refresh(hipStream_t s, const int *dst, const int *src, int n, T *u);

template <typename TI, typename TO>
void launch_cast(hipStream_t s, const TI *in, TO *out, long long n);

// coefficient pipeline
void launch_coarsen_k(hipStream_t s, const double *kf, int Nf, double *kc, int Nc);
void launch_vol_weights(hipStream_t s, const VolGeom &vfull, const int *tetinfo, int m, int N, double h,
                        const double *k, double *w0, double *w1, double *w2);
void launch_ifc_weights(hipStream_t s, int n_ifc, const int *ifc_xyz, int N, double h, const double *k, double *wi);
// general macro meshes: one SOR pass over one of the 4 classes (vg lists its
// interior nodes, g.ifcq its masters; ig gives base, stride, ghosts, frozen)
template <typename T>
void launch_colour15(hipStream_t s, const VolGeom &vg, const IfcGeom &ig, const Gen15 &g, T *u, const T *b,
                     double omega);
// workgroups of such a class pass
int colour15_blocks(const VolGeom &vg, const Gen15 &g);
// class pass that also leaves per-workgroup sums of ((1 - omega) r)^2 over
// its nodes (FP64), or writes (1 - omega) r to r at its nodes: with r the
// residual before the update, that is the node's residual after the pass
// (no 15-point stencil couples two nodes of one class)
int launch_colour15_norm(hipStream_t s, const VolGeom &vg, const IfcGeom &ig, const Gen15 &g, double *u,
                         const double *b, double omega, double *partial);
template <typename T>
void launch_colour15_res(hipStream_t s, const VolGeom &vg, const IfcGeom &ig, const Gen15 &g, T *u, const T *b,
                         double omega, T *r);
// general macro meshes: r = b - A u over the interior list of vg and the
// masters g.ifcq[0 .. g.nq) if g.ifcq is set, else every master of ig (r
// and/or partial sums of r^2 per block, as launch_residual)
template <typename T, typename TO>
int launch_residual15(hipStream_t s, const VolGeom &vg, const IfcGeom &ig, const Gen15 &g, const T *u, const T *b,
                      TO *r, double *partial);
// coarsest level of a general macro mesh: Jacobi-PCG with 15 entries per row
template <typename T>
void launch_coarse_pcg15(hipStream_t s, int n, const long long *slot, const int *col, const double *val,
                         const unsigned char *frozen, const T *b, T *u, const int *cptr, const int *cidx,
                         double rtol, int maxit, int *iters);
// local coarsest level of a general macro mesh: u = b / diagonal at the single interior node
void launch_local_coarse15(hipStream_t s, const VolDesc *vd, int nvol, int slot, const Gen15 &g, const double *b,
                           double *u);
// per-element coefficient on a general macro mesh: closure-slot weights of
// every tetrahedron in vfull (full closure lists), interface weights, and the
// coarsest-level rows (kGrid15 order, zero for boundary columns)
void launch_gen_weights(hipStream_t s, const VolGeom &vfull, const int *tetinfo, const GenK &G, double *wv,
                        long long ws);
void launch_gen_ifc_weights(hipStream_t s, int n_ifc, const int *ifc_xyz, const GenK &G, double *wi15);
void launch_gen_coarse_vals(hipStream_t s, int n, const int *pos, const int *col15, const GenK &G, double *val);
// y = S x on a general macro mesh (interior nodes of vint, masters of ig)
// with the stencils of g, e.g. the mass matrix
void launch_apply15(hipStream_t s, const VolGeom &vint, const IfcGeom &ig, const Gen15 &g, const double *x, double *y);
// dJ/dk per element of a general macro mesh (u, lam in vector order)
void launch_grad_k15(hipStream_t s, int N, int m, int n_sub, const double *kel, const double *u, const double *lam,
                     double *out);
// Dirichlet-Neumann Neumann data on a general macro mesh (see launch_neumann_rhs)
void launch_neumann_rhs15(hipStream_t s, int n_ifc, long long base, const int *nb15, const double *wi15,
                          const unsigned char *gamma, const double *u, double *b_out);
// eliminated Dirichlet data on a general macro mesh into b (slot order):
// interior nodes of vint and masters [0, ig.i1) of ig
void launch_gen_dirichlet(hipStream_t s, const VolGeom &vint, const IfcGeom &ig, const Gen15 &g, const int *tetinfo,
                          const int *ifc_xyz, int N, const double *gfull, double *b);
// b = eliminated Dirichlet data g (full (N+1)^3 grid, x fastest), vector order
void launch_dirichlet_load(hipStream_t s, int N, double h, const double *k, const double *g, double *b);
void launch_coarse_vals(hipStream_t s, int n, const int *pos, const int *col, int N, double h, const double *k,
                        double *val);

// Dirichlet-Neumann recovery: interface and coarsest-level operators over the
// elements of intact macro tetrahedra only (k == nullptr: k = 1; faulty[t] for
// each macro tetrahedron), and the static Neumann data b_out = A^I u at the
// interface nodes flagged in gamma
void launch_ifc_weights_intact(hipStream_t s, int n_ifc, const int *ifc_xyz, int N, int m, int n_sub, double h,
                               const double *k, const unsigned char *faulty, double *wi);
void launch_coarse_vals_intact(hipStream_t s, int n, const int *pos, const int *col, int N, int m, int n_sub, double h,
                               const double *k, const unsigned char *faulty, double *val);
void launch_neumann_rhs(hipStream_t s, int n_ifc, long long base, const int *nbr, const double *wi,
                        const unsigned char *gamma, const double *u, double *b_out);

// frozen / Gamma flags and the intact-side ghost list of a Dirichlet-Neumann recovery
void launch_dn_masks(hipStream_t s, int n_ifc, long long base, long long C_pad, const int *gptr, const int *gidx,
                     const unsigned char *faulty, unsigned char *frozen, unsigned char *gamma, int *gidx_dn);

// dJ/dk per element from user-order u and lambda
void launch_grad_k(hipStream_t s, const double *u, const double *lam, int N, double h, double *out);

}  // namespace hhgr
