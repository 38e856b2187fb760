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

// structured part of a launch: every listed volume x either a list of nodes
// (list mode: packed (i,j,k), the same for every volume, with the row offset
// tables of the level) or every chunk of its closure (chunk mode)
struct VolGeom {
    const VolDesc *vd = nullptr;
    int nvol = 0;
    const unsigned *list = nullptr;  // list mode
    int nlist = 0;
    const int4 *rowA = nullptr;      // per row (j,k): (slot of (0,j,k), length, to (j-1,k+1), to (j+1,k-1))
    const int4 *rowB = nullptr;      // per row: (to (j,k+1), to (j,k-1), 0, 0)
    const int2 *chunks = nullptr;    // chunk mode: (plane k, first offset) per chunk of bs slots
    int nchunks = 0;
    int M = 0;   // nodes per macro edge at this level (2^l + 1)
    int bs = 256;
    int remap = 1;  // 1: contiguous block ranges per XCD, 0: hardware order
    int cpb = 4;    // list mode: nodes per thread (1 or 4), all loads issued before the stores
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
};

template <typename T>
struct Weights {
    const T *w0 = nullptr, *w1 = nullptr, *w2 = nullptr;  // volume edge weights per slot, local dirs a,b,c
    const T *wi = nullptr;                                // [6][n_ifc] interface edge weights
};

// colour pass of red-black SOR (colour 0 = red = even x+y+z).  own0: the
// nodes of this colour start from zero; nb0: all neighbours are zero.
// uvol: where interface nodes read their volume-interior neighbours (the
// volume interiors may live in a second buffer during fused sweeps); u holds
// the interface masters and the ghost copies.
template <typename T>
void launch_colour(hipStream_t s, const VolGeom &vg, const IfcGeom &ig, T *u, const T *uvol, const T *b,
                   const Weights<T> &w, bool vk, double h, double omega, int colour, bool own0, bool nb0);

// tiles of the fused sweep: (j0, k0, i0) of an 8x8 block of rows and a
// 62-node segment along i
constexpr int kFusedTile = 8;
constexpr int kFusedSeg = 62;
struct FusedGeom {
    const VolDesc *vd = nullptr;
    const int4 *tiles = nullptr;
    const int4 *rowA = nullptr;
    int ntiles = 0;
    int nvol = 0;
    int M = 0;
    int remap = 1;
};

// one red-black SOR sweep of the volume interiors: reads uin (interiors) and
// ughost (ghost copies, red ones already updated), writes uout (interiors).
// zero: uin is logically zero (first sweep of a correction).
template <typename T>
void launch_fused_sweep(hipStream_t s, const FusedGeom &fg, const T *uin, T *uout, const T *ughost, const T *b,
                        const Weights<T> &w, bool vk, double h, double omega, bool zero);

// r = b - A u on volume interiors and interface nodes; r (of type TO) may be
// nullptr; partial (one double per block) receives block sums of r^2 if not
// nullptr.  Returns the number of blocks launched.
template <typename T, typename TO>
int launch_residual(hipStream_t s, const VolGeom &vg, const IfcGeom &ig, const T *u, const T *b, const Weights<T> &w,
                    bool vk, double h, TO *r, double *partial);

// b_c = P^T r_f.  vc: coarse volumes (interior list of the coarse level),
// vdf: matching fine volumes, fA/fB: row tables of the fine level;
// rst: [15][n_ifc_c] fine slots per coarse interface node.
template <typename T>
void launch_restrict(hipStream_t s, const VolGeom &vc, const VolDesc *vdf, const int4 *fA, const int4 *fB,
                     const IfcGeom &igc, const int *rst, const T *rf, T *bc);

// u_f += P e_c.  vf: fine volumes (interior list), vdc: matching coarse
// volumes, cA: row table and Mc node count per edge of the coarse level;
// prl: [2][n_ifc_f] coarse slots per fine interface node.  The volume part
// writes uo = uf + P e_c (uo may differ from uf); the interface part updates
// uf in place and its ghost copies.
template <typename T>
void launch_prolong(hipStream_t s, const VolGeom &vf, const VolDesc *vdc, const int4 *cA, int Mc, const IfcGeom &igf,
                    const int *prl, const T *ec, T *uf, T *uo);

// Jacobi-PCG on the coarsest level in one workgroup
template <typename T>
void launch_coarse_pcg(hipStream_t s, int n, const long long *slot, const int *col, const double *val,
                       const unsigned char *frozen, const T *b, T *u, const int *cptr, const int *cidx, double rtol,
                       int maxit, int *iters);

// one-unknown coarsest level of local (single tetrahedron) hierarchies
template <typename T>
void launch_local_coarse(hipStream_t s, const VolDesc *vd, int nvol, int M, const T *b, T *u, const Weights<T> &w,
                         bool vk, double h);

void launch_reduce(hipStream_t s, const double *partial, int n, double *out);

template <typename T>
void launch_fill(hipStream_t s, T *p, long long n, T v);

// user vector (global lexicographic interior order) <-> slot space
template <typename T>
void launch_user_to_slots(hipStream_t s, const VolGeom &vfull, const int *tetinfo, int m, int N, const IfcGeom &ig,
                          const int *ifc_dof, const double *user, T *vec);
template <typename T>
void launch_slots_to_user(hipStream_t s, const VolGeom &vint, const int *tetinfo, int m, int N, const IfcGeom &ig,
                          const int *ifc_dof, const T *vec, double *user);

// y = M x (consistent P1 mass matrix) at volume-interior and interface slots
void launch_mass(hipStream_t s, const VolGeom &vint, const IfcGeom &ig, const int *nb15, const double *x, double *y,
                 double h);

// u64 += e32 over the closures of the listed volumes and all interface slots
void launch_update_add(hipStream_t s, const VolGeom &vfull, const IfcGeom &ig, double *u, const float *e);

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
void launch_coarse_vals(hipStream_t s, int n, const int *pos, const int *col, int N, double h, const double *k,
                        double *val);

// dJ/dk per element from user-order u and lambda
void launch_grad_k(hipStream_t s, const double *u, const double *lam, int N, double h, double *out);

}  // namespace hhgr
