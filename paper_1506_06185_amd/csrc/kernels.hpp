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

// structured part of a launch: every listed volume x every chunk of its closure
struct VolGeom {
    const VolDesc *vd = nullptr;
    const int2 *chunks = nullptr;  // (plane k, first offset) per chunk of bs slots
    int nchunks = 0;
    int nvol = 0;
    int M = 0;   // nodes per macro edge at this level (2^l + 1)
    int bs = 256;
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
template <typename T>
void launch_colour(hipStream_t s, const VolGeom &vg, const IfcGeom &ig, T *u, const T *b, const Weights<T> &w, bool vk,
                   double h, double omega, int colour, bool own0, bool nb0);

// r = b - A u on volume interiors and interface nodes; r (of type TO) may be
// nullptr; partial (one double per block) receives block sums of r^2 if not
// nullptr.  Returns the number of blocks launched.
template <typename T, typename TO>
int launch_residual(hipStream_t s, const VolGeom &vg, const IfcGeom &ig, const T *u, const T *b, const Weights<T> &w,
                    bool vk, double h, TO *r, double *partial);

// b_c = P^T r_f.  vc: coarse volumes (interior chunks of the coarse level),
// vdf: matching fine volumes; rst: [15][n_ifc_c] fine slots per coarse interface node.
template <typename T>
void launch_restrict(hipStream_t s, const VolGeom &vc, const VolDesc *vdf, int Mf, const IfcGeom &igc, const int *rst,
                     const T *rf, T *bc);

// u_f += P e_c.  vf: fine volumes (interior chunks), vdc: matching coarse
// volumes; prl: [2][n_ifc_f] coarse slots per fine interface node.
template <typename T>
void launch_prolong(hipStream_t s, const VolGeom &vf, const VolDesc *vdc, int Mc, const IfcGeom &igf, const int *prl,
                    const T *ec, T *uf);

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
