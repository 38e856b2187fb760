// Solver engine and C ABI of the HHG multigrid library (declarations and
// semantics in include/hhgr.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <tuple>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/hhgr.h"
#include "geometry.hpp"
#include "kernels.hpp"
#include "topology.hpp"

namespace hhgr {

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(x)                                                                                  \
    do {                                                                                           \
        hipError_t e_ = (x);                                                                       \
        if (e_ != hipSuccess) return fail(HHGR_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define CHKLAUNCH()                                                                                   \
    do {                                                                                              \
        hipError_t e_ = hipGetLastError();                                                            \
        if (e_ != hipSuccess) return fail(HHGR_EHIP, std::string("kernel launch: ") + hipGetErrorString(e_)); \
    } while (0)

constexpr int kBS[3] = {128, 256, 512};
constexpr double kCoarseRtol = 1e-14;
constexpr int kCoarseMaxit = 2000;
// largest coarsest level (unknowns) solved with a precomputed dense inverse
// (k = 1; 512^2 FP64 = 2 MiB of workspace)
constexpr int kDenseCoarseMax = 512;
// ... on an unstructured macro mesh, whose coarsest level has no other solver
constexpr int kDenseCoarseMaxMesh = 2048;
constexpr int kMaxLevels = 10;

// bump allocator over the caller's workspace; with base == nullptr it only sizes
struct Carver {
    char *base = nullptr;
    size_t off = 0;
    template <typename T>
    T *take(size_t n) {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += std::max<size_t>(n, 1) * sizeof(T);
        return p;
    }
};

struct LevelDev {
    int l = 0, m = 0, M = 0, N = 0;
    double h = 0;
    long long C = 0, C_pad = 0, ifc_base = 0, n_slots = 0;
    int n_ifc = 0, n_ifc_red = 0;
    int bs_sel = 1;  // colour pass
    int remap = 1;   // XCD-contiguous block order (autotuned)
    int cpb = 1;     // nodes per thread of the list-mode kernels (autotuned)
    int cpb_res = 1; // ... of the residual, of the prolongation and of the red
    int cpb_prl = 1; // post-smoothing pass that adds the correction (autotuned
    int cpb_fus = 1; // separately)
    int nbw = 15;    // entries per master of the general-mesh stencil and restriction tables
    long long vbase = 0, nint = 0;  // unstructured macro meshes: user order of the volume interiors
    int *nbr = nullptr, *gptr = nullptr, *gidx = nullptr, *rst = nullptr, *prl = nullptr, *nb15 = nullptr;
    int *ifc_dof = nullptr, *ifc_xyz = nullptr, *tg_dst = nullptr, *tg_src = nullptr;
    std::vector<int> tg_ptr;
    double *u = nullptr, *b = nullptr, *r = nullptr;
    float *u32 = nullptr, *b32 = nullptr, *r32 = nullptr;
    // node lists: interior (all, red, black), every closure node
    unsigned *ilist = nullptr, *rlist = nullptr, *blist = nullptr, *flist = nullptr;
    int nilist = 0, nrlist = 0, nblist = 0, nflist = 0;
    int2 *rowC = nullptr;  // row table of the colour-split closure layout
    int4 *rowN = nullptr;  // neighbour bases per (colour, row)
    int nrows = 0;
    int4 lc_sl{0, 0, 0, 0};  // slots of (1,1,1) and its -a, -b, -c neighbours (local coarsest level)
    double *w[3] = {}, *wi = nullptr;
    float *w32[3] = {}, *wi32 = nullptr;
    double *kc = nullptr;
    VolDesc *vd_all = nullptr, *vd_masked = nullptr, *vd_loc = nullptr;
    int n_masked = 0, n_loc = 0;
    unsigned char *frozen = nullptr;
    double *lu = nullptr, *lb = nullptr, *lr = nullptr;  // local hierarchy (levels < L)
    // Dirichlet-Neumann recovery: intact-side interface weights, ghost copies
    // outside the faulty closures, interface nodes with static Neumann data
    double *wi_dn = nullptr;
    int *gidx_dn = nullptr;  // same layout as gidx (gptr)
    unsigned char *gamma = nullptr;
    // general macro meshes: interior nodes and interface masters of each of
    // the 4 classes, 15-point row bases, the volume stencil of every
    // tetrahedron, and per master the index of its stencil in a table of the
    // level's distinct stencils (one per primitive)
    unsigned *qlist[4] = {};
    int nqlist[4] = {};
    int *ifcq[4] = {};
    int nifcq[4] = {};
    int *rowN15 = nullptr;
    double *w15 = nullptr, *wtab = nullptr;
    int *sid = nullptr;
    int wtab_cap = 0;
    // ... with a per-element coefficient: 7 forward edge weights and the
    // diagonal per closure slot ([e n_slots + slot]), 15 entries per master
    double *wv = nullptr, *wi15 = nullptr;
    double *wi15_dn = nullptr;  // intact-side master entries of a Dirichlet-Neumann recovery
    double *mw15 = nullptr, *mwtab = nullptr;  // finest level: mass stencils (indexed like w15, wtab)
    double *mwi = nullptr;                     // ... the masters' own mass rows (unstructured meshes)
    float *w15f = nullptr, *wtabf = nullptr, *wvf = nullptr, *wi15f = nullptr;  // FP32 copies (mixed precision)
    // fused red-black sweeps (cube, k = 1, unmasked cycles): a second slot
    // vector of u in the cycle's precision (the pair of sweeps goes u -> ualt
    // -> u), plane starts and tiles (FusedGeom)
    double *ualt = nullptr;
    float *u32alt = nullptr;
    int *fz_ps = nullptr;
    int4 *fz_tiles = nullptr;
    std::vector<int> fz_ps_host;
    std::vector<int4> fz_tiles_host;
    int fz_TJ = 0, fz_TK = 0;
    long long fz_black0 = 0;
    bool fz_on = false;  // the cycles use fused pairs on this level (autotuner: where faster)
};

template <typename T>
struct LevView {
    T *u = nullptr, *b = nullptr, *r = nullptr;
    T *ualt = nullptr;  // second buffer of fused sweep pairs (unmasked cube cycles with k = 1), or nullptr
    Weights<T> w;
    const VolDesc *vd = nullptr;
    int nvol = 0;
    bool ifc = false;
    const unsigned char *frozen = nullptr;
    const int *gptr = nullptr, *gidx = nullptr;  // ghost copies to update (nullptr: all of the level's)
    const double *wi15 = nullptr;                // general macro mesh: master entries (nullptr: the level's)
};

template <typename T>
struct HView {
    LevView<T> lv[kMaxLevels];
    int L = 0, Lc = 0;
    bool local = false;
    const unsigned char *cfrozen = nullptr;
    const double *cval = nullptr;  // coarsest-level operator (nullptr: the context's)
    double *partial = nullptr;
    unsigned int *counter = nullptr;
    bool timed = false;
};

}  // namespace
}  // namespace hhgr

using namespace hhgr;

struct hhgr_ctx {
    hhgr_desc d{};
    std::shared_ptr<const Topology> topo_hold;  // shared by contexts of the same mesh and levels
    const Topology *topo = nullptr;
    std::vector<LevelDev> lev;
    int L = 0, Lc = 0, n_tets = 0;
    long long n_dofs = 0, n_elems = 0;
    hipStream_t stream = nullptr, stream2 = nullptr;
    hipStream_t cap = nullptr;  // graphs are captured here (the caller's stream may be the legacy default stream)
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    double *partial[2] = {};
    unsigned int *counter = nullptr;  // [2] last-block detection of the norm reductions
    int partial_cap = 0;
    double *dnorm = nullptr;
    double *hnorm = nullptr;  // pinned, or hnorm_local in a context without HIP objects of its own
    double hnorm_local[8] = {};
    int *tetinfo = nullptr;
    // coarsest level
    long long *cslot = nullptr;
    int *ccol = nullptr, *cptr = nullptr, *cidx = nullptr, *cpos = nullptr, *citers = nullptr;
    double *cval = nullptr, *cval_dn = nullptr;
    unsigned char *cfrozen = nullptr, *dn_faulty = nullptr;
    int cn = 0;
    // dense inverse of the unmasked coarsest-level operator (k = 1, at most
    // kDenseCoarseMax unknowns): workspace room in cinv, valid once
    // dense_coarse is set (at create on the cube, by hhgr_set_geometry on a
    // general mesh); the other operators use PCG
    bool dense_coarse = false;
    double *cinv = nullptr;
    // unstructured macro meshes: dense inverse of the coarsest operator with
    // the unknowns frozen by a Dirichlet-Dirichlet recovery left out (their
    // rows and columns zero), set by dd_setup
    double *cinv_dd = nullptr;
    // ... and the couplings of interior rows to Dirichlet boundary nodes
    int *dir_rows = nullptr, *dir_ptr = nullptr, *dir_col = nullptr;
    double *dir_val = nullptr;
    int n_dir_rows = 0;
    // general macro meshes: 15-point coarsest-level operator
    bool gen = false, geom_set = false;
    bool mesh = false;  // unstructured macro mesh (hhgr_create_mesh): gen, operator fixed at creation
    int *ccol15 = nullptr;
    double *cval15 = nullptr;
    double *kel = nullptr;  // unit-size element matrices per macro tet and axis order
    double *cval15_dn = nullptr;  // intact-side coarsest-level rows of a Dirichlet-Neumann recovery
    std::vector<double> cval_host;
    // adjoint temporaries
    double *aux_u = nullptr, *aux_b = nullptr, *user_u = nullptr, *user_l = nullptr;
    double bnorm = 0.0;
    bool rhs_set = false, coeff_set = false;
    bool vk = false, mixed = false;
    // graphs
    bool use_graph = false;
    hipGraphExec_t gexec = nullptr;
    bool graph_ok = false;
    // local recovery: its kernels are small enough that launching them one
    // by one leaves the GPU waiting for the host, so its cycles replay a
    // captured graph, kept for one (tetrahedron, cycle count)
    hipGraphExec_t lgexec = nullptr;
    int lg_tet = -1, lg_n = -1;
    std::vector<int> loc_tets;  // the tetrahedra whose local hierarchy vd_loc holds
    // unstructured mesh with a coefficient per tetrahedron (empty: k = 1):
    // the values, the master rows of every level and the coarsest rows
    std::vector<double> mesh_k;
    std::vector<std::vector<double>> mesh_k_wi;
    std::vector<double> mesh_k_valw;
    double *mesh_kel = nullptr;  // unit-k matrices of the 6 element types per tetrahedron (finest level)
    // kernel timing
    bool timing = false;
    std::vector<hipEvent_t> tev;
    size_t tev_used = 0;
    void *ws = nullptr;
    size_t ws_bytes = 0;
};

// a Dirichlet-Dirichlet recovery armed on a batch member
struct BatchDD {
    bool armed = false;
    std::vector<int> tets;
    int n_intact = 0, n_local = 0;
    int step = 0;  // steps of the recovery done
};

struct hhgr_batch {
    std::vector<hhgr_ctx *> ctx;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;
    std::vector<hipStream_t> branch, branch2;  // per member: main branch, local-recovery branch
    std::vector<hipEvent_t> ev;                // [0] fork, [1 + q] member join
    std::vector<hipEvent_t> evl;               // [2q] local fork, [2q + 1] local join
    std::vector<BatchDD> dd;
    hipGraphExec_t gexec = nullptr;
    std::vector<int> sig_in_graph;  // (member, mode) pairs the graph was captured for
    double *hnorm = nullptr;        // pinned, one per member
};

namespace hhgr {
namespace {

// ----------------------------------------------------------------------------
// fused sweep tables of one level: plane starts of each colour, tile shape
// (i extent fixed by the kernel, rows TJ, planes TK) and the tiles that hold
// interior nodes
// ----------------------------------------------------------------------------
// planes and rows per tile (the LDS of one FP64 workgroup is 288 (7 TJ + 22)
// bytes with tiles of 64 i values, under 64 KiB for TJ <= 28)
#ifndef HHGR_FUSED_TK
#define HHGR_FUSED_TK 16
#endif
#ifndef HHGR_FUSED_TJ
#define HHGR_FUSED_TJ 28
#endif
constexpr int kFusedTK = HHGR_FUSED_TK;
constexpr int kFusedTJ = HHGR_FUSED_TJ;

// false: the kernel cannot take this level (the level keeps two colour passes per sweep)
bool fused_tables(const TopoLevel &T, LevelDev &D) {
    const int m = T.m, M = T.M;
    const ClosureLayout &ly = T.lay;
    D.fz_black0 = ly.black0;
    D.fz_ps_host.assign(2 * (size_t)(m + 2), 0);
    for (int c = 0; c < 2; c++) {
        for (int k = 0; k <= m; k++)
            D.fz_ps_host[c * (m + 2) + k] = ly.row0[2 * (size_t)row_id(M, 0, k) + c] - (c ? (int)ly.black0 : 0);
        D.fz_ps_host[c * (m + 2) + m + 1] = (int)(c ? ly.n_black : ly.n_red);
    }
    D.fz_TJ = std::min(kFusedTJ, m);
    D.fz_TK = std::min(kFusedTK, m);
    FusedGeom g;
    g.m = m;
    g.TJ = D.fz_TJ;
    g.TK = D.fz_TK;
    if (!fused_shape_ok(g)) {
        D.fz_ps_host.clear();
        D.fz_tiles_host.clear();
        return false;
    }
    const int ti = fused_tile_i();
    D.fz_tiles_host.clear();
    for (int k0 = 1; k0 <= m - 3; k0 += D.fz_TK)
        for (int j0 = 1; j0 <= m - 3; j0 += D.fz_TJ)
            for (int i0 = 1; i0 <= m - 3; i0 += ti)
                if (i0 + j0 + k0 <= m - 1) D.fz_tiles_host.push_back(make_int4(i0, j0, k0, 0));
    return true;
}

// ----------------------------------------------------------------------------
// user vector <-> slot space of one level (D of context c).  to_slots sets
// every slot of the closures (ghost copies from their masters, Dirichlet
// ghosts zero) and the masters; to_user reads the interior nodes and masters.
// ----------------------------------------------------------------------------
VolGeom vgeom(const LevelDev &D, const VolDesc *vd, int nvol, bool full, int bsq, int colour);
IfcGeom igeom(const LevelDev &D, int i0, int i1, const unsigned char *frozen, bool scatter);

void to_slots(const hhgr_ctx &c, const LevelDev &D, const double *user, double *vec, hipStream_t s) {
    const IfcGeom ig = igeom(D, 0, D.n_ifc, nullptr, false);
    if (c.mesh) {
        launch_mesh_user_to_slots<double>(s, vgeom(D, D.vd_all, c.n_tets, false, -1, -1), D.vbase, D.nint, ig,
                                          D.ifc_dof, user, vec);
        launch_ghost_refresh<double>(s, D.tg_dst, D.tg_src, D.tg_ptr.back(), vec);
    } else {
        launch_user_to_slots<double>(s, vgeom(D, D.vd_all, c.n_tets, true, -1, -1), c.tetinfo, D.m, D.N, ig,
                                     D.ifc_dof, user, vec);
    }
}

void to_user(const hhgr_ctx &c, const LevelDev &D, const double *vec, double *user, hipStream_t s) {
    const IfcGeom ig = igeom(D, 0, D.n_ifc, nullptr, false);
    const VolGeom vint = vgeom(D, D.vd_all, c.n_tets, false, -1, -1);
    if (c.mesh)
        launch_mesh_slots_to_user<double>(s, vint, D.vbase, D.nint, ig, D.ifc_dof, vec, user);
    else
        launch_slots_to_user<double>(s, vint, c.tetinfo, D.m, D.N, ig, D.ifc_dof, vec, user);
}

// ----------------------------------------------------------------------------
// layout of the workspace (sizing and carving share this code)
// ----------------------------------------------------------------------------
void carve(hhgr_ctx &c, Carver &cv) {
    const Topology &tp = *c.topo;
    const int nf = std::max(c.d.max_faults, 1);
    c.lev.assign(c.L + 1, LevelDev());
    int max_blocks = 0;
    for (int l = c.Lc; l <= c.L; l++) {
        const TopoLevel &T = tp.lev[l];
        LevelDev &D = c.lev[l];
        D.l = l;
        D.m = T.m;
        D.M = T.M;
        D.N = T.N;
        D.h = T.h;
        D.C = T.C;
        D.C_pad = T.C_pad;
        D.ifc_base = T.ifc_base;
        D.n_slots = T.n_slots;
        D.n_ifc = T.n_ifc;
        D.n_ifc_red = T.n_ifc_red;
        D.nbw = tp.nbw;
        D.vbase = T.vbase;
        D.nint = T.nint;
        const size_t W = (size_t)tp.nbw;
        {
            // most blocks of a launch with per-block partial sums: smallest
            // workgroup, one node per thread, the longest node list
            const int nib = ((T.n_ifc + kBS[0] - 1) / kBS[0] + 7) & ~7;
            const long long nb = nib + (long long)((T.flist.size() + kBS[0] - 1) / kBS[0]) * c.n_tets;
            max_blocks = (int)std::max<long long>(max_blocks, nb);
        }
        D.nbr = cv.take<int>(6 * (size_t)T.n_ifc);
        D.gptr = cv.take<int>(T.n_ifc + 1);
        D.gidx = cv.take<int>(T.gidx.size());
        if (l > c.Lc) D.prl = cv.take<int>(2 * (size_t)T.n_ifc);
        if (l < c.L) D.rst = cv.take<int>(W * T.n_ifc);
        if (l == c.L || c.gen) D.nb15 = cv.take<int>(W * T.n_ifc);
        if (c.gen) {
            // the class lists (nodes, masters) back to back, so that classes
            // 0..2 form a prefix of each
            size_t nq_all = 0, nf_all = 0;
            for (int q = 0; q < 4; q++) {
                D.nqlist[q] = (int)T.qlist[q].size();
                D.nifcq[q] = (int)T.ifcq[q].size();
                nq_all += D.nqlist[q];
                nf_all += D.nifcq[q];
            }
            unsigned *qall = cv.take<unsigned>(nq_all);
            int *fall = cv.take<int>(nf_all);
            for (int q = 0, oq = 0, of = 0; q < 4; q++) {
                D.qlist[q] = qall ? qall + oq : nullptr;
                D.ifcq[q] = fall ? fall + of : nullptr;
                oq += D.nqlist[q];
                of += D.nifcq[q];
            }
            D.rowN15 = cv.take<int>(16 * T.rowN15.size());
            D.w15 = cv.take<double>(15 * (size_t)c.n_tets);
            // distinct master stencils: at most one per primitive (4 faces,
            // 6 edges, 4 vertices per tetrahedron), one zero stencil first
            D.wtab_cap = c.mesh ? 1 : 1 + 14 * c.n_tets;
            D.wtab = cv.take<double>(15 * (size_t)D.wtab_cap);
            D.sid = cv.take<int>(T.n_ifc);
            if (c.mesh) {
                // masters carry their own stencils (and, on the finest
                // level, their own mass-matrix rows), and the intact-side
                // rows of a Dirichlet-Neumann recovery
                D.wi15 = cv.take<double>(W * T.n_ifc);
                if (c.d.max_faults > 0) D.wi15_dn = cv.take<double>(W * T.n_ifc);
                if (l == c.L) {
                    D.mw15 = cv.take<double>(15 * (size_t)c.n_tets);
                    D.mwi = cv.take<double>(W * T.n_ifc);
                }
                if (c.mixed) {
                    D.w15f = cv.take<float>(15 * (size_t)c.n_tets);
                    D.wi15f = cv.take<float>(W * T.n_ifc);
                }
            } else {
                D.wi15_dn = cv.take<double>(15 * (size_t)T.n_ifc);
            }
            if (l == c.L && !c.mesh) {
                D.mw15 = cv.take<double>(15 * (size_t)c.n_tets);
                D.mwtab = cv.take<double>(15 * (size_t)D.wtab_cap);
            }
            if (c.mesh) {
            } else if (c.mixed && c.vk) {
                D.wvf = cv.take<float>(8 * (size_t)T.n_slots);
                D.wi15f = cv.take<float>(15 * (size_t)T.n_ifc);
            } else if (c.mixed) {
                D.w15f = cv.take<float>(15 * (size_t)c.n_tets);
                D.wtabf = cv.take<float>(15 * (size_t)D.wtab_cap);
            }
        }
        D.ifc_dof = cv.take<int>(T.n_ifc);
        D.ifc_xyz = cv.take<int>(3 * (size_t)T.n_ifc);
        D.tg_dst = cv.take<int>(T.tg_dst.size());
        D.tg_src = cv.take<int>(T.tg_src.size());
        D.tg_ptr = T.tg_ptr;
        D.u = cv.take<double>(T.n_slots);
        D.b = cv.take<double>(T.n_slots);
        D.r = cv.take<double>(T.n_slots);
        if (c.mixed) {
            D.u32 = cv.take<float>(T.n_slots);
            D.b32 = cv.take<float>(T.n_slots);
            D.r32 = cv.take<float>(T.n_slots);
        }
        if (!c.gen && !c.vk && l > c.Lc && T.m >= 8 && fused_tables(T, D)) {
            D.fz_ps = cv.take<int>(D.fz_ps_host.size());
            D.fz_tiles = cv.take<int4>(D.fz_tiles_host.size());
            if (c.mixed)
                D.u32alt = cv.take<float>(T.n_slots);
            else
                D.ualt = cv.take<double>(T.n_slots);
        }
        D.nilist = (int)T.ilist.size();
        D.nrlist = (int)T.rlist.size();
        D.nblist = (int)T.blist.size();
        D.nflist = (int)T.flist.size();
        D.ilist = cv.take<unsigned>(D.nilist);
        D.rlist = cv.take<unsigned>(D.nrlist);
        D.blist = cv.take<unsigned>(D.nblist);
        D.flist = cv.take<unsigned>(D.nflist);
        D.nrows = (int)T.rowC.size();
        D.rowC = cv.take<int2>(T.rowC.size());
        D.rowN = cv.take<int4>(2 * T.rowN.size());
        if (l == c.Lc) {
            const ClosureLayout &ly = T.lay;
            D.lc_sl = make_int4((int)ly.index(1, 1, 1), (int)ly.index(0, 1, 1), (int)ly.index(2, 0, 1),
                                (int)ly.index(1, 2, 0));
        }
        if (c.vk && c.gen) {
            D.wv = cv.take<double>(8 * (size_t)T.n_slots);
            D.wi15 = cv.take<double>(15 * (size_t)T.n_ifc);
            D.kc = cv.take<double>(6 * (size_t)T.N * T.N * T.N);
        } else if (c.vk) {
            for (int s = 0; s < 3; s++) D.w[s] = cv.take<double>(T.n_slots);
            D.wi = cv.take<double>(6 * (size_t)T.n_ifc);
            if (c.mixed) {
                for (int s = 0; s < 3; s++) D.w32[s] = cv.take<float>(T.n_slots);
                D.wi32 = cv.take<float>(6 * (size_t)T.n_ifc);
            }
            D.kc = cv.take<double>(6 * (size_t)T.N * T.N * T.N);
        }
        D.vd_all = cv.take<VolDesc>(c.n_tets);
        D.vd_masked = cv.take<VolDesc>(c.n_tets);
        D.vd_loc = cv.take<VolDesc>(nf);
        D.frozen = cv.take<unsigned char>(T.n_ifc);
        if (l < c.L) {
            D.lu = cv.take<double>((size_t)nf * T.C_pad);
            D.lb = cv.take<double>((size_t)nf * T.C_pad);
            D.lr = cv.take<double>((size_t)nf * T.C_pad);
        }
        D.wi_dn = cv.take<double>(6 * (size_t)T.n_ifc);
        D.gidx_dn = cv.take<int>(T.gidx.size());
        if (l == c.L) D.gamma = cv.take<unsigned char>(T.n_ifc);
    }
    c.partial_cap = max_blocks;
    c.partial[0] = cv.take<double>(max_blocks);
    c.partial[1] = cv.take<double>(max_blocks);
    c.counter = cv.take<unsigned int>(64);
    c.dnorm = cv.take<double>(8);
    c.tetinfo = cv.take<int>(6 * (size_t)c.n_tets);
    c.cn = tp.coarse.n;
    c.cslot = cv.take<long long>(c.cn);
    c.ccol = cv.take<int>(7 * (size_t)c.cn);
    c.cval = cv.take<double>(7 * (size_t)c.cn);
    c.cptr = cv.take<int>(c.cn + 1);
    c.cidx = cv.take<int>(tp.coarse.cidx.size());
    c.cpos = cv.take<int>(3 * (size_t)c.cn);
    c.cfrozen = cv.take<unsigned char>(c.cn);
    c.cval_dn = cv.take<double>(7 * (size_t)c.cn);
    c.dn_faulty = cv.take<unsigned char>(c.n_tets);
    c.citers = cv.take<int>(4);
    if (!c.vk && c.cn <= (c.mesh ? kDenseCoarseMaxMesh : kDenseCoarseMax)) c.cinv = cv.take<double>((size_t)c.cn * c.cn);
    if (c.mesh && c.d.max_faults > 0) c.cinv_dd = cv.take<double>((size_t)c.cn * c.cn);
    if (c.mesh) {
        c.mesh_kel = cv.take<double>(96 * (size_t)c.n_tets);
        c.n_dir_rows = (int)tp.dir_rows.size();
        c.dir_rows = cv.take<int>(tp.dir_rows.size());
        c.dir_ptr = cv.take<int>(tp.dir_ptr.size());
        c.dir_col = cv.take<int>(tp.dir_col.size());
        c.dir_val = cv.take<double>(tp.dir_val.size());
    }
    if (c.gen) {
        c.ccol15 = cv.take<int>(15 * (size_t)c.cn);
        c.cval15 = cv.take<double>(15 * (size_t)c.cn);
        c.cval15_dn = cv.take<double>(15 * (size_t)c.cn);
        c.kel = cv.take<double>(96 * (size_t)c.n_tets);
    }
    const TopoLevel &TL = tp.lev[c.L];
    c.aux_u = cv.take<double>(TL.n_slots);
    c.aux_b = cv.take<double>(TL.n_slots);
    if (c.vk) {
        c.user_u = cv.take<double>(c.n_dofs);
        c.user_l = cv.take<double>(c.n_dofs);
    }
}

// host topologies are immutable after construction and shared by every
// context of the same (n_sub, level, coarse_level); the cache keeps the most
// recent few
std::string get_topology(int n_sub, int L, int Lc, std::shared_ptr<const Topology> &out) {
    static std::mutex mu;
    static std::vector<std::pair<std::tuple<int, int, int>, std::shared_ptr<const Topology>>> cache;
    const auto key = std::make_tuple(n_sub, L, Lc);
    {
        std::lock_guard<std::mutex> g(mu);
        for (auto &e : cache)
            if (e.first == key) {
                out = e.second;
                return "";
            }
    }
    auto t = std::make_shared<Topology>();
    std::string err = t->build(n_sub, L, Lc);
    if (!err.empty()) return err;
    std::lock_guard<std::mutex> g(mu);
    cache.push_back({key, t});
    if (cache.size() > 6) cache.erase(cache.begin());
    out = t;
    return "";
}

// unstructured macro meshes: the same cache, keyed by a hash of the mesh
std::string get_mesh_topology(int nv, const double *xyz, int nt, const int *tets, int L, int Lc,
                              std::shared_ptr<const Topology> &out) {
    if (!xyz || !tets || nv < 1 || nt < 1) return "null or empty mesh";
    uint64_t h = 1469598103934665603ULL;
    auto mix = [&](const void *p, size_t n) {
        const unsigned char *b = (const unsigned char *)p;
        for (size_t q = 0; q < n; q++) h = (h ^ b[q]) * 1099511628211ULL;
    };
    mix(xyz, 3 * sizeof(double) * (size_t)nv);
    mix(tets, 4 * sizeof(int) * (size_t)nt);
    static std::mutex mu;
    static std::vector<std::pair<std::tuple<uint64_t, int, int, int, int>, std::shared_ptr<const Topology>>> cache;
    const auto key = std::make_tuple(h, nv, nt, L, Lc);
    {
        std::lock_guard<std::mutex> g(mu);
        for (auto &e : cache)
            if (e.first == key) {
                out = e.second;
                return "";
            }
    }
    auto t = std::make_shared<Topology>();
    std::string err = t->build_mesh(nv, xyz, nt, tets, L, Lc);
    if (!err.empty()) return err;
    if (t->coarse.n > kDenseCoarseMaxMesh) return "the coarsest level has more unknowns than the dense solver takes";
    t->mesh_hash = h;
    std::lock_guard<std::mutex> g(mu);
    cache.push_back({key, t});
    if (cache.size() > 4) cache.erase(cache.begin());
    out = t;
    return "";
}

std::string check_desc(const hhgr_desc *d) {
    if (!d) return "null descriptor";
    if (d->n_sub < 1 || d->n_sub > 8) return "n_sub must be in 1..8";
    if (d->coarse_level < 2) return "coarse_level must be >= 2";
    if (d->level <= d->coarse_level || d->level > 9) return "need coarse_level < level <= 9";
    if (d->nu_pre < 0 || d->nu_post < 0 || d->nu_pre + d->nu_post < 1) return "need nu_pre, nu_post >= 0, sum >= 1";
    if (!(d->omega > 0.0 && d->omega < 2.0)) return "omega must be in (0, 2)";
    if (d->precision != HHGR_FP64 && d->precision != HHGR_MIXED) return "bad precision";
    if (d->variable_coeff != 0 && d->variable_coeff != 1) return "variable_coeff must be 0 or 1";
    if (d->max_faults < 0 || d->max_faults > 8) return "max_faults must be in 0..8";
    if (d->general_geometry != 0 && d->general_geometry != 1) return "general_geometry must be 0 or 1";
    return "";
}

// ----------------------------------------------------------------------------
// launch geometry
// ----------------------------------------------------------------------------
// full = true: every node of the closures; otherwise the interior nodes, or
// only one colour of them with colour = 0 (red) / 1 (black)
VolGeom vgeom(const LevelDev &D, const VolDesc *vd, int nvol, bool full, int bsq = -1, int colour = -1) {
    const int q = bsq < 0 ? D.bs_sel : bsq;
    VolGeom g;
    g.vd = vd;
    g.nvol = nvol;
    g.M = D.M;
    g.bs = kBS[q];
    g.rowC = D.rowC;
    g.rowN = D.rowN;
    g.nrows = D.nrows;
    g.remap = D.remap;
    g.cpb = D.cpb;
    if (full) {
        g.list = D.flist;
        g.nlist = D.nflist;
    } else {
        g.list = colour == 0 ? D.rlist : colour == 1 ? D.blist : D.ilist;
        g.nlist = colour == 0 ? D.nrlist : colour == 1 ? D.nblist : D.nilist;
    }
    return g;
}

IfcGeom igeom(const LevelDev &D, int i0, int i1, const unsigned char *frozen, bool scatter) {
    IfcGeom g;
    g.i0 = i0;
    g.i1 = i1;
    g.base = D.ifc_base;
    g.stride = D.n_ifc;
    g.nbr = D.nbr;
    g.gptr = scatter ? D.gptr : nullptr;
    g.gidx = scatter ? D.gidx : nullptr;
    g.frozen = frozen;
    g.w = D.nbw;
    return g;
}

IfcGeom ig_none() { return IfcGeom(); }

// interface part of a launch on a view's level (its frozen nodes and ghost lists)
template <typename T>
IfcGeom igeom_v(const LevelDev &D, const LevView<T> &v, int i0, int i1, bool scatter) {
    IfcGeom g = igeom(D, i0, i1, v.frozen, scatter);
    if (scatter && v.gptr) {
        g.gptr = v.gptr;
        g.gidx = v.gidx;
    }
    return g;
}

// 15-point data of a level; q >= 0 selects the interface masters of class q
// (none unless ifc)
Gen15 gen15(const LevelDev &D, int q, bool ifc) {
    Gen15 g;
    g.rowN15 = D.rowN15;
    g.w15 = D.w15;
    g.sid = D.sid;
    g.wtab = D.wtab;
    g.nb15 = D.nb15;
    g.ifcq = q >= 0 ? D.ifcq[q] : nullptr;
    g.nq = q >= 0 && ifc ? D.nifcq[q] : 0;
    g.wv = D.wv;
    g.ws = D.n_slots;
    g.wi15 = D.wi15;
    g.w15f = D.w15f;
    g.wtabf = D.wtabf;
    g.wvf = D.wvf;
    g.wi15f = D.wi15f;
    return g;
}

// the finest level's mass matrix of a general macro mesh
Gen15 gen15mass(const LevelDev &D) {
    Gen15 g;
    g.rowN15 = D.rowN15;
    g.w15 = D.mw15;
    g.sid = D.sid;
    g.wtab = D.mwtab;
    g.nb15 = D.nb15;
    g.wi15 = D.mwi;  // unstructured meshes: per-master rows
    return g;
}

// ... of a view's level (a view may bring its own master entries)
template <typename T>
Gen15 gen15v(const LevelDev &D, const LevView<T> &v, int q) {
    Gen15 g = gen15(D, q, v.ifc);
    if (v.wi15) g.wi15 = v.wi15;
    return g;
}

template <typename T>
Weights<T> weights(const LevelDev &D);
template <>
Weights<double> weights<double>(const LevelDev &D) {
    Weights<double> w;
    w.w0 = D.w[0];
    w.w1 = D.w[1];
    w.w2 = D.w[2];
    w.wi = D.wi;
    return w;
}
template <>
Weights<float> weights<float>(const LevelDev &D) {
    Weights<float> w;
    w.w0 = D.w32[0];
    w.w1 = D.w32[1];
    w.w2 = D.w32[2];
    w.wi = D.wi32;
    return w;
}

template <typename T>
T *lvec(LevelDev &D, int which);
template <>
double *lvec<double>(LevelDev &D, int which) {
    return which == 0 ? D.u : which == 1 ? D.b : which == 2 ? D.r : D.ualt;
}
template <>
float *lvec<float>(LevelDev &D, int which) {
    return which == 0 ? D.u32 : which == 1 ? D.b32 : which == 2 ? D.r32 : D.u32alt;
}

// global (all tetrahedra) or masked (intact tetrahedra, frozen interface) view
template <typename T>
HView<T> global_view(hhgr_ctx &c, bool masked, int stream_idx) {
    HView<T> V;
    V.L = c.L;
    V.Lc = c.Lc;
    V.local = false;
    V.cfrozen = masked ? c.cfrozen : nullptr;
    V.partial = c.partial[stream_idx];
    V.counter = c.counter + 16 * stream_idx;
    V.timed = !masked;
    for (int l = c.Lc; l <= c.L; l++) {
        LevelDev &D = c.lev[l];
        LevView<T> &v = V.lv[l];
        v.u = lvec<T>(D, 0);
        v.b = lvec<T>(D, 1);
        v.r = lvec<T>(D, 2);
        v.ualt = masked ? nullptr : lvec<T>(D, 3);
        v.w = weights<T>(D);
        v.vd = masked ? D.vd_masked : D.vd_all;
        v.nvol = masked ? D.n_masked : c.n_tets;
        v.ifc = true;
        v.frozen = masked ? D.frozen : nullptr;
    }
    return V;
}

// local hierarchy of the faulty tetrahedra currently in vd_loc (FP64)
HView<double> local_view(hhgr_ctx &c, int stream_idx, double *finest_r = nullptr) {
    HView<double> V;
    V.L = c.L;
    V.Lc = c.Lc;
    V.local = true;
    V.partial = c.partial[stream_idx];
    V.counter = c.counter + 16 * stream_idx;
    for (int l = c.Lc; l <= c.L; l++) {
        LevelDev &D = c.lev[l];
        LevView<double> &v = V.lv[l];
        if (l == c.L) {
            v.u = D.u;
            v.b = D.b;
            v.r = finest_r ? finest_r : D.r;
        } else {
            v.u = D.lu;
            v.b = D.lb;
            v.r = D.lr;
        }
        v.w = weights<double>(D);
        v.vd = D.vd_loc;
        v.nvol = D.n_loc;
        v.ifc = false;
    }
    return V;
}

// ----------------------------------------------------------------------------
// V-cycle
// ----------------------------------------------------------------------------
void timed_begin(hhgr_ctx &c, hipStream_t s) {
    if (c.tev_used + 2 > c.tev.size()) {
        for (int q = 0; q < 64; q++) {
            hipEvent_t e;
            if (hipEventCreate(&e) == hipSuccess) c.tev.push_back(e);
        }
    }
    if (c.tev_used + 2 <= c.tev.size()) hipEventRecord(c.tev[c.tev_used], s);
}
void timed_end(hhgr_ctx &c, hipStream_t s) {
    if (c.tev_used + 2 <= c.tev.size()) {
        hipEventRecord(c.tev[c.tev_used + 1], s);
        c.tev_used += 2;
    }
}

// vector length of a view's level (a local hierarchy below the finest
// level holds max_faults closures)
template <typename T>
long long view_len(const hhgr_ctx &c, const HView<T> &V, int l) {
    const LevelDev &D = c.lev[l];
    return V.local && l < c.L ? (long long)std::max(c.d.max_faults, 1) * D.C_pad : D.n_slots;
}

// per-workgroup sums of the squared residual that the last black pass (or
// class-3 pass) of an FP64 cycle leaves (see launch_colour_norm)
struct NormOut {
    double *partial = nullptr;
    int blocks = 0;
};

template <typename T>
bool fused_ok(const hhgr_ctx &c, const HView<T> &V, int l, bool any = false);

// general macro meshes: one 4-colour sweep, classes 0, 1, 2, 3 (a start
// from zero clears the level's vector first).  The class-3 pass also sums
// the squared residual of its nodes (nout) or writes it to rout.
template <typename T>
void sweep15(hhgr_ctx &c, const HView<T> &V, int l, bool zero, hipStream_t s, NormOut *nout = nullptr,
             T *rout = nullptr) {
    const LevelDev &D = c.lev[l];
    const LevView<T> &v = V.lv[l];
    if (zero) launch_fill<T>(s, v.u, view_len(c, V, l), T(0));
    for (int q = 0; q < 4; q++) {
        VolGeom vg = vgeom(D, v.vd, v.nvol, false);
        vg.list = D.qlist[q];
        vg.nlist = D.nqlist[q];
        const IfcGeom ig = v.ifc ? igeom_v(D, v, 0, D.n_ifc, true) : ig_none();
        if constexpr (std::is_same<T, double>::value) {
            if (nout && q == 3) {
                nout->blocks = launch_colour15_norm(s, vg, ig, gen15v(D, v, q), v.u, v.b, c.d.omega, nout->partial);
                continue;
            }
        }
        if (rout && q == 3) {
            launch_colour15_res<T>(s, vg, ig, gen15v(D, v, q), v.u, v.b, c.d.omega, rout);
            continue;
        }
        const bool timed = c.timing && V.timed && l == c.L;
        if (timed) timed_begin(c, s);
        launch_colour15<T>(s, vg, ig, gen15v(D, v, q), v.u, v.b, c.d.omega);
        if (timed) timed_end(c, s);
    }
}

// general macro meshes: the classes 0..2 (whose lists are stored back to
// back) as one node list and one master list, for residuals after a sweep
template <typename T>
void classes012(const LevelDev &D, const LevView<T> &v, VolGeom &vg, Gen15 &g) {
    vg.list = D.qlist[0];
    vg.nlist = D.nqlist[0] + D.nqlist[1] + D.nqlist[2];
    g.ifcq = v.ifc ? D.ifcq[0] : nullptr;
    g.nq = v.ifc ? D.nifcq[0] + D.nifcq[1] + D.nifcq[2] : 0;
}

// one red-black sweep in place: two colour passes.  pr: the red pass first
// adds the coarse-grid correction to its nodes (the black nodes hold theirs).
// nout: the black pass also sums the squared residual of its nodes; rout:
// the black pass also writes the residual of its nodes there.
template <typename T>
void sweep(hhgr_ctx &c, const HView<T> &V, int l, bool zero, hipStream_t s, const Prol<T> *pr = nullptr,
           NormOut *nout = nullptr, T *rout = nullptr) {
    if (c.gen) {
        sweep15<T>(c, V, l, zero, s, nout, rout);
        return;
    }
    const LevelDev &D = c.lev[l];
    const LevView<T> &v = V.lv[l];
    for (int colour = 0; colour < 2; colour++) {
        const VolGeom vg = vgeom(D, v.vd, v.nvol, false, -1, colour);
        const IfcGeom ig = v.ifc ? igeom_v(D, v, colour == 0 ? 0 : D.n_ifc_red, colour == 0 ? D.n_ifc_red : D.n_ifc,
                                           true)
                                 : ig_none();
        if (pr && colour == 0) {
            VolGeom vgf = vg;
            vgf.cpb = D.cpb_fus;
            launch_colour_prol<T>(s, vgf, ig, v.u, v.b, v.w, c.vk, D.h, c.d.omega, *pr);
            continue;
        }
        if constexpr (std::is_same<T, double>::value) {
            if (nout && colour == 1) {
                nout->blocks = launch_colour_norm(s, vg, ig, v.u, v.b, v.w, c.vk, D.h, c.d.omega, nout->partial);
                continue;
            }
        }
        if (rout && colour == 1 && !zero) {
            launch_colour_res<T>(s, vg, ig, v.u, v.b, v.w, c.vk, D.h, c.d.omega, rout);
            continue;
        }
        const bool timed = c.timing && V.timed && l == c.L && !fused_ok(c, V, l);
        if (timed) timed_begin(c, s);
        launch_colour<T>(s, vg, ig, v.u, v.b, v.w, c.vk, D.h, c.d.omega, zero, zero && colour == 0);
        if (timed) timed_end(c, s);
    }
}

// the fused kernels apply: the cube with k = 1, every tetrahedron and
// every master of the level (no frozen nodes, no intact-side stencils), a
// second buffer for the level; and the level uses them (any = true: whether
// or not the autotuner chose them)
template <typename T>
bool fused_ok(const hhgr_ctx &c, const HView<T> &V, int l, bool any) {
    const LevelDev &D = c.lev[l];
    const LevView<T> &v = V.lv[l];
    return !c.gen && !c.vk && !V.local && v.ualt && v.ifc && !v.frozen && !v.w.wi && !v.gptr && D.fz_ps &&
           v.vd == D.vd_all && v.nvol == c.n_tets && (any || D.fz_on);
}

template <typename T>
FusedGeom fgeom(const LevelDev &D, const LevView<T> &v) {
    FusedGeom g;
    g.vd = v.vd;
    g.nvol = v.nvol;
    g.tiles = D.fz_tiles;
    g.ntiles = (int)D.fz_tiles_host.size();
    g.m = D.m;
    g.TJ = D.fz_TJ;
    g.TK = D.fz_TK;
    g.black0 = D.fz_black0;
    g.ps = D.fz_ps;
    g.remap = D.remap;
    return g;
}

// one red-black sweep from us into ud: red masters, the volume interiors
// (fused kernel), black masters.  zero: from u = 0; rout: black residual tail.
template <typename T>
void fused_sweep(hhgr_ctx &c, const HView<T> &V, int l, const T *us, T *ud, bool zero, hipStream_t s, T *rout) {
    const LevelDev &D = c.lev[l];
    const LevView<T> &v = V.lv[l];
    const IfcGeom red = igeom(D, 0, D.n_ifc_red, nullptr, true), black = igeom(D, D.n_ifc_red, D.n_ifc, nullptr, true);
    launch_ifc_sor<T>(s, red, us, us, ud, v.b, D.h, c.d.omega, zero, zero, (T *)nullptr);
    const bool timed = c.timing && V.timed && l == c.L && !zero && !rout;
    if (timed) timed_begin(c, s);
    launch_sweep_fused_vol<T>(s, fgeom(D, v), us, ud, v.b, D.h, c.d.omega, zero, rout);
    if (timed) timed_end(c, s);
    launch_ifc_sor<T>(s, black, us, ud, ud, v.b, D.h, c.d.omega, zero, false, rout);
}

// nsweeps red-black sweeps in place.  Two sweeps in a row run fused where
// fused_ok holds, the first into the level's second buffer and the second
// back (the first sweep may start from zero, the second may write the
// residual tail); a sweep that adds the coarse-grid correction (pr) or sums
// the squared residual (nout) runs as two colour passes.
template <typename T>
void smooth(hhgr_ctx &c, const HView<T> &V, int l, int nsweeps, bool zero, hipStream_t s,
            const Prol<T> *pr = nullptr, NormOut *nout = nullptr, T *rout = nullptr, bool force_fused = false) {
    const LevView<T> &v = V.lv[l];
    for (int k = 0; k < nsweeps; k++) {
        const bool last = k == nsweeps - 1;
        if (k + 1 < nsweeps && fused_ok(c, V, l, force_fused) && !(k == 0 && pr) && !(k + 1 == nsweeps - 1 && nout)) {
            fused_sweep<T>(c, V, l, v.u, v.ualt, zero && k == 0, s, (T *)nullptr);
            fused_sweep<T>(c, V, l, v.ualt, v.u, false, s, k + 1 == nsweeps - 1 ? rout : nullptr);
            k++;
            continue;
        }
        sweep(c, V, l, zero && k == 0, s, k == 0 ? pr : nullptr, last ? nout : nullptr, last ? rout : nullptr);
    }
}

template <typename T>
void coarse_solve(hhgr_ctx &c, const HView<T> &V, hipStream_t s) {
    const LevelDev &D = c.lev[c.Lc];
    const LevView<T> &v = V.lv[c.Lc];
    if (c.gen) {
        if constexpr (std::is_same<T, double>::value) {
            if (V.local) {
                launch_local_coarse15(s, v.vd, v.nvol, D.lc_sl.x, gen15(D, -1, false), v.b, v.u);
                return;
            }
        }
        if (c.dense_coarse && !V.cfrozen && !V.cval) {
            launch_coarse_dense<T>(s, c.cn, c.cslot, c.cinv, v.b, v.u, c.cptr, c.cidx);
            return;
        }
        if (c.mesh && V.cfrozen && !V.cval) {
            // frozen unknowns: zero rows of the masked inverse (coarse levels
            // hold corrections, zero at the frozen nodes)
            launch_coarse_dense<T>(s, c.cn, c.cslot, c.cinv_dd, v.b, v.u, c.cptr, c.cidx);
            return;
        }
        launch_coarse_pcg15<T>(s, c.cn, c.cslot, c.ccol15, V.cval ? V.cval : c.cval15, V.cfrozen, v.b, v.u, c.cptr,
                               c.cidx, kCoarseRtol, kCoarseMaxit, c.citers);
        return;
    }
    if (V.local) {
        launch_local_coarse<T>(s, v.vd, v.nvol, D.lc_sl, v.b, v.u, v.w, c.vk, D.h);
    } else if (c.dense_coarse && !V.cfrozen && !V.cval) {
        launch_coarse_dense<T>(s, c.cn, c.cslot, c.cinv, v.b, v.u, c.cptr, c.cidx);
    } else {
        launch_coarse_pcg<T>(s, c.cn, c.cslot, c.ccol, V.cval ? V.cval : c.cval, V.cfrozen, v.b, v.u, c.cptr, c.cidx,
                             kCoarseRtol, kCoarseMaxit, c.citers);
    }
}

// nout (top level, at least one post-smoothing sweep): the last black pass
// leaves the squared residual of the black nodes (launch_colour_norm)
template <typename T>
void vcycle(hhgr_ctx &c, const HView<T> &V, int l, bool zero, hipStream_t s, NormOut *nout = nullptr) {
    if (l == V.Lc) {
        coarse_solve(c, V, s);
        return;
    }
    LevelDev &D = c.lev[l];
    LevelDev &Dc = c.lev[l - 1];
    const LevView<T> &v = V.lv[l];
    const LevView<T> &vc = V.lv[l - 1];
    // On the cube the last pre-smoothing pass (black, not the first pass from
    // zero) writes the residual of the black nodes, and the residual launch
    // covers the red nodes only
    // (a general mesh's class-3 pass has no zero-start variant)
    const bool split_res = c.gen ? c.d.nu_pre >= 1 : (c.d.nu_pre >= 2 || (c.d.nu_pre == 1 && !zero));
    smooth(c, V, l, c.d.nu_pre, zero, s, (const Prol<T> *)nullptr, (NormOut *)nullptr, split_res ? v.r : nullptr);
    if (c.d.nu_pre == 0 && zero) launch_fill<T>(s, v.u, view_len(c, V, l), T(0));
    VolGeom vg = vgeom(D, v.vd, v.nvol, false, -1, split_res && !c.gen ? 0 : -1);
    const IfcGeom ig =
        v.ifc ? igeom(D, 0, split_res && !c.gen ? D.n_ifc_red : D.n_ifc, v.frozen, false) : ig_none();
    vg.cpb = D.cpb_res;
    const VolGeom vgc = vgeom(Dc, vc.vd, vc.nvol, false);
    const IfcGeom igc = vc.ifc ? igeom(Dc, 0, Dc.n_ifc, vc.frozen, false) : ig_none();
    if (c.gen) {
        Gen15 g = gen15v(D, v, -1);
        if (split_res) classes012(D, v, vg, g);
        launch_residual15<T, T>(s, vg, ig, g, v.u, v.b, v.r, nullptr);
    } else
        launch_residual<T, T>(s, vg, ig, v.u, v.b, v.w, c.vk, D.h, v.r, nullptr);
    launch_restrict<T>(s, vgc, v.vd, D.rowC, igc, Dc.rst, v.r, vc.b);
    vcycle(c, V, l - 1, true, s);
    // u += P e_c.  With a red-black post-smoother only the black nodes are
    // corrected here; the first red pass corrects its own nodes as it reads
    // them (it reads nothing else of its colour), so no red value is written
    // twice.
    const bool fuse = !c.gen && c.d.nu_post > 0;
    const IfcGeom igp = v.ifc ? igeom_v(D, v, fuse ? D.n_ifc_red : 0, D.n_ifc, true) : ig_none();
    VolGeom vgp = vgeom(D, v.vd, v.nvol, false, -1, fuse ? 1 : -1);
    vgp.cpb = D.cpb_prl;
    launch_prolong<T>(s, vgp, vc.vd, Dc.rowC, Dc.M, igp, D.prl, vc.u, v.u);
    if (fuse) {
        Prol<T> pr;
        pr.vdc = vc.vd;
        pr.cC = Dc.rowC;
        pr.Mc = Dc.M;
        pr.prl = D.prl;
        pr.ec = vc.u;
        smooth(c, V, l, c.d.nu_post, false, s, &pr, nout);
    } else {
        smooth(c, V, l, c.d.nu_post, false, s, (const Prol<T> *)nullptr, nout);
    }
}

// ||b - A u||^2 (or with TO output: r = b - A u written as TO) on level L of a view
template <typename TO>
void finest_residual(hhgr_ctx &c, const HView<double> &V, TO *rout, hipStream_t s, double *dst) {
    const LevelDev &D = c.lev[c.L];
    const LevView<double> &v = V.lv[c.L];
    VolGeom vg = vgeom(D, v.vd, v.nvol, false);
    vg.cpb = D.cpb_res;
    const IfcGeom ig = v.ifc ? igeom(D, 0, D.n_ifc, v.frozen, false) : ig_none();
    const int nb = c.gen ? launch_residual15<double, TO>(s, vg, ig, gen15v(D, v, -1), v.u, v.b, rout, V.partial)
                         : launch_residual<double, TO>(s, vg, ig, v.u, v.b, v.w, c.vk, D.h, rout, V.partial);
    if (nb > 0)
        launch_reduce(s, V.partial, nb, dst);
    else
        launch_fill<double>(s, dst, 1, 0.0);
}

// one FP64 cycle + residual norm into dnorm[slot]
// one FP64 cycle on view V and ||b - A u||^2 on its finest level into *dst.
// On the cube the cycle ends with a black pass, which leaves the squared
// residual of the black nodes: ((1 - omega) r)^2 with r its residual before
// the update.  The red nodes' residual then comes from a red-only residual
// launch, so the norm costs one pass over the red nodes instead of one over
// all (frozen masters are left out on both sides, as in the full residual).
// On a general mesh the class-3 pass and classes 0..2 play those parts.
void cycle_and_norm(hhgr_ctx &c, const HView<double> &V, hipStream_t s, double *dst) {
    if (!c.gen && c.d.nu_post > 0) {
        const LevelDev &D = c.lev[c.L];
        const LevView<double> &v = V.lv[c.L];
        const VolGeom vb = vgeom(D, v.vd, v.nvol, false, -1, 1);
        const IfcGeom igb = v.ifc ? igeom_v(D, v, D.n_ifc_red, D.n_ifc, true) : ig_none();
        VolGeom vr = vgeom(D, v.vd, v.nvol, false, -1, 0);
        vr.cpb = D.cpb_res;
        const IfcGeom igr = v.ifc ? igeom(D, 0, D.n_ifc_red, v.frozen, false) : ig_none();
        if ((long long)colour_blocks(vb, igb) + colour_blocks(vr, igr) <= c.partial_cap) {
            NormOut no;
            no.partial = V.partial;
            vcycle<double>(c, V, c.L, false, s, &no);
            const int nr = launch_residual<double, double>(s, vr, igr, v.u, v.b, v.w, c.vk, D.h, (double *)nullptr,
                                                           V.partial + no.blocks);
            if (no.blocks + nr > 0)
                launch_reduce(s, V.partial, no.blocks + nr, dst);
            else
                launch_fill<double>(s, dst, 1, 0.0);
            return;
        }
    }
    if (c.gen && c.d.nu_post > 0) {
        // general mesh: the last class-3 pass and a residual over classes 0..2
        const LevelDev &D = c.lev[c.L];
        const LevView<double> &v = V.lv[c.L];
        VolGeom v3 = vgeom(D, v.vd, v.nvol, false);
        v3.list = D.qlist[3];
        v3.nlist = D.nqlist[3];
        const Gen15 g3 = gen15v(D, v, 3);
        VolGeom vr = vgeom(D, v.vd, v.nvol, false);
        Gen15 gr = gen15v(D, v, -1);
        classes012(D, v, vr, gr);
        const IfcGeom igr = v.ifc ? igeom(D, 0, D.n_ifc, v.frozen, false) : ig_none();
        if ((long long)colour15_blocks(v3, g3) + colour15_blocks(vr, gr) <= c.partial_cap) {
            NormOut no;
            no.partial = V.partial;
            vcycle<double>(c, V, c.L, false, s, &no);
            const int nr =
                launch_residual15<double, double>(s, vr, igr, gr, v.u, v.b, (double *)nullptr, V.partial + no.blocks);
            if (no.blocks + nr > 0)
                launch_reduce(s, V.partial, no.blocks + nr, dst);
            else
                launch_fill<double>(s, dst, 1, 0.0);
            return;
        }
    }
    vcycle<double>(c, V, c.L, false, s);
    finest_residual<double>(c, V, (double *)nullptr, s, dst);
}

void step_fp64(hhgr_ctx &c, const HView<double> &V, hipStream_t s, int slot) {
    cycle_and_norm(c, V, s, c.dnorm + slot);
}

// mixed step: e32 = V32(b32) from zero, u += e32, then b32 = round32(b - A u) and its norm
void step_mixed(hhgr_ctx &c, const HView<double> &V64, const HView<float> &V32, hipStream_t s, int slot) {
    vcycle<float>(c, V32, c.L, true, s);
    LevelDev &D = c.lev[c.L];
    launch_update_add(s, V64.lv[c.L].vd, V64.lv[c.L].nvol, D.C_pad, igeom(D, 0, D.n_ifc, nullptr, false), D.u, D.u32);
    finest_residual<float>(c, V64, D.b32, s, c.dnorm + slot);
}

int read_norm(hhgr_ctx &c, int slot, double *out) {
    HIPCHK(hipMemcpyAsync(c.hnorm + slot, c.dnorm + slot, sizeof(double), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    *out = std::sqrt(std::max(c.hnorm[slot], 0.0));
    return HHGR_OK;
}

void invalidate_graph(hhgr_ctx &c) {
    if (c.gexec) hipGraphExecDestroy(c.gexec);
    c.gexec = nullptr;
    c.graph_ok = false;
    if (c.lgexec) hipGraphExecDestroy(c.lgexec);
    c.lgexec = nullptr;
    c.lg_tet = c.lg_n = -1;
}

// enqueue one global step (FP64 cycle or mixed refinement step) ending with
// the residual norm in dnorm[0] copied to hnorm[0]
void enqueue_step(hhgr_ctx &c, hipStream_t s) {
    HView<double> V64 = global_view<double>(c, false, 0);
    if (c.mixed) {
        HView<float> V32 = global_view<float>(c, false, 0);
        step_mixed(c, V64, V32, s, 0);
    } else {
        step_fp64(c, V64, s, 0);
    }
    hipMemcpyAsync(c.hnorm, c.dnorm, sizeof(double), hipMemcpyDeviceToHost, s);
}

int run_step(hhgr_ctx &c) {
    if (c.use_graph && !c.timing) {
        if (!c.graph_ok) {
            hipGraph_t g = nullptr;
            HIPCHK(hipStreamBeginCapture(c.cap, hipStreamCaptureModeRelaxed));
            enqueue_step(c, c.cap);
            HIPCHK(hipStreamEndCapture(c.cap, &g));
            hipError_t e = hipGraphInstantiate(&c.gexec, g, nullptr, nullptr, 0);
            hipGraphDestroy(g);
            if (e != hipSuccess) return fail(HHGR_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
            c.graph_ok = true;
        }
        HIPCHK(hipGraphLaunch(c.gexec, c.stream));
    } else {
        enqueue_step(c, c.stream);
        CHKLAUNCH();
    }
    return HHGR_OK;
}

// in mixed mode the residual (and b32) of the current u must be ready before a step
void prime_mixed(hhgr_ctx &c, hipStream_t s) {
    HView<double> V64 = global_view<double>(c, false, 0);
    finest_residual<float>(c, V64, c.lev[c.L].b32, s, c.dnorm);
}

void set_loc(hhgr_ctx &c, const std::vector<int> &tets) {
    if (tets == c.loc_tets) return;  // vd_loc already holds them
    std::vector<std::vector<VolDesc>> h(c.L + 1);
    for (int l = c.Lc; l <= c.L; l++) {
        LevelDev &D = c.lev[l];
        h[l].resize(tets.size());
        for (size_t f = 0; f < tets.size(); f++) {
            h[l][f].vec = (l == c.L ? (long long)tets[f] : (long long)f) * D.C_pad;
            h[l][f].w = (long long)tets[f] * D.C_pad;
            h[l][f].tet = tets[f];
            h[l][f].pad = 0;
        }
        hipMemcpyAsync(D.vd_loc, h[l].data(), h[l].size() * sizeof(VolDesc), hipMemcpyHostToDevice, c.stream);
        D.n_loc = (int)tets.size();
    }
    hipStreamSynchronize(c.stream);  // the copies read h
    c.loc_tets = tets;
}

// restore ghost copies of tet t on the finest level from the interface masters,
// after zeroing its closure (interior re-initialised with zero)
void restore_tet(hhgr_ctx &c, int t, hipStream_t s) {
    LevelDev &D = c.lev[c.L];
    launch_fill<double>(s, D.u + (long long)t * D.C_pad, D.C_pad, 0.0);
    const int a = D.tg_ptr[t], b = D.tg_ptr[t + 1];
    launch_ghost_refresh<double>(s, D.tg_dst + a, D.tg_src + a, b - a, D.u);
}

int upload(hhgr_ctx &c, void *dst, const void *src, size_t bytes) {
    if (bytes == 0) return HHGR_OK;
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c.stream));
    return HHGR_OK;
}

// ----------------------------------------------------------------------------
// Dirichlet-Dirichlet recovery (Sec. 4.2, Alg. 1 b)): the intact part cycles
// with the closures of the faulty tetrahedra frozen as Dirichlet data while
// the faulty tetrahedra run local cycles; the two share no unknowns
// ----------------------------------------------------------------------------
int dd_check(const hhgr_ctx &c, const int *tets, int n_tets, int n_intact, int n_local, std::vector<int> &ft) {
    if (!tets || n_tets < 1 || n_tets > c.d.max_faults) return fail(HHGR_EINVAL, "need 1..max_faults tets");
    if (n_intact < 0 || n_local < 0) return fail(HHGR_EINVAL, "negative cycle count");
    if (c.Lc != 2) return fail(HHGR_ESTATE, "local recovery needs coarse_level = 2 (one unknown per tetrahedron)");
    ft.assign(tets, tets + n_tets);
    std::vector<char> isf(c.n_tets, 0);
    for (int t : ft) {
        if (t < 0 || t >= c.n_tets) return fail(HHGR_EINVAL, "tet id out of range");
        if (isf[t]) return fail(HHGR_EINVAL, "duplicate tet id");
        isf[t] = 1;
    }
    return HHGR_OK;
}

// masks of the intact volumes and of the frozen interface nodes on every
// level, the local hierarchy of the faulty tetrahedra, their ghost copies
// restored and interiors zeroed, coarse corrections zeroed; synchronises
int dd_setup(hhgr_ctx &c, const std::vector<int> &ft) {
    std::vector<char> isf(c.n_tets, 0);
    for (int t : ft) isf[t] = 1;
    std::vector<std::vector<VolDesc>> vds(c.L + 1);
    std::vector<std::vector<unsigned char>> frz(c.L + 1);
    int rc = HHGR_OK;
    for (int l = c.Lc; l <= c.L; l++) {
        LevelDev &D = c.lev[l];
        const TopoLevel &T = c.topo->lev[l];
        for (int t = 0; t < c.n_tets; t++)
            if (!isf[t]) vds[l].push_back(VolDesc{(long long)t * D.C_pad, (long long)t * D.C_pad, t, 0});
        frz[l].assign(D.n_ifc, 0);
        for (int t : ft)
            for (int q = T.tg_ptr[t]; q < T.tg_ptr[t + 1]; q++) {
                long long s = T.tg_src[q];
                if (s >= T.ifc_base && s < T.ifc_base + T.n_ifc) frz[l][s - T.ifc_base] = 1;
            }
        D.n_masked = (int)vds[l].size();
        rc = rc ? rc : upload(c, D.vd_masked, vds[l].data(), vds[l].size() * sizeof(VolDesc));
        rc = rc ? rc : upload(c, D.frozen, frz[l].data(), frz[l].size());
    }
    const CoarseSystem &cs = c.topo->coarse;
    std::vector<unsigned char> cf(cs.n, 0);
    for (int q = 0; q < cs.n; q++) cf[q] = cs.is_vol[q] ? (unsigned char)isf[cs.tet[q]] : frz[c.Lc][cs.ifc[q]];
    rc = rc ? rc : upload(c, c.cfrozen, cf.data(), cf.size());
    std::vector<double> inv_full;
    if (c.mesh) {
        // the coarsest operator on the unfrozen unknowns, inverted densely
        const std::vector<double> &valw = c.mesh_k.empty() ? cs.valw : c.mesh_k_valw;
        std::vector<int> keep(cs.n, -1);
        int nk = 0;
        for (int q = 0; q < cs.n; q++)
            if (!cf[q]) keep[q] = nk++;
        std::vector<int> colk((size_t)nk * cs.cw, -1);
        std::vector<double> valk((size_t)nk * cs.cw, 0.0);
        for (int q = 0; q < cs.n; q++) {
            if (keep[q] < 0) continue;
            for (int e = 0; e < cs.cw; e++) {
                const int cq = cs.colw[(size_t)cs.cw * q + e];
                if (cq < 0 || keep[cq] < 0) continue;
                colk[(size_t)cs.cw * keep[q] + e] = keep[cq];
                valk[(size_t)cs.cw * keep[q] + e] = valw[(size_t)cs.cw * q + e];
            }
        }
        std::vector<double> inv;
        if (nk > 0 && !coarse_inverse(nk, cs.cw, colk, valk, inv)) {
            HIPCHK(hipStreamSynchronize(c.stream));
            return fail(HHGR_EINVAL, "the masked coarsest-level operator is not positive definite");
        }
        inv_full.assign((size_t)cs.n * cs.n, 0.0);
        for (int q = 0; q < cs.n; q++)
            for (int r = 0; r < cs.n; r++)
                if (keep[q] >= 0 && keep[r] >= 0) inv_full[(size_t)q * cs.n + r] = inv[(size_t)keep[q] * nk + keep[r]];
        rc = rc ? rc : upload(c, c.cinv_dd, inv_full.data(), inv_full.size() * sizeof(double));
    }
    // copies already queued read the host vectors above: wait before any return
    HIPCHK(hipStreamSynchronize(c.stream));
    if (rc) return rc;
    set_loc(c, ft);
    for (int t : ft) restore_tet(c, t, c.stream);
    for (int l = c.Lc; l <= c.L; l++) {
        LevelDev &D = c.lev[l];
        if (l < c.L) launch_fill<double>(c.stream, D.u, D.n_slots, 0.0);
        if (c.mixed) launch_fill<float>(c.stream, D.u32, D.n_slots, 0.0f);
    }
    CHKLAUNCH();
    HIPCHK(hipStreamSynchronize(c.stream));
    return HHGR_OK;
}

// one intact-side step on the masked hierarchy (an FP64 cycle, or a mixed
// refinement step); with norm (or in mixed mode) the squared norm of the
// intact residual goes to dnorm[slot]
void dd_intact_step(hhgr_ctx &c, hipStream_t s, bool first, bool norm, int slot) {
    HView<double> V64 = global_view<double>(c, true, 0);
    if (c.mixed) {
        HView<float> V32 = global_view<float>(c, true, 0);
        if (first) finest_residual<float>(c, V64, c.lev[c.L].b32, s, c.dnorm + slot);
        step_mixed(c, V64, V32, s, slot);
    } else if (norm) {
        cycle_and_norm(c, V64, s, c.dnorm + slot);
    } else {
        vcycle<double>(c, V64, c.L, false, s);
    }
}

void dd_local(hhgr_ctx &c, int n_local, hipStream_t s) {
    HView<double> VL = local_view(c, 1);
    for (int q = 0; q < n_local; q++) vcycle<double>(c, VL, c.L, false, s);
}

// residual of the whole problem once a recovery is complete (and, in mixed
// mode, the FP32 right-hand side of the next refinement step) into dnorm[0]
void dd_final_norm(hhgr_ctx &c, hipStream_t s) {
    if (c.mixed) {
        prime_mixed(c, s);
    } else {
        HView<double> V = global_view<double>(c, false, 0);
        finest_residual<double>(c, V, (double *)nullptr, s, c.dnorm);
    }
}

// ----------------------------------------------------------------------------
// Dirichlet-Neumann recovery (Sec. 4.3, Alg. 2, eq. (5)): the intact side
// cycles on a Neumann problem (stiffness over the elements of intact macro
// tetrahedra only, interface nodes free, static Neumann data on the
// interface); the faulty side runs local Dirichlet cycles whose boundary
// values are refreshed from the interface at the start of every round
// ----------------------------------------------------------------------------
int dn_setup(hhgr_ctx &c, const std::vector<int> &ft) {
    std::vector<unsigned char> isf(c.n_tets, 0);
    for (int t : ft) isf[t] = 1;
    int rc = upload(c, c.dn_faulty, isf.data(), isf.size());
    std::vector<std::vector<VolDesc>> vds(c.L + 1);
    for (int l = c.Lc; l <= c.L; l++) {
        LevelDev &D = c.lev[l];
        for (int t = 0; t < c.n_tets; t++)
            if (!isf[t]) vds[l].push_back(VolDesc{(long long)t * D.C_pad, (long long)t * D.C_pad, t, 0});
        D.n_masked = (int)vds[l].size();
        rc = rc ? rc : upload(c, D.vd_masked, vds[l].data(), vds[l].size() * sizeof(VolDesc));
    }
    if (rc) {
        hipStreamSynchronize(c.stream);  // queued copies read vds
        return rc;
    }
    // an interface node lies in the closures of the tetrahedra holding its
    // ghost copies: frozen if all of them are faulty, on the interface Gamma
    // if some are; ghost copies in faulty closures are not written
    for (int l = c.Lc; l <= c.L; l++) {
        LevelDev &D = c.lev[l];
        launch_dn_masks(c.stream, D.n_ifc, D.ifc_base, D.C_pad, D.gptr, D.gidx, c.dn_faulty, D.frozen, D.gamma,
                        D.gidx_dn);
    }
    // frozen flags of the coarsest level's unknowns (a small host loop)
    const TopoLevel &Tc = c.topo->lev[c.Lc];
    std::vector<unsigned char> frc(Tc.n_ifc, 0);
    for (int f = 0; f < Tc.n_ifc; f++) {
        int ni = 0;
        for (int g = Tc.gptr[f]; g < Tc.gptr[f + 1]; g++) ni += !isf[(int)(Tc.gidx[g] / Tc.C_pad)];
        frc[f] = ni == 0;
    }
    const CoarseSystem &cs = c.topo->coarse;
    std::vector<unsigned char> cf(cs.n, 0);
    for (int q = 0; q < cs.n; q++) cf[q] = cs.is_vol[q] ? isf[cs.tet[q]] : frc[cs.ifc[q]];
    rc = upload(c, c.cfrozen, cf.data(), cf.size());
    if (rc) {
        hipStreamSynchronize(c.stream);  // queued copies read vds and cf
        return rc;
    }
    // intact-side operators on every level
    if (c.mesh) {
        // master rows over the elements of intact tetrahedra (host), and the
        // coarsest-level operator on the unfrozen unknowns, inverted densely
        std::vector<double> wt(c.n_tets);
        for (int t = 0; t < c.n_tets; t++) wt[t] = isf[t] ? 0.0 : c.mesh_k.empty() ? 1.0 : c.mesh_k[t];
        Topology::MeshOps I;
        const std::string e =
            c.topo->mesh_weighted_operators(wt.data(), isf.data(), c.mesh_k.empty() ? nullptr : &c.mesh_k_wi, I, false);
        if (!e.empty()) {
            HIPCHK(hipStreamSynchronize(c.stream));
            return fail(HHGR_EINVAL, e);
        }
        const std::vector<std::vector<double>> &wi = I.wi;
        const std::vector<double> &valw = I.valw;
        for (int l = c.Lc; l <= c.L && !rc; l++) rc = upload(c, c.lev[l].wi15_dn, wi[l].data(), wi[l].size() * sizeof(double));
        std::vector<int> keep(cs.n, -1);
        int nk = 0;
        for (int q = 0; q < cs.n; q++)
            if (!cf[q]) keep[q] = nk++;
        std::vector<int> colk((size_t)nk * cs.cw, -1);
        std::vector<double> valk((size_t)nk * cs.cw, 0.0);
        for (int q = 0; q < cs.n; q++) {
            if (keep[q] < 0) continue;
            for (int e2 = 0; e2 < cs.cw; e2++) {
                const int cq = cs.colw[(size_t)cs.cw * q + e2];
                if (cq < 0 || keep[cq] < 0) continue;
                colk[(size_t)cs.cw * keep[q] + e2] = keep[cq];
                valk[(size_t)cs.cw * keep[q] + e2] = valw[(size_t)cs.cw * q + e2];
            }
        }
        std::vector<double> inv, inv_full;
        if (nk > 0 && !coarse_inverse(nk, cs.cw, colk, valk, inv)) {
            HIPCHK(hipStreamSynchronize(c.stream));
            return fail(HHGR_EINVAL, "the intact side's coarsest-level operator is not positive definite");
        }
        inv_full.assign((size_t)cs.n * cs.n, 0.0);
        for (int q = 0; q < cs.n; q++)
            for (int r = 0; r < cs.n; r++)
                if (keep[q] >= 0 && keep[r] >= 0) inv_full[(size_t)q * cs.n + r] = inv[(size_t)keep[q] * nk + keep[r]];
        rc = rc ? rc : upload(c, c.cinv_dd, inv_full.data(), inv_full.size() * sizeof(double));
        // the copies read wi and inv_full
        HIPCHK(hipStreamSynchronize(c.stream));
        if (rc) return rc;
    } else if (c.gen) {
        GenK G;
        G.kel = c.kel;
        G.faulty = c.dn_faulty;
        G.n_sub = c.d.n_sub;
        for (int l = c.Lc; l <= c.L; l++) {
            LevelDev &D = c.lev[l];
            G.k = c.vk ? D.kc : nullptr;
            G.N = D.N;
            G.m = D.m;
            launch_gen_ifc_weights(c.stream, D.n_ifc, D.ifc_xyz, G, D.wi15_dn);
            if (l == c.Lc) launch_gen_coarse_vals(c.stream, c.cn, c.cpos, c.ccol15, G, c.cval15_dn);
        }
    } else {
        for (int l = c.Lc; l <= c.L; l++) {
            LevelDev &D = c.lev[l];
            launch_ifc_weights_intact(c.stream, D.n_ifc, D.ifc_xyz, D.N, D.m, c.d.n_sub, D.h, c.vk ? D.kc : nullptr,
                                      c.dn_faulty, D.wi_dn);
        }
        const LevelDev &Dc = c.lev[c.Lc];
        launch_coarse_vals_intact(c.stream, c.cn, c.cpos, c.ccol, Dc.N, Dc.m, c.d.n_sub, Dc.h, c.vk ? Dc.kc : nullptr,
                                  c.dn_faulty, c.cval_dn);
    }
    CHKLAUNCH();
    HIPCHK(hipStreamSynchronize(c.stream));
    set_loc(c, ft);
    LevelDev &F = c.lev[c.L];
    // static Neumann data from the data at the time of the fault (u_F plays
    // no part: its edges have zero intact-side weight)
    HIPCHK(hipMemcpyAsync(c.aux_b, F.b, F.n_slots * sizeof(double), hipMemcpyDeviceToDevice, c.stream));
    if (c.mesh)
        launch_neumann_rhs_w(c.stream, F.n_ifc, F.ifc_base, F.nb15, F.wi15_dn, F.nbw, F.gamma, F.u, c.aux_b);
    else if (c.gen)
        launch_neumann_rhs15(c.stream, F.n_ifc, F.ifc_base, F.nb15, F.wi15_dn, F.gamma, F.u, c.aux_b);
    else
        launch_neumann_rhs(c.stream, F.n_ifc, F.ifc_base, F.nbr, F.wi_dn, F.gamma, F.u, c.aux_b);
    for (int t : ft) restore_tet(c, t, c.stream);
    for (int l = c.Lc; l <= c.L; l++) {
        LevelDev &D = c.lev[l];
        if (l < c.L) launch_fill<double>(c.stream, D.u, D.n_slots, 0.0);
        // the intact side never writes residuals inside faulty closures; its
        // restriction reads them there as zero
        launch_fill<double>(c.stream, D.r, D.n_slots, 0.0);
    }
    CHKLAUNCH();
    HIPCHK(hipStreamSynchronize(c.stream));
    return HHGR_OK;
}

// the intact side's Neumann hierarchy (FP64)
HView<double> dn_view(hhgr_ctx &c) {
    HView<double> V = global_view<double>(c, true, 0);
    for (int l = c.Lc; l <= c.L; l++) {
        LevelDev &D = c.lev[l];
        LevView<double> &v = V.lv[l];
        v.w.wi = D.wi_dn;
        v.wi15 = D.wi15_dn;
        v.gptr = D.gptr;
        v.gidx = D.gidx_dn;
    }
    V.lv[c.L].b = c.aux_b;
    // a mesh's intact-side coarsest level is the dense inverse of dn_setup
    V.cval = c.mesh ? nullptr : c.gen ? c.cval15_dn : c.cval_dn;
    return V;
}

// ghost copies of the faulty tetrahedra from the interface masters (their
// interiors are kept)
void refresh_faulty_ghosts(hhgr_ctx &c, const std::vector<int> &ft, hipStream_t s) {
    LevelDev &D = c.lev[c.L];
    for (int t : ft) {
        const int a = D.tg_ptr[t], b = D.tg_ptr[t + 1];
        launch_ghost_refresh<double>(s, D.tg_dst + a, D.tg_src + a, b - a, D.u);
    }
}

// masks inactive again; later global cycles use the whole hierarchy
void dd_end(hhgr_ctx &c) {
    for (int l = c.Lc; l <= c.L; l++) c.lev[l].n_masked = 0;
}

// general macro mesh with a per-element coefficient: the per-node stencils
// of every level and the coarsest-level rows from the level's k and the
// element matrices; synchronises
int gen_weights(hhgr_ctx &c) {
    GenK G;
    G.kel = c.kel;
    G.n_sub = c.d.n_sub;
    for (int l = c.Lc; l <= c.L; l++) {
        LevelDev &D = c.lev[l];
        G.k = D.kc;
        G.N = D.N;
        G.m = D.m;
        launch_gen_weights(c.stream, vgeom(D, D.vd_all, c.n_tets, true), c.tetinfo, G, D.wv, D.n_slots);
        launch_gen_ifc_weights(c.stream, D.n_ifc, D.ifc_xyz, G, D.wi15);
        if (c.mixed) {
            launch_cast<double, float>(c.stream, D.wv, D.wvf, 8 * D.n_slots);
            launch_cast<double, float>(c.stream, D.wi15, D.wi15f, 15LL * D.n_ifc);
        }
        if (l == c.Lc) launch_gen_coarse_vals(c.stream, c.cn, c.cpos, c.ccol15, G, c.cval15);
    }
    CHKLAUNCH();
    HIPCHK(hipStreamSynchronize(c.stream));
    return HHGR_OK;
}

}  // namespace
}  // namespace hhgr

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

void hhgr_desc_default(hhgr_desc *d) {
    if (!d) return;
    d->n_sub = 2;
    d->level = 7;
    d->coarse_level = 2;
    d->nu_pre = 2;
    d->nu_post = 1;
    d->omega = 1.25;
    d->precision = HHGR_FP64;
    d->variable_coeff = 0;
    d->max_faults = 8;
    d->general_geometry = 0;
}

const char *hhgr_last_error(void) { return g_err.c_str(); }

int hhgr_workspace_bytes(const hhgr_desc *desc, size_t *bytes) {
    std::string e = check_desc(desc);
    if (!e.empty()) return fail(HHGR_EINVAL, e);
    if (!bytes) return fail(HHGR_EINVAL, "null bytes pointer");
    hhgr_ctx c;
    c.d = *desc;
    c.L = desc->level;
    c.Lc = desc->coarse_level;
    c.n_tets = 6 * desc->n_sub * desc->n_sub * desc->n_sub;
    long long N = (long long)desc->n_sub << desc->level;
    c.n_dofs = (N - 1) * (N - 1) * (N - 1);
    c.vk = desc->variable_coeff != 0;
    c.mixed = desc->precision == HHGR_MIXED;
    c.gen = desc->general_geometry != 0;
    std::string te = get_topology(desc->n_sub, c.L, c.Lc, c.topo_hold);
    if (!te.empty()) return fail(HHGR_EINVAL, te);
    c.topo = c.topo_hold.get();
    Carver cv;
    carve(c, cv);
    *bytes = cv.off + 256;
    return HHGR_OK;
}

}  // extern "C"

namespace hhgr {
namespace {

// hhgr_create and the context of hhgr_solve_static.  own_objects: create the
// second stream, the capture stream, the fork/join events and the pinned
// read-back buffer; without them (a context that allocates nothing) the
// norms are read back into pageable host memory and the context supports
// set_rhs, solve and get_solution only (no graphs, recoveries or batches).
int create_ctx(const hhgr_desc *desc, std::shared_ptr<const Topology> mesh_topo, void *dev_ws, size_t ws_bytes,
               void *hip_stream, bool own_objects, hhgr_ctx **out) {
    if (!out) return fail(HHGR_EINVAL, "null output pointer");
    *out = nullptr;
    std::string e = check_desc(desc);
    if (!e.empty()) return fail(HHGR_EINVAL, e);
    if (mesh_topo && desc->variable_coeff) return fail(HHGR_EINVAL, "an unstructured macro mesh takes k = 1 only");
    if (!dev_ws) return fail(HHGR_EINVAL, "null workspace");
    if ((reinterpret_cast<uintptr_t>(dev_ws) & 255) != 0) return fail(HHGR_EINVAL, "workspace must be 256-byte aligned");
    hhgr_ctx *c = new hhgr_ctx();
    c->d = *desc;
    c->L = desc->level;
    c->Lc = desc->coarse_level;
    c->n_tets = 6 * desc->n_sub * desc->n_sub * desc->n_sub;
    long long N = (long long)desc->n_sub << desc->level;
    c->n_dofs = (N - 1) * (N - 1) * (N - 1);
    c->n_elems = 6 * N * N * N;
    c->vk = desc->variable_coeff != 0;
    c->mixed = desc->precision == HHGR_MIXED;
    c->gen = desc->general_geometry != 0;
    c->stream = (hipStream_t)hip_stream;
    if (mesh_topo) {
        c->topo_hold = mesh_topo;
        c->mesh = c->gen = true;
        c->n_tets = mesh_topo->n_tets;
        c->n_dofs = mesh_topo->n_dofs;
        c->n_elems = (long long)c->n_tets << (3 * c->L);
    } else {
        std::string te = get_topology(desc->n_sub, c->L, c->Lc, c->topo_hold);
        if (!te.empty()) {
            delete c;
            return fail(HHGR_EINVAL, te);
        }
    }
    c->topo = c->topo_hold.get();
    Carver sz;
    carve(*c, sz);
    if (sz.off + 256 > ws_bytes) {
        delete c;
        return fail(HHGR_ENOMEM, "workspace too small");
    }
    Carver cv;
    cv.base = (char *)dev_ws;
    carve(*c, cv);
    c->ws = dev_ws;
    c->ws_bytes = ws_bytes;
    auto bail = [&](int code) {
        hhgr_destroy(c);
        return code;
    };
    if (own_objects) {
        if (hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess)
            return bail(fail(HHGR_EHIP, "stream create"));
        if (hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess)
            return bail(fail(HHGR_EHIP, "event create"));
        if (hipHostMalloc((void **)&c->hnorm, 8 * sizeof(double), hipHostMallocDefault) != hipSuccess)
            return bail(fail(HHGR_EHIP, "pinned host allocation"));
    } else {
        c->hnorm = c->hnorm_local;
    }

    const Topology &tp = *c->topo;
    // host-side staging of all tables; kept alive until the final synchronise
    std::vector<std::vector<VolDesc>> vd_store;
    std::vector<std::vector<int4>> rown_store;
    int rc = HHGR_OK;
    for (int l = c->Lc; l <= c->L && rc == HHGR_OK; l++) {
        const TopoLevel &T = tp.lev[l];
        LevelDev &D = c->lev[l];
        rc = rc ? rc : upload(*c, D.nbr, T.nbr.data(), T.nbr.size() * sizeof(int));
        rc = rc ? rc : upload(*c, D.gptr, T.gptr.data(), T.gptr.size() * sizeof(int));
        rc = rc ? rc : upload(*c, D.gidx, T.gidx.data(), T.gidx.size() * sizeof(int));
        if (D.prl) rc = rc ? rc : upload(*c, D.prl, T.prl.data(), T.prl.size() * sizeof(int));
        if (D.rst) rc = rc ? rc : upload(*c, D.rst, T.rst.data(), T.rst.size() * sizeof(int));
        if (D.nb15) rc = rc ? rc : upload(*c, D.nb15, T.nb15.data(), T.nb15.size() * sizeof(int));
        rc = rc ? rc : upload(*c, D.ifc_dof, T.ifc_dof.data(), T.ifc_dof.size() * sizeof(int));
        rc = rc ? rc : upload(*c, D.ifc_xyz, T.ifc_X.data(), T.ifc_X.size() * 3 * sizeof(int));
        rc = rc ? rc : upload(*c, D.tg_dst, T.tg_dst.data(), T.tg_dst.size() * sizeof(int));
        rc = rc ? rc : upload(*c, D.tg_src, T.tg_src.data(), T.tg_src.size() * sizeof(int));
        std::vector<VolDesc> vd(c->n_tets);
        for (int t = 0; t < c->n_tets; t++) vd[t] = VolDesc{(long long)t * T.C_pad, (long long)t * T.C_pad, t, 0};
        vd_store.push_back(vd);
        rc = rc ? rc : upload(*c, D.vd_all, vd_store.back().data(), vd.size() * sizeof(VolDesc));
        rc = rc ? rc : upload(*c, D.ilist, T.ilist.data(), T.ilist.size() * sizeof(unsigned));
        rc = rc ? rc : upload(*c, D.rlist, T.rlist.data(), T.rlist.size() * sizeof(unsigned));
        rc = rc ? rc : upload(*c, D.blist, T.blist.data(), T.blist.size() * sizeof(unsigned));
        rc = rc ? rc : upload(*c, D.flist, T.flist.data(), T.flist.size() * sizeof(unsigned));
        rc = rc ? rc : upload(*c, D.rowC, T.rowC.data(), T.rowC.size() * sizeof(int2));
        {
            std::vector<int4> rn(2 * T.rowN.size());
            for (size_t q = 0; q < T.rowN.size(); q++) {
                const auto &e = T.rowN[q];
                rn[2 * q] = make_int4(e[0], e[1], e[2], e[3]);
                rn[2 * q + 1] = make_int4(e[4], e[5], e[6], e[7]);
            }
            rown_store.push_back(std::move(rn));
            rc = rc ? rc : upload(*c, D.rowN, rown_store.back().data(), rown_store.back().size() * sizeof(int4));
        }
        if (c->gen) {
            for (int q = 0; q < 4; q++) {
                rc = rc ? rc : upload(*c, D.qlist[q], T.qlist[q].data(), T.qlist[q].size() * sizeof(unsigned));
                rc = rc ? rc : upload(*c, D.ifcq[q], T.ifcq[q].data(), T.ifcq[q].size() * sizeof(int));
            }
            rc = rc ? rc : upload(*c, D.rowN15, T.rowN15.data(), T.rowN15.size() * 16 * sizeof(int));
            if (c->mesh) {
                // the operator of a mesh comes with its topology
                rc = rc ? rc : upload(*c, D.w15, T.mesh_w15.data(), T.mesh_w15.size() * sizeof(double));
                rc = rc ? rc : upload(*c, D.wi15, T.mesh_wi.data(), T.mesh_wi.size() * sizeof(double));
                if (D.mwi) {
                    rc = rc ? rc : upload(*c, D.mw15, T.mesh_mw15.data(), T.mesh_mw15.size() * sizeof(double));
                    rc = rc ? rc : upload(*c, D.mwi, T.mesh_mwi.data(), T.mesh_mwi.size() * sizeof(double));
                }
                launch_fill<double>(c->stream, D.wtab, 15LL * D.wtab_cap, 0.0);
                launch_fill<unsigned int>(c->stream, reinterpret_cast<unsigned int *>(D.sid), T.n_ifc, 0u);
                if (c->mixed) {
                    launch_cast<double, float>(c->stream, D.w15, D.w15f, 15LL * c->n_tets);
                    launch_cast<double, float>(c->stream, D.wi15, D.wi15f, (long long)tp.nbw * T.n_ifc);
                }
            }
        }
        if (c->gen && !c->mesh) {
            // no operator until hhgr_set_geometry
            launch_fill<double>(c->stream, D.w15, 15LL * c->n_tets, 0.0);
            launch_fill<double>(c->stream, D.wtab, 15LL * D.wtab_cap, 0.0);
            launch_fill<unsigned int>(c->stream, reinterpret_cast<unsigned int *>(D.sid), T.n_ifc, 0u);
            if (D.mw15) {
                launch_fill<double>(c->stream, D.mw15, 15LL * c->n_tets, 0.0);
                launch_fill<double>(c->stream, D.mwtab, 15LL * D.wtab_cap, 0.0);
            }
        }
        if (D.fz_ps) {
            rc = rc ? rc : upload(*c, D.fz_ps, D.fz_ps_host.data(), D.fz_ps_host.size() * sizeof(int));
            rc = rc ? rc : upload(*c, D.fz_tiles, D.fz_tiles_host.data(), D.fz_tiles_host.size() * sizeof(int4));
        }
        // zero every vector (also the Dirichlet ghosts and the zero slot)
        if (D.ualt) launch_fill<double>(c->stream, D.ualt, T.n_slots, 0.0);
        if (D.u32alt) launch_fill<float>(c->stream, D.u32alt, T.n_slots, 0.0f);
        launch_fill<double>(c->stream, D.u, T.n_slots, 0.0);
        launch_fill<double>(c->stream, D.b, T.n_slots, 0.0);
        launch_fill<double>(c->stream, D.r, T.n_slots, 0.0);
        if (c->mixed) {
            launch_fill<float>(c->stream, D.u32, T.n_slots, 0.0f);
            launch_fill<float>(c->stream, D.b32, T.n_slots, 0.0f);
            launch_fill<float>(c->stream, D.r32, T.n_slots, 0.0f);
        }
        if (D.lu) {
            const long long n = (long long)std::max(c->d.max_faults, 1) * T.C_pad;
            launch_fill<double>(c->stream, D.lu, n, 0.0);
            launch_fill<double>(c->stream, D.lb, n, 0.0);
            launch_fill<double>(c->stream, D.lr, n, 0.0);
        }
        launch_fill<unsigned char>(c->stream, D.frozen, T.n_ifc, 0);
        if (c->vk && c->gen) {
            launch_fill<double>(c->stream, D.wv, 8 * T.n_slots, 0.0);
            launch_fill<double>(c->stream, D.wi15, 15LL * T.n_ifc, 0.0);
        } else if (c->vk) {
            for (int s = 0; s < 3; s++) launch_fill<double>(c->stream, D.w[s], T.n_slots, 0.0);
            if (c->mixed)
                for (int s = 0; s < 3; s++) launch_fill<float>(c->stream, D.w32[s], T.n_slots, 0.0f);
        }
    }
    std::vector<int> tinfo(6 * (size_t)c->n_tets, 0);  // (cube position and axis order; unused on a mesh)
    for (int t = 0; t < c->n_tets && !c->mesh; t++)
        for (int a = 0; a < 3; a++) {
            tinfo[6 * t + a] = tp.V0[t][a];
            tinfo[6 * t + 3 + a] = tp.perm[t][a];
        }
    rc = rc ? rc : upload(*c, c->tetinfo, tinfo.data(), tinfo.size() * sizeof(int));
    const CoarseSystem &cs = tp.coarse;
    std::vector<int> cpos(3 * (size_t)cs.n);
    for (int q = 0; q < cs.n; q++)
        for (int a = 0; a < 3; a++) cpos[3 * q + a] = cs.pos[q][a];
    c->cval_host = cs.val;
    rc = rc ? rc : upload(*c, c->cslot, cs.slot.data(), cs.slot.size() * sizeof(long long));
    rc = rc ? rc : upload(*c, c->ccol, cs.col.data(), cs.col.size() * sizeof(int));
    rc = rc ? rc : upload(*c, c->cval, c->cval_host.data(), c->cval_host.size() * sizeof(double));
    std::vector<double> cinv_host;
    if (!c->gen && c->cinv && coarse_inverse(cs.n, 7, cs.col, cs.val, cinv_host)) {
        rc = rc ? rc : upload(*c, c->cinv, cinv_host.data(), cinv_host.size() * sizeof(double));
        c->dense_coarse = true;
    }
    if (c->mesh) {
        rc = rc ? rc : upload(*c, c->dir_rows, tp.dir_rows.data(), tp.dir_rows.size() * sizeof(int));
        rc = rc ? rc : upload(*c, c->dir_ptr, tp.dir_ptr.data(), tp.dir_ptr.size() * sizeof(int));
        rc = rc ? rc : upload(*c, c->dir_col, tp.dir_col.data(), tp.dir_col.size() * sizeof(int));
        rc = rc ? rc : upload(*c, c->dir_val, tp.dir_val.data(), tp.dir_val.size() * sizeof(double));
        std::vector<double> kel;
        tp.mesh_kuhn_matrices(c->L, kel);
        rc = rc ? rc : upload(*c, c->mesh_kel, kel.data(), kel.size() * sizeof(double));
        // the copies read kel before it goes out of scope
        if (hipStreamSynchronize(c->stream) != hipSuccess) return bail(fail(HHGR_EHIP, "stream synchronize"));
        if (!c->cinv || !coarse_inverse(cs.n, cs.cw, cs.colw, cs.valw, cinv_host))
            return bail(fail(HHGR_EINVAL, "the coarsest-level operator of the mesh is not positive definite"));
        rc = rc ? rc : upload(*c, c->cinv, cinv_host.data(), cinv_host.size() * sizeof(double));
        c->dense_coarse = true;
        c->geom_set = true;
    }
    rc = rc ? rc : upload(*c, c->cptr, cs.cptr.data(), cs.cptr.size() * sizeof(int));
    rc = rc ? rc : upload(*c, c->cidx, cs.cidx.data(), cs.cidx.size() * sizeof(int));
    rc = rc ? rc : upload(*c, c->cpos, cpos.data(), cpos.size() * sizeof(int));
    if (c->gen) {
        rc = rc ? rc : upload(*c, c->ccol15, cs.col15.data(), cs.col15.size() * sizeof(int));
        launch_fill<double>(c->stream, c->cval15, 15LL * cs.n, 0.0);
    }
    launch_fill<unsigned char>(c->stream, c->cfrozen, cs.n, 0);
    // the scratch vectors' zero slot and Dirichlet ghosts must read zero
    launch_fill<double>(c->stream, c->aux_u, tp.lev[c->L].n_slots, 0.0);
    launch_fill<double>(c->stream, c->aux_b, tp.lev[c->L].n_slots, 0.0);
    launch_fill<double>(c->stream, c->dnorm, 8, 0.0);
    launch_fill<unsigned int>(c->stream, c->counter, 64, 0u);
    if (rc != HHGR_OK) return bail(rc);
    if (hipGetLastError() != hipSuccess) return bail(fail(HHGR_EHIP, "kernel launch during setup"));
    if (hipStreamSynchronize(c->stream) != hipSuccess) return bail(fail(HHGR_EHIP, "setup synchronise"));
    *out = c;
    return HHGR_OK;
}

}  // namespace
}  // namespace hhgr

extern "C" {

int hhgr_create(const hhgr_desc *desc, void *dev_ws, size_t ws_bytes, void *hip_stream, hhgr_ctx **out) {
    return create_ctx(desc, nullptr, dev_ws, ws_bytes, hip_stream, true, out);
}

// a mesh context ignores n_sub and general_geometry
static hhgr_desc mesh_desc(const hhgr_desc *desc) {
    hhgr_desc d = *desc;
    d.n_sub = 1;
    d.general_geometry = 1;
    return d;
}

int hhgr_mesh_boundary(const hhgr_ctx *c, long long *n_boundary, double *host_xyz) {
    if (!c) return fail(HHGR_EINVAL, "null context");
    if (!c->mesh) return fail(HHGR_EINVAL, "not an unstructured macro mesh context");
    if (n_boundary) *n_boundary = c->topo->n_bnd;
    if (host_xyz) std::copy(c->topo->bnd_xyz.begin(), c->topo->bnd_xyz.end(), host_xyz);
    return HHGR_OK;
}

int hhgr_mesh_set_coeff(hhgr_ctx *c, const double *host_k) {
    if (!c) return fail(HHGR_EINVAL, "null context");
    if (!c->mesh) return fail(HHGR_EINVAL, "not an unstructured macro mesh context");
    const Topology &tp = *c->topo;
    const CoarseSystem &cs = tp.coarse;
    Topology::MeshOps K;
    if (host_k) {
        for (int t = 0; t < c->n_tets; t++)
            if (!(host_k[t] > 0.0) || !std::isfinite(host_k[t]))
                return fail(HHGR_EINVAL, "the coefficient must be positive and finite on every tetrahedron");
        const std::vector<unsigned char> all(c->n_tets, 1);
        const std::string e = tp.mesh_weighted_operators(host_k, all.data(), nullptr, K);
        if (!e.empty()) return fail(HHGR_EINVAL, e);
    } else {
        // back to k = 1: the topology's own tables
        K.w15.assign(c->L + 1, {});
        K.wi.assign(c->L + 1, {});
        for (int l = c->Lc; l <= c->L; l++) {
            K.w15[l] = tp.lev[l].mesh_w15;
            K.wi[l] = tp.lev[l].mesh_wi;
        }
        K.valw = cs.valw;
        K.dir_val = tp.dir_val;
    }
    std::vector<double> inv;
    if (!coarse_inverse(cs.n, cs.cw, cs.colw, K.valw, inv))
        return fail(HHGR_EINVAL, "the coarsest-level operator is not positive definite");
    invalidate_graph(*c);
    int rc = HHGR_OK;
    for (int l = c->Lc; l <= c->L; l++) {
        LevelDev &D = c->lev[l];
        rc = rc ? rc : upload(*c, D.w15, K.w15[l].data(), K.w15[l].size() * sizeof(double));
        rc = rc ? rc : upload(*c, D.wi15, K.wi[l].data(), K.wi[l].size() * sizeof(double));
        if (c->mixed) {
            launch_cast<double, float>(c->stream, D.w15, D.w15f, 15LL * c->n_tets);
            launch_cast<double, float>(c->stream, D.wi15, D.wi15f, (long long)tp.nbw * D.n_ifc);
        }
    }
    rc = rc ? rc : upload(*c, c->cinv, inv.data(), inv.size() * sizeof(double));
    rc = rc ? rc : upload(*c, c->dir_val, K.dir_val.data(), K.dir_val.size() * sizeof(double));
    const hipError_t le = hipGetLastError();
    HIPCHK(hipStreamSynchronize(c->stream));  // the copies read K and inv
    if (le != hipSuccess) return fail(HHGR_EHIP, std::string("kernel launch: ") + hipGetErrorString(le));
    if (rc) return rc;
    if (host_k) {
        c->mesh_k.assign(host_k, host_k + c->n_tets);
        c->mesh_k_wi = std::move(K.wi);
        c->mesh_k_valw = std::move(K.valw);
    } else {
        c->mesh_k.clear();
        c->mesh_k_wi.clear();
        c->mesh_k_valw.clear();
    }
    return HHGR_OK;
}

int hhgr_mesh_workspace_bytes(const hhgr_desc *desc_in, int nv, const double *host_xyz, int nt, const int *host_tets,
                              size_t *bytes) {
    if (!desc_in) return fail(HHGR_EINVAL, "null descriptor");
    const hhgr_desc dd = mesh_desc(desc_in);
    const hhgr_desc *desc = &dd;
    std::string e = check_desc(desc);
    if (!e.empty()) return fail(HHGR_EINVAL, e);
    if (!bytes) return fail(HHGR_EINVAL, "null bytes pointer");
    if (desc->variable_coeff) return fail(HHGR_EINVAL, "an unstructured macro mesh takes k = 1 only");
    hhgr_ctx c;
    c.d = *desc;
    c.L = desc->level;
    c.Lc = desc->coarse_level;
    c.mixed = desc->precision == HHGR_MIXED;
    c.gen = c.mesh = true;
    std::string te = get_mesh_topology(nv, host_xyz, nt, host_tets, c.L, c.Lc, c.topo_hold);
    if (!te.empty()) return fail(HHGR_EINVAL, te);
    c.topo = c.topo_hold.get();
    c.n_tets = c.topo->n_tets;
    c.n_dofs = c.topo->n_dofs;
    Carver cv;
    carve(c, cv);
    *bytes = cv.off + 256;
    return HHGR_OK;
}

int hhgr_create_mesh(const hhgr_desc *desc_in, int nv, const double *host_xyz, int nt, const int *host_tets,
                     void *dev_ws, size_t ws_bytes, void *hip_stream, hhgr_ctx **out) {
    if (!out) return fail(HHGR_EINVAL, "null output pointer");
    *out = nullptr;
    if (!desc_in) return fail(HHGR_EINVAL, "null descriptor");
    const hhgr_desc dd = mesh_desc(desc_in);
    const hhgr_desc *desc = &dd;
    std::string e = check_desc(desc);
    if (!e.empty()) return fail(HHGR_EINVAL, e);
    std::shared_ptr<const Topology> tp;
    std::string te = get_mesh_topology(nv, host_xyz, nt, host_tets, desc->level, desc->coarse_level, tp);
    if (!te.empty()) return fail(HHGR_EINVAL, te);
    return create_ctx(desc, tp, dev_ws, ws_bytes, hip_stream, true, out);
}

void hhgr_destroy(hhgr_ctx *c) {
    if (!c) return;
    hipStreamSynchronize(c->stream);  // also the legacy default stream (nullptr)
    if (c->stream2) {
        hipStreamSynchronize(c->stream2);
        hipStreamDestroy(c->stream2);
    }
    if (c->cap) hipStreamDestroy(c->cap);
    if (c->ev_fork) hipEventDestroy(c->ev_fork);
    if (c->ev_join) hipEventDestroy(c->ev_join);
    for (hipEvent_t e : c->tev) hipEventDestroy(e);
    if (c->gexec) hipGraphExecDestroy(c->gexec);
    if (c->lgexec) hipGraphExecDestroy(c->lgexec);
    if (c->hnorm && c->hnorm != c->hnorm_local) hipHostFree(c->hnorm);
    delete c;
}

int hhgr_sizes(const hhgr_ctx *c, long long *n_dofs, int *n_tets, long long *n_elems) {
    if (!c) return fail(HHGR_EINVAL, "null context");
    if (n_dofs) *n_dofs = c->n_dofs;
    if (n_tets) *n_tets = c->n_tets;
    if (n_elems) *n_elems = c->n_elems;
    return HHGR_OK;
}

int hhgr_set_rhs(hhgr_ctx *c, const double *dev_vec, int kind) {
    if (!c || !dev_vec) return fail(HHGR_EINVAL, "null argument");
    if (kind != HHGR_RHS_LOAD && kind != HHGR_RHS_NODAL_F && kind != HHGR_RHS_DIRICHLET)
        return fail(HHGR_EINVAL, "bad rhs kind");
    if (c->gen && kind != HHGR_RHS_LOAD && !c->geom_set)
        return fail(HHGR_ESTATE, "this right-hand side on a general macro mesh needs hhgr_set_geometry first");
    if (kind == HHGR_RHS_DIRICHLET && c->vk && !c->coeff_set)
        return fail(HHGR_ESTATE, "Dirichlet data with variable_coeff = 1 needs hhgr_set_coeff first");
    LevelDev &D = c->lev[c->L];
    const VolGeom vfull = vgeom(D, D.vd_all, c->n_tets, true);
    const VolGeom vint = vgeom(D, D.vd_all, c->n_tets, false);
    const IfcGeom ig = igeom(D, 0, D.n_ifc, nullptr, false);
    bool aux_used = false;  // aux_u held the load in vector order

    if (kind == HHGR_RHS_DIRICHLET && c->mesh) {
        // g at the boundary nodes (hhgr_mesh_boundary order): b = -A_IB g
        launch_fill<double>(c->stream, D.b, D.n_slots, 0.0);
        launch_dirichlet_rows(c->stream, c->n_dir_rows, c->dir_rows, c->dir_ptr, c->dir_col, c->dir_val, dev_vec, D.b);
    } else if (kind == HHGR_RHS_LOAD) {
        to_slots(*c, D, dev_vec, D.b, c->stream);
    } else if (kind == HHGR_RHS_DIRICHLET && c->gen) {
        launch_gen_dirichlet(c->stream, vint, ig, gen15(D, -1, false), c->tetinfo, D.ifc_xyz, D.N, dev_vec, D.b);
    } else if (kind == HHGR_RHS_DIRICHLET) {
        // the load in vector order goes through aux_u (n_slots >= (N-1)^3 entries)
        if (D.n_slots < (long long)(D.N - 1) * (D.N - 1) * (D.N - 1)) return fail(HHGR_EINVAL, "aux buffer too small");
        launch_dirichlet_load(c->stream, D.N, D.h, c->vk ? D.kc : nullptr, dev_vec, c->aux_u);
        launch_user_to_slots<double>(c->stream, vfull, c->tetinfo, D.m, D.N, ig, D.ifc_dof, c->aux_u, D.b);
        aux_used = true;
    } else if (c->gen) {
        to_slots(*c, D, dev_vec, D.r, c->stream);
        launch_apply15(c->stream, vint, ig, gen15mass(D), D.r, D.b);
    } else {
        // b = M f on the grid in vector order (through aux_u), then into the slots
        if (D.n_slots < (long long)(D.N - 1) * (D.N - 1) * (D.N - 1)) return fail(HHGR_EINVAL, "aux buffer too small");
        launch_mass_grid(c->stream, D.N, D.h, dev_vec, c->aux_u);
        launch_user_to_slots<double>(c->stream, vfull, c->tetinfo, D.m, D.N, ig, D.ifc_dof, c->aux_u, D.b);
        aux_used = true;
    }
    // aux_u is a scratch slot vector again (zero slot and boundary ghosts zero)
    if (aux_used) launch_fill<double>(c->stream, c->aux_u, D.n_slots, 0.0);
    // ||b|| over every interior node once
    const int nb = launch_norm2(c->stream, vint, ig, D.b, c->partial[0]);
    if (nb > 0)
        launch_reduce(c->stream, c->partial[0], nb, c->dnorm + 1);
    else
        launch_fill<double>(c->stream, c->dnorm + 1, 1, 0.0);
    CHKLAUNCH();
    double bn;
    int rc = read_norm(*c, 1, &bn);
    if (rc) return rc;
    c->bnorm = bn;
    c->rhs_set = true;
    return HHGR_OK;
}

int hhgr_set_coeff(hhgr_ctx *c, const double *dev_k) {
    if (!c || !dev_k) return fail(HHGR_EINVAL, "null argument");
    if (!c->vk) return fail(HHGR_ESTATE, "context created with variable_coeff = 0");
    invalidate_graph(*c);
    LevelDev &F = c->lev[c->L];
    HIPCHK(hipMemcpyAsync(F.kc, dev_k, sizeof(double) * 6 * (size_t)F.N * F.N * F.N, hipMemcpyDeviceToDevice,
                          c->stream));
    for (int l = c->L - 1; l >= c->Lc; l--) launch_coarsen_k(c->stream, c->lev[l + 1].kc, c->lev[l + 1].N, c->lev[l].kc, c->lev[l].N);
    if (c->gen) {
        CHKLAUNCH();
        HIPCHK(hipStreamSynchronize(c->stream));
        c->coeff_set = true;
        return c->geom_set ? gen_weights(*c) : HHGR_OK;
    }
    for (int l = c->Lc; l <= c->L; l++) {
        LevelDev &D = c->lev[l];
        launch_vol_weights(c->stream, vgeom(D, D.vd_all, c->n_tets, true), c->tetinfo, D.m, D.N, D.h, D.kc, D.w[0],
                           D.w[1], D.w[2]);
        launch_ifc_weights(c->stream, D.n_ifc, D.ifc_xyz, D.N, D.h, D.kc, D.wi);
        if (c->mixed) {
            for (int s = 0; s < 3; s++) launch_cast<double, float>(c->stream, D.w[s], D.w32[s], D.n_slots);
            launch_cast<double, float>(c->stream, D.wi, D.wi32, 6LL * D.n_ifc);
        }
    }
    const LevelDev &Dc = c->lev[c->Lc];
    launch_coarse_vals(c->stream, c->cn, c->cpos, c->ccol, Dc.N, Dc.h, Dc.kc, c->cval);
    CHKLAUNCH();
    HIPCHK(hipStreamSynchronize(c->stream));
    c->coeff_set = true;
    return HHGR_OK;
}

int hhgr_set_geometry(hhgr_ctx *c, const double *host_xyz) {
    if (!c || !host_xyz) return fail(HHGR_EINVAL, "null argument");
    if (!c->gen) return fail(HHGR_ESTATE, "context created with general_geometry = 0");
    if (c->mesh) return fail(HHGR_EINVAL, "an unstructured macro mesh takes its geometry at creation");
    const Topology &tp = *c->topo;
    std::string e = check_macro_mesh(tp, host_xyz);
    if (!e.empty()) return fail(HHGR_EINVAL, e);
    invalidate_graph(*c);
    int rc = HHGR_OK;
    // host staging vectors must outlive the copies (synchronised below)
    std::vector<LevelStencils> G(c->L + 1);
    std::vector<double> cval, kel;
    // element matrices: per-node stencils of a variable k and the intact side
    // of a Dirichlet-Neumann recovery are computed from them on the GPU
    element_matrices(tp, host_xyz, kel);
    // k = 1: the stiffness stencils of every level; the finest level's mass
    // stencils (and master ids) in either case.  Everything is computed
    // before the first copy, so a failure leaves the context as it was.
    const int l0 = c->vk ? c->L : c->Lc;
    for (int l = l0; l <= c->L; l++) {
        e = level_stencils(tp, host_xyz, l, c->lev[l].wtab_cap, G[l]);
        if (!e.empty()) return fail(HHGR_EINVAL, e);
    }
    std::vector<double> cinv_host;
    bool dense = false;
    if (!c->vk) {
        coarse_stencils(tp, host_xyz, cval);
        dense = c->cinv && coarse_inverse(tp.coarse.n, 15, tp.coarse.col15, cval, cinv_host);
    }
    rc = upload(*c, c->kel, kel.data(), kel.size() * sizeof(double));
    for (int l = l0; l <= c->L; l++) {
        LevelDev &D = c->lev[l];
        rc = rc ? rc : upload(*c, D.w15, G[l].w15.data(), G[l].w15.size() * sizeof(double));
        rc = rc ? rc : upload(*c, D.wtab, G[l].wtab.data(), G[l].wtab.size() * sizeof(double));
        rc = rc ? rc : upload(*c, D.sid, G[l].sid.data(), G[l].sid.size() * sizeof(int));
        if (l == c->L) {
            rc = rc ? rc : upload(*c, D.mw15, G[l].mw15.data(), G[l].mw15.size() * sizeof(double));
            rc = rc ? rc : upload(*c, D.mwtab, G[l].mwtab.data(), G[l].mwtab.size() * sizeof(double));
        }
    }
    c->dense_coarse = false;
    if (dense) {
        rc = rc ? rc : upload(*c, c->cinv, cinv_host.data(), cinv_host.size() * sizeof(double));
        c->dense_coarse = true;
    }
    if (!c->vk) {
        rc = rc ? rc : upload(*c, c->cval15, cval.data(), cval.size() * sizeof(double));
        if (c->mixed)
            for (int l = c->Lc; l <= c->L; l++) {
                LevelDev &D = c->lev[l];
                launch_cast<double, float>(c->stream, D.w15, D.w15f, 15LL * c->n_tets);
                launch_cast<double, float>(c->stream, D.wtab, D.wtabf, 15LL * D.wtab_cap);
            }
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    if (rc) return rc;
    c->geom_set = true;
    if (c->vk && c->coeff_set) return gen_weights(*c);
    return HHGR_OK;
}

int hhgr_set_solution(hhgr_ctx *c, const double *dev_u) {
    if (!c) return fail(HHGR_EINVAL, "null context");
    LevelDev &D = c->lev[c->L];
    if (!dev_u) {
        // u = 0 in every slot (ghost copies and the zero slot included)
        launch_fill<double>(c->stream, D.u, D.n_slots, 0.0);
        CHKLAUNCH();
        return HHGR_OK;
    }
    to_slots(*c, D, dev_u, D.u, c->stream);
    CHKLAUNCH();
    return HHGR_OK;
}

int hhgr_get_solution(const hhgr_ctx *cc, double *dev_u) {
    hhgr_ctx *c = const_cast<hhgr_ctx *>(cc);
    if (!c || !dev_u) return fail(HHGR_EINVAL, "null argument");
    LevelDev &D = c->lev[c->L];
    to_user(*c, D, D.u, dev_u, c->stream);
    CHKLAUNCH();
    return HHGR_OK;
}

static int check_ready(hhgr_ctx *c) {
    if (!c) return fail(HHGR_EINVAL, "null context");
    if (!c->rhs_set) return fail(HHGR_ESTATE, "no right-hand side set");
    if (c->vk && !c->coeff_set) return fail(HHGR_ESTATE, "no coefficient set");
    if (c->gen && !c->geom_set) return fail(HHGR_ESTATE, "no geometry set");
    return HHGR_OK;
}

int hhgr_vcycle(hhgr_ctx *c, int n, double *rel_res_out) {
    int rc = check_ready(c);
    if (rc) return rc;
    if (n < 0) return fail(HHGR_EINVAL, "negative cycle count");
    if (c->mixed) {
        prime_mixed(*c, c->stream);
        CHKLAUNCH();
    }
    for (int q = 0; q < n; q++) {
        rc = run_step(*c);
        if (rc) return rc;
    }
    if (rel_res_out) {
        double rn;
        if (n == 0 || c->timing || !c->use_graph) {
            if (n == 0) {
                HView<double> V = global_view<double>(*c, false, 0);
                finest_residual<double>(*c, V, (double *)nullptr, c->stream, c->dnorm);
            }
            rc = read_norm(*c, 0, &rn);
            if (rc) return rc;
        } else {
            HIPCHK(hipStreamSynchronize(c->stream));
            rn = std::sqrt(std::max(c->hnorm[0], 0.0));
        }
        *rel_res_out = c->bnorm > 0 ? rn / c->bnorm : 0.0;
    }
    return HHGR_OK;
}

int hhgr_solve(hhgr_ctx *c, double rel_tol, int max_cycles, hhgr_report *rep) {
    int rc = check_ready(c);
    if (rc) return rc;
    if (max_cycles < 0) return fail(HHGR_EINVAL, "negative max_cycles");
    HView<double> V = global_view<double>(*c, false, 0);
    if (c->mixed)
        prime_mixed(*c, c->stream);
    else
        finest_residual<double>(*c, V, (double *)nullptr, c->stream, c->dnorm);
    CHKLAUNCH();
    double rn;
    rc = read_norm(*c, 0, &rn);
    if (rc) return rc;
    double rel = c->bnorm > 0 ? rn / c->bnorm : 0.0;
    if (rep && rep->history && rep->history_cap > 0) rep->history[0] = rel;
    int cyc = 0;
    while (rel > rel_tol && cyc < max_cycles) {
        rc = run_step(*c);
        if (rc) return rc;
        HIPCHK(hipStreamSynchronize(c->stream));
        rn = std::sqrt(std::max(c->hnorm[0], 0.0));
        rel = c->bnorm > 0 ? rn / c->bnorm : 0.0;
        cyc++;
        if (rep && rep->history && cyc < rep->history_cap) rep->history[cyc] = rel;
        if (!std::isfinite(rel)) break;
    }
    if (rep) {
        rep->cycles = cyc;
        rep->rel_res = rel;
    }
    return rel <= rel_tol ? HHGR_OK : fail(HHGR_ENOCONV, "tolerance not reached in max_cycles");
}

int hhgr_inject_fault(hhgr_ctx *c, int tet) {
    if (!c) return fail(HHGR_EINVAL, "null context");
    if (tet < 0 || tet >= c->n_tets) return fail(HHGR_EINVAL, "tet id out of range");
    // the closure is lost; its ghost copies come back from the surviving
    // masters (eq. (4)) before any cycle reads them
    restore_tet(*c, tet, c->stream);
    CHKLAUNCH();
    return HHGR_OK;
}

int hhgr_recover_local(hhgr_ctx *c, int tet, int n_cycles, double *local_rel) {
    int rc = check_ready(c);
    if (rc) return rc;
    if (tet < 0 || tet >= c->n_tets) return fail(HHGR_EINVAL, "tet id out of range");
    if (n_cycles < 0) return fail(HHGR_EINVAL, "negative cycle count");
    if (c->d.max_faults < 1) return fail(HHGR_ESTATE, "context created with max_faults = 0");
    if (c->Lc != 2) return fail(HHGR_ESTATE, "local recovery needs coarse_level = 2 (one unknown per tetrahedron)");
    set_loc(*c, {tet});
    // restored ghosts, the local residual before and after the cycles
    auto enqueue = [&](hipStream_t s) {
        restore_tet(*c, tet, s);
        HView<double> V = local_view(*c, 0);
        finest_residual<double>(*c, V, (double *)nullptr, s, c->dnorm + 2);
        for (int q = 0; q < n_cycles; q++) vcycle<double>(*c, V, c->L, false, s);
        finest_residual<double>(*c, V, (double *)nullptr, s, c->dnorm + 3);
    };
    if (!c->cap) {
        enqueue(c->stream);  // a context without a capture stream
    } else if (!(c->lgexec && c->lg_tet == tet && c->lg_n == n_cycles)) {
        if (c->lgexec) hipGraphExecDestroy(c->lgexec);
        c->lgexec = nullptr;
        c->lg_tet = c->lg_n = -1;
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(c->cap, hipStreamCaptureModeRelaxed));
        enqueue(c->cap);
        HIPCHK(hipStreamEndCapture(c->cap, &g));
        hipError_t e = hipGraphInstantiate(&c->lgexec, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (e != hipSuccess) {
            c->lgexec = nullptr;
            return fail(HHGR_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        }
        c->lg_tet = tet;
        c->lg_n = n_cycles;
    }
    if (c->lgexec) HIPCHK(hipGraphLaunch(c->lgexec, c->stream));
    CHKLAUNCH();
    double r0, r1;
    rc = read_norm(*c, 2, &r0);
    if (rc) return rc;
    rc = read_norm(*c, 3, &r1);
    if (rc) return rc;
    if (local_rel) *local_rel = r0 > 0 ? r1 / r0 : 0.0;
    return HHGR_OK;
}

int hhgr_recover_dd(hhgr_ctx *c, const int *tets, int n_tets, int n_intact, int n_local) {
    int rc = check_ready(c);
    if (rc) return rc;
    std::vector<int> ft;
    rc = dd_check(*c, tets, n_tets, n_intact, n_local, ft);
    if (rc) return rc;
    invalidate_graph(*c);
    rc = dd_setup(*c, ft);
    if (rc) return rc;
    HIPCHK(hipEventRecord(c->ev_fork, c->stream));
    HIPCHK(hipStreamWaitEvent(c->stream2, c->ev_fork, 0));
    // intact side on the main stream, faulty side on the second stream
    for (int q = 0; q < n_intact; q++) dd_intact_step(*c, c->stream, q == 0, false, 4);
    dd_local(*c, n_local, c->stream2);
    HIPCHK(hipEventRecord(c->ev_join, c->stream2));
    HIPCHK(hipStreamWaitEvent(c->stream, c->ev_join, 0));
    CHKLAUNCH();
    HIPCHK(hipStreamSynchronize(c->stream));
    dd_end(*c);
    return HHGR_OK;
}

int hhgr_recover_dn(hhgr_ctx *c, const int *tets, int n_tets, int n_intact, int eta) {
    int rc = check_ready(c);
    if (rc) return rc;
    std::vector<int> ft;
    rc = dd_check(*c, tets, n_tets, n_intact, eta, ft);
    if (rc) return rc;
    invalidate_graph(*c);
    rc = dn_setup(*c, ft);
    if (rc) return rc;
    HView<double> VI = dn_view(*c);
    HView<double> VL = local_view(*c, 1, c->aux_u);
    for (int q = 0; q < n_intact; q++) {
        // the faulty side reads the interface values of the start of the round
        refresh_faulty_ghosts(*c, ft, c->stream);
        HIPCHK(hipEventRecord(c->ev_fork, c->stream));
        HIPCHK(hipStreamWaitEvent(c->stream2, c->ev_fork, 0));
        // the intact cycle first: its launches then reach the GPU while the
        // host is still launching the many small local kernels
        vcycle<double>(*c, VI, c->L, false, c->stream);
        for (int e = 0; e < eta; e++) vcycle<double>(*c, VL, c->L, false, c->stream2);
        HIPCHK(hipEventRecord(c->ev_join, c->stream2));
        HIPCHK(hipStreamWaitEvent(c->stream, c->ev_join, 0));
    }
    refresh_faulty_ghosts(*c, ft, c->stream);
    CHKLAUNCH();
    HIPCHK(hipStreamSynchronize(c->stream));
    dd_end(*c);
    return HHGR_OK;
}

int hhgr_mass_apply(hhgr_ctx *c, const double *dev_x, double *dev_y) {
    if (!c || !dev_x || !dev_y) return fail(HHGR_EINVAL, "null argument");
    if (c->gen && !c->geom_set) return fail(HHGR_ESTATE, "no geometry set");
    LevelDev &D = c->lev[c->L];
    const IfcGeom ig = igeom(D, 0, D.n_ifc, nullptr, false);
    to_slots(*c, D, dev_x, c->aux_b, c->stream);
    if (c->gen)
        launch_apply15(c->stream, vgeom(D, D.vd_all, c->n_tets, false), ig, gen15mass(D), c->aux_b, c->aux_u);
    else
        launch_mass(c->stream, vgeom(D, D.vd_all, c->n_tets, false), ig, D.nb15, c->aux_b, c->aux_u, D.h);
    to_user(*c, D, c->aux_u, dev_y, c->stream);
    CHKLAUNCH();
    return HHGR_OK;
}

int hhgr_adjoint_grad(hhgr_ctx *c, const double *dev_g, double rel_tol, int max_cycles, double *dev_dJdf,
                      double *dev_dJdk) {
    int rc = check_ready(c);
    if (rc) return rc;
    if (!dev_g) return fail(HHGR_EINVAL, "null g");
    if (dev_dJdk && !c->vk && !c->mesh) return fail(HHGR_ESTATE, "dJ/dk needs variable_coeff = 1");
    LevelDev &D = c->lev[c->L];
    const long long ns = D.n_slots;
    const IfcGeom ig = igeom(D, 0, D.n_ifc, nullptr, false);
    const VolGeom vfull = vgeom(D, D.vd_all, c->n_tets, true), vint = vgeom(D, D.vd_all, c->n_tets, false);
    // save u and b, solve A lambda = g from zero in FP64
    HIPCHK(hipMemcpyAsync(c->aux_u, D.u, ns * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->aux_b, D.b, ns * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    if (dev_dJdk && !c->mesh)
        launch_slots_to_user<double>(c->stream, vint, c->tetinfo, D.m, D.N, ig, D.ifc_dof, D.u, c->user_u);
    to_slots(*c, D, dev_g, D.b, c->stream);
    launch_fill<double>(c->stream, D.u, ns, 0.0);
    const double bnorm_saved = c->bnorm;
    const bool mixed_saved = c->mixed;
    c->mixed = false;
    invalidate_graph(*c);
    {
        HView<double> V = global_view<double>(*c, false, 0);
        launch_fill<double>(c->stream, D.r, ns, 0.0);
        HView<double> Vz = V;
        Vz.lv[c->L].u = D.r;
        finest_residual<double>(*c, Vz, (double *)nullptr, c->stream, c->dnorm + 1);
    }
    CHKLAUNCH();
    double gn;
    rc = read_norm(*c, 1, &gn);
    int result = HHGR_OK;
    if (!rc) {
        c->bnorm = gn;
        hhgr_report rep{0, 0.0, nullptr, 0};
        result = gn > 0 ? hhgr_solve(c, rel_tol, max_cycles, &rep) : HHGR_OK;
        if (dev_dJdf) {
            if (c->gen)
                launch_apply15(c->stream, vint, ig, gen15mass(D), D.u, D.r);
            else
                launch_mass(c->stream, vint, ig, D.nb15, D.u, D.r, D.h);
            to_user(*c, D, D.r, dev_dJdf, c->stream);
        }
        if (dev_dJdk && c->mesh) {
            // per macro tetrahedron from the saved u and lambda in slot space
            // (D.r is free here: it serves as the partial sums)
            launch_mesh_grad_tet(c->stream, c->n_tets, D.m, D.M, D.rowC, D.C_pad, c->mesh_kel, c->aux_u, D.u, D.r,
                                 dev_dJdk);
        } else if (dev_dJdk) {
            launch_slots_to_user<double>(c->stream, vint, c->tetinfo, D.m, D.N, ig, D.ifc_dof, D.u, c->user_l);
            if (c->gen)
                launch_grad_k15(c->stream, D.N, D.m, c->d.n_sub, c->kel, c->user_u, c->user_l, dev_dJdk);
            else
                launch_grad_k(c->stream, c->user_u, c->user_l, D.N, D.h, dev_dJdk);
        }
    }
    // restore the forward state
    hipMemcpyAsync(D.u, c->aux_u, ns * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
    hipMemcpyAsync(D.b, c->aux_b, ns * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
    c->bnorm = bnorm_saved;
    c->mixed = mixed_saved;
    invalidate_graph(*c);
    CHKLAUNCH();
    HIPCHK(hipStreamSynchronize(c->stream));
    if (rc) return rc;
    return result;
}

int hhgr_set_graph(hhgr_ctx *c, int use_graph) {
    if (!c) return fail(HHGR_EINVAL, "null context");
    c->use_graph = use_graph != 0;
    invalidate_graph(*c);
    return HHGR_OK;
}

int hhgr_tuning_info(const hhgr_ctx *c, int level, int *block_size, int *xcd_order, int *nodes_per_thread) {
    if (!c) return fail(HHGR_EINVAL, "null context");
    if (level <= c->Lc || level > c->L) return fail(HHGR_EINVAL, "level outside coarse_level+1..level");
    const LevelDev &D = c->lev[level];
    if (block_size) *block_size = kBS[D.bs_sel];
    if (xcd_order) *xcd_order = D.remap;
    if (nodes_per_thread) *nodes_per_thread = D.cpb;
    return HHGR_OK;
}

int hhgr_set_fused_sweeps(hhgr_ctx *c, int level, int on) {
    if (!c) return fail(HHGR_EINVAL, "null context");
    if (level <= c->Lc || level > c->L) return fail(HHGR_EINVAL, "level outside coarse_level+1..level");
    LevelDev &D = c->lev[level];
    if (on && !D.fz_ps) return fail(HHGR_EINVAL, "no fused sweeps on this level of this context");
    D.fz_on = on != 0;
    invalidate_graph(*c);
    return HHGR_OK;
}

int hhgr_set_tuning(hhgr_ctx *c, int level, int block_size, int xcd_order, int nodes_per_thread) {
    if (!c) return fail(HHGR_EINVAL, "null context");
    if (level != 0 && (level <= c->Lc || level > c->L)) return fail(HHGR_EINVAL, "level outside coarse_level+1..level");
    int q = -1;
    for (int k = 0; k < 3; k++)
        if (kBS[k] == block_size) q = k;
    if (q < 0) return fail(HHGR_EINVAL, "block_size must be 128, 256 or 512");
    if (xcd_order != 0 && xcd_order != 1) return fail(HHGR_EINVAL, "xcd_order must be 0 or 1");
    if (nodes_per_thread != 1 && nodes_per_thread != 4) return fail(HHGR_EINVAL, "nodes_per_thread must be 1 or 4");
    for (int l = c->Lc + 1; l <= c->L; l++) {
        if (level != 0 && l != level) continue;
        LevelDev &D = c->lev[l];
        D.bs_sel = q;
        D.remap = xcd_order;
        D.cpb = nodes_per_thread;
        D.cpb_res = nodes_per_thread;
        D.cpb_prl = nodes_per_thread;
        D.cpb_fus = nodes_per_thread;
    }
    invalidate_graph(*c);
    return HHGR_OK;
}

int hhgr_kernel_timing(hhgr_ctx *c, int enable) {
    if (!c) return fail(HHGR_EINVAL, "null context");
    HIPCHK(hipStreamSynchronize(c->stream));
    c->timing = enable != 0;
    c->tev_used = 0;
    return HHGR_OK;
}

int hhgr_kernel_stats(hhgr_ctx *c, long long *launches, double *mean_ms, double *alg_bytes) {
    if (!c) return fail(HHGR_EINVAL, "null context");
    HIPCHK(hipStreamSynchronize(c->stream));
    double tot = 0.0;
    long long n = 0;
    for (size_t q = 0; q + 1 < c->tev_used; q += 2) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->tev[q], c->tev[q + 1]) == hipSuccess) {
            tot += ms;
            n++;
        }
    }
    if (launches) *launches = n;
    if (mean_ms) *mean_ms = n ? tot / n : 0.0;
    // a colour pass reads the other colour's u and its own b and old u and
    // writes its own u: 4 words per updated node, 2 words per unknown; a
    // class pass of the 4-colour sweep reads the other 3 classes' u
    // (3/4 word per unknown) and 3 words per node of its class (1/4)
    const double w = c->mixed ? 4.0 : 8.0;
    const LevelDev &F = c->lev[c->L];
    if (F.fz_on && (c->mixed ? F.u32alt != nullptr : F.ualt != nullptr)) {
        // the fused sweep's volume kernel: u (both colours) and b read once,
        // u written once, over the volume-interior nodes
        const double mm = F.m;
        if (alg_bytes) *alg_bytes = 3.0 * w * (double)c->n_tets * (mm - 1) * (mm - 2) * (mm - 3) / 6.0;
    } else if (alg_bytes) {
        *alg_bytes = (c->gen ? 1.5 : 2.0) * w * (double)c->n_dofs;
    }
    return HHGR_OK;
}

int hhgr_autotune(hhgr_ctx *c, const char *cache_path) {
    if (!c) return fail(HHGR_EINVAL, "null context");
    if (c->gen && !c->geom_set) return fail(HHGR_ESTATE, "no geometry set");
    hipDeviceProp_t prop;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    std::string devname = prop.gcnArchName;
    std::map<std::string, int> cache;
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string key;
        int v;
        while (in >> key >> v) cache[key] = v;
    }
    invalidate_graph(*c);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    for (int l = c->Lc + 1; l <= c->L; l++) {
        LevelDev &D = c->lev[l];
        std::ostringstream ks;
        ks << devname << ":n" << c->d.n_sub << ":l" << l << ":" << (c->mixed ? "f32" : "f64") << ":vk" << c->vk
           << (c->gen ? ":g15" : "");
        if (c->mesh) ks << ":mesh" << std::hex << c->topo->mesh_hash << std::dec << ":t" << c->n_tets;
        auto it = cache.find(ks.str());
        auto itr = cache.find(ks.str() + ":remap");
        auto itc = cache.find(ks.str() + ":cpb");
        auto itcr = cache.find(ks.str() + ":cpb_res");
        auto itcp = cache.find(ks.str() + ":cpb_prl");
        auto itcf = cache.find(ks.str() + ":cpb_fus");
        auto itfz = cache.find(ks.str() + ":fused");
        if (it != cache.end() && itr != cache.end() && itc != cache.end() && itcr != cache.end() &&
            itcp != cache.end() && itcf != cache.end() && (itfz != cache.end() || !D.fz_ps)) {
            D.bs_sel = it->second;
            D.remap = itr->second;
            D.cpb = itc->second;
            D.cpb_res = itcr->second;
            D.cpb_prl = itcp->second;
            D.cpb_fus = itcf->second;
            D.fz_on = D.fz_ps && itfz->second != 0;
            continue;
        }
        auto time_it = [&](auto run, int reps) -> float {
            run();
            if (hipEventRecord(e0, c->stream) != hipSuccess) return 1e30f;
            for (int r = 0; r < reps; r++) run();
            if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return 1e30f;
            float ms = 0;
            return hipEventElapsedTime(&ms, e0, e1) == hipSuccess ? ms : 1e30f;
        };
        double best = 1e30;
        int bq = 1, br = 1, bc = 1;
        if (c->gen) {
            // general macro mesh: workgroup size and block order of the class
            // pass (one node per thread); the residual takes the same shape
            for (int rq = 0; rq < 6; rq++) {
                const int q = rq % 3;
                D.remap = rq < 3 ? 1 : 0;
                VolGeom vg = vgeom(D, D.vd_all, c->n_tets, false, q);
                vg.list = D.qlist[0];
                vg.nlist = D.nqlist[0];
                const float ms = time_it([&]() {
                    launch_colour15(c->stream, vg, igeom(D, 0, D.n_ifc, nullptr, true), gen15(D, 0, true), D.r, D.b,
                                    c->d.omega);
                }, l >= 6 ? 5 : 20);
                if (ms < best) {
                    best = ms;
                    bq = q;
                    br = D.remap;
                }
            }
            D.bs_sel = bq;
            D.remap = br;
            D.cpb = D.cpb_res = D.cpb_prl = D.cpb_fus = 1;
            cache[ks.str()] = bq;
            cache[ks.str() + ":remap"] = br;
            cache[ks.str() + ":cpb"] = 1;
            cache[ks.str() + ":cpb_res"] = 1;
            cache[ks.str() + ":cpb_prl"] = 1;
            cache[ks.str() + ":cpb_fus"] = 1;
            launch_fill<double>(c->stream, D.r, D.n_slots, 0.0);
            continue;
        }
        for (int rq = 0; rq < 12; rq++) {
            const int q = rq % 3;
            D.remap = (rq / 3) % 2 == 0 ? 1 : 0;
            D.cpb = rq < 6 ? 1 : 4;
            const VolGeom vg = vgeom(D, D.vd_all, c->n_tets, false, q, 0);
            const IfcGeom ig = igeom(D, 0, D.n_ifc_red, nullptr, false);
            auto run = [&]() {
                if (c->mixed)
                    launch_colour<float>(c->stream, vg, ig, D.r32, D.b32, weights<float>(D), c->vk, D.h, c->d.omega,
                                         false, false);
                else
                    launch_colour<double>(c->stream, vg, ig, D.r, D.b, weights<double>(D), c->vk, D.h, c->d.omega,
                                          false, false);
            };
            run();
            HIPCHK(hipEventRecord(e0, c->stream));
            const int reps = l >= 6 ? 5 : 20;
            for (int r = 0; r < reps; r++) run();
            HIPCHK(hipEventRecord(e1, c->stream));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                bq = q;
                br = D.remap;
                bc = D.cpb;
            }
        }
        D.bs_sel = bq;
        D.remap = br;
        D.cpb = bc;
        cache[ks.str()] = bq;
        cache[ks.str() + ":remap"] = br;
        cache[ks.str() + ":cpb"] = bc;
        // nodes per thread of the residual (norm form), of the prolongation
        // (black nodes, as in the cycle) and of the red pass that adds the
        // correction, at that workgroup size and block order; the scratch
        // vectors r of this level and of the next coarser one stand in for
        // u and the coarse correction
        const int reps = l >= 6 ? 5 : 20;
        float tr[2], tp[2], tf[2];
        const LevelDev &Dc = c->lev[l - 1];
        for (int qc = 0; qc < 2; qc++) {
            VolGeom vg = vgeom(D, D.vd_all, c->n_tets, false);
            vg.cpb = qc ? 4 : 1;
            VolGeom vgb = vgeom(D, D.vd_all, c->n_tets, false, -1, 1);
            vgb.cpb = vg.cpb;
            VolGeom vgr = vgeom(D, D.vd_all, c->n_tets, false, -1, 0);
            vgr.cpb = vg.cpb;
            tr[qc] = time_it([&]() {
                if (c->mixed)
                    launch_residual<float, float>(c->stream, vg, igeom(D, 0, D.n_ifc, nullptr, false), D.r32, D.b32,
                                                  weights<float>(D), c->vk, D.h, (float *)nullptr, c->partial[0]);
                else
                    launch_residual<double, double>(c->stream, vg, igeom(D, 0, D.n_ifc, nullptr, false), D.r, D.b,
                                                    weights<double>(D), c->vk, D.h, (double *)nullptr, c->partial[0]);
            }, reps);
            tp[qc] = time_it([&]() {
                const IfcGeom igb = igeom(D, D.n_ifc_red, D.n_ifc, nullptr, true);
                if (c->mixed)
                    launch_prolong<float>(c->stream, vgb, Dc.vd_all, Dc.rowC, Dc.M, igb, D.prl, Dc.r32, D.r32);
                else
                    launch_prolong<double>(c->stream, vgb, Dc.vd_all, Dc.rowC, Dc.M, igb, D.prl, Dc.r, D.r);
            }, reps);
            tf[qc] = time_it([&]() {
                const IfcGeom igr = igeom(D, 0, D.n_ifc_red, nullptr, true);
                if (c->mixed) {
                    Prol<float> pr;
                    pr.vdc = Dc.vd_all;
                    pr.cC = Dc.rowC;
                    pr.Mc = Dc.M;
                    pr.prl = D.prl;
                    pr.ec = Dc.r32;
                    launch_colour_prol<float>(c->stream, vgr, igr, D.r32, D.b32, weights<float>(D), c->vk, D.h,
                                              c->d.omega, pr);
                } else {
                    Prol<double> pr;
                    pr.vdc = Dc.vd_all;
                    pr.cC = Dc.rowC;
                    pr.Mc = Dc.M;
                    pr.prl = D.prl;
                    pr.ec = Dc.r;
                    launch_colour_prol<double>(c->stream, vgr, igr, D.r, D.b, weights<double>(D), c->vk, D.h,
                                               c->d.omega, pr);
                }
            }, reps);
        }
        D.cpb_res = tr[1] < tr[0] ? 4 : 1;
        D.cpb_prl = tp[1] < tp[0] ? 4 : 1;
        D.cpb_fus = tf[1] < tf[0] ? 4 : 1;
        cache[ks.str() + ":cpb_res"] = D.cpb_res;
        cache[ks.str() + ":cpb_prl"] = D.cpb_prl;
        cache[ks.str() + ":cpb_fus"] = D.cpb_fus;
        // two sweeps as a fused pair (through the level's second buffer)
        // against two sweeps of two colour passes each, from the scratch
        // vector r; the cycles use the pair only where it is faster
        if (D.fz_ps && (c->mixed ? D.u32alt != nullptr : D.ualt != nullptr)) {
            HView<double> V64 = global_view<double>(*c, false, 0);
            HView<float> V32 = global_view<float>(*c, false, 0);
            V64.lv[l].u = D.r;
            V32.lv[l].u = D.r32;
            V64.timed = V32.timed = false;
            const float t_pair = time_it([&]() {
                if (c->mixed)
                    smooth<float>(*c, V32, l, 2, false, c->stream, nullptr, nullptr, nullptr, true);
                else
                    smooth<double>(*c, V64, l, 2, false, c->stream, nullptr, nullptr, nullptr, true);
            }, reps);
            const float t_plain = time_it([&]() {
                if (c->mixed)
                    for (int q = 0; q < 2; q++) sweep<float>(*c, V32, l, false, c->stream);
                else
                    for (int q = 0; q < 2; q++) sweep<double>(*c, V64, l, false, c->stream);
            }, reps);
            D.fz_on = t_pair < t_plain;
            cache[ks.str() + ":fused"] = D.fz_on ? 1 : 0;
        }
        // scratch vector used for timing goes back to zero
        launch_fill<double>(c->stream, D.r, D.n_slots, 0.0);
        if (c->mixed) launch_fill<float>(c->stream, D.r32, D.n_slots, 0.0f);
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    CHKLAUNCH();
    HIPCHK(hipStreamSynchronize(c->stream));
    if (cache_path) {
        std::ofstream o(cache_path);
        for (auto &kv : cache) o << kv.first << " " << kv.second << "\n";
    }
    return HHGR_OK;
}

int hhgr_debug_op(hhgr_ctx *c, int op, int l, const double *in0, const double *in1, double *out) {
    if (!c || !in0 || !out) return fail(HHGR_EINVAL, "null argument");
    const bool class_op = c->gen && op >= 9 && op <= 23;
    const bool fused_op = !c->gen && (op == 9 || op == 10);
    if (l < c->Lc || l > c->L || op < 0 || (op > 7 && !class_op && !fused_op))
        return fail(HHGR_EINVAL, "bad op or level");
    if (fused_op && !fused_ok(*c, global_view<double>(*c, false, 0), l, true))
        return fail(HHGR_EINVAL, "no fused sweeps on this level of this context");
    if (c->gen && (op == 1 || op == 2)) return fail(HHGR_EINVAL, "general_geometry: class passes are op 8 + class mask");
    if ((op == 4 || op == 5) && l <= c->Lc) return fail(HHGR_EINVAL, "transfer needs level > coarse_level");
    if ((op == 6 || op == 7) && l != c->Lc) return fail(HHGR_EINVAL, "coarse solve needs level = coarse_level");
    if ((op <= 3 || op == 5 || class_op || fused_op) && !in1) return fail(HHGR_EINVAL, "null second input");
    if (c->vk && !c->coeff_set) return fail(HHGR_ESTATE, "no coefficient set");
    if (c->gen && !c->geom_set && op != 4 && op != 5) return fail(HHGR_ESTATE, "no geometry set");
    if (op == 7 && !c->dense_coarse) return fail(HHGR_EINVAL, "no dense coarsest-level inverse in this context");
    if (op == 6 && c->mesh) return fail(HHGR_EINVAL, "an unstructured macro mesh solves its coarsest level densely (op 7)");
    invalidate_graph(*c);
    hipStream_t s = c->stream;
    auto to_slots = [&](const double *user, double *vec, LevelDev &D) { hhgr::to_slots(*c, D, user, vec, s); };
    auto to_user = [&](const double *vec, double *user, LevelDev &D) { hhgr::to_user(*c, D, vec, user, s); };
    LevelDev &D = c->lev[l];
    const VolGeom vint = vgeom(D, D.vd_all, c->n_tets, false);
    const Weights<double> w = weights<double>(D);
    if (c->gen && (op == 0 || op == 3 || op == 6 || op == 7 || class_op)) {
        if (op == 0) {
            to_slots(in0, D.u, D);
            to_slots(in1, D.b, D);
            launch_residual15(s, vint, igeom(D, 0, D.n_ifc, nullptr, false), gen15(D, -1, false), D.u, D.b, D.r,
                              nullptr);
            to_user(D.r, out, D);
        } else if (op == 6) {
            to_slots(in0, D.b, D);
            launch_coarse_pcg15(s, c->cn, c->cslot, c->ccol15, c->cval15, nullptr, D.b, D.u, c->cptr, c->cidx,
                                kCoarseRtol, kCoarseMaxit, c->citers);
            to_user(D.u, out, D);
        } else if (op == 7) {
            to_slots(in0, D.b, D);
            launch_coarse_dense<double>(s, c->cn, c->cslot, c->cinv, D.b, D.u, c->cptr, c->cidx);
            to_user(D.u, out, D);
        } else {
            const int mask = op == 3 ? 15 : op - 8;
            to_slots(in0, D.u, D);
            to_slots(in1, D.b, D);
            for (int q = 0; q < 4; q++) {
                if (!((mask >> q) & 1)) continue;
                VolGeom vg = vint;
                vg.list = D.qlist[q];
                vg.nlist = D.nqlist[q];
                launch_colour15(s, vg, igeom(D, 0, D.n_ifc, nullptr, true), gen15(D, q, true), D.u, D.b, c->d.omega);
            }
            to_user(D.u, out, D);
        }
        op = -1;  // done
    }
    switch (op) {
    case 0:
        to_slots(in0, D.u, D);
        to_slots(in1, D.b, D);
        launch_residual<double, double>(s, vint, igeom(D, 0, D.n_ifc, nullptr, false), D.u, D.b, w, c->vk, D.h, D.r,
                                        nullptr);
        to_user(D.r, out, D);
        break;
    case 1:
    case 2:
    case 3:
        to_slots(in0, D.u, D);
        to_slots(in1, D.b, D);
        for (int colour = 0; colour < 2; colour++) {
            if (!((op == 3) || (op == 1 && colour == 0) || (op == 2 && colour == 1))) continue;
            const IfcGeom ig = igeom(D, colour == 0 ? 0 : D.n_ifc_red, colour == 0 ? D.n_ifc_red : D.n_ifc, nullptr, true);
            launch_colour<double>(s, vgeom(D, D.vd_all, c->n_tets, false, -1, colour), ig, D.u, D.b, w, c->vk, D.h,
                                  c->d.omega, false, false);
        }
        to_user(D.u, out, D);
        break;
    case 4: {
        LevelDev &Dc = c->lev[l - 1];
        to_slots(in0, D.r, D);
        launch_restrict<double>(s, vgeom(Dc, Dc.vd_all, c->n_tets, false), D.vd_all, D.rowC,
                                igeom(Dc, 0, Dc.n_ifc, nullptr, false), Dc.rst, D.r, Dc.b);
        to_user(Dc.b, out, Dc);
        break;
    }
    case 5: {
        LevelDev &Dc = c->lev[l - 1];
        to_slots(in0, Dc.u, Dc);
        to_slots(in1, D.u, D);
        launch_prolong<double>(s, vint, Dc.vd_all, Dc.rowC, Dc.M, igeom(D, 0, D.n_ifc, nullptr, true), D.prl, Dc.u,
                               D.u);
        to_user(D.u, out, D);
        break;
    }
    case 6:
        to_slots(in0, D.b, D);
        launch_coarse_pcg<double>(s, c->cn, c->cslot, c->ccol, c->cval, nullptr, D.b, D.u, c->cptr, c->cidx,
                                  kCoarseRtol, kCoarseMaxit, c->citers);
        to_user(D.u, out, D);
        break;
    case 7:
        to_slots(in0, D.b, D);
        launch_coarse_dense<double>(s, c->cn, c->cslot, c->cinv, D.b, D.u, c->cptr, c->cidx);
        to_user(D.u, out, D);
        break;
    case 9:
    case 10: {
        // two sweeps as a fused pair (op 10: the first from u = 0)
        to_slots(in0, D.u, D);
        to_slots(in1, D.b, D);
        HView<double> V = global_view<double>(*c, false, 0);
        smooth<double>(*c, V, l, 2, op == 10, s, nullptr, nullptr, nullptr, true);
        to_user(D.u, out, D);
        break;
    }
    }
    CHKLAUNCH();
    HIPCHK(hipStreamSynchronize(s));
    return HHGR_OK;
}

// ---------------------------------------------------------------------------
// batch: members' steps as parallel branches of one captured graph
// ---------------------------------------------------------------------------
int hhgr_batch_create(hhgr_ctx **ctxs, int n, void *hip_stream, hhgr_batch **out) {
    if (!out) return fail(HHGR_EINVAL, "null output");
    *out = nullptr;
    if (!ctxs || n < 1) return fail(HHGR_EINVAL, "need at least one member");
    for (int q = 0; q < n; q++) {
        if (!ctxs[q]) return fail(HHGR_EINVAL, "null member");
        for (int p = 0; p < q; p++)
            if (ctxs[p] == ctxs[q]) return fail(HHGR_EINVAL, "a context appears twice in the batch");
    }
    hhgr_batch *b = new hhgr_batch();
    b->ctx.assign(ctxs, ctxs + n);
    b->stream = (hipStream_t)hip_stream;
    b->branch.resize(n);
    b->branch2.resize(n);
    b->ev.resize(n + 1);
    b->evl.resize(2 * n);
    b->dd.resize(n);
    auto bail = [&](const char *what) {
        hhgr_batch_destroy(b);
        return fail(HHGR_EHIP, what);
    };
    if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) return bail("stream create");
    for (int q = 0; q < n; q++)
        if (hipStreamCreateWithFlags(&b->branch[q], hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&b->branch2[q], hipStreamNonBlocking) != hipSuccess)
            return bail("stream create");
    for (auto *evs : {&b->ev, &b->evl})
        for (auto &e : *evs)
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return bail("event create");
    if (hipHostMalloc((void **)&b->hnorm, sizeof(double) * n, hipHostMallocDefault) != hipSuccess)
        return bail("pinned host allocation");
    *out = b;
    return HHGR_OK;
}

void hhgr_batch_destroy(hhgr_batch *b) {
    if (!b) return;
    if (b->stream) hipStreamSynchronize(b->stream);
    if (b->gexec) hipGraphExecDestroy(b->gexec);
    for (auto *ss : {&b->branch, &b->branch2})
        for (auto s : *ss)
            if (s) hipStreamDestroy(s);
    if (b->cap) hipStreamDestroy(b->cap);
    for (auto *evs : {&b->ev, &b->evl})
        for (auto e : *evs)
            if (e) hipEventDestroy(e);
    if (b->hnorm) hipHostFree(b->hnorm);
    delete b;
}

int hhgr_batch_arm_dd(hhgr_batch *b, int member, const int *tets, int n_tets, int n_intact, int n_local) {
    if (!b) return fail(HHGR_EINVAL, "null batch");
    if (member < 0 || member >= (int)b->ctx.size()) return fail(HHGR_EINVAL, "member index out of range");
    std::vector<int> ft;
    int rc = dd_check(*b->ctx[member], tets, n_tets, n_intact, n_local, ft);
    if (rc) return rc;
    BatchDD &d = b->dd[member];
    d.armed = true;
    d.tets = ft;
    d.n_intact = n_intact;
    d.n_local = n_local;
    d.step = 0;
    return HHGR_OK;
}

// mode bits of a member in one batch step
enum { kModeMasked = 1, kModeLocal = 2, kModeFinal = 4 };

int hhgr_batch_run(hhgr_batch *b, double rel_tol, int max_cycles, hhgr_report *reps) {
    if (!b) return fail(HHGR_EINVAL, "null batch");
    const int n = (int)b->ctx.size();
    std::vector<double> rel(n, 0.0);
    std::vector<int> cyc(n, 0), active;
    for (int q = 0; q < n; q++) {
        int rc = check_ready(b->ctx[q]);
        if (rc) return rc;
    }
    // armed recoveries: masks, local hierarchies, restored ghosts (eager, synchronous)
    for (int q = 0; q < n; q++)
        if (b->dd[q].armed) {
            invalidate_graph(*b->ctx[q]);
            int rc = dd_setup(*b->ctx[q], b->dd[q].tets);
            if (rc) return rc;
            b->dd[q].step = 0;
        }
    // initial residuals (and FP32 right-hand sides of mixed members)
    for (int q = 0; q < n; q++) {
        hhgr_ctx *c = b->ctx[q];
        HView<double> V = global_view<double>(*c, false, 0);
        if (c->mixed)
            prime_mixed(*c, b->stream);
        else
            finest_residual<double>(*c, V, (double *)nullptr, b->stream, c->dnorm);
        HIPCHK(hipMemcpyAsync(b->hnorm + q, c->dnorm, sizeof(double), hipMemcpyDeviceToHost, b->stream));
    }
    CHKLAUNCH();
    HIPCHK(hipStreamSynchronize(b->stream));
    auto in_dd = [&](int q) { return b->dd[q].armed && b->dd[q].step < std::max(b->dd[q].n_intact, 1); };
    for (int q = 0; q < n; q++) {
        rel[q] = b->ctx[q]->bnorm > 0 ? std::sqrt(std::max(b->hnorm[q], 0.0)) / b->ctx[q]->bnorm : 0.0;
        if (reps && reps[q].history && reps[q].history_cap > 0) reps[q].history[0] = rel[q];
        if ((rel[q] > rel_tol || in_dd(q)) && max_cycles > 0) active.push_back(q);
    }
    while (!active.empty()) {
        // (member, mode) signature of this step; the graph is re-captured when it changes
        std::vector<int> sig;
        for (int q : active) {
            int mode = 0;
            if (in_dd(q)) {
                const BatchDD &d = b->dd[q];
                if (d.step < d.n_intact) mode |= kModeMasked;
                if (d.step == 0) mode |= kModeLocal;
                if (d.step == std::max(d.n_intact, 1) - 1) mode |= kModeFinal;
            }
            sig.push_back(q);
            sig.push_back(mode);
        }
        // the step graph holds every member's cycle (and a recovering member's
        // intact-side cycle); local recovery cycles run beside the graph launch
        // on the member's second stream, forked and joined by events
        auto in_graph = [](int mode) { return mode == 0 || (mode & kModeMasked) || !(mode & kModeLocal); };
        if (sig != b->sig_in_graph || !b->gexec) {
            if (b->gexec) hipGraphExecDestroy(b->gexec);
            b->gexec = nullptr;
            hipGraph_t g = nullptr;
            HIPCHK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
            HIPCHK(hipEventRecord(b->ev[0], b->cap));
            for (size_t a = 0; a < active.size(); a++) {
                const int q = sig[2 * a], mode = sig[2 * a + 1];
                if (!in_graph(mode)) continue;
                hhgr_ctx *c = b->ctx[q];
                hipStream_t s = b->branch[q];
                hipStreamWaitEvent(s, b->ev[0], 0);
                if (mode == 0) {
                    HView<double> V64 = global_view<double>(*c, false, 0);
                    if (c->mixed) {
                        HView<float> V32 = global_view<float>(*c, false, 0);
                        step_mixed(*c, V64, V32, s, 0);
                    } else {
                        step_fp64(*c, V64, s, 0);
                    }
                } else {
                    if (mode & kModeMasked) dd_intact_step(*c, s, b->dd[q].step == 0, true, 0);
                    if ((mode & kModeFinal) && !(mode & kModeLocal)) dd_final_norm(*c, s);
                }
                hipMemcpyAsync(b->hnorm + q, c->dnorm, sizeof(double), hipMemcpyDeviceToHost, s);
                hipEventRecord(b->ev[1 + q], s);
                hipStreamWaitEvent(b->cap, b->ev[1 + q], 0);
            }
            hipError_t ce = hipStreamEndCapture(b->cap, &g);
            if (ce != hipSuccess) return fail(HHGR_EHIP, std::string("batch capture: ") + hipGetErrorString(ce));
            ce = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
            hipGraphDestroy(g);
            if (ce != hipSuccess) return fail(HHGR_EHIP, std::string("batch instantiate: ") + hipGetErrorString(ce));
            b->sig_in_graph = sig;
        }
        // local cycles of recoveries starting now, concurrent with the graph:
        // forked before the graph launch, launched after it (the host then
        // launches the many small local kernels while the graph runs)
        for (size_t a = 0; a < active.size(); a++) {
            const int q = sig[2 * a], mode = sig[2 * a + 1];
            if (!(mode & kModeLocal)) continue;
            HIPCHK(hipEventRecord(b->evl[2 * q], b->stream));
            HIPCHK(hipStreamWaitEvent(b->branch2[q], b->evl[2 * q], 0));
        }
        HIPCHK(hipGraphLaunch(b->gexec, b->stream));
        for (size_t a = 0; a < active.size(); a++) {
            const int q = sig[2 * a], mode = sig[2 * a + 1];
            if (!(mode & kModeLocal)) continue;
            dd_local(*b->ctx[q], b->dd[q].n_local, b->branch2[q]);
            HIPCHK(hipEventRecord(b->evl[2 * q + 1], b->branch2[q]));
        }
        for (size_t a = 0; a < active.size(); a++) {
            const int q = sig[2 * a], mode = sig[2 * a + 1];
            if (!(mode & kModeLocal)) continue;
            HIPCHK(hipStreamWaitEvent(b->stream, b->evl[2 * q + 1], 0));
            if (mode & kModeFinal) {
                hhgr_ctx *c = b->ctx[q];
                dd_final_norm(*c, b->stream);
                HIPCHK(hipMemcpyAsync(b->hnorm + q, c->dnorm, sizeof(double), hipMemcpyDeviceToHost, b->stream));
            }
        }
        CHKLAUNCH();
        HIPCHK(hipStreamSynchronize(b->stream));
        std::vector<int> next;
        for (size_t a = 0; a < active.size(); a++) {
            const int q = sig[2 * a], mode = sig[2 * a + 1];
            // during a recovery the norm is that of the intact part's residual;
            // a step without an intact cycle (local recovery only) is not a cycle
            rel[q] = b->ctx[q]->bnorm > 0 ? std::sqrt(std::max(b->hnorm[q], 0.0)) / b->ctx[q]->bnorm : 0.0;
            if (mode == 0 || (mode & kModeMasked)) {
                cyc[q]++;
                if (reps && reps[q].history && cyc[q] < reps[q].history_cap) reps[q].history[cyc[q]] = rel[q];
            }
            if (mode != 0) {
                b->dd[q].step++;
                if (mode & kModeFinal) {
                    dd_end(*b->ctx[q]);
                    b->dd[q].armed = false;
                }
            }
            const bool more = in_dd(q) || (rel[q] > rel_tol && std::isfinite(rel[q]));
            if (more && (cyc[q] < max_cycles || in_dd(q))) next.push_back(q);
        }
        active.swap(next);
    }
    // a recovery cut short by max_cycles: masks off, the member stays as it is
    for (int q = 0; q < n; q++)
        if (b->dd[q].armed) {
            dd_end(*b->ctx[q]);
            b->dd[q].armed = false;
        }
    bool all = true;
    for (int q = 0; q < n; q++) {
        if (reps) {
            reps[q].cycles = cyc[q];
            reps[q].rel_res = rel[q];
        }
        all = all && rel[q] <= rel_tol;
    }
    return all ? HHGR_OK : fail(HHGR_ENOCONV, "some batch members did not converge");
}

}  // extern "C"

// ----------------------------------------------------------------------------
// Solve without device allocation (hhgr_solve_static)
// ----------------------------------------------------------------------------
// The whole workspace of one solve lives in this file-scope device array.
// Every GPU the library runs on holds its own copy until the process ends.
// Host code never uses the array's name as an address: the device address of
// each GPU's copy comes from hipGetSymbolAddress, once per device.
namespace {
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
constexpr int kStaticMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
struct StaticScratch {
    std::mutex m;          // held for a whole hhgr_solve_static call on the device
    void *ptr = nullptr;   // device address of this device's copy of scratch
};
StaticScratch g_static[kStaticMaxDevices];
}  // namespace

extern "C" {

int hhgr_solve_static(const hhgr_desc *desc, const double *dev_rhs, int kind, double rel_tol, int max_cycles,
                      double *dev_u, hhgr_report *report, void *hip_stream) {
    if (!desc || !dev_rhs || !dev_u) return fail(HHGR_EINVAL, "null argument");
    if (desc->variable_coeff || desc->general_geometry)
        return fail(HHGR_EINVAL, "hhgr_solve_static takes k = 1 on the unit cube only");
    if (kind != HHGR_RHS_LOAD && kind != HHGR_RHS_NODAL_F && kind != HHGR_RHS_DIRICHLET)
        return fail(HHGR_EINVAL, "bad rhs kind");
    if (max_cycles < 0) return fail(HHGR_EINVAL, "negative max_cycles");
    size_t need = 0;
    int rc = hhgr_workspace_bytes(desc, &need);
    if (rc) return rc;
    if (need > kStaticScratchBytes)
        return fail(HHGR_EINVAL, "problem needs " + std::to_string(need) + " bytes of workspace; the static scratch of "
                                     "hhgr_solve_static holds " + std::to_string(kStaticScratchBytes));
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kStaticMaxDevices) return fail(HHGR_EINVAL, "device ordinal out of range");
    StaticScratch &S = g_static[dev];
    std::lock_guard<std::mutex> lock(S.m);
    if (!S.ptr) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || (reinterpret_cast<uintptr_t>(p) & 255) != 0) return fail(HHGR_EHIP, "static scratch address");
        S.ptr = p;
    }
    // the context carves S.ptr and clears every vector it reads (zero slot,
    // Dirichlet ghosts, partial sums, counters), so the previous call's
    // contents do not matter
    hhgr_ctx *c = nullptr;
    rc = create_ctx(desc, nullptr, S.ptr, kStaticScratchBytes, hip_stream, false, &c);
    if (rc) return rc;
    rc = hhgr_set_rhs(c, dev_rhs, kind);
    hhgr_report rep{0, 0.0, nullptr, 0};
    if (report) rep = *report;
    int src = rc ? rc : hhgr_solve(c, rel_tol, max_cycles, &rep);
    if (report && !rc) {
        report->cycles = rep.cycles;
        report->rel_res = rep.rel_res;
    }
    if (src == HHGR_OK || src == HHGR_ENOCONV) {
        const std::string keep = g_err;
        rc = hhgr_get_solution(c, dev_u);
        if (!rc && hipStreamSynchronize(c->stream) != hipSuccess) rc = fail(HHGR_EHIP, "synchronise");
        if (!rc && src == HHGR_ENOCONV) g_err = keep;
        if (!rc) rc = src;
    } else {
        rc = src;
    }
    hhgr_destroy(c);
    return rc;
}

}  // extern "C"
