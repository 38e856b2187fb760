/*
 * hhgr.h -- C ABI of the MI355X hierarchical-hybrid-grid (HHG) multigrid
 * library with fault recovery (Huber, Gmeiner, Ruede, Wohlmuth, "Resilience
 * for Multigrid Software at the Extreme Scale").
 *
 * Problem (Sec. 2.1, eqs. (1)-(2)): -div(k grad u) = f on the unit cube with
 * u = 0 on its boundary, conforming P1 finite elements on a hierarchy of
 * uniformly refined tetrahedral meshes.  The base mesh splits the cube into
 * n^3 subcubes, each into 6 Kuhn tetrahedra (the macro tetrahedra, one per
 * process in the paper); level L is L uniform refinements of it, so a level
 * has N = n 2^L cells per axis and h = 1/N.  The paper's coarsest level, with
 * one inner node per macro tetrahedron, is level 2 here.
 *
 * Data orders seen by callers
 *   vectors  (FP64, length (N-1)^3): interior grid node (x,y,z), 1 <= x,y,z <= N-1,
 *            at index (x-1) + (N-1)*((y-1) + (N-1)*(z-1)), x fastest;
 *   elements (FP64, length 6 N^3): element 6*cell + perm, cell = cx + N*(cy + N*cz)
 *            is its lowest corner and perm indexes its axis steps in the order
 *            (0,1,2),(0,2,1),(1,0,2),(1,2,0),(2,0,1),(2,1,0);
 *   macro tetrahedra: tet id = 6*subcube + perm in the same way on the n^3 grid.
 *
 * Memory and streams
 *   The caller owns every device buffer: the workspace handed to hhgr_create
 *   (size from hhgr_workspace_bytes) and all vectors.  The library borrows the
 *   workspace for the lifetime of the context and never allocates device
 *   memory; it allocates a few bytes of pinned host memory per context for
 *   residual read-back.  Work is enqueued on the stream given at creation;
 *   calls that return a host scalar synchronise that stream.  Device pointers
 *   passed to a call must stay valid until that stream reaches the call.
 *
 * Errors
 *   Every int-returning call returns HHGR_OK or a negative code; no exception
 *   crosses the ABI.  hhgr_last_error() returns a thread-local description of
 *   the last failure on the calling thread.
 */
#ifndef HHGR_H
#define HHGR_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hhgr_ctx hhgr_ctx;
typedef struct hhgr_batch hhgr_batch;

enum {
    HHGR_OK = 0,
    HHGR_EINVAL = -1,  /* bad argument: level, tet id, null pointer, size */
    HHGR_ENOMEM = -2,  /* workspace smaller than hhgr_workspace_bytes */
    HHGR_EHIP = -3,    /* a HIP runtime call failed */
    HHGR_ESTATE = -4,  /* call not valid in the current state (e.g. no right-hand side yet) */
    HHGR_ENOCONV = -5  /* max_cycles reached before the tolerance; outputs still filled */
};

enum { HHGR_FP64 = 0, HHGR_MIXED = 1 };
enum { HHGR_RHS_LOAD = 0, HHGR_RHS_NODAL_F = 1, HHGR_RHS_DIRICHLET = 2 };

/* Solver description.  hhgr_desc_default fills the defaults shown. */
typedef struct {
    int n_sub;          /* subcubes per axis (>= 1); 6 n^3 macro tetrahedra            */
    int level;          /* finest level L, coarse_level+1 <= L <= 9                      */
    int coarse_level;   /* coarsest level, default 2 (Sec. 2.1: one inner node per tet) */
    int nu_pre;         /* pre-smoothing sweeps, default 2                              */
    int nu_post;        /* post-smoothing sweeps, default 1                             */
    double omega;       /* SOR factor of the red-black smoother, default 1.25 (1 = GS)  */
    int precision;      /* HHGR_FP64 or HHGR_MIXED (FP32 cycle, FP64 refinement)        */
    int variable_coeff; /* 0: k = 1; 1: per-element k from hhgr_set_coeff               */
    int max_faults;     /* faulty tetrahedra recoverable at once, 0..8, default 8       */
    int general_geometry; /* 0: the unit cube; 1: moved macro vertices from
                             hhgr_set_geometry, default 0                        */
} hhgr_desc;

/* Convergence report.  history (optional, caller-owned, history_cap entries)
 * receives ||b - A u|| / ||b|| before the first and after every cycle. */
typedef struct {
    int cycles;
    double rel_res;
    double *history;
    int history_cap;
} hhgr_report;

void hhgr_desc_default(hhgr_desc *desc);

/* Size in bytes of the device workspace a context with this description
 * needs.  Host-only, no HIP calls.  EINVAL for an invalid description. */
int hhgr_workspace_bytes(const hhgr_desc *desc, size_t *bytes);

/* Mesh and level setup (Sec. 2.1; Sec. 3.1 data structures): builds the macro
 * mesh, the volume/face/edge/vertex containers of every level with their ghost
 * copies, and uploads the index tables into dev_ws (device memory of at least
 * hhgr_workspace_bytes bytes, 256-byte aligned), all on hip_stream (a
 * hipStream_t, NULL = default stream).  The solution starts at zero.
 * EINVAL/ENOMEM/EHIP on failure; *out is then NULL. */
int hhgr_create(const hhgr_desc *desc, void *dev_ws, size_t ws_bytes, void *hip_stream, hhgr_ctx **out);
void hhgr_destroy(hhgr_ctx *ctx);

/* Sizes: interior unknowns (N-1)^3, macro tetrahedra 6 n^3, elements 6 N^3. */
int hhgr_sizes(const hhgr_ctx *ctx, long long *n_dofs, int *n_tets, long long *n_elems);

/* General macro meshes (Sec. 3.1: unstructured macro mesh, each macro
 * element refined regularly): needs general_geometry = 1.  host_xyz (host
 * memory, read during the call) holds the positions of the (n+1)^3 macro
 * vertices, vertex (x,y,z) at 3*(x + (n+1)*(y + (n+1)*z)) + {0,1,2}; the
 * connectivity stays the Kuhn split of the cube described above, every
 * macro tetrahedron is refined regularly and mapped affinely (so a refined
 * node is the midpoint of its parent edge) and the operator of level l is the
 * P1 stiffness matrix assembled in physical coordinates.  With k = 1 an
 * affine element has a constant stencil, so every node of one primitive
 * (tetrahedron interior, face, edge, vertex) shares one 15-point stencil;
 * these are computed on the host and uploaded (with k = 1 and at most 512
 * coarsest unknowns, also the dense inverse of the coarsest-level matrix,
 * which the cycles then apply as on the cube).  With variable_coeff = 1 the
 * element coefficients of hhgr_set_coeff (element order above; coarse levels
 * take the mean of the 8 children) weight the element matrices, and the GPU
 * computes per-node stencils on every level and the coarsest-level matrix
 * (after both calls, in either order).  The smoother colours the nodes in the
 * 4 classes (x+y+z) mod 4, which no 15-point stencil couples to themselves; a
 * sweep visits classes 0, 1, 2, 3.  Vectors keep the grid-node order above;
 * HHGR_RHS_DIRICHLET takes the boundary values g at the moved boundary nodes
 * and sets b_i = -sum of A_ij g_j over the boundary neighbours j (after this
 * call, and after hhgr_set_coeff with variable_coeff = 1; ESTATE otherwise).
 * Cycles, solves and recoveries return ESTATE until this call.  EINVAL for
 * an inverted or degenerate macro tetrahedron (the context keeps its previous
 * geometry); may be called again to move the vertices (a right-hand side set
 * from Dirichlet data or nodal values before is not recomputed).  The recoveries work as on the cube; the intact side of a
 * Dirichlet-Neumann recovery takes the 15-point entries assembled over the
 * elements of intact macro tetrahedra.  HHGR_RHS_NODAL_F, hhgr_mass_apply and
 * hhgr_adjoint_grad use the consistent P1 mass matrix and the element
 * matrices of the moved elements (after this call); hhgr_autotune times the
 * class pass (after this call); mixed precision keeps FP32 copies of the
 * stencil tables for its FP32 cycle. */
int hhgr_set_geometry(hhgr_ctx *ctx, const double *host_xyz);

/* Unstructured macro meshes (Sec. 3.1: the macro mesh is an arbitrary
 * conforming tetrahedral mesh whose elements are refined regularly; eq. (2)
 * assembled with P1 elements in physical coordinates, k = 1 until
 * hhgr_mesh_set_coeff).  Host arrays,
 * read during the call: nv vertices (host_xyz, 3 doubles each) and nt
 * tetrahedra (host_tets, 4 vertex ids each).  Every tetrahedron lists its
 * vertices by a proper 4-colouring of the mesh: a vertex takes the same
 * position 0..3 in every tetrahedron that contains it (the smoother's 4
 * classes are (sum of colour x weight) mod 4 of a refined node, which no
 * element edge couples to themselves; a sweep visits classes 0, 1, 2, 3).
 * Closure node (i,j,k) of a tetrahedron has the weights (m-i-j-k, i, j, k),
 * m = 2^level, on its vertices 0..3.  The Dirichlet boundary (u = 0) is the
 * union of the faces that belong to one tetrahedron.  Vectors list the
 * interior nodes in this order: interior macro vertices by id; interior
 * edges (a < b, by vertex pair) with their nodes by the weight of b; interior
 * faces (a < b < c) with their nodes by the weight of c, then of b; then the
 * interiors of the tetrahedra by id, each in plane k, row j, i order (i, j,
 * k >= 1, i + j + k < m).  desc: level, coarse_level (>= 2), nu_pre, nu_post,
 * omega, precision and max_faults as above; n_sub and general_geometry are
 * ignored; variable_coeff must be 0 (a coefficient per tetrahedron comes
 * with hhgr_mesh_set_coeff).  The coarsest level is solved with a
 * dense inverse (at most 2048 unknowns).  A mesh context takes hhgr_set_rhs
 * with HHGR_RHS_LOAD, HHGR_RHS_NODAL_F (b = M f with the consistent P1 mass
 * matrix of the finest level, per-master rows like the stiffness) or
 * HHGR_RHS_DIRICHLET (Laplace's equation with the boundary values g of
 * eq. (1): the vector holds g at the boundary nodes in the order of
 * hhgr_mesh_boundary, and b = -A_IB g, the stiffness couplings of the
 * interior nodes to the boundary nodes applied to g),
 * hhgr_mass_apply, hhgr_adjoint_grad (dJ/df, and dJ/dk per macro
 * tetrahedron), hhgr_set_solution/get_solution, hhgr_vcycle,
 * hhgr_solve, hhgr_inject_fault, hhgr_recover_local, hhgr_recover_dd (its
 * masked coarsest level with a dense inverse of the unfrozen unknowns,
 * computed on the host for each fault set), hhgr_recover_dn (the intact
 * side's master rows summed over the elements of intact tetrahedra and its
 * coarsest level inverted densely, both on the host for each fault set;
 * eq. (5)), hhgr_set_graph, the hhgr_batch_* calls, hhgr_autotune (the
 * class pass, as on a general mesh; cache entries keyed by a hash of the
 * vertex and tetrahedron lists), hhgr_mesh_set_coeff,
 * hhgr_kernel_timing/stats and hhgr_debug_op (ops 0, 3 to 5, 7, 8 + class
 * mask); every other call returns EINVAL for it.  hhgr_sizes reports the
 * interior unknowns, nt and nt 8^level.  EINVAL for a mesh that is not
 * coloured that way, has an id out of range, a vertex in no tetrahedron, a
 * flat tetrahedron, a face of more than two tetrahedra, or a coarsest level
 * that is too large; the message names the reason. */
int hhgr_mesh_workspace_bytes(const hhgr_desc *desc, int nv, const double *host_xyz, int nt, const int *host_tets,
                              size_t *bytes);
/* Boundary nodes of the finest level of a mesh context (the nodes where u is
 * prescribed, eq. (1)): their number, and (host_xyz, optional, host memory
 * of 3 * n doubles) their positions, in this order: boundary macro vertices
 * by id, then boundary edges (a < b) with their nodes by the weight of b,
 * then boundary faces (a < b < c) with their nodes by the weight of c, then
 * of b.  EINVAL for a context not made by hhgr_create_mesh. */
int hhgr_mesh_boundary(const hhgr_ctx *ctx, long long *n_boundary, double *host_xyz);
/* Coefficient of eq. (2) constant on each macro tetrahedron of a mesh
 * context (Sec. 2.1: other scalar elliptic problems; HHG keeps one stencil
 * per macro element): host_k holds nt values > 0, read during the call
 * (NULL: back to k = 1).  Every level takes the same k (the mean of 8
 * children of a constant), so the volume stencils are scaled per
 * tetrahedron, and the host sums the master rows, the coarsest-level
 * operator (inverted again densely) and the Dirichlet couplings A_IB again
 * with k times each element matrix.  Later cycles, solves, recoveries
 * (the intact side of Dirichlet-Neumann keeps its k), batches and
 * HHGR_RHS_DIRICHLET use it; a right-hand side set before is not
 * recomputed.  hhgr_adjoint_grad gives dJ/df and dJ/dk per tetrahedron.
 * EINVAL for a context
 * not made by hhgr_create_mesh or a k that is not positive and finite. */
int hhgr_mesh_set_coeff(hhgr_ctx *ctx, const double *host_k);
int hhgr_create_mesh(const hhgr_desc *desc, int nv, const double *host_xyz, int nt, const int *host_tets,
                     void *dev_ws, size_t ws_bytes, void *hip_stream, hhgr_ctx **out);

/* Right-hand side of eq. (2) from a device vector in the vector order above.
 * kind = HHGR_RHS_LOAD: the vector is the load vector b itself;
 * kind = HHGR_RHS_NODAL_F: the vector holds nodal values of f (zero on the
 * boundary) and b = M f with the consistent P1 mass matrix;
 * kind = HHGR_RHS_DIRICHLET: Laplace's equation with inhomogeneous Dirichlet
 * data, eq. (1) (f = 0, u = g on the boundary).  The vector holds the values
 * of the (N+1)^3 grid nodes, node (x,y,z), 0 <= x,y,z <= N, at index
 * x + (N+1)*(y + (N+1)*z); only the boundary entries (g) are read.  The known
 * boundary values are moved to the right-hand side as in eq. (2):
 * b_i = sum over the axis neighbours j of node i on the boundary of
 * w_ij g_j, w_ij = h for k = 1, else the edge weight of the coefficient set
 * by hhgr_set_coeff (ESTATE if none was set; a later hhgr_set_coeff does not
 * update b).  The solution holds the interior values; g is not stored.
 * Every kind records ||b|| as the reference for relative residuals. */
int hhgr_set_rhs(hhgr_ctx *ctx, const double *dev_vec, int kind);

/* Per-element diffusion coefficient of -div(k grad u) = f, one of the
 * "other scalar elliptic problems" the model problem generalises to (Sec. 2.1,
 * after eq. (1)); the operator of eq. (2) becomes the P1 stiffness matrix
 * weighted by k on every element.  dev_k: device, element order, length
 * 6 N^3, positive; needs variable_coeff = 1 (ESTATE otherwise).  Coarse
 * levels use the mean over the 8 children of each coarse element (the
 * Galerkin-consistent choice).  EINVAL for a null pointer. */
int hhgr_set_coeff(hhgr_ctx *ctx, const double *dev_k);

/* Copy a device vector into / out of the solver's containers (vector order).
 * hhgr_set_solution with dev_u = NULL sets u = 0 (a fill, no copy). */
int hhgr_set_solution(hhgr_ctx *ctx, const double *dev_u);
int hhgr_get_solution(const hhgr_ctx *ctx, double *dev_u);

/* n multigrid V-cycles of the correction scheme (Sec. 2.1): red-black SOR
 * smoothing, restriction by the transpose of linear interpolation, the
 * coarsest level solved to round-off (Jacobi-PCG to a relative residual of
 * 1e-14; with k = 1 on the cube and at most 512 coarsest unknowns, a dense
 * inverse factorised on the host at hhgr_create), linear interpolation of
 * the correction.
 * With precision = HHGR_MIXED one cycle is one refinement step
 * u += V32(b - A u) with the residual and update in FP64.  rel_res_out
 * (optional) receives ||b - A u|| / ||b||.  ESTATE without a right-hand side. */
int hhgr_vcycle(hhgr_ctx *ctx, int n, double *rel_res_out);

/* V-cycles until ||b - A u|| <= rel_tol ||b|| or max_cycles (Sec. 2.2: the
 * solution process continues with multigrid cycles).  ENOCONV if max_cycles
 * was reached; the report is filled either way. */
int hhgr_solve(hhgr_ctx *ctx, double rel_tol, int max_cycles, hhgr_report *report);

/* Fail-stop fault of one macro tetrahedron (Sec. 2.2): the unknowns strictly
 * inside it are lost and set to zero (re-initialisation).  Its ghost copies of
 * face/edge/vertex values are lost too; the face, edge and vertex containers
 * (stored redundantly, eq. (4)) survive, and the copies are filled again
 * from them at once, as the ghost update of Sec. 3.1 would do before any
 * stencil reads them.  So a cycle run right after the fault (the do-nothing
 * strategy) sees the interface values and a zero interior.  Only between
 * cycles.  EINVAL for a bad tet id. */
int hhgr_inject_fault(hhgr_ctx *ctx, int tet);

/* Local recovery (Sec. 4; Alg. 1 a)): restores the tetrahedron's
 * ghost copies from the surviving interface containers (eq. (4), row 4), sets
 * its interior to zero and runs n_cycles multigrid V-cycles restricted to the
 * tetrahedron's interior on every level for A_FF u_F = f_F - A_FG u_G (a
 * Dirichlet problem; coarsest level: one unknown, solved exactly).
 * local_rel_res_out (optional) receives the local residual relative to the
 * local right-hand side.  The restore, the residuals and the cycles run as
 * one captured HIP graph, captured on the first call for a (tet, n_cycles)
 * pair and replayed while later calls repeat that pair (calls that change
 * launch shapes or run other recoveries drop it).  ESTATE without a
 * right-hand side or with coarse_level != 2. */
int hhgr_recover_local(hhgr_ctx *ctx, int tet, int n_cycles, double *local_rel_res_out);

/* Dirichlet-Dirichlet recovery (Alg. 1): for the listed faulty tetrahedra,
 * restores their ghost copies and zeroes their interiors, then runs
 * concurrently (two streams) n_intact V-cycles on the intact part with the
 * closures of the faulty tetrahedra frozen as Dirichlet data and n_local
 * local V-cycles on each faulty tetrahedron.  Returns after both finish.
 * n_tets <= max_faults.  ESTATE without a right-hand side or with
 * coarse_level != 2. */
int hhgr_recover_dd(hhgr_ctx *ctx, const int *tets, int n_tets, int n_intact, int n_local);

/* Dirichlet-Neumann recovery (Sec. 4.3, Alg. 2, eq. (5)) of the listed faulty
 * tetrahedra (after hhgr_inject_fault on them).  The intact side cycles on a
 * Neumann problem: the stiffness assembled over the elements of intact
 * macro tetrahedra only (the sub-stencils of eq. (5)), with the interface
 * nodes free and, on the interface, the static Neumann data A^I u of the
 * data at call time (lambda of Alg. 2).  The faulty side starts from zero and
 * runs local Dirichlet cycles with boundary values from the interface.
 * n_intact rounds: eta local cycles with the interface values of the start
 * of the round, concurrently (second stream) with one intact cycle.  Faces,
 * edges and vertices inside the faulty region stay as stored.  Returns after
 * both sides finish; later cycles use the whole problem again.  Same
 * argument rules as hhgr_recover_dd (eta in place of n_local). */
int hhgr_recover_dn(hhgr_ctx *ctx, const int *tets, int n_tets, int n_intact, int eta);

/* Adjoint gradients for J = 1/2 ||u - u_obs||^2 with A(k) u = M f: given
 * dev_g = u - u_obs (device, vector order), solves A lambda = g with the same
 * multigrid (A is symmetric) to rel_tol and returns dJ/df = M lambda (vector
 * order) and, when variable_coeff = 1 and dev_dJdk != NULL,
 * dJ/dk_T = -lambda^T A_T u (element order, A_T the unit-coefficient element
 * stiffness).  On a mesh context dev_dJdk (optional) receives one value per
 * macro tetrahedron, dJ/dk_t = -lambda^T A_t u with A_t the unit-coefficient
 * stiffness of its elements (the coefficient of hhgr_mesh_set_coeff, or
 * k = 1).  Dirichlet nodes count with u = lambda = 0.  The current solution
 * u is used and left unchanged.  ENOCONV if the adjoint solve did not
 * converge in max_cycles. */
int hhgr_adjoint_grad(hhgr_ctx *ctx, const double *dev_g, double rel_tol, int max_cycles, double *dev_dJdf,
                      double *dev_dJdk);

/* Apply the consistent P1 mass matrix M to a device vector (vector order). */
int hhgr_mass_apply(hhgr_ctx *ctx, const double *dev_x, double *dev_y);

/* Batched solves: independent contexts (each with its own workspace and
 * right-hand side) run their V-cycles as concurrent branches of captured HIP
 * graphs on hip_stream, one graph launch per step of all members; every
 * member stops at its own tolerance.  The batch borrows the contexts (each at
 * most once); members may be cube, general or unstructured-mesh contexts.
 * reps: one report per member (may be NULL).
 *
 * hhgr_batch_arm_dd arms a Dirichlet-Dirichlet recovery (Sec. 4.2, Alg. 1)
 * of the listed faulty tetrahedra of one member (after hhgr_inject_fault on
 * them) for the next hhgr_batch_run: its first max(n_intact, 1) steps are
 * intact-side cycles with the faulty closures frozen as Dirichlet data, and
 * its n_local local cycles run on a stream of their own beside the first
 * step's graph launch, concurrently with every other member's work; the
 * member then goes on with global cycles.  Intact-side cycles count as cycles and their history
 * entries are the intact part's residual; with n_intact = 0 the first step
 * (local cycles only) is not counted.  Same argument rules as hhgr_recover_dd. */
int hhgr_batch_create(hhgr_ctx **ctxs, int n, void *hip_stream, hhgr_batch **out);
int hhgr_batch_arm_dd(hhgr_batch *batch, int member, const int *tets, int n_tets, int n_intact, int n_local);
int hhgr_batch_run(hhgr_batch *batch, double rel_tol, int max_cycles, hhgr_report *reps);
void hhgr_batch_destroy(hhgr_batch *batch);

/* Execution controls.  use_graph = 1 replays a captured HIP graph per
 * V-cycle instead of launching kernel by kernel (same results). */
int hhgr_set_graph(hhgr_ctx *ctx, int use_graph);

/* Autotuner: times the candidate workgroup sizes, nodes per thread and block
 * orders of the volume colour pass on every level and keeps the fastest per
 * (level, precision, coefficient mode) for all volume kernels of that level;
 * at that shape it then picks 1 or 4 nodes per thread separately for the
 * residual, the prolongation and the red post-smoothing pass that adds the
 * coarse-grid correction.  cache_path (optional) is a text file read before
 * and written after tuning, keyed by device name.  Enqueues work and
 * synchronises. */
int hhgr_autotune(hhgr_ctx *ctx, const char *cache_path);

/* The tuning choices in use on `level` (any output may be NULL): workgroup
 * size of the volume kernels, XCD-contiguous block order (1) or hardware
 * order (0), nodes per thread (1 or 4).  EINVAL for a level outside
 * coarse_level+1..level. */
int hhgr_tuning_info(const hhgr_ctx *ctx, int level, int *block_size, int *xcd_order, int *nodes_per_thread);

/* Fused red-black sweeps (cube, k = 1; Sec. 2.1 smoother): on level
 * `level` (coarse_level < level <= level of the context), on = 1 runs every
 * two consecutive sweeps of an unmasked cycle as a pair of single-launch
 * sweeps (red and black of each plane in one kernel, planes marched through
 * LDS), on = 0 as two colour passes per sweep.  The iterates are the same
 * bit for bit.  hhgr_autotune sets it where the pair is faster; this call
 * overrides that (e.g. to time the kernel).  EINVAL where the fused kernel
 * cannot take the level (general or unstructured meshes, variable k, levels
 * with fewer than 8 segments per edge). */
int hhgr_set_fused_sweeps(hhgr_ctx *ctx, int level, int on);

/* Set the tuning choices of one level (level = 0: every level above the
 * coarsest) instead of the autotuner's: block_size 128, 256 or 512,
 * xcd_order 0 or 1, nodes_per_thread 1 or 4.  Results do not depend on them.
 * EINVAL for other values. */
int hhgr_set_tuning(hhgr_ctx *ctx, int level, int block_size, int xcd_order, int nodes_per_thread);

/* Kernel timing for roofline reports: when enabled, every launch of the
 * finest-level volume smoother kernel is bracketed by HIP events on the
 * context's stream; hhgr_kernel_stats returns the launch count and mean
 * duration in milliseconds since the last enable and the bytes the
 * algorithm moves per launch. */
int hhgr_kernel_timing(hhgr_ctx *ctx, int enable);
int hhgr_kernel_stats(hhgr_ctx *ctx, long long *launches, double *mean_ms, double *algorithmic_bytes);

/* Single multigrid operator on level `level`, for testing the kernels one by
 * one (Sec. 2.1 components).  Vectors are device FP64 in the vector order of
 * that level (length (N_level - 1)^3).  Clobbers the context's vectors on the
 * levels involved.
 *   op 0: out = in1 - A in0                     (residual)
 *   op 1: out = in0 after one red SOR pass with right-hand side in1
 *   op 2: out = in0 after one black pass;  op 3: red then black (one sweep)
 *   op 4: out (level-1) = P^T in0               (restriction)
 *   op 5: out = in1 + P in0, in0 on level-1     (interpolation and correction)
 *   op 6: out = coarsest-level PCG solution for right-hand side in0 (level = coarse_level)
 *   op 7: the same through the dense inverse (EINVAL where the context has none)
 * With general_geometry = 1, ops 1 and 2 are EINVAL, op 3 is one 4-class
 * sweep and op 8 + mask (mask 1..15) runs the passes of the classes whose
 * bits are set in mask, lowest class first.
 * EINVAL for a bad op/level combination. */
int hhgr_debug_op(hhgr_ctx *ctx, int op, int level, const double *in0, const double *in1, double *out);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc, such as tight serving loops or harnesses that forbid it): a
 * variant of hhgr_create + hhgr_set_rhs + hhgr_solve + hhgr_get_solution that
 * brings no workspace.  The workspace of the solve lives in a static device
 * array of the library, 64 MiB per GPU (held by every GPU the library runs
 * on until the process ends); problems whose hhgr_workspace_bytes exceed it
 * are rejected with EINVAL and a message naming both sizes (64 MiB holds
 * n_sub = 2 up to level 5 and n_sub = 1 up to level 6).  k = 1 on the unit
 * cube only (variable_coeff and general_geometry must be 0, else EINVAL).
 * dev_rhs: device vector of the given kind, as for hhgr_set_rhs; dev_u:
 * device vector (vector order) that receives the solution, computed from
 * u = 0 with V-cycles until ||b - A u|| <= rel_tol ||b|| or max_cycles
 * (ENOCONV; dev_u and the report are still filled).  report (optional, as
 * for hhgr_solve) receives the cycle count, the final relative residual and
 * the history.  Work runs on hip_stream and the call synchronises it before
 * returning; it allocates no device or pinned memory and creates no streams,
 * events or graphs.  Every call on one GPU uses that GPU's one array and
 * keeps nothing from the previous call; calls from several host threads on
 * the same device are serialised by the library.  Work of the caller that
 * overlaps a call on the same GPU must not touch the array (it cannot: its
 * address is not exported). */
int hhgr_solve_static(const hhgr_desc *desc, const double *dev_rhs, int kind, double rel_tol, int max_cycles,
                      double *dev_u, hhgr_report *report, void *hip_stream);

const char *hhgr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HHGR_H */
