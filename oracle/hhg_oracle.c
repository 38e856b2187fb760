/*
 * hhg_oracle.c -- CPU oracle for the resilient hierarchical-hybrid-grid (HHG)
 * multigrid method of Huber, Gmeiner, Ruede and Wohlmuth, "Resilience for
 * Multigrid Software at the Extreme Scale".
 *
 * TEST INFRASTRUCTURE ONLY.  This library is loaded by the tests, by the smoke
 * check and by the benchmark's CPU-baseline leg; the product path never links,
 * loads or calls it, and it shares no code, header or table with the GPU path.
 *
 * It is deliberately plain and slow:
 *   - the macro mesh is a list of tetrahedra (each subcube of the unit cube
 *     split into 6 Kuhn tetrahedra), refined by Bey's regular refinement
 *     (Sec. 2.1: hierarchy T_0 ... T_L built by uniform refinement);
 *   - P1 stiffness and mass matrices are assembled element by element into CSR
 *     with the Dirichlet nodes eliminated (Sec. 2.1, eq. (2));
 *   - multigrid is a textbook V-cycle on those CSR matrices: red-black SOR
 *     smoothing, residual, restriction by the transpose of linear
 *     interpolation, prolongation by linear interpolation, Jacobi-PCG on the
 *     coarsest level (Sec. 2.1);
 *   - a fault zeroes the unknowns strictly inside one macro tetrahedron
 *     (Sec. 2.2); local recovery solves the Dirichlet problem on that
 *     tetrahedron with multigrid restricted to its interior (Sec. 4, Alg. 1 a));
 *     the Dirichlet-Dirichlet intact cycles freeze the closure of the faulty
 *     tetrahedra (Alg. 1 b));
 *   - mixed precision runs the same V-cycle in FP32 inside an FP64 residual
 *     correction loop; gradients use the adjoint solution.
 *
 * Level numbering: level 0 is the macro mesh (n^3 subcubes, 6 n^3 tetrahedra),
 * level l has N = n 2^l cells per axis and h = 1/N.  The paper's coarsest
 * level (one inner node per macro tetrahedron, Sec. 2.1) is level 2 here.
 *
 * Orders shared with callers: interior node (x,y,z) in grid units has index
 * (x-1) + (N-1)((y-1) + (N-1)(z-1)); an element has index 6*cell + perm,
 * cell = cx + N(cy + N cz) its lowest corner and perm the position of its
 * axis sequence in (0,1,2),(0,2,1),(1,0,2),(1,2,0),(2,0,1),(2,1,0).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef int64_t i64;

#define MAXLEV 12

static void die(const char *msg) {
    fprintf(stderr, "hhg_oracle: %s\n", msg);
    abort();
}
static void *xmalloc(size_t n) {
    void *p = malloc(n ? n : 1);
    if (!p) die("out of memory");
    return p;
}
static void *xcalloc(size_t n, size_t s) {
    void *p = calloc(n ? n : 1, s ? s : 1);
    if (!p) die("out of memory");
    return p;
}
static double now_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

/* ------------------------------------------------------------------------- */
/* Sparse matrices                                                            */
/* ------------------------------------------------------------------------- */
typedef struct {
    i64 nrow, ncol;
    i64 *ptr;
    int *col;
    double *val;
} csr;

static void csr_free(csr *m) {
    free(m->ptr);
    free(m->col);
    free(m->val);
    memset(m, 0, sizeof(*m));
}

/* y = A x */
static void spmv(const csr *A, const double *x, double *y) {
#pragma omp parallel for schedule(static)
    for (i64 i = 0; i < A->nrow; i++) {
        double s = 0.0;
        for (i64 q = A->ptr[i]; q < A->ptr[i + 1]; q++) s += A->val[q] * x[A->col[q]];
        y[i] = s;
    }
}

/* r = b - A x */
static void residual(const csr *A, const double *x, const double *b, double *r) {
#pragma omp parallel for schedule(static)
    for (i64 i = 0; i < A->nrow; i++) {
        double s = b[i];
        for (i64 q = A->ptr[i]; q < A->ptr[i + 1]; q++) s -= A->val[q] * x[A->col[q]];
        r[i] = s;
    }
}

static double dot(i64 n, const double *a, const double *b) {
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (i64 i = 0; i < n; i++) s += a[i] * b[i];
    return s;
}

static double norm2(i64 n, const double *a) { return sqrt(dot(n, a, a)); }

static csr csr_transpose(const csr *A) {
    csr T;
    T.nrow = A->ncol;
    T.ncol = A->nrow;
    i64 nnz = A->ptr[A->nrow];
    T.ptr = xcalloc((size_t)T.nrow + 1, sizeof(i64));
    T.col = xmalloc((size_t)nnz * sizeof(int));
    T.val = xmalloc((size_t)nnz * sizeof(double));
    for (i64 q = 0; q < nnz; q++) T.ptr[A->col[q] + 1]++;
    for (i64 i = 0; i < T.nrow; i++) T.ptr[i + 1] += T.ptr[i];
    i64 *fill = xmalloc((size_t)T.nrow * sizeof(i64));
    memcpy(fill, T.ptr, (size_t)T.nrow * sizeof(i64));
    for (i64 i = 0; i < A->nrow; i++)
        for (i64 q = A->ptr[i]; q < A->ptr[i + 1]; q++) {
            i64 d = fill[A->col[q]]++;
            T.col[d] = (int)i;
            T.val[d] = A->val[q];
        }
    free(fill);
    return T;
}

/* Submatrix A[rows, cols]; rmap/cmap give the new index of an old one or -1. */
static csr csr_sub(const csr *A, const i64 *rmap, i64 nrow_new, const i64 *cmap, i64 ncol_new) {
    csr S;
    S.nrow = nrow_new;
    S.ncol = ncol_new;
    S.ptr = xcalloc((size_t)nrow_new + 1, sizeof(i64));
    for (i64 i = 0; i < A->nrow; i++) {
        if (rmap[i] < 0) continue;
        i64 c = 0;
        for (i64 q = A->ptr[i]; q < A->ptr[i + 1]; q++)
            if (cmap[A->col[q]] >= 0) c++;
        S.ptr[rmap[i] + 1] = c;
    }
    for (i64 i = 0; i < nrow_new; i++) S.ptr[i + 1] += S.ptr[i];
    S.col = xmalloc((size_t)S.ptr[nrow_new] * sizeof(int));
    S.val = xmalloc((size_t)S.ptr[nrow_new] * sizeof(double));
    for (i64 i = 0; i < A->nrow; i++) {
        if (rmap[i] < 0) continue;
        i64 d = S.ptr[rmap[i]];
        for (i64 q = A->ptr[i]; q < A->ptr[i + 1]; q++) {
            i64 c = cmap[A->col[q]];
            if (c < 0) continue;
            S.col[d] = (int)c;
            S.val[d] = A->val[q];
            d++;
        }
    }
    return S;
}

/* ------------------------------------------------------------------------- */
/* Mesh: macro mesh, Bey refinement, Kuhn/Freudenthal facts                   */
/* ------------------------------------------------------------------------- */
static const int PERM[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

static int perm_index(int a, int b, int c) {
    for (int q = 0; q < 6; q++)
        if (PERM[q][0] == a && PERM[q][1] == b && PERM[q][2] == c) return q;
    die("not an axis permutation");
    return -1;
}

static inline i64 vid(int N, i64 x, i64 y, i64 z) { return x + (i64)(N + 1) * (y + (i64)(N + 1) * z); }
static inline void vxyz(int N, i64 v, int *x, int *y, int *z) {
    *x = (int)(v % (N + 1));
    v /= (N + 1);
    *y = (int)(v % (N + 1));
    *z = (int)(v / (N + 1));
}
static inline i64 dof_xyz(int N, int x, int y, int z) {
    if (x <= 0 || y <= 0 || z <= 0 || x >= N || y >= N || z >= N) return -1;
    return (i64)(x - 1) + (i64)(N - 1) * ((i64)(y - 1) + (i64)(N - 1) * (z - 1));
}
static inline i64 dof_vid(int N, i64 v) {
    int x, y, z;
    vxyz(N, v, &x, &y, &z);
    return dof_xyz(N, x, y, z);
}

typedef struct {
    int N;
    double h;
    i64 ne;
    int *ev;    /* 4 vertex ids per element, listed along the element's Kuhn path */
    i64 *ecl;   /* cell-lexicographic element index of each element */
    double *k;  /* coefficient per element, cell-lexicographic order */
    int *par;   /* 2 parent vertex ids (previous level) per vertex */
    i64 ndof;
    int built;  /* A, diag, colours assembled */
    csr A, P, R, M;
    double *diag;
    i64 nred, nblack;
    i64 *red, *black;
    /* general geometry: colours (x+y+z) mod 4; red = classes 0 then 2 (the
     * first nred0 entries are class 0), black = classes 1 then 3 */
    i64 nred0, nblack1;
    double *xyz; /* vertex positions (3 per vertex) when the geometry is given */
    float *A32, *diag32;
    /* general macro mesh (vertex and tetrahedron lists): nodes of the level in
     * creation order; per node its user index (or -1 on the boundary) and its
     * key: up to 4 (macro vertex, weight) pairs, vertex ascending, -1 padded,
     * the weights its barycentric coordinates times 2^level */
    i64 nnode;
    i64 *dof, *node_of_dof;
    int *key;
} olevel;

typedef struct {
    int n_sub, L, Lc;
    int var_k;
    int geom; /* 1: vertex positions given, 4-colour smoother */
    olevel lev[MAXLEV];
    double setup_s;
    /* general macro mesh: macro vertices (colour = the position of the vertex
     * in the vertex list of each of its tetrahedra) and tetrahedra */
    int mesh, nv, nt;
    int *tet_v, *vcol;
} oproblem;

/* Macro mesh (Sec. 2.1, base mesh): each subcube c of the n^3 split becomes 6
 * Kuhn tetrahedra v0=c, v1=v0+e_p0, v2=v1+e_p1, v3=v2+e_p2; all subcubes are
 * translated copies, so the mesh is conforming.  Tet id = 6*cell + perm. */
static void macro_mesh(olevel *L0, int n) {
    L0->N = n;
    L0->h = 1.0 / n;
    L0->ne = 6 * (i64)n * n * n;
    L0->ev = xmalloc((size_t)L0->ne * 4 * sizeof(int));
    for (int cz = 0; cz < n; cz++)
        for (int cy = 0; cy < n; cy++)
            for (int cx = 0; cx < n; cx++)
                for (int p = 0; p < 6; p++) {
                    i64 e = 6 * (cx + (i64)n * (cy + (i64)n * cz)) + p;
                    int x[3] = {cx, cy, cz};
                    L0->ev[4 * e + 0] = (int)vid(n, x[0], x[1], x[2]);
                    for (int s = 0; s < 3; s++) {
                        x[PERM[p][s]] += 1;
                        L0->ev[4 * e + 1 + s] = (int)vid(n, x[0], x[1], x[2]);
                    }
                }
}

/* Bey's regular refinement (Sec. 2.1, uniform refinement): the 4 corner
 * tetrahedra plus the octahedron cut along the x02-x13 diagonal.  Children of
 * element e are stored at 8e..8e+7.  par[] records, for each fine vertex, the
 * coarse edge (a,b) it bisects, or (a,a) for an old vertex. */
static void refine(const olevel *C, olevel *F) {
    static const int CH[8][4] = {{0, 4, 5, 6}, {4, 1, 7, 8}, {5, 7, 2, 9}, {6, 8, 9, 3},
                                 {4, 5, 6, 8}, {4, 5, 7, 8}, {5, 6, 8, 9}, {5, 7, 8, 9}};
    /* node slots: 0..3 corners, 4=x01 5=x02 6=x03 7=x12 8=x13 9=x23 */
    static const int MID[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
    F->N = 2 * C->N;
    F->h = 1.0 / F->N;
    F->ne = 8 * C->ne;
    F->ev = xmalloc((size_t)F->ne * 4 * sizeof(int));
    i64 nv = (i64)(F->N + 1) * (F->N + 1) * (F->N + 1);
    F->par = xmalloc((size_t)nv * 2 * sizeof(int));
    for (i64 v = 0; v < 2 * nv; v++) F->par[v] = -1;
    for (i64 e = 0; e < C->ne; e++) {
        int cx[4][3];
        for (int a = 0; a < 4; a++) vxyz(C->N, C->ev[4 * e + a], &cx[a][0], &cx[a][1], &cx[a][2]);
        i64 node[10];
        int pa[10], pb[10];
        for (int a = 0; a < 4; a++) {
            node[a] = vid(F->N, 2 * cx[a][0], 2 * cx[a][1], 2 * cx[a][2]);
            pa[a] = pb[a] = C->ev[4 * e + a];
        }
        for (int s = 0; s < 6; s++) {
            int a = MID[s][0], b = MID[s][1];
            node[4 + s] = vid(F->N, cx[a][0] + cx[b][0], cx[a][1] + cx[b][1], cx[a][2] + cx[b][2]);
            pa[4 + s] = C->ev[4 * e + a];
            pb[4 + s] = C->ev[4 * e + b];
        }
        for (int s = 0; s < 10; s++) {
            int *pp = &F->par[2 * node[s]];
            int lo = pa[s] < pb[s] ? pa[s] : pb[s], hi = pa[s] < pb[s] ? pb[s] : pa[s];
            if (pp[0] < 0) {
                pp[0] = lo;
                pp[1] = hi;
            } else if (pp[0] != lo || pp[1] != hi) {
                die("inconsistent parents in refinement");
            }
        }
        for (int c = 0; c < 8; c++)
            for (int a = 0; a < 4; a++) F->ev[4 * (8 * e + c) + a] = (int)node[CH[c][a]];
    }
}

/* Every element is a Kuhn tetrahedron: consecutive vertices differ by distinct
 * unit axis steps.  Its cell is its first vertex and its permutation is the
 * step sequence.  Returns 0 if some element is not of that form. */
static int classify_elements(olevel *Lv) {
    Lv->ecl = xmalloc((size_t)Lv->ne * sizeof(i64));
    int ok = 1;
#pragma omp parallel for schedule(static) reduction(& : ok)
    for (i64 e = 0; e < Lv->ne; e++) {
        int x[4][3], ax[3];
        for (int a = 0; a < 4; a++) vxyz(Lv->N, Lv->ev[4 * e + a], &x[a][0], &x[a][1], &x[a][2]);
        int good = 1;
        for (int s = 0; s < 3; s++) {
            int d[3] = {x[s + 1][0] - x[s][0], x[s + 1][1] - x[s][1], x[s + 1][2] - x[s][2]};
            int nz = 0, which = -1;
            for (int c = 0; c < 3; c++) {
                if (d[c] == 1) {
                    nz++;
                    which = c;
                } else if (d[c] != 0) {
                    good = 0;
                }
            }
            if (nz != 1) good = 0;
            ax[s] = which;
        }
        if (good && (ax[0] == ax[1] || ax[0] == ax[2] || ax[1] == ax[2])) good = 0;
        if (!good) {
            ok = 0;
            Lv->ecl[e] = -1;
            continue;
        }
        i64 cell = x[0][0] + (i64)Lv->N * (x[0][1] + (i64)Lv->N * x[0][2]);
        Lv->ecl[e] = 6 * cell + perm_index(ax[0], ax[1], ax[2]);
    }
    return ok;
}

/* Element matrices in grid units (vertex coordinates are integers).  P1
 * stiffness scales like h and mass like h^3 under x -> h x, so the physical
 * matrices are h*K and h^3*Mm.  K_ab = |T| grad(l_a).grad(l_b) with the
 * barycentric gradients taken from the inverse of the edge matrix;
 * Mm_ab = |T| (1 + delta_ab) / 20 (consistent P1 mass). */
static void elem_mats(int N, const int *ev, double K[4][4], double Mm[4][4]) {
    int x[4][3];
    for (int a = 0; a < 4; a++) vxyz(N, ev[a], &x[a][0], &x[a][1], &x[a][2]);
    double J[3][3];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) J[r][c] = (double)(x[c + 1][r] - x[0][r]);
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                 J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                 J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (det == 0.0) die("degenerate element");
    double inv[3][3];
    inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    double g[4][3];
    for (int c = 0; c < 3; c++) {
        g[1][c] = inv[0][c];
        g[2][c] = inv[1][c];
        g[3][c] = inv[2][c];
        g[0][c] = -(inv[0][c] + inv[1][c] + inv[2][c]);
    }
    double vol = fabs(det) / 6.0;
    for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++) {
            K[a][b] = vol * (g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2]);
            Mm[a][b] = vol * (a == b ? 2.0 : 1.0) / 20.0;
        }
}

/* The same element matrices from physical vertex positions (general macro
 * meshes): no scaling afterwards. */
static void elem_mats_xyz(const double *xyz, const int *ev, double K[4][4], double Mm[4][4]) {
    double J[3][3];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) J[r][c] = xyz[3 * (i64)ev[c + 1] + r] - xyz[3 * (i64)ev[0] + r];
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                 J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                 J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (det == 0.0) die("degenerate element");
    double inv[3][3];
    inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    double g[4][3];
    for (int c = 0; c < 3; c++) {
        g[1][c] = inv[0][c];
        g[2][c] = inv[1][c];
        g[3][c] = inv[2][c];
        g[0][c] = -(inv[0][c] + inv[1][c] + inv[2][c]);
    }
    double vol = fabs(det) / 6.0;
    for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++) {
            K[a][b] = vol * (g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2]);
            Mm[a][b] = vol * (a == b ? 2.0 : 1.0) / 20.0;
        }
}

static double elem_volume_grid(int N, const int *ev) {
    int x[4][3];
    for (int a = 0; a < 4; a++) vxyz(N, ev[a], &x[a][0], &x[a][1], &x[a][2]);
    double J[3][3];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) J[r][c] = (double)(x[c + 1][r] - x[0][r]);
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                 J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                 J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    return fabs(det) / 6.0;
}

/* vertex -> elements adjacency, elements listed in increasing order */
static void vertex_adjacency(const olevel *Lv, i64 **off_out, int **lst_out) {
    i64 nv = (i64)(Lv->N + 1) * (Lv->N + 1) * (Lv->N + 1);
    i64 *off = xcalloc((size_t)nv + 1, sizeof(i64));
    for (i64 q = 0; q < 4 * Lv->ne; q++) off[Lv->ev[q] + 1]++;
    for (i64 v = 0; v < nv; v++) off[v + 1] += off[v];
    int *lst = xmalloc((size_t)(4 * Lv->ne) * sizeof(int));
    i64 *fill = xmalloc((size_t)nv * sizeof(i64));
    memcpy(fill, off, (size_t)nv * sizeof(i64));
    for (i64 e = 0; e < Lv->ne; e++)
        for (int a = 0; a < 4; a++) lst[fill[Lv->ev[4 * e + a]]++] = (int)e;
    free(fill);
    *off_out = off;
    *lst_out = lst;
}

/* Element-by-element assembly of the stiffness (which=0, scaled by the
 * element coefficient) or mass (which=1) matrix.  interior=1: rows and
 * columns are the interior nodes (Dirichlet nodes eliminated with value 0,
 * eq. (2)); interior=0: all vertices.  Rows are filled in parallel, each row
 * summing the local matrices of the elements that contain its vertex. */
#define ROWCAP 64
static csr assemble(const olevel *Lv, const double *kcoef, int which, int interior) {
    i64 *off;
    int *lst;
    vertex_adjacency(Lv, &off, &lst);
    const int N = Lv->N;
    i64 nv = (i64)(N + 1) * (N + 1) * (N + 1);
    i64 nrow = interior ? (i64)(N - 1) * (N - 1) * (N - 1) : nv;
    csr A;
    A.nrow = A.ncol = nrow;
    A.ptr = xcalloc((size_t)nrow + 1, sizeof(i64));
    const double scale = Lv->xyz ? 1.0 : which == 0 ? Lv->h : Lv->h * Lv->h * Lv->h;
    for (int pass = 0; pass < 2; pass++) {
        if (pass == 1) {
            for (i64 i = 0; i < nrow; i++) A.ptr[i + 1] += A.ptr[i];
            A.col = xmalloc((size_t)A.ptr[nrow] * sizeof(int));
            A.val = xmalloc((size_t)A.ptr[nrow] * sizeof(double));
        }
#pragma omp parallel for schedule(dynamic, 1024)
        for (i64 r = 0; r < nrow; r++) {
            i64 v;
            if (interior) {
                i64 t = r;
                int x = (int)(t % (N - 1)) + 1;
                t /= (N - 1);
                int y = (int)(t % (N - 1)) + 1;
                int z = (int)(t / (N - 1)) + 1;
                v = vid(N, x, y, z);
            } else {
                v = r;
            }
            int cols[ROWCAP];
            double vals[ROWCAP];
            int cnt = 0;
            for (i64 q = off[v]; q < off[v + 1]; q++) {
                i64 e = lst[q];
                const int *ev = &Lv->ev[4 * e];
                int a = -1;
                for (int s = 0; s < 4; s++)
                    if (ev[s] == v) a = s;
                double K[4][4], Mm[4][4];
                double ke = 1.0;
                if (pass == 1) {
                    if (Lv->xyz)
                        elem_mats_xyz(Lv->xyz, ev, K, Mm);
                    else
                        elem_mats(N, ev, K, Mm);
                    if (which == 0 && kcoef) ke = kcoef[Lv->ecl[e]];
                }
                for (int b = 0; b < 4; b++) {
                    i64 c = interior ? dof_vid(N, ev[b]) : ev[b];
                    if (c < 0) continue;
                    double add = pass == 1 ? scale * ke * (which == 0 ? K[a][b] : Mm[a][b]) : 0.0;
                    int s;
                    for (s = 0; s < cnt; s++)
                        if (cols[s] == c) break;
                    if (s == cnt) {
                        if (cnt == ROWCAP) die("row capacity exceeded");
                        cols[cnt] = (int)c;
                        vals[cnt] = 0.0;
                        cnt++;
                    }
                    vals[s] += add;
                }
            }
            if (pass == 0) {
                A.ptr[r + 1] = cnt;
            } else {
                /* insertion sort by column */
                for (int s = 1; s < cnt; s++) {
                    int c = cols[s];
                    double w = vals[s];
                    int t = s - 1;
                    while (t >= 0 && cols[t] > c) {
                        cols[t + 1] = cols[t];
                        vals[t + 1] = vals[t];
                        t--;
                    }
                    cols[t + 1] = c;
                    vals[t + 1] = w;
                }
                i64 d = A.ptr[r];
                for (int s = 0; s < cnt; s++) {
                    A.col[d + s] = cols[s];
                    A.val[d + s] = vals[s];
                }
            }
        }
    }
    free(off);
    free(lst);
    return A;
}

/* Linear interpolation from level l-1 to level l (Sec. 2.1, intergrid
 * transfer): an old vertex keeps its value, a new vertex takes the mean of the
 * two ends of the coarse edge it bisects.  interior=1 drops Dirichlet rows and
 * columns. */
static csr prolongation(const olevel *C, const olevel *F, int interior) {
    const int N = F->N;
    i64 nvf = (i64)(N + 1) * (N + 1) * (N + 1);
    i64 nvc = (i64)(C->N + 1) * (C->N + 1) * (C->N + 1);
    i64 nrow = interior ? F->ndof : nvf;
    csr P;
    P.nrow = nrow;
    P.ncol = interior ? C->ndof : nvc;
    P.ptr = xcalloc((size_t)nrow + 1, sizeof(i64));
    P.col = xmalloc((size_t)nrow * 2 * sizeof(int));
    P.val = xmalloc((size_t)nrow * 2 * sizeof(double));
    i64 d = 0;
    for (i64 r = 0; r < nrow; r++) {
        i64 v;
        if (interior) {
            i64 t = r;
            int x = (int)(t % (N - 1)) + 1;
            t /= (N - 1);
            int y = (int)(t % (N - 1)) + 1;
            int z = (int)(t / (N - 1)) + 1;
            v = vid(N, x, y, z);
        } else {
            v = r;
        }
        int a = F->par[2 * v], b = F->par[2 * v + 1];
        if (a < 0) die("vertex without parents");
        i64 ca = interior ? dof_vid(C->N, a) : a;
        i64 cb = interior ? dof_vid(C->N, b) : b;
        if (a == b) {
            if (ca >= 0) {
                P.col[d] = (int)ca;
                P.val[d] = 1.0;
                d++;
            }
        } else {
            i64 lo = ca < cb ? ca : cb, hi = ca < cb ? cb : ca;
            if (lo >= 0) {
                P.col[d] = (int)lo;
                P.val[d] = 0.5;
                d++;
            }
            if (hi >= 0) {
                P.col[d] = (int)hi;
                P.val[d] = 0.5;
                d++;
            }
        }
        P.ptr[r + 1] = d;
    }
    return P;
}

static void build_level_operators(oproblem *p, int l) {
    olevel *Lv = &p->lev[l];
    if (Lv->built) return;
    Lv->A = assemble(Lv, p->var_k ? Lv->k : NULL, 0, 1);
    Lv->diag = xmalloc((size_t)Lv->ndof * sizeof(double));
    for (i64 i = 0; i < Lv->ndof; i++) {
        Lv->diag[i] = 0.0;
        for (i64 q = Lv->A.ptr[i]; q < Lv->A.ptr[i + 1]; q++)
            if (Lv->A.col[q] == i) Lv->diag[i] = Lv->A.val[q];
    }
    /* red = even x+y+z, black = odd (grid units of this level).  With a
     * general geometry every edge of the mesh couples (x+y+z) classes that
     * differ by 1, 2 or 3, so the classes mod 4 are the colours: red holds
     * class 0 then class 2, black class 1 then class 3. */
    const int N = Lv->N;
    Lv->nred = Lv->nblack = 0;
    Lv->red = xmalloc((size_t)Lv->ndof * sizeof(i64));
    Lv->black = xmalloc((size_t)Lv->ndof * sizeof(i64));
    for (int pass = 0; pass < (p->geom ? 2 : 1); pass++) {
        for (i64 i = 0; i < Lv->ndof; i++) {
            i64 t = i;
            int x = (int)(t % (N - 1)) + 1;
            t /= (N - 1);
            int y = (int)(t % (N - 1)) + 1;
            int z = (int)(t / (N - 1)) + 1;
            const int c4 = (x + y + z) & 3;
            if (p->geom && (c4 >> 1) != pass) continue;
            if (((x + y + z) & 1) == 0)
                Lv->red[Lv->nred++] = i;
            else
                Lv->black[Lv->nblack++] = i;
        }
        if (pass == 0) {
            Lv->nred0 = Lv->nred;
            Lv->nblack1 = Lv->nblack;
        }
    }
    if (l > p->Lc) {
        Lv->P = prolongation(&p->lev[l - 1], Lv, 1);
        Lv->R = csr_transpose(&Lv->P);
    }
    Lv->built = 1;
}

/* ------------------------------------------------------------------------- */
/* Problem creation                                                           */
/* ------------------------------------------------------------------------- */
void ohhg_destroy(void *vp);

/* xyz_macro (optional): positions of the (n+1)^3 macro vertices, x fastest;
 * a refined vertex sits at the midpoint of the coarse edge it bisects (Bey's
 * refinement), so every macro tetrahedron is refined affinely. */
void *ohhg_create_geom(int n_sub, int L, int Lc, const double *k_fine, const double *xyz_macro) {
    if (n_sub < 1 || L < 1 || L >= MAXLEV || Lc < 1 || Lc > L) return NULL;
    double t0 = now_s();
    oproblem *p = xcalloc(1, sizeof(oproblem));
    p->n_sub = n_sub;
    p->L = L;
    p->Lc = Lc;
    p->var_k = k_fine != NULL;
    p->geom = xyz_macro != NULL;
    macro_mesh(&p->lev[0], n_sub);
    for (int l = 1; l <= L; l++) refine(&p->lev[l - 1], &p->lev[l]);
    if (p->geom) {
        const i64 nv0 = (i64)(n_sub + 1) * (n_sub + 1) * (n_sub + 1);
        p->lev[0].xyz = xmalloc((size_t)nv0 * 3 * sizeof(double));
        memcpy(p->lev[0].xyz, xyz_macro, (size_t)nv0 * 3 * sizeof(double));
        for (int l = 1; l <= L; l++) {
            olevel *C = &p->lev[l - 1], *F = &p->lev[l];
            const i64 nv = (i64)(F->N + 1) * (F->N + 1) * (F->N + 1);
            F->xyz = xmalloc((size_t)nv * 3 * sizeof(double));
            for (i64 v = 0; v < nv; v++)
                for (int a = 0; a < 3; a++)
                    F->xyz[3 * v + a] = 0.5 * (C->xyz[3 * (i64)F->par[2 * v] + a] + C->xyz[3 * (i64)F->par[2 * v + 1] + a]);
        }
    }
    for (int l = 0; l <= L; l++) {
        olevel *Lv = &p->lev[l];
        if (!classify_elements(Lv)) die("refined element is not a Kuhn tetrahedron");
        Lv->ndof = (i64)(Lv->N - 1) * (Lv->N - 1) * (Lv->N - 1);
        Lv->k = xmalloc((size_t)Lv->ne * sizeof(double));
    }
    /* coefficient: given on the finest level; on a coarser element it is the
     * mean over its 8 children, which makes the rediscretised coarse operator
     * the Galerkin product P^T A P. */
    olevel *F = &p->lev[L];
    for (i64 e = 0; e < F->ne; e++) F->k[e] = k_fine ? k_fine[e] : 1.0;
    for (int l = L - 1; l >= 0; l--) {
        olevel *C = &p->lev[l], *Fn = &p->lev[l + 1];
        for (i64 e = 0; e < C->ne; e++) {
            double s = 0.0;
            for (int c = 0; c < 8; c++) s += Fn->k[Fn->ecl[8 * e + c]];
            C->k[C->ecl[e]] = s / 8.0;
        }
    }
    for (int l = Lc; l <= L; l++) build_level_operators(p, l);
    p->setup_s = now_s() - t0;
    return p;
}

void *ohhg_create(int n_sub, int L, int Lc, const double *k_fine) { return ohhg_create_geom(n_sub, L, Lc, k_fine, NULL); }

void ohhg_destroy(void *vp) {
    oproblem *p = vp;
    if (!p) return;
    for (int l = 0; l < MAXLEV; l++) {
        olevel *Lv = &p->lev[l];
        free(Lv->ev);
        free(Lv->ecl);
        free(Lv->k);
        free(Lv->par);
        csr_free(&Lv->A);
        csr_free(&Lv->P);
        csr_free(&Lv->R);
        csr_free(&Lv->M);
        free(Lv->diag);
        free(Lv->red);
        free(Lv->black);
        free(Lv->xyz);
        free(Lv->A32);
        free(Lv->diag32);
        free(Lv->dof);
        free(Lv->node_of_dof);
        free(Lv->key);
    }
    free(p->tet_v);
    free(p->vcol);
    free(p);
}

int ohhg_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* number of OpenMP threads of later calls (timing of the CPU baseline) */
void ohhg_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

double ohhg_setup_seconds(void *vp) { return ((oproblem *)vp)->setup_s; }
long long ohhg_ndof(void *vp, int l) { return ((oproblem *)vp)->lev[l].ndof; }
long long ohhg_nelem(void *vp, int l) { return ((oproblem *)vp)->lev[l].ne; }
int ohhg_cells(void *vp, int l) { return ((oproblem *)vp)->lev[l].N; }

/* vertex positions of level l ((N+1)^3 x 3, x fastest); the grid points
 * (x/N, y/N, z/N) when no geometry was given */
void ohhg_positions(void *vp, int l, double *out) {
    olevel *Lv = &((oproblem *)vp)->lev[l];
    const int N = Lv->N;
    const i64 nv = (i64)(N + 1) * (N + 1) * (N + 1);
    for (i64 v = 0; v < nv; v++) {
        int x, y, z;
        vxyz(N, v, &x, &y, &z);
        const double g[3] = {(double)x / N, (double)y / N, (double)z / N};
        for (int a = 0; a < 3; a++) out[3 * v + a] = Lv->xyz ? Lv->xyz[3 * v + a] : g[a];
    }
}

/* element export: vertex ids (grid (N+1)^3 numbering) and cell-lex index */
void ohhg_elements(void *vp, int l, int *ev, long long *ecl) {
    olevel *Lv = &((oproblem *)vp)->lev[l];
    memcpy(ev, Lv->ev, (size_t)Lv->ne * 4 * sizeof(int));
    for (i64 e = 0; e < Lv->ne; e++) ecl[e] = Lv->ecl[e];
}

void ohhg_coeff(void *vp, int l, double *k) {
    olevel *Lv = &((oproblem *)vp)->lev[l];
    memcpy(k, Lv->k, (size_t)Lv->ne * sizeof(double));
}

double ohhg_volume_sum(void *vp, int l) {
    olevel *Lv = &((oproblem *)vp)->lev[l];
    double s = 0.0;
    for (i64 e = 0; e < Lv->ne; e++) s += elem_volume_grid(Lv->N, &Lv->ev[4 * e]);
    return s * Lv->h * Lv->h * Lv->h;
}

/* Freudenthal triangulation of the N^3 grid built independently (each cell
 * split into its 6 Kuhn tetrahedra); returns 1 if it equals the Bey-refined
 * element set as a set of vertex quadruples. */
static int cmp4(const void *a, const void *b) {
    const int *x = a, *y = b;
    for (int s = 0; s < 4; s++)
        if (x[s] != y[s]) return x[s] < y[s] ? -1 : 1;
    return 0;
}
static void sort4(int *v) {
    for (int s = 1; s < 4; s++) {
        int c = v[s], t = s - 1;
        while (t >= 0 && v[t] > c) {
            v[t + 1] = v[t];
            t--;
        }
        v[t + 1] = c;
    }
}
int ohhg_check_freudenthal(void *vp, int l) {
    olevel *Lv = &((oproblem *)vp)->lev[l];
    const int N = Lv->N;
    i64 ne = 6 * (i64)N * N * N;
    if (ne != Lv->ne) return 0;
    int *a = xmalloc((size_t)ne * 4 * sizeof(int));
    int *b = xmalloc((size_t)ne * 4 * sizeof(int));
    memcpy(a, Lv->ev, (size_t)ne * 4 * sizeof(int));
    i64 e = 0;
    for (int cz = 0; cz < N; cz++)
        for (int cy = 0; cy < N; cy++)
            for (int cx = 0; cx < N; cx++)
                for (int p = 0; p < 6; p++, e++) {
                    int x[3] = {cx, cy, cz};
                    b[4 * e] = (int)vid(N, x[0], x[1], x[2]);
                    for (int s = 0; s < 3; s++) {
                        x[PERM[p][s]]++;
                        b[4 * e + 1 + s] = (int)vid(N, x[0], x[1], x[2]);
                    }
                }
    for (i64 q = 0; q < ne; q++) {
        sort4(&a[4 * q]);
        sort4(&b[4 * q]);
    }
    qsort(a, (size_t)ne, 4 * sizeof(int), cmp4);
    qsort(b, (size_t)ne, 4 * sizeof(int), cmp4);
    int eq = memcmp(a, b, (size_t)ne * 4 * sizeof(int)) == 0;
    free(a);
    free(b);
    return eq;
}

/* ------------------------------------------------------------------------- */
/* General macro meshes from vertex and tetrahedron lists (Sec. 3.1: an       */
/* unstructured macro mesh, every macro element refined regularly)            */
/* ------------------------------------------------------------------------- */
/* Input: nv macro vertices (3 coordinates each) and nt tetrahedra (4 vertex
 * ids each).  The vertex order of every tetrahedron is its order for Bey's
 * refinement, and it must list the vertices by a proper 4-colouring of the
 * macro mesh: a vertex is at the same position (its colour 0..3) in every
 * tetrahedron it belongs to.  A refined node then has the colour class
 * (sum over macro vertices v of colour(v) x weight(v)) mod 4, weights being
 * its barycentric coordinates times 2^level; two nodes joined by a refined
 * edge always differ in class (an edge is parallel to a macro edge, whose
 * ends differ in colour, or is the octahedron diagonal x02-x13 of Bey's
 * rule, which changes the class by 2), so the 4 classes are independent sets
 * of the stiffness matrix and the smoother sweeps them in the order 0, 1, 2, 3.
 *
 * Boundary: the faces of exactly one tetrahedron; a node whose support (the
 * macro vertices with nonzero weight) lies in a boundary face is a Dirichlet
 * node (value 0).
 *
 * Order of the interior nodes (the vector order of callers): vertices by id;
 * then edges by their vertex pair (a < b), nodes by weight of b; then faces by
 * their vertex triple (a < b < c), nodes by weight of c, then of b; then
 * tetrahedra by id, nodes by weight of their vertex 3, then 2, then 1 (the
 * tetrahedron's own order). */

static int mesh_in_tet(const oproblem *p, const int *key, int tet, int closure);

/* (lo, hi) node pair -> midpoint node: open addressing */
typedef struct {
    i64 *k;
    i64 *v;
    i64 cap;
} pairmap;

static void pm_init(pairmap *m, i64 n) {
    m->cap = 16;
    while (m->cap < 2 * n) m->cap *= 2;
    m->k = xmalloc((size_t)m->cap * sizeof(i64));
    m->v = xmalloc((size_t)m->cap * sizeof(i64));
    for (i64 i = 0; i < m->cap; i++) m->k[i] = -1;
}
static i64 pm_get(pairmap *m, i64 a, i64 b, i64 *next) {
    const i64 lo = a < b ? a : b, hi = a < b ? b : a;
    const i64 key = lo * 4294967296LL + hi;
    i64 h = (i64)(((uint64_t)key * 0x9E3779B97F4A7C15ULL) >> 20) & (m->cap - 1);
    while (m->k[h] >= 0 && m->k[h] != key) h = (h + 1) & (m->cap - 1);
    if (m->k[h] < 0) {
        m->k[h] = key;
        m->v[h] = (*next)++;
    }
    return m->v[h];
}

/* key of the midpoint of nodes with keys ka, kb of the previous level: the
 * union of the supports, weights added (each key sums to 2^(l-1), the result
 * to 2^l) */
static void key_mid(const int *ka, const int *kb, int *out) {
    int v[8], w[8], n = 0;
    for (int s = 0; s < 2; s++) {
        const int *k = s ? kb : ka;
        for (int a = 0; a < 4 && k[2 * a] >= 0; a++) {
            int q = 0;
            while (q < n && v[q] != k[2 * a]) q++;
            if (q == n) {
                v[n] = k[2 * a];
                w[n++] = 0;
            }
            w[q] += k[2 * a + 1];
        }
    }
    if (n > 4) die("midpoint outside every macro tetrahedron");
    for (int a = 0; a < n; a++)
        for (int b = a + 1; b < n; b++)
            if (v[b] < v[a]) {
                int t = v[a];
                v[a] = v[b];
                v[b] = t;
                t = w[a];
                w[a] = w[b];
                w[b] = t;
            }
    for (int a = 0; a < 4; a++) {
        out[2 * a] = a < n ? v[a] : -1;
        out[2 * a + 1] = a < n ? w[a] : 0;
    }
}

static int key_size(const int *k) {
    int n = 0;
    while (n < 4 && k[2 * n] >= 0) n++;
    return n;
}

static int cmp_int3(const void *a, const void *b) {
    const int *x = a, *y = b;
    for (int q = 0; q < 3; q++)
        if (x[q] != y[q]) return x[q] < y[q] ? -1 : 1;
    return 0;
}

/* sorted unique list of the boundary faces (vertex triples, ascending) */
static int *boundary_faces(const oproblem *p, int *nbf) {
    const int nf = 4 * p->nt;
    int *f = xmalloc((size_t)nf * 3 * sizeof(int));
    for (int t = 0; t < p->nt; t++)
        for (int o = 0; o < 4; o++) {
            int q = 0;
            int *fr = &f[3 * (4 * t + o)];
            for (int r = 0; r < 4; r++)
                if (r != o) fr[q++] = p->tet_v[4 * t + r];
            for (int a = 0; a < 3; a++)
                for (int b = a + 1; b < 3; b++)
                    if (fr[b] < fr[a]) {
                        int tt = fr[a];
                        fr[a] = fr[b];
                        fr[b] = tt;
                    }
        }
    qsort(f, (size_t)nf, 3 * sizeof(int), cmp_int3);
    int *out = xmalloc((size_t)nf * 3 * sizeof(int));
    int n = 0;
    for (int i = 0; i < nf;) {
        int j = i;
        while (j < nf && cmp_int3(&f[3 * i], &f[3 * j]) == 0) j++;
        if (j - i == 1) memcpy(&out[3 * n++], &f[3 * i], 3 * sizeof(int));
        if (j - i > 2) die("a face belongs to more than two tetrahedra");
        i = j;
    }
    free(f);
    *nbf = n;
    return out;
}

/* is the support of key k inside some boundary face? */
static int mesh_on_boundary(const int *bf, int nbf, const int *k) {
    const int n = key_size(k);
    if (n == 4) return 0;
    for (int q = 0; q < nbf; q++) {
        int all = 1;
        for (int a = 0; a < n; a++) {
            const int v = k[2 * a];
            all &= bf[3 * q] == v || bf[3 * q + 1] == v || bf[3 * q + 2] == v;
        }
        if (all) return 1;
    }
    return 0;
}

typedef struct {
    int dim;     /* support size - 1 */
    int prim[4]; /* sorted support vertices, or (tet id, 0, 0, 0) for tetrahedron interiors */
    int w[3];    /* order within the primitive, most significant first */
    i64 node;
} mrec;

static int cmp_mrec(const void *a, const void *b) {
    const mrec *x = a, *y = b;
    if (x->dim != y->dim) return x->dim < y->dim ? -1 : 1;
    for (int q = 0; q < 4; q++)
        if (x->prim[q] != y->prim[q]) return x->prim[q] < y->prim[q] ? -1 : 1;
    for (int q = 0; q < 3; q++)
        if (x->w[q] != y->w[q]) return x->w[q] < y->w[q] ? -1 : 1;
    return 0;
}

static int weight_of(const int *k, int v) {
    for (int a = 0; a < 4; a++)
        if (k[2 * a] == v) return k[2 * a + 1];
    return 0;
}

/* the tetrahedron whose vertex set is the support of k (size 4) */
static int mesh_tet_of(const oproblem *p, const int *k) {
    for (int t = 0; t < p->nt; t++)
        if (mesh_in_tet(p, k, t, 0)) return t;
    die("interior node outside every tetrahedron");
    return -1;
}

/* user order of the interior nodes of level l (see above) */
static void mesh_order(oproblem *p, int l, const int *bf, int nbf) {
    olevel *Lv = &p->lev[l];
    mrec *r = xmalloc((size_t)(Lv->nnode ? Lv->nnode : 1) * sizeof(mrec));
    i64 n = 0;
    for (i64 v = 0; v < Lv->nnode; v++) {
        const int *k = &Lv->key[8 * v];
        if (mesh_on_boundary(bf, nbf, k)) continue;
        mrec *e = &r[n++];
        memset(e, 0, sizeof(*e));
        e->node = v;
        const int ns = key_size(k);
        e->dim = ns - 1;
        if (ns == 4) {
            const int t = mesh_tet_of(p, k);
            e->prim[0] = t;
            for (int q = 0; q < 3; q++) e->w[q] = weight_of(k, p->tet_v[4 * t + 3 - q]);
        } else {
            for (int a = 0; a < ns; a++) e->prim[a] = k[2 * a];
            for (int a = ns; a < 4; a++) e->prim[a] = -1;
            /* edge (a, b): weight of b; face (a, b, c): of c, then of b */
            if (ns == 2) e->w[0] = k[3];
            if (ns == 3) {
                e->w[0] = k[5];
                e->w[1] = k[3];
            }
        }
    }
    qsort(r, (size_t)n, sizeof(mrec), cmp_mrec);
    Lv->ndof = n;
    Lv->dof = xmalloc((size_t)(Lv->nnode ? Lv->nnode : 1) * sizeof(i64));
    Lv->node_of_dof = xmalloc((size_t)(n ? n : 1) * sizeof(i64));
    for (i64 v = 0; v < Lv->nnode; v++) Lv->dof[v] = -1;
    for (i64 q = 0; q < n; q++) {
        Lv->dof[r[q].node] = q;
        Lv->node_of_dof[q] = r[q].node;
    }
    free(r);
}

/* triplets (row, col, val) summed into a CSR matrix of nrow x ncol */
typedef struct {
    i64 r, c;
    double v;
} trip;
static int cmp_trip(const void *a, const void *b) {
    const trip *x = a, *y = b;
    if (x->r != y->r) return x->r < y->r ? -1 : 1;
    if (x->c != y->c) return x->c < y->c ? -1 : 1;
    return 0;
}
static csr csr_from_trip(trip *t, i64 nt, i64 nrow, i64 ncol) {
    qsort(t, (size_t)nt, sizeof(trip), cmp_trip);
    csr m;
    m.nrow = nrow;
    m.ncol = ncol;
    m.ptr = xcalloc((size_t)nrow + 1, sizeof(i64));
    i64 nnz = 0;
    for (i64 q = 0; q < nt; q++)
        if (q == 0 || t[q].r != t[q - 1].r || t[q].c != t[q - 1].c) nnz++;
    m.col = xmalloc((size_t)(nnz ? nnz : 1) * sizeof(int));
    m.val = xmalloc((size_t)(nnz ? nnz : 1) * sizeof(double));
    i64 z = -1;
    for (i64 q = 0; q < nt; q++) {
        if (q == 0 || t[q].r != t[q - 1].r || t[q].c != t[q - 1].c) {
            z++;
            m.col[z] = (int)t[q].c;
            m.val[z] = 0.0;
            m.ptr[t[q].r + 1]++;
        }
        m.val[z] += t[q].v;
    }
    for (i64 i = 0; i < nrow; i++) m.ptr[i + 1] += m.ptr[i];
    return m;
}

/* element-by-element stiffness (which = 0) or mass (which = 1) matrix of a
 * mesh level in physical coordinates, element e scaled by kcoef[e] (NULL: 1);
 * rows and columns through map (node -> index or -1 to drop), n indices */
static csr mesh_assemble(const olevel *Lv, const double *kcoef, int which, const i64 *map, i64 n) {
    trip *t = xmalloc((size_t)(16 * Lv->ne + 1) * sizeof(trip));
    i64 nt = 0;
    for (i64 e = 0; e < Lv->ne; e++) {
        double K[4][4], Mm[4][4];
        elem_mats_xyz(Lv->xyz, &Lv->ev[4 * e], K, Mm);
        const double ke = kcoef ? kcoef[e] : 1.0;
        for (int a = 0; a < 4; a++) {
            const i64 r = map ? map[Lv->ev[4 * e + a]] : Lv->ev[4 * e + a];
            if (r < 0) continue;
            for (int b = 0; b < 4; b++) {
                const i64 c = map ? map[Lv->ev[4 * e + b]] : Lv->ev[4 * e + b];
                if (c < 0) continue;
                t[nt].r = r;
                t[nt].c = c;
                t[nt].v = which ? Mm[a][b] : ke * K[a][b];
                nt++;
            }
        }
    }
    csr m = csr_from_trip(t, nt, n, n);
    free(t);
    return m;
}

/* linear interpolation from level l-1: an old node keeps its value, a new
 * node takes the mean of the two nodes of the coarse edge it bisects; through
 * the maps (-1: dropped) */
static csr mesh_prolongation(const olevel *C, const olevel *F, const i64 *mapf, i64 nf, const i64 *mapc, i64 nc) {
    trip *t = xmalloc((size_t)(2 * F->nnode + 1) * sizeof(trip));
    i64 nt = 0;
    for (i64 v = 0; v < F->nnode; v++) {
        const i64 r = mapf ? mapf[v] : v;
        if (r < 0) continue;
        const i64 a = F->par[2 * v], b = F->par[2 * v + 1];
        const i64 ca = mapc ? mapc[a] : a, cb = mapc ? mapc[b] : b;
        if (a == b) {
            if (ca >= 0) t[nt++] = (trip){r, ca, 1.0};
        } else {
            if (ca >= 0) t[nt++] = (trip){r, ca, 0.5};
            if (cb >= 0) t[nt++] = (trip){r, cb, 0.5};
        }
    }
    csr m = csr_from_trip(t, nt, nf, nc);
    free(t);
    (void)C;
    return m;
}

static void mesh_level_operators(oproblem *p, int l) {
    olevel *Lv = &p->lev[l];
    Lv->A = mesh_assemble(Lv, p->var_k ? Lv->k : NULL, 0, Lv->dof, Lv->ndof);
    Lv->diag = xmalloc((size_t)(Lv->ndof ? Lv->ndof : 1) * sizeof(double));
    for (i64 i = 0; i < Lv->ndof; i++) {
        Lv->diag[i] = 0.0;
        for (i64 q = Lv->A.ptr[i]; q < Lv->A.ptr[i + 1]; q++)
            if (Lv->A.col[q] == i) Lv->diag[i] = Lv->A.val[q];
    }
    /* classes 0, 2 (red) and 1, 3 (black), each list in dof order */
    Lv->red = xmalloc((size_t)(Lv->ndof ? Lv->ndof : 1) * sizeof(i64));
    Lv->black = xmalloc((size_t)(Lv->ndof ? Lv->ndof : 1) * sizeof(i64));
    Lv->nred = Lv->nblack = 0;
    for (int pass = 0; pass < 2; pass++) {
        for (i64 i = 0; i < Lv->ndof; i++) {
            const int *k = &Lv->key[8 * Lv->node_of_dof[i]];
            int c = 0;
            for (int a = 0; a < 4 && k[2 * a] >= 0; a++) c += p->vcol[k[2 * a]] * k[2 * a + 1];
            c &= 3;
            if ((c >> 1) != pass) continue;
            if ((c & 1) == 0)
                Lv->red[Lv->nred++] = i;
            else
                Lv->black[Lv->nblack++] = i;
        }
        if (pass == 0) {
            Lv->nred0 = Lv->nred;
            Lv->nblack1 = Lv->nblack;
        }
    }
    if (l > p->Lc) {
        const olevel *C = &p->lev[l - 1];
        Lv->P = mesh_prolongation(C, Lv, Lv->dof, Lv->ndof, C->dof, C->ndof);
        Lv->R = csr_transpose(&Lv->P);
    }
    Lv->built = 1;
}

/* k_tet (NULL: k = 1): the coefficient of eq. (2) on each macro
 * tetrahedron, so element e of level l (a descendant of macro element
 * e >> 3l) has k = k_tet[e >> 3l] on every level */
void *ohhg_create_mesh_k(int nv, const double *xyz, int nt, const int *tets, int L, int Lc, const double *k_tet) {
    if (nv < 4 || nt < 1 || !xyz || !tets || L < 1 || L >= MAXLEV || Lc < 1 || Lc > L) return NULL;
    if (k_tet)
        for (int t = 0; t < nt; t++)
            if (!(k_tet[t] > 0.0) || !isfinite(k_tet[t])) return NULL;
    double t0 = now_s();
    oproblem *p = xcalloc(1, sizeof(oproblem));
    p->mesh = 1;
    p->geom = 1;
    p->L = L;
    p->Lc = Lc;
    p->nv = nv;
    p->nt = nt;
    p->tet_v = xmalloc((size_t)nt * 4 * sizeof(int));
    memcpy(p->tet_v, tets, (size_t)nt * 4 * sizeof(int));
    p->vcol = xmalloc((size_t)nv * sizeof(int));
    for (int v = 0; v < nv; v++) p->vcol[v] = -1;
    for (int t = 0; t < nt; t++)
        for (int r = 0; r < 4; r++) {
            const int v = tets[4 * t + r];
            if (v < 0 || v >= nv || (p->vcol[v] >= 0 && p->vcol[v] != r)) {
                ohhg_destroy(p);
                return NULL;
            }
            p->vcol[v] = r;
        }
    /* level 0: the macro mesh */
    olevel *M0 = &p->lev[0];
    M0->nnode = nv;
    M0->ne = nt;
    M0->ev = xmalloc((size_t)nt * 4 * sizeof(int));
    memcpy(M0->ev, tets, (size_t)nt * 4 * sizeof(int));
    M0->xyz = xmalloc((size_t)nv * 3 * sizeof(double));
    memcpy(M0->xyz, xyz, (size_t)nv * 3 * sizeof(double));
    M0->key = xmalloc((size_t)nv * 8 * sizeof(int));
    M0->par = xmalloc((size_t)nv * 2 * sizeof(int));
    for (int v = 0; v < nv; v++) {
        for (int a = 0; a < 8; a++) M0->key[8 * v + a] = a == 0 ? v : a == 1 ? 1 : a % 2 == 0 ? -1 : 0;
        M0->par[2 * v] = M0->par[2 * v + 1] = v;
    }
    for (int t = 0; t < nt; t++) {
        /* reject flat macro tetrahedra (6 x volume = det of the edge vectors) */
        const int *e = &M0->ev[4 * t];
        double J[3][3];
        for (int r = 0; r < 3; r++)
            for (int c = 0; c < 3; c++) J[r][c] = xyz[3 * e[c + 1] + r] - xyz[3 * e[0] + r];
        const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                           J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        if (!(fabs(det) > 0.0)) {
            ohhg_destroy(p);
            return NULL;
        }
    }
    /* Bey's regular refinement, as on the cube (children of element e at
     * 8e..8e+7); midpoints are shared between the elements of an edge */
    static const int CH[8][4] = {{0, 4, 5, 6}, {4, 1, 7, 8}, {5, 7, 2, 9}, {6, 8, 9, 3},
                                 {4, 5, 6, 8}, {4, 5, 7, 8}, {5, 6, 8, 9}, {5, 7, 8, 9}};
    static const int MID[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
    for (int l = 1; l <= L; l++) {
        olevel *C = &p->lev[l - 1], *F = &p->lev[l];
        pairmap pm;
        pm_init(&pm, 6 * C->ne + 16);
        i64 next = C->nnode;
        F->ne = 8 * C->ne;
        F->ev = xmalloc((size_t)F->ne * 4 * sizeof(int));
        int *mid = xmalloc((size_t)C->ne * 6 * sizeof(int));
        for (i64 e = 0; e < C->ne; e++)
            for (int q = 0; q < 6; q++)
                mid[6 * e + q] = (int)pm_get(&pm, C->ev[4 * e + MID[q][0]], C->ev[4 * e + MID[q][1]], &next);
        F->nnode = next;
        F->xyz = xmalloc((size_t)F->nnode * 3 * sizeof(double));
        F->key = xmalloc((size_t)F->nnode * 8 * sizeof(int));
        F->par = xmalloc((size_t)F->nnode * 2 * sizeof(int));
        for (i64 v = 0; v < C->nnode; v++) {
            for (int a = 0; a < 3; a++) F->xyz[3 * v + a] = C->xyz[3 * v + a];
            for (int a = 0; a < 4; a++) {
                F->key[8 * v + 2 * a] = C->key[8 * v + 2 * a];
                F->key[8 * v + 2 * a + 1] = 2 * C->key[8 * v + 2 * a + 1];
            }
            F->par[2 * v] = F->par[2 * v + 1] = (int)v;
        }
        for (i64 e = 0; e < C->ne; e++) {
            int node[10];
            for (int a = 0; a < 4; a++) node[a] = C->ev[4 * e + a];
            for (int q = 0; q < 6; q++) {
                const int a = C->ev[4 * e + MID[q][0]], b = C->ev[4 * e + MID[q][1]], v = mid[6 * e + q];
                node[4 + q] = v;
                F->par[2 * v] = a;
                F->par[2 * v + 1] = b;
                for (int d = 0; d < 3; d++) F->xyz[3 * v + d] = 0.5 * (C->xyz[3 * a + d] + C->xyz[3 * b + d]);
                key_mid(&C->key[8 * a], &C->key[8 * b], &F->key[8 * v]);
            }
            for (int c = 0; c < 8; c++)
                for (int a = 0; a < 4; a++) F->ev[4 * (8 * e + c) + a] = node[CH[c][a]];
        }
        free(mid);
        free(pm.k);
        free(pm.v);
    }
    int nbf = 0;
    int *bf = boundary_faces(p, &nbf);
    for (int l = 0; l <= L; l++) mesh_order(p, l, bf, nbf);
    free(bf);
    p->var_k = k_tet != NULL;
    for (int l = 0; l <= L; l++) {
        olevel *Lv = &p->lev[l];
        Lv->k = xmalloc((size_t)Lv->ne * sizeof(double));
        for (i64 e = 0; e < Lv->ne; e++) Lv->k[e] = k_tet ? k_tet[e >> (3 * l)] : 1.0;
        Lv->ecl = xmalloc((size_t)Lv->ne * sizeof(i64));
        for (i64 e = 0; e < Lv->ne; e++) Lv->ecl[e] = e;
    }
    for (int l = Lc; l <= L; l++) mesh_level_operators(p, l);
    p->setup_s = now_s() - t0;
    return p;
}

void *ohhg_create_mesh(int nv, const double *xyz, int nt, const int *tets, int L, int Lc) {
    return ohhg_create_mesh_k(nv, xyz, nt, tets, L, Lc, NULL);
}

/* nodes of level l of a general macro mesh in creation order: positions
 * (3 each) and user index (-1 on the boundary); returns the node count */
long long ohhg_mesh_nodes(void *vp, int l, double *xyz, long long *dof) {
    const olevel *Lv = &((oproblem *)vp)->lev[l];
    if (xyz) memcpy(xyz, Lv->xyz, (size_t)Lv->nnode * 3 * sizeof(double));
    if (dof)
        for (i64 v = 0; v < Lv->nnode; v++) dof[v] = Lv->dof[v];
    return Lv->nnode;
}

/* keys of the nodes of level l (8 ints each, see olevel) */
void ohhg_mesh_keys(void *vp, int l, int *keys) {
    const olevel *Lv = &((oproblem *)vp)->lev[l];
    memcpy(keys, Lv->key, (size_t)Lv->nnode * 8 * sizeof(int));
}

/* ------------------------------------------------------------------------- */
/* Matrix export (for the tests' independent checks)                          */
/* ------------------------------------------------------------------------- */
/* which: 0 = A, 1 = M, 2 = P (level <- level-1); +3 for the variants that keep
 * the boundary vertices.  Returns a handle to a freshly built matrix. */
void *ohhg_matrix(void *vp, int l, int which) {
    oproblem *p = vp;
    olevel *Lv = &p->lev[l];
    csr *m = xcalloc(1, sizeof(csr));
    int interior = which < 3;
    int kind = which % 3;
    if (p->mesh) {
        /* general macro mesh: interior rows in user order, or every node in
         * creation order */
        if (kind == 2) {
            if (l < 1) die("no prolongation into level 0");
            const olevel *C = &p->lev[l - 1];
            *m = interior ? mesh_prolongation(C, Lv, Lv->dof, Lv->ndof, C->dof, C->ndof)
                          : mesh_prolongation(C, Lv, NULL, Lv->nnode, NULL, C->nnode);
        } else {
            const double *k = kind == 0 && p->var_k ? Lv->k : NULL;
            *m = interior ? mesh_assemble(Lv, k, kind, Lv->dof, Lv->ndof)
                          : mesh_assemble(Lv, k, kind, NULL, Lv->nnode);
        }
        return m;
    }
    if (kind == 2) {
        if (l < 1) die("no prolongation into level 0");
        *m = prolongation(&p->lev[l - 1], Lv, interior);
    } else {
        *m = assemble(Lv, p->var_k ? Lv->k : NULL, kind, interior);
    }
    return m;
}
long long ohhg_matrix_rows(void *m) { return ((csr *)m)->nrow; }
long long ohhg_matrix_cols(void *m) { return ((csr *)m)->ncol; }
long long ohhg_matrix_nnz(void *m) { return ((csr *)m)->ptr[((csr *)m)->nrow]; }
void ohhg_matrix_copy(void *vm, long long *ptr, int *col, double *val) {
    csr *m = vm;
    for (i64 i = 0; i <= m->nrow; i++) ptr[i] = m->ptr[i];
    memcpy(col, m->col, (size_t)m->ptr[m->nrow] * sizeof(int));
    memcpy(val, m->val, (size_t)m->ptr[m->nrow] * sizeof(double));
}
void ohhg_matrix_free(void *vm) {
    csr_free(vm);
    free(vm);
}

/* ------------------------------------------------------------------------- */
/* Macro-primitive membership (Sec. 3.1: volume, face, edge, vertex nodes)    */
/* ------------------------------------------------------------------------- */
static i64 det3(const i64 a[3], const i64 b[3], const i64 c[3]) {
    return a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
           a[2] * (b[0] * c[1] - b[1] * c[0]);
}

/* Barycentric test of grid point X (level-l units) against macro tet `tet`:
 * returns 2 if strictly inside, 1 if on its boundary, 0 if outside. */
static int tet_locate(const oproblem *p, int tet, int l, const i64 X[3]) {
    const olevel *M0 = &p->lev[0];
    i64 P[4][3];
    for (int a = 0; a < 4; a++) {
        int x, y, z;
        vxyz(M0->N, M0->ev[4 * tet + a], &x, &y, &z);
        P[a][0] = (i64)x << l;
        P[a][1] = (i64)y << l;
        P[a][2] = (i64)z << l;
    }
    i64 e1[3], e2[3], e3[3];
    for (int c = 0; c < 3; c++) {
        e1[c] = P[1][c] - P[0][c];
        e2[c] = P[2][c] - P[0][c];
        e3[c] = P[3][c] - P[0][c];
    }
    i64 D = det3(e1, e2, e3);
    int zero = 0;
    for (int a = 0; a < 4; a++) {
        i64 Q[4][3];
        memcpy(Q, P, sizeof(Q));
        for (int c = 0; c < 3; c++) Q[a][c] = X[c];
        i64 f1[3], f2[3], f3[3];
        for (int c = 0; c < 3; c++) {
            f1[c] = Q[1][c] - Q[0][c];
            f2[c] = Q[2][c] - Q[0][c];
            f3[c] = Q[3][c] - Q[0][c];
        }
        i64 Da = det3(f1, f2, f3);
        if ((Da > 0 && D < 0) || (Da < 0 && D > 0)) return 0;
        if (Da == 0) zero++;
    }
    return zero == 0 ? 2 : 1;
}

/* general macro mesh: 1 if the node's support (the macro vertices with a
 * nonzero weight in its key) lies in tetrahedron tet; with closure = 0 only
 * nodes strictly inside it (support = all four of its vertices) count */
static int mesh_in_tet(const oproblem *p, const int *key, int tet, int closure) {
    int ns = 0;
    for (int a = 0; a < 4; a++) {
        if (key[2 * a] < 0) continue;
        ns++;
        int found = 0;
        for (int r = 0; r < 4; r++) found |= p->tet_v[4 * tet + r] == key[2 * a];
        if (!found) return 0;
    }
    return closure ? 1 : ns == 4;
}

/* mask over interior dofs of level l: nodes strictly inside (closure=0) or in
 * the closed tetrahedron (closure=1). */
void ohhg_tet_mask(void *vp, int l, int tet, int closure, unsigned char *mask) {
    oproblem *p = vp;
    if (p->mesh) {
        const olevel *Lv = &p->lev[l];
        for (i64 i = 0; i < Lv->ndof; i++) mask[i] = (unsigned char)mesh_in_tet(p, &Lv->key[8 * Lv->node_of_dof[i]], tet, closure);
        return;
    }
    const int N = p->lev[l].N;
#pragma omp parallel for schedule(static)
    for (i64 i = 0; i < p->lev[l].ndof; i++) {
        i64 t = i;
        i64 X[3];
        X[0] = t % (N - 1) + 1;
        t /= (N - 1);
        X[1] = t % (N - 1) + 1;
        X[2] = t / (N - 1) + 1;
        int w = tet_locate(p, tet, l, X);
        mask[i] = closure ? (w > 0) : (w == 2);
    }
}

/* per interior dof: number of macro tetrahedra whose closure contains it */
void ohhg_containment_counts(void *vp, int l, int *count) {
    oproblem *p = vp;
    if (p->mesh) {
        const olevel *Lv = &p->lev[l];
        for (i64 i = 0; i < Lv->ndof; i++) {
            int c = 0;
            for (int q = 0; q < p->nt; q++) c += mesh_in_tet(p, &Lv->key[8 * Lv->node_of_dof[i]], q, 1);
            count[i] = c;
        }
        return;
    }
    const int N = p->lev[l].N;
    const int nt = (int)p->lev[0].ne;
#pragma omp parallel for schedule(static)
    for (i64 i = 0; i < p->lev[l].ndof; i++) {
        i64 t = i;
        i64 X[3];
        X[0] = t % (N - 1) + 1;
        t /= (N - 1);
        X[1] = t % (N - 1) + 1;
        X[2] = t / (N - 1) + 1;
        int c = 0;
        for (int q = 0; q < nt; q++) c += tet_locate(p, q, l, X) > 0;
        count[i] = c;
    }
}

/* ------------------------------------------------------------------------- */
/* Multigrid (Sec. 2.1): V-cycles of the correction scheme                    */
/* ------------------------------------------------------------------------- */
typedef struct {
    i64 n;
    csr A, P, R; /* P from the level below; R = P^T */
    double *diag;
    i64 nred, nblack;
    i64 *red, *black;
    int four;            /* 4-colour sweep: red[0..nred0), black[0..nblack1), then the rest of each */
    i64 nred0, nblack1;
    float *A32, *diag32;
    int owned;
} mglev;

typedef struct {
    int Lc, L;
    mglev lv[MAXLEV];
} mghier;

typedef struct {
    double omega;
    int nu1, nu2;
} mgopt;

static void hier_global(oproblem *p, mghier *H) {
    memset(H, 0, sizeof(*H));
    H->Lc = p->Lc;
    H->L = p->L;
    for (int l = p->Lc; l <= p->L; l++) {
        olevel *Lv = &p->lev[l];
        mglev *m = &H->lv[l];
        m->n = Lv->ndof;
        m->A = Lv->A;
        m->P = Lv->P;
        m->R = Lv->R;
        m->diag = Lv->diag;
        m->nred = Lv->nred;
        m->nblack = Lv->nblack;
        m->red = Lv->red;
        m->black = Lv->black;
        m->four = p->geom;
        m->nred0 = Lv->nred0;
        m->nblack1 = Lv->nblack1;
        m->owned = 0;
    }
}

/* Restriction of the global hierarchy to the subsets keep[l] (masks over the
 * interior dofs of each level): A_l[S_l,S_l] and P_l[S_l,S_{l-1}]. */
static void hier_sub(oproblem *p, unsigned char **keep, mghier *H, i64 **map_out) {
    memset(H, 0, sizeof(*H));
    H->Lc = p->Lc;
    H->L = p->L;
    i64 *map[MAXLEV] = {0};
    for (int l = p->Lc; l <= p->L; l++) {
        olevel *Lv = &p->lev[l];
        map[l] = xmalloc((size_t)Lv->ndof * sizeof(i64));
        i64 c = 0;
        for (i64 i = 0; i < Lv->ndof; i++) map[l][i] = keep[l][i] ? c++ : -1;
        mglev *m = &H->lv[l];
        m->n = c;
        m->owned = 1;
        m->A = csr_sub(&Lv->A, map[l], c, map[l], c);
        m->diag = xmalloc((size_t)(c ? c : 1) * sizeof(double));
        m->red = xmalloc((size_t)(c ? c : 1) * sizeof(i64));
        m->black = xmalloc((size_t)(c ? c : 1) * sizeof(i64));
        for (i64 i = 0; i < Lv->ndof; i++)
            if (map[l][i] >= 0) m->diag[map[l][i]] = Lv->diag[i];
        for (i64 q = 0; q < Lv->nred; q++) {
            if (q == Lv->nred0) m->nred0 = m->nred;
            if (map[l][Lv->red[q]] >= 0) m->red[m->nred++] = map[l][Lv->red[q]];
        }
        if (Lv->nred0 >= Lv->nred) m->nred0 = m->nred;
        for (i64 q = 0; q < Lv->nblack; q++) {
            if (q == Lv->nblack1) m->nblack1 = m->nblack;
            if (map[l][Lv->black[q]] >= 0) m->black[m->nblack++] = map[l][Lv->black[q]];
        }
        if (Lv->nblack1 >= Lv->nblack) m->nblack1 = m->nblack;
        m->four = p->geom;
        if (l > p->Lc) {
            m->P = csr_sub(&Lv->P, map[l], c, map[l - 1], H->lv[l - 1].n);
            m->R = csr_transpose(&m->P);
        }
    }
    if (map_out)
        for (int l = 0; l < MAXLEV; l++) map_out[l] = map[l];
    else
        for (int l = 0; l < MAXLEV; l++) free(map[l]);
}

static void hier_free(mghier *H) {
    for (int l = H->Lc; l <= H->L; l++) {
        mglev *m = &H->lv[l];
        if (m->owned) {
            csr_free(&m->A);
            csr_free(&m->P);
            csr_free(&m->R);
            free(m->diag);
            free(m->red);
            free(m->black);
        }
        free(m->A32);
        free(m->diag32);
    }
}

/* One colour pass of SOR: every node i of the colour gets
 * u_i <- u_i + omega (b - A u)_i / a_ii, all computed from the values before
 * the pass (nodes of one colour are not coupled, so this is Gauss-Seidel
 * within the colour). */
static void colour_pass64(const mglev *m, const i64 *list, i64 cnt, double *u, const double *b,
                          double omega) {
    double *nv = xmalloc((size_t)(cnt ? cnt : 1) * sizeof(double));
#pragma omp parallel for schedule(static)
    for (i64 q = 0; q < cnt; q++) {
        i64 i = list[q];
        double s = b[i];
        for (i64 t = m->A.ptr[i]; t < m->A.ptr[i + 1]; t++) s -= m->A.val[t] * u[m->A.col[t]];
        nv[q] = u[i] + omega * s / m->diag[i];
    }
#pragma omp parallel for schedule(static)
    for (i64 q = 0; q < cnt; q++) u[list[q]] = nv[q];
    free(nv);
}

/* smoother (Sec. 2.1 names a Gauss-Seidel variant): red-black SOR sweep, red
 * (even x+y+z) first */
static void sweep64(const mglev *m, double *u, const double *b, double omega) {
    if (m->four) {
        /* classes 0, 1, 2, 3 of (x+y+z) mod 4 */
        colour_pass64(m, m->red, m->nred0, u, b, omega);
        colour_pass64(m, m->black, m->nblack1, u, b, omega);
        colour_pass64(m, m->red + m->nred0, m->nred - m->nred0, u, b, omega);
        colour_pass64(m, m->black + m->nblack1, m->nblack - m->nblack1, u, b, omega);
        return;
    }
    colour_pass64(m, m->red, m->nred, u, b, omega);
    colour_pass64(m, m->black, m->nblack, u, b, omega);
}

/* Jacobi-preconditioned CG (Sec. 2.1: PCG coarse solver), from the given x,
 * until ||r|| <= rtol ||r_0||.  Returns the iteration count. */
static int pcg64(const csr *A, const double *diag, const double *b, double *x, double rtol, int maxit) {
    i64 n = A->nrow;
    double *r = xmalloc((size_t)(n ? n : 1) * sizeof(double));
    double *z = xmalloc((size_t)(n ? n : 1) * sizeof(double));
    double *pv = xmalloc((size_t)(n ? n : 1) * sizeof(double));
    double *q = xmalloc((size_t)(n ? n : 1) * sizeof(double));
    residual(A, x, b, r);
    double r0 = norm2(n, r);
    int it = 0;
    if (r0 > 0.0) {
        for (i64 i = 0; i < n; i++) {
            z[i] = r[i] / diag[i];
            pv[i] = z[i];
        }
        double rz = dot(n, r, z);
        for (it = 1; it <= maxit; it++) {
            spmv(A, pv, q);
            double alpha = rz / dot(n, pv, q);
            for (i64 i = 0; i < n; i++) {
                x[i] += alpha * pv[i];
                r[i] -= alpha * q[i];
            }
            if (norm2(n, r) <= rtol * r0) break;
            for (i64 i = 0; i < n; i++) z[i] = r[i] / diag[i];
            double rz1 = dot(n, r, z);
            double beta = rz1 / rz;
            rz = rz1;
            for (i64 i = 0; i < n; i++) pv[i] = z[i] + beta * pv[i];
        }
    }
    free(r);
    free(z);
    free(pv);
    free(q);
    return it;
}

#define COARSE_RTOL 1e-14
#define COARSE_MAXIT 2000

/* V-cycle of the correction scheme on level l (Sec. 2.1): nu1 pre-sweeps,
 * residual, restriction by P^T, recursive correction from zero, linear
 * interpolation of the correction, nu2 post-sweeps; on the coarsest level the
 * correction comes from PCG. */
static void vcycle64(const mghier *H, int l, double *u, const double *b, const mgopt *o) {
    const mglev *m = &H->lv[l];
    i64 n = m->n;
    double *r = xmalloc((size_t)(n ? n : 1) * sizeof(double));
    if (l == H->Lc) {
        double *e = xcalloc((size_t)(n ? n : 1), sizeof(double));
        residual(&m->A, u, b, r);
        pcg64(&m->A, m->diag, r, e, COARSE_RTOL, COARSE_MAXIT);
        for (i64 i = 0; i < n; i++) u[i] += e[i];
        free(e);
        free(r);
        return;
    }
    for (int s = 0; s < o->nu1; s++) sweep64(m, u, b, o->omega);
    residual(&m->A, u, b, r);
    const mglev *mc = &H->lv[l - 1];
    double *bc = xmalloc((size_t)(mc->n ? mc->n : 1) * sizeof(double));
    double *ec = xcalloc((size_t)(mc->n ? mc->n : 1), sizeof(double));
    spmv(&m->R, r, bc);
    vcycle64(H, l - 1, ec, bc, o);
    spmv(&m->P, ec, r); /* r <- P e_c */
    for (i64 i = 0; i < n; i++) u[i] += r[i];
    for (int s = 0; s < o->nu2; s++) sweep64(m, u, b, o->omega);
    free(bc);
    free(ec);
    free(r);
}

static double resnorm(const csr *A, const double *u, const double *b) {
    double *r = xmalloc((size_t)(A->nrow ? A->nrow : 1) * sizeof(double));
    residual(A, u, b, r);
    double s = norm2(A->nrow, r);
    free(r);
    return s;
}

/* ------------------------------------------------------------------------- */
/* Public entry points: operators                                             */
/* ------------------------------------------------------------------------- */
static void ensure_mass(oproblem *p, int l) {
    olevel *Lv = &p->lev[l];
    if (Lv->M.ptr == NULL) Lv->M = p->mesh ? mesh_assemble(Lv, NULL, 1, Lv->dof, Lv->ndof) : assemble(Lv, NULL, 1, 1);
}

void ohhg_apply_A(void *vp, int l, const double *u, double *out) {
    oproblem *p = vp;
    build_level_operators(p, l);
    spmv(&p->lev[l].A, u, out);
}

void ohhg_apply_M(void *vp, int l, const double *u, double *out) {
    oproblem *p = vp;
    ensure_mass(p, l);
    spmv(&p->lev[l].M, u, out);
}

void ohhg_residual(void *vp, int l, const double *u, const double *b, double *r) {
    oproblem *p = vp;
    build_level_operators(p, l);
    residual(&p->lev[l].A, u, b, r);
}

/* colours: 1 red pass, 2 black pass, 3 full sweep (red then black); with a
 * general geometry bits 1, 2, 4, 8 select the classes 0..3 of (x+y+z) mod 4
 * (15 = full sweep) */
void ohhg_smooth(void *vp, int l, double *u, const double *b, double omega, int colours) {
    oproblem *p = vp;
    mghier H;
    hier_global(p, &H);
    const mglev *m = &H.lv[l];
    if (m->four) {
        if (colours & 1) colour_pass64(m, m->red, m->nred0, u, b, omega);
        if (colours & 2) colour_pass64(m, m->black, m->nblack1, u, b, omega);
        if (colours & 4) colour_pass64(m, m->red + m->nred0, m->nred - m->nred0, u, b, omega);
        if (colours & 8) colour_pass64(m, m->black + m->nblack1, m->nblack - m->nblack1, u, b, omega);
        return;
    }
    if (colours & 1) colour_pass64(m, m->red, m->nred, u, b, omega);
    if (colours & 2) colour_pass64(m, m->black, m->nblack, u, b, omega);
}

/* b_c = P^T r (level l -> l-1) */
void ohhg_restrict(void *vp, int l, const double *r, double *bc) {
    oproblem *p = vp;
    spmv(&p->lev[l].R, r, bc);
}

/* u += P e_c (level l-1 -> l) */
void ohhg_prolong_add(void *vp, int l, const double *ec, double *u) {
    oproblem *p = vp;
    olevel *Lv = &p->lev[l];
    double *t = xmalloc((size_t)Lv->ndof * sizeof(double));
    spmv(&Lv->P, ec, t);
    for (i64 i = 0; i < Lv->ndof; i++) u[i] += t[i];
    free(t);
}

/* coarsest-level PCG from x (in/out); returns iterations */
int ohhg_coarse_solve(void *vp, const double *b, double *x, double rtol) {
    oproblem *p = vp;
    olevel *Lv = &p->lev[p->Lc];
    return pcg64(&Lv->A, Lv->diag, b, x, rtol, COARSE_MAXIT);
}

/* one V-cycle on the finest level; returns ||b - A u|| afterwards */
double ohhg_vcycle(void *vp, double *u, const double *b, double omega, int nu1, int nu2) {
    oproblem *p = vp;
    mghier H;
    hier_global(p, &H);
    mgopt o = {omega, nu1, nu2};
    vcycle64(&H, p->L, u, b, &o);
    return resnorm(&p->lev[p->L].A, u, b);
}

/* V-cycles until ||b - A u|| <= rtol * r0 (r0_ref > 0: given reference, else
 * the residual of the initial u).  hist[c] = ||r_c|| / r0 for c = 0..cycles.
 * Returns the number of cycles, or -1 if max_cycles was reached. */
int ohhg_solve(void *vp, double *u, const double *b, double omega, int nu1, int nu2, double rtol,
               int max_cycles, double r0_ref, double *hist) {
    oproblem *p = vp;
    mghier H;
    hier_global(p, &H);
    mgopt o = {omega, nu1, nu2};
    const csr *A = &p->lev[p->L].A;
    double rn = resnorm(A, u, b);
    double r0 = r0_ref > 0 ? r0_ref : rn;
    if (hist) hist[0] = r0 > 0 ? rn / r0 : 0.0;
    if (rn <= rtol * r0) return 0;
    for (int c = 1; c <= max_cycles; c++) {
        vcycle64(&H, p->L, u, b, &o);
        rn = resnorm(A, u, b);
        if (hist) hist[c] = rn / r0;
        if (rn <= rtol * r0) return c;
    }
    return -1;
}

/* ------------------------------------------------------------------------- */
/* Fault and recovery (Sec. 2.2, Sec. 4, Alg. 1)                              */
/* ------------------------------------------------------------------------- */
/* A fault re-initialises with zero the unknowns strictly inside the faulty
 * macro tetrahedron; nodes on its faces, edges and vertices survive in their
 * own containers. */
void ohhg_inject_fault(void *vp, int tet, double *u) {
    oproblem *p = vp;
    olevel *Lv = &p->lev[p->L];
    unsigned char *mask = xmalloc((size_t)Lv->ndof);
    ohhg_tet_mask(p, p->L, tet, 0, mask);
    for (i64 i = 0; i < Lv->ndof; i++)
        if (mask[i]) u[i] = 0.0;
    free(mask);
}

/* rhs of a subproblem with the other unknowns as Dirichlet data:
 * (b - A u~)[S] with u~ = u and u~[S] = 0, i.e. f_S - A_{S,not S} u_{not S} */
static void sub_rhs(const csr *A, const i64 *map, i64 nsub, const double *u, const double *b, double *rhs) {
    i64 n = A->nrow;
    double *ut = xmalloc((size_t)n * sizeof(double));
    double *r = xmalloc((size_t)n * sizeof(double));
    for (i64 i = 0; i < n; i++) ut[i] = map[i] >= 0 ? 0.0 : u[i];
    residual(A, ut, b, r);
    for (i64 i = 0; i < n; i++)
        if (map[i] >= 0) rhs[map[i]] = r[i];
    (void)nsub;
    free(ut);
    free(r);
}

static void build_masks(oproblem *p, const int *tets, int nt, int closure, int invert, unsigned char **keep) {
    for (int l = p->Lc; l <= p->L; l++) {
        i64 n = p->lev[l].ndof;
        keep[l] = xcalloc((size_t)n, 1);
        unsigned char *m = xmalloc((size_t)n);
        for (int q = 0; q < nt; q++) {
            ohhg_tet_mask(p, l, tets[q], closure, m);
            for (i64 i = 0; i < n; i++) keep[l][i] |= m[i];
        }
        if (invert)
            for (i64 i = 0; i < n; i++) keep[l][i] = !keep[l][i];
        free(m);
    }
}

/* Local recovery (Alg. 1 a), Sec. 4): u_F <- 0, then n_cycles V-cycles of the
 * multigrid restricted to the interiors of the faulty tetrahedra on every
 * level for A_FF u_F = f_F - A_FG u_G, the interface values acting as
 * Dirichlet data.  res[c] = ||local residual|| / ||local rhs|| after cycle c. */
void ohhg_recover_local(void *vp, const int *tets, int nt, double *u, const double *b, int n_cycles,
                        double omega, int nu1, int nu2, double *res) {
    oproblem *p = vp;
    unsigned char *keep[MAXLEV] = {0};
    i64 *map[MAXLEV] = {0};
    build_masks(p, tets, nt, 0, 0, keep);
    mghier H;
    hier_sub(p, keep, &H, map);
    mgopt o = {omega, nu1, nu2};
    i64 ns = H.lv[p->L].n;
    double *rhs = xmalloc((size_t)(ns ? ns : 1) * sizeof(double));
    double *x = xcalloc((size_t)(ns ? ns : 1), sizeof(double));
    sub_rhs(&p->lev[p->L].A, map[p->L], ns, u, b, rhs);
    double r0 = norm2(ns, rhs);
    for (int c = 0; c < n_cycles; c++) {
        vcycle64(&H, p->L, x, rhs, &o);
        if (res) res[c] = r0 > 0 ? resnorm(&H.lv[p->L].A, x, rhs) / r0 : 0.0;
    }
    const i64 *mp = map[p->L];
    for (i64 i = 0; i < p->lev[p->L].ndof; i++)
        if (mp[i] >= 0) u[i] = x[mp[i]];
    free(rhs);
    free(x);
    hier_free(&H);
    for (int l = 0; l < MAXLEV; l++) {
        free(keep[l]);
        free(map[l]);
    }
}

/* Dirichlet-Dirichlet intact cycles (Alg. 1 b)): n_cycles V-cycles for
 * A_II u_I = f_I - A_IG u_G, where the closure of every faulty tetrahedron is
 * frozen on all levels; starts from the current u_I. */
void ohhg_dd_intact(void *vp, const int *tets, int nt, double *u, const double *b, int n_cycles, double omega,
                    int nu1, int nu2) {
    oproblem *p = vp;
    unsigned char *keep[MAXLEV] = {0};
    i64 *map[MAXLEV] = {0};
    build_masks(p, tets, nt, 1, 1, keep);
    mghier H;
    hier_sub(p, keep, &H, map);
    mgopt o = {omega, nu1, nu2};
    i64 ns = H.lv[p->L].n;
    double *rhs = xmalloc((size_t)(ns ? ns : 1) * sizeof(double));
    double *x = xmalloc((size_t)(ns ? ns : 1) * sizeof(double));
    sub_rhs(&p->lev[p->L].A, map[p->L], ns, u, b, rhs);
    const i64 *mp = map[p->L];
    for (i64 i = 0; i < p->lev[p->L].ndof; i++)
        if (mp[i] >= 0) x[mp[i]] = u[i];
    for (int c = 0; c < n_cycles; c++) vcycle64(&H, p->L, x, rhs, &o);
    for (i64 i = 0; i < p->lev[p->L].ndof; i++)
        if (mp[i] >= 0) u[i] = x[mp[i]];
    free(rhs);
    free(x);
    hier_free(&H);
    for (int l = 0; l < MAXLEV; l++) {
        free(keep[l]);
        free(map[l]);
    }
}

/* ------------------------------------------------------------------------- */
/* Dirichlet-Neumann recovery (Sec. 4.3, Alg. 2, eq. (5))                      */
/* ------------------------------------------------------------------------- */
/* Element coefficient restricted to one side of the fault: k of the element
 * (1 without variable k) where its macro tetrahedron is intact (side 0) or
 * faulty (side 1), else 0.  Element e of level l descends from macro element
 * e >> 3l (Bey children of e are 8e..8e+7). */
static double *side_coeff(const oproblem *p, int l, const unsigned char *faulty, int side) {
    const olevel *Lv = &p->lev[l];
    double *k = xmalloc((size_t)Lv->ne * sizeof(double));
    for (i64 e = 0; e < Lv->ne; e++) {
        const int f = faulty[e >> (3 * l)];
        const double ke = p->var_k ? Lv->k[Lv->ecl[e]] : 1.0;
        k[Lv->ecl[e]] = (side == 0 ? !f : f) ? ke : 0.0;
    }
    return k;
}

/* Stiffness matrix of level l assembled over the elements of one side only:
 * the sub-stencils of eq. (5) (A_II, A_{I Gamma_I}, A_{Gamma_I Gamma_I} for
 * side 0).  A^intact + A^faulty = A. */
static csr side_matrix(const oproblem *p, int l, const int *tets, int nt, int side) {
    unsigned char *faulty = xcalloc((size_t)p->lev[0].ne, 1);
    for (int q = 0; q < nt; q++) faulty[tets[q]] = 1;
    double *k = side_coeff(p, l, faulty, side);
    csr A = p->mesh ? mesh_assemble(&p->lev[l], k, 0, p->lev[l].dof, p->lev[l].ndof) : assemble(&p->lev[l], k, 0, 1);
    free(k);
    free(faulty);
    return A;
}

/* Multigrid hierarchy of given operators ops[l], restricted to keep[l]; the
 * transfers are the restrictions of the global ones */
static void hier_ops(oproblem *p, csr *ops, unsigned char **keep, mghier *H, i64 **map_out) {
    memset(H, 0, sizeof(*H));
    H->Lc = p->Lc;
    H->L = p->L;
    i64 *map[MAXLEV] = {0};
    for (int l = p->Lc; l <= p->L; l++) {
        olevel *Lv = &p->lev[l];
        map[l] = xmalloc((size_t)Lv->ndof * sizeof(i64));
        i64 c = 0;
        for (i64 i = 0; i < Lv->ndof; i++) map[l][i] = keep[l][i] ? c++ : -1;
        mglev *m = &H->lv[l];
        m->n = c;
        m->owned = 1;
        m->A = csr_sub(&ops[l], map[l], c, map[l], c);
        m->diag = xcalloc((size_t)(c ? c : 1), sizeof(double));
        m->red = xmalloc((size_t)(c ? c : 1) * sizeof(i64));
        m->black = xmalloc((size_t)(c ? c : 1) * sizeof(i64));
        for (i64 i = 0; i < c; i++)
            for (i64 q = m->A.ptr[i]; q < m->A.ptr[i + 1]; q++)
                if (m->A.col[q] == i) m->diag[i] = m->A.val[q];
        for (i64 q = 0; q < Lv->nred; q++) {
            if (q == Lv->nred0) m->nred0 = m->nred;
            if (map[l][Lv->red[q]] >= 0) m->red[m->nred++] = map[l][Lv->red[q]];
        }
        if (Lv->nred0 >= Lv->nred) m->nred0 = m->nred;
        for (i64 q = 0; q < Lv->nblack; q++) {
            if (q == Lv->nblack1) m->nblack1 = m->nblack;
            if (map[l][Lv->black[q]] >= 0) m->black[m->nblack++] = map[l][Lv->black[q]];
        }
        if (Lv->nblack1 >= Lv->nblack) m->nblack1 = m->nblack;
        m->four = p->geom;
        if (l > p->Lc) {
            m->P = csr_sub(&Lv->P, map[l], c, map[l - 1], H->lv[l - 1].n);
            m->R = csr_transpose(&m->P);
        }
    }
    for (int l = 0; l < MAXLEV; l++) {
        if (map_out)
            map_out[l] = map[l];
        else
            free(map[l]);
    }
}

/* Alg. 2.  Intact side: V-cycles for the Neumann problem (the first two
 * block rows of eq. (5)) on the nodes the intact operator couples (intact
 * interiors and the interface Gamma), right-hand side b off Gamma and, on
 * Gamma, the intact-side action A^I u of the data at the time of the fault
 * (lambda of Alg. 2 taken with static data).  Faulty side: u_F starts at
 * zero; its local Dirichlet problems take their boundary values from the
 * interface values on Gamma.
 * n_intact rounds: in round i the faulty side runs eta local cycles with the
 * interface values of the start of the round, continuing from its current
 * u_F, and the intact side runs one V-cycle; the two sides share no unknown
 * within a round, so their order inside it does not matter. */
void ohhg_dn_recover(void *vp, const int *tets, int nt, double *u, const double *b, int n_intact, int eta,
                     double omega, int nu1, int nu2) {
    oproblem *p = vp;
    const int L = p->L;
    const olevel *F = &p->lev[L];
    mgopt o = {omega, nu1, nu2};
    /* intact side */
    csr ops[MAXLEV];
    memset(ops, 0, sizeof(ops));
    unsigned char *keep[MAXLEV] = {0};
    for (int l = p->Lc; l <= L; l++) {
        ops[l] = side_matrix(p, l, tets, nt, 0);
        keep[l] = xcalloc((size_t)p->lev[l].ndof, 1);
        for (i64 i = 0; i < p->lev[l].ndof; i++)
            for (i64 q = ops[l].ptr[i]; q < ops[l].ptr[i + 1]; q++)
                if (ops[l].col[q] == i && ops[l].val[q] > 0.0) keep[l][i] = 1;
    }
    i64 *mapI[MAXLEV] = {0};
    mghier HI;
    hier_ops(p, ops, keep, &HI, mapI);
    unsigned char *onF = xcalloc((size_t)F->ndof, 1), *m = xmalloc((size_t)F->ndof);
    for (int q = 0; q < nt; q++) {
        ohhg_tet_mask(p, L, tets[q], 1, m);
        for (i64 i = 0; i < F->ndof; i++) onF[i] |= m[i];
    }
    const i64 nI = HI.lv[L].n;
    double *Au = xmalloc((size_t)F->ndof * sizeof(double));
    spmv(&ops[L], u, Au);
    double *bI = xmalloc((size_t)(nI ? nI : 1) * sizeof(double));
    double *xI = xmalloc((size_t)(nI ? nI : 1) * sizeof(double));
    for (i64 i = 0; i < F->ndof; i++) {
        const i64 j = mapI[L][i];
        if (j < 0) continue;
        bI[j] = onF[i] ? Au[i] : b[i]; /* Gamma: static Neumann data */
        xI[j] = u[i];
    }
    /* faulty side */
    unsigned char *keepF[MAXLEV] = {0};
    i64 *mapF[MAXLEV] = {0};
    build_masks(p, tets, nt, 0, 0, keepF);
    mghier HF;
    hier_sub(p, keepF, &HF, mapF);
    const i64 nF = HF.lv[L].n;
    double *bF = xmalloc((size_t)(nF ? nF : 1) * sizeof(double));
    double *xF = xcalloc((size_t)(nF ? nF : 1), sizeof(double));
    for (i64 i = 0; i < F->ndof; i++)
        if (mapF[L][i] >= 0) u[i] = 0.0;
    for (int r = 0; r < n_intact; r++) {
        sub_rhs(&F->A, mapF[L], nF, u, b, bF); /* interface values of the start of the round */
        for (int c = 0; c < eta; c++) vcycle64(&HF, L, xF, bF, &o);
        vcycle64(&HI, L, xI, bI, &o);
        for (i64 i = 0; i < F->ndof; i++) {
            if (mapF[L][i] >= 0) u[i] = xF[mapF[L][i]];
            if (mapI[L][i] >= 0) u[i] = xI[mapI[L][i]];
        }
    }
    free(Au);
    free(bI);
    free(xI);
    free(bF);
    free(xF);
    free(onF);
    free(m);
    hier_free(&HI);
    hier_free(&HF);
    for (int l = 0; l < MAXLEV; l++) {
        csr_free(&ops[l]);
        free(keep[l]);
        free(keepF[l]);
        free(mapI[l]);
        free(mapF[l]);
    }
}

/* The side matrices for tests: side 0 = intact, 1 = faulty (matrix handle) */
void *ohhg_side_matrix(void *vp, int l, const int *tets, int nt, int side) {
    csr *A = xmalloc(sizeof(csr));
    *A = side_matrix(vp, l, tets, nt, side);
    return A;
}

/* The same on a general macro mesh (Sec. 3.1): dJ/dk_e = -lambda^T A_e u for
 * every element e of the finest level, in element order (children of
 * element e at 8e..8e+7, so macro tetrahedron t owns elements
 * t 8^L .. (t+1) 8^L - 1); A_e in physical coordinates, u = lambda = 0 at
 * Dirichlet nodes. */
void ohhg_mesh_grad_k(void *vp, const double *u, const double *lam, double *out) {
    oproblem *p = vp;
    olevel *Lv = &p->lev[p->L];
#pragma omp parallel for schedule(static)
    for (i64 e = 0; e < Lv->ne; e++) {
        double K[4][4], Mm[4][4], ul[4], ll[4];
        elem_mats_xyz(Lv->xyz, &Lv->ev[4 * e], K, Mm);
        for (int a = 0; a < 4; a++) {
            const i64 d = Lv->dof[Lv->ev[4 * e + a]];
            ul[a] = d >= 0 ? u[d] : 0.0;
            ll[a] = d >= 0 ? lam[d] : 0.0;
        }
        double g = 0.0;
        for (int a = 0; a < 4; a++)
            for (int b = 0; b < 4; b++) g += ll[a] * K[a][b] * ul[b];
        out[e] = -g;
    }
}

/* ------------------------------------------------------------------------- */
/* Mixed precision: FP32 V-cycle inside an FP64 residual-correction loop      */
/* ------------------------------------------------------------------------- */
static void ensure_fp32(mghier *H) {
    for (int l = H->Lc; l <= H->L; l++) {
        mglev *m = &H->lv[l];
        if (m->A32) continue;
        i64 nnz = m->A.ptr[m->n];
        m->A32 = xmalloc((size_t)(nnz ? nnz : 1) * sizeof(float));
        m->diag32 = xmalloc((size_t)(m->n ? m->n : 1) * sizeof(float));
        for (i64 q = 0; q < nnz; q++) m->A32[q] = (float)m->A.val[q];
        for (i64 i = 0; i < m->n; i++) m->diag32[i] = (float)m->diag[i];
    }
}

static void colour_pass32(const mglev *m, const i64 *list, i64 cnt, float *u, const float *b, float omega) {
    float *nv = xmalloc((size_t)(cnt ? cnt : 1) * sizeof(float));
#pragma omp parallel for schedule(static)
    for (i64 q = 0; q < cnt; q++) {
        i64 i = list[q];
        float s = b[i];
        for (i64 t = m->A.ptr[i]; t < m->A.ptr[i + 1]; t++) s -= m->A32[t] * u[m->A.col[t]];
        nv[q] = u[i] + omega * s / m->diag32[i];
    }
#pragma omp parallel for schedule(static)
    for (i64 q = 0; q < cnt; q++) u[list[q]] = nv[q];
    free(nv);
}

static void residual32(const mglev *m, const float *u, const float *b, float *r) {
#pragma omp parallel for schedule(static)
    for (i64 i = 0; i < m->n; i++) {
        float s = b[i];
        for (i64 t = m->A.ptr[i]; t < m->A.ptr[i + 1]; t++) s -= m->A32[t] * u[m->A.col[t]];
        r[i] = s;
    }
}

/* one FP32 sweep in the order of sweep64 */
static void sweep32(const mglev *m, float *u, const float *b, float omega) {
    if (m->four) {
        colour_pass32(m, m->red, m->nred0, u, b, omega);
        colour_pass32(m, m->black, m->nblack1, u, b, omega);
        colour_pass32(m, m->red + m->nred0, m->nred - m->nred0, u, b, omega);
        colour_pass32(m, m->black + m->nblack1, m->nblack - m->nblack1, u, b, omega);
        return;
    }
    colour_pass32(m, m->red, m->nred, u, b, omega);
    colour_pass32(m, m->black, m->nblack, u, b, omega);
}

static void spmv32(const csr *A, const float *x, float *y) {
#pragma omp parallel for schedule(static)
    for (i64 i = 0; i < A->nrow; i++) {
        float s = 0.0f;
        for (i64 q = A->ptr[i]; q < A->ptr[i + 1]; q++) s += (float)A->val[q] * x[A->col[q]];
        y[i] = s;
    }
}

/* The FP32 V-cycle: same steps as vcycle64 in FP32; the coarsest correction is
 * computed by FP64 PCG on the FP64 operator and rounded to FP32. */
static void vcycle32(const mghier *H, int l, float *u, const float *b, const mgopt *o) {
    const mglev *m = &H->lv[l];
    i64 n = m->n;
    if (l == H->Lc) {
        double *r64 = xmalloc((size_t)(n ? n : 1) * sizeof(double));
        double *e64 = xcalloc((size_t)(n ? n : 1), sizeof(double));
        double *u64 = xmalloc((size_t)(n ? n : 1) * sizeof(double));
        double *b64 = xmalloc((size_t)(n ? n : 1) * sizeof(double));
        for (i64 i = 0; i < n; i++) {
            u64[i] = u[i];
            b64[i] = b[i];
        }
        residual(&m->A, u64, b64, r64);
        pcg64(&m->A, m->diag, r64, e64, COARSE_RTOL, COARSE_MAXIT);
        for (i64 i = 0; i < n; i++) u[i] = (float)(u64[i] + e64[i]);
        free(r64);
        free(e64);
        free(u64);
        free(b64);
        return;
    }
    float om = (float)o->omega;
    for (int s = 0; s < o->nu1; s++) sweep32(m, u, b, om);
    float *r = xmalloc((size_t)(n ? n : 1) * sizeof(float));
    residual32(m, u, b, r);
    const mglev *mc = &H->lv[l - 1];
    float *bc = xmalloc((size_t)(mc->n ? mc->n : 1) * sizeof(float));
    float *ec = xcalloc((size_t)(mc->n ? mc->n : 1), sizeof(float));
    spmv32(&m->R, r, bc);
    vcycle32(H, l - 1, ec, bc, o);
    spmv32(&m->P, ec, r);
    for (i64 i = 0; i < n; i++) u[i] += r[i];
    for (int s = 0; s < o->nu2; s++) sweep32(m, u, b, om);
    free(bc);
    free(ec);
    free(r);
}

/* x_{k+1} = x_k + V32(round32(b - A x_k)) until ||b - A x|| <= rtol * r0.
 * hist[c] = ||r_c|| / r0.  Returns the step count or -1. */
int ohhg_solve_mixed(void *vp, double *u, const double *b, double omega, int nu1, int nu2, double rtol,
                     int max_steps, double r0_ref, double *hist) {
    oproblem *p = vp;
    mghier H;
    hier_global(p, &H);
    ensure_fp32(&H);
    mgopt o = {omega, nu1, nu2};
    const csr *A = &p->lev[p->L].A;
    i64 n = A->nrow;
    double *r = xmalloc((size_t)n * sizeof(double));
    float *r32 = xmalloc((size_t)n * sizeof(float));
    float *e32 = xmalloc((size_t)n * sizeof(float));
    residual(A, u, b, r);
    double rn = norm2(n, r);
    double r0 = r0_ref > 0 ? r0_ref : rn;
    if (hist) hist[0] = r0 > 0 ? rn / r0 : 0.0;
    int result = -1;
    if (rn <= rtol * r0) result = 0;
    for (int c = 1; result < 0 && c <= max_steps; c++) {
        for (i64 i = 0; i < n; i++) {
            r32[i] = (float)r[i];
            e32[i] = 0.0f;
        }
        vcycle32(&H, p->L, e32, r32, &o);
        for (i64 i = 0; i < n; i++) u[i] += (double)e32[i];
        residual(A, u, b, r);
        rn = norm2(n, r);
        if (hist) hist[c] = rn / r0;
        if (rn <= rtol * r0) result = c;
    }
    free(r);
    free(r32);
    free(e32);
    hier_free(&H); /* frees only the FP32 copies: the FP64 parts are borrowed */
    return result;
}

/* ------------------------------------------------------------------------- */
/* Adjoint gradient with respect to the element coefficients                  */
/* ------------------------------------------------------------------------- */
/* J(u) with A(k) u = b and A(k) = sum_T k_T A_T: dJ/dk_T = -lambda^T A_T u,
 * where A lambda = dJ/du.  A_T is the unit-coefficient element stiffness (in
 * physical coordinates when the geometry is given, the same matrices the
 * assembly uses); Dirichlet nodes carry u = lambda = 0.  out is in cell-lex
 * element order. */
void ohhg_grad_k(void *vp, const double *u, const double *lam, double *out) {
    oproblem *p = vp;
    olevel *Lv = &p->lev[p->L];
    const int N = Lv->N;
#pragma omp parallel for schedule(static)
    for (i64 e = 0; e < Lv->ne; e++) {
        double K[4][4], Mm[4][4], ul[4], ll[4];
        if (Lv->xyz)
            elem_mats_xyz(Lv->xyz, &Lv->ev[4 * e], K, Mm);
        else
            elem_mats(N, &Lv->ev[4 * e], K, Mm);
        for (int a = 0; a < 4; a++) {
            i64 d = dof_vid(N, Lv->ev[4 * e + a]);
            ul[a] = d >= 0 ? u[d] : 0.0;
            ll[a] = d >= 0 ? lam[d] : 0.0;
        }
        double g = 0.0;
        for (int a = 0; a < 4; a++)
            for (int b = 0; b < 4; b++) g += ll[a] * K[a][b] * ul[b];
        /* the reference matrices of elem_mats are scaled by h in the assembly */
        out[Lv->ecl[e]] = -(Lv->xyz ? 1.0 : Lv->h) * g;
    }
}
