"""Pins of the oracle on general macro meshes (the Kuhn connectivity with moved
macro vertices, so every macro tetrahedron has its own shape and the stiffness
a full 15-point stencil), against facts that do not come from the oracle:

* refined vertices are the affine images of the reference lattice of their
  macro tetrahedron (Bey's refinement of an affine tetrahedron);
* P1 elements reproduce linear functions on any mesh: with linear Dirichlet
  data the discrete solution is that function at every interior vertex;
* the stiffness is symmetric with zero row sums over all vertices, and its
  interior block is positive definite;
* with the macro vertices on the grid the operator is the Kuhn operator;
* every edge joins vertices whose (x+y+z) classes mod 4 differ, so the
  4-colour SOR sweep is a Gauss-Seidel sweep, and the moved mesh couples all
  14 neighbours of a vertex;
* the discretisation error of a smooth solution decays like h^2 and the
  V(2,1) cycle still contracts."""
import numpy as np
import pytest
import scipy.sparse.linalg as sla

import oracle
from paper_1506_06185_amd import inputs


def grid_idx(N):
    t = np.arange(N + 1)
    z, y, x = np.meshgrid(t, t, t, indexing="ij")
    return x.ravel(), y.ravel(), z.ravel()


def interior_mask(N):
    x, y, z = grid_idx(N)
    return (x > 0) & (y > 0) & (z > 0) & (x < N) & (y < N) & (z < N)


@pytest.mark.parametrize("n_sub,level", [(1, 3), (2, 2)])
def test_refined_vertices_are_affine_images(n_sub, level):
    V = inputs.perturbed_vertices(n_sub, seed=1)
    p = oracle.Problem(n_sub, level, vertices=V)
    X = p.positions(level)
    N, m = n_sub << level, 1 << level
    perms = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))
    for tet in range(6 * n_sub ** 3):
        P = inputs.macro_tet_corners(V, n_sub, tet)
        cube, q = divmod(tet, 6)
        c = np.array([cube % n_sub, (cube // n_sub) % n_sub, cube // (n_sub * n_sub)])
        a, b, cc = (np.eye(3, dtype=int)[perms[q][s]] for s in range(3))
        for i in range(m + 1):
            for j in range(m + 1 - i):
                for k in range(m + 1 - i - j):
                    g = m * c + i * a + j * (a + b) + k * (a + b + cc)
                    v = g[0] + (N + 1) * (g[1] + (N + 1) * g[2])
                    want = P[0] + (i * (P[1] - P[0]) + j * (P[2] - P[0]) + k * (P[3] - P[0])) / m
                    assert np.allclose(X[v], want, atol=1e-14)
    p.close()


@pytest.mark.parametrize("n_sub,level", [(1, 3), (2, 3)])
def test_linear_data_reproduced_on_a_general_mesh(n_sub, level):
    V = inputs.perturbed_vertices(n_sub, seed=2)
    p = oracle.Problem(n_sub, level, vertices=V)
    X = p.positions(level)
    g = 0.3 + 1.5 * X[:, 0] - 2.0 * X[:, 1] + 0.75 * X[:, 2]
    b = p.dirichlet_load(g)
    u = sla.spsolve(p.matrix(level, "A").tocsc(), b)
    N = n_sub << level
    assert np.abs(u - g[interior_mask(N)]).max() < 1e-11
    p.close()


def test_stiffness_structure_on_a_general_mesh():
    n_sub, level = 2, 2
    V = inputs.perturbed_vertices(n_sub, seed=3)
    p = oracle.Problem(n_sub, level, vertices=V)
    A = p.matrix(level, "A", full=True)
    assert abs(A - A.T).max() < 1e-14
    assert np.abs(np.asarray(A.sum(axis=1))).max() < 1e-13
    Ai = p.matrix(level, "A").toarray()
    assert np.linalg.eigvalsh(Ai).min() > 0
    # same-class couplings vanish; all 14 neighbours of an interior vertex couple
    N = n_sub << level
    x, y, z = grid_idx(N)
    cls = (x + y + z) % 4
    Ac = A.tocoo()
    off = Ac.row != Ac.col
    assert np.all(cls[Ac.row[off]] != cls[Ac.col[off]])
    nnz = np.diff(A.tocsr().indptr)[interior_mask(N)]
    assert nnz.min() == 15 and nnz.max() == 15
    p.close()


def test_grid_vertices_give_the_kuhn_operator():
    n_sub, level = 2, 3
    V = inputs.perturbed_vertices(n_sub, seed=0, amplitude=0.0)
    pg = oracle.Problem(n_sub, level, vertices=V)
    pk = oracle.Problem(n_sub, level)
    assert abs(pg.matrix(level, "A") - pk.matrix(level, "A")).max() < 1e-14
    assert abs(pg.matrix(level, "M") - pk.matrix(level, "M")).max() < 1e-16
    pg.close()
    pk.close()


def test_four_colour_sweep_is_gauss_seidel():
    # sweeping the 4 classes one by one equals the sequential Gauss-Seidel of
    # those classes (SOR factor 1): each class sees the updated earlier ones
    n_sub, level = 2, 2
    V = inputs.perturbed_vertices(n_sub, seed=4)
    p = oracle.Problem(n_sub, level, vertices=V)
    A = p.matrix(level, "A").toarray()
    rng = np.random.default_rng(0)
    u0, b = rng.standard_normal(A.shape[0]), rng.standard_normal(A.shape[0])
    got = p.smooth(u0, b, omega=1.0, colours=15)
    N = n_sub << level
    x, y, z = grid_idx(N)
    cls = ((x + y + z) % 4)[interior_mask(N)]
    u = u0.copy()
    for c in range(4):
        for i in np.nonzero(cls == c)[0]:
            u[i] += (b[i] - A[i] @ u) / A[i, i]
    assert np.abs(got - u).max() < 1e-12
    p.close()


def test_convergence_and_contraction_on_a_general_mesh():
    # -Laplace(u) = f with u = g on the boundary, u = exp(x) sin(y) + z^2
    # (f = -2), on the moved mesh at levels 3 and 4: nodal errors fall like h^2
    n_sub = 2
    V = inputs.perturbed_vertices(n_sub, seed=5)
    errs = []
    for level in (3, 4):
        p = oracle.Problem(n_sub, level, vertices=V)
        X = p.positions(level)
        ue = np.exp(X[:, 0]) * np.sin(X[:, 1]) + X[:, 2] ** 2
        f = np.full(len(X), -2.0)
        N = n_sub << level
        inn = interior_mask(N)
        Mf = p.matrix(level, "M", full=True) @ f
        b = Mf[inn] + p.dirichlet_load(ue)
        u, cyc, hist = p.solve(b, rtol=1e-12, max_cycles=60)
        rates = hist[1:cyc + 1] / hist[:cyc]
        assert rates[2:].max() < 0.3, rates
        errs.append(np.abs(u - ue[inn]).max())
        p.close()
    assert 3.0 < errs[0] / errs[1] < 5.0, errs
