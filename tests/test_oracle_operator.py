"""Oracle operator pins: P1 stiffness/mass assembly on the Kuhn meshes
(eq. (2)), linear interpolation and its adjoint (Sec. 2.1)."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_1506_06185_amd import inputs


def lap1d(n):
    return sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1])


def seven_point(N):
    """Textbook 7-point Laplacian (unscaled) on the (N-1)^3 interior grid, x fastest."""
    n = N - 1
    I = sp.identity(n)
    T = lap1d(n)
    return (sp.kron(sp.kron(I, I), T) + sp.kron(sp.kron(I, T), I) + sp.kron(sp.kron(T, I), I)).tocsr()


@pytest.mark.parametrize("n_sub,level", [(1, 3), (2, 3), (3, 2)])
def test_stiffness_is_h_times_seven_point(n_sub, level):
    # For the Kuhn/Freudenthal triangulation the P1 stiffness matrix of the
    # Laplacian is h times the 7-point finite-difference matrix; the other
    # Freudenthal neighbours carry exactly zero.
    p = oracle.Problem(n_sub, level, coarse_level=1)
    A = p.matrix(level, "A")
    N = n_sub << level
    D = (A - seven_point(N) / N).tocoo()
    assert np.abs(D.data).max() < 1e-15 * N
    A.eliminate_zeros()
    assert A.nnz == seven_point(N).nnz


def test_stiffness_symmetric_and_row_sums_zero():
    k = inputs.lognormal_k(2, 2, seed=3)
    p = oracle.Problem(2, 2, coarse_level=1, k=k)
    A = p.matrix(2, "A")
    assert abs(A - A.T).max() < 1e-15
    Af = p.matrix(2, "A", full=True)  # all vertices, before Dirichlet elimination
    assert np.abs(Af @ np.ones(Af.shape[0])).max() < 1e-14
    # with k = 1, linear functions are discrete-harmonic at interior nodes
    Af = oracle.Problem(2, 2, coarse_level=1).matrix(2, "A", full=True)
    N = 8
    v = np.arange((N + 1) ** 3)
    x = (v % (N + 1)) / N
    interior = ((v % (N + 1)) % N != 0) & (((v // (N + 1)) % (N + 1)) % N != 0) & ((v // (N + 1) ** 2) % N != 0)
    assert np.abs((Af @ x)[interior]).max() < 1e-14


def test_spd():
    p = oracle.Problem(1, 3, coarse_level=1, k=inputs.lognormal_k(1, 3, seed=1))
    A = p.matrix(3, "A").toarray()
    np.linalg.cholesky(A)  # raises if not positive definite


def test_single_element_coefficient_is_path_laplacian():
    # A(k) is linear in k and a unit coefficient on one Kuhn tetrahedron adds
    # (h/6) times the Laplacian of its vertex path v0-v1-v2-v3 (the element
    # stiffness from the barycentric gradients).  Checks the element order
    # (cell-lex x permutation) and the scale of the per-element coefficient.
    n_sub, level = 1, 3
    N = n_sub << level
    ne = 6 * N ** 3
    base = oracle.Problem(n_sub, level, coarse_level=1, k=np.ones(ne)).matrix(level, "A", full=True)
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    for cell, q in [((3, 4, 2), 0), ((1, 1, 1), 3), ((5, 2, 6), 5), ((0, 7, 3), 4)]:
        e = 6 * (cell[0] + N * (cell[1] + N * cell[2])) + q
        k = np.ones(ne)
        k[e] = 3.0
        A = oracle.Problem(n_sub, level, coarse_level=1, k=k).matrix(level, "A", full=True)
        D = (A - base).toarray()
        x = list(cell)
        path = [x[0] + (N + 1) * (x[1] + (N + 1) * x[2])]
        for s in range(3):
            x[perms[q][s]] += 1
            path.append(x[0] + (N + 1) * (x[1] + (N + 1) * x[2]))
        Lp = np.array([[1, -1, 0, 0], [-1, 2, -1, 0], [0, -1, 2, -1], [0, 0, -1, 1]], float)
        E = np.zeros_like(D)
        E[np.ix_(path, path)] = 2.0 * Lp / (6 * N)
        assert np.abs(D - E).max() < 1e-14


@pytest.mark.parametrize("var_k", [False, True])
def test_galerkin_identity(var_k):
    # Rediscretised coarse operators equal P^T A P: for k = 1 by nestedness,
    # for per-element k when the coarse coefficient is the mean of the 8 Bey
    # children.
    n_sub, L = 2, 4
    k = inputs.lognormal_k(n_sub, L, seed=7) if var_k else None
    p = oracle.Problem(n_sub, L, coarse_level=2, k=k)
    for l in range(3, L + 1):
        P = p.matrix(l, "P")
        G = (P.T @ p.matrix(l, "A") @ P - p.matrix(l - 1, "A")).tocoo()
        assert np.abs(G.data).max() < 1e-14 * np.abs(p.matrix(l - 1, "A").data).max() * 8


def test_coarse_coefficient_is_child_mean():
    n_sub, L = 1, 2
    k = inputs.lognormal_k(n_sub, L, seed=2)
    p = oracle.Problem(n_sub, L, coarse_level=1, k=k)
    kc = p.coeff(1)
    assert abs(kc.mean() - k.mean()) < 1e-14  # children are 8 per parent, equal volume
    assert np.allclose(p.coeff(L), k)


def test_prolongation_reproduces_linear_functions():
    n_sub, L = 2, 3
    p = oracle.Problem(n_sub, L, coarse_level=1)
    for l in (2, 3):
        P = p.matrix(l, "P", full=True)
        Nf, Nc = n_sub << l, n_sub << (l - 1)

        def lin(N):
            v = np.arange((N + 1) ** 3)
            x, y, z = v % (N + 1) / N, (v // (N + 1)) % (N + 1) / N, v // (N + 1) ** 2 / N
            return 0.3 + 1.7 * x - 2.2 * y + 0.9 * z

        assert np.abs(P @ lin(Nc) - lin(Nf)).max() < 1e-14
        Pi = p.matrix(l, "P")
        assert np.allclose(np.asarray(Pi.sum(axis=1)).ravel()[:5], Pi.sum(axis=1).A1[:5])


def test_mass_matrix_integrals():
    n_sub, L = 2, 2
    p = oracle.Problem(n_sub, L, coarse_level=1)
    Mf = p.matrix(L, "M", full=True)
    N = n_sub << L
    one = np.ones(Mf.shape[0])
    assert abs(one @ Mf @ one - 1.0) < 1e-13  # integral of 1 over the cube
    v = np.arange((N + 1) ** 3)
    x = (v % (N + 1)) / N
    assert abs(one @ Mf @ x - 0.5) < 1e-13  # integral of x
    assert abs(x @ Mf @ x - 1.0 / 3.0) < 1e-13  # integral of x^2, exact for P1 functions
    # an interior node's row sums to the integral of its hat function, h^3
    M = p.matrix(L, "M")
    rs = np.asarray(M.sum(axis=1)).ravel()
    center = ((N // 2 - 1) * (1 + (N - 1) + (N - 1) ** 2))
    Mfull_row = Mf[(N // 2) * (1 + (N + 1) + (N + 1) ** 2)].sum()
    assert abs(Mfull_row - 1.0 / N ** 3) < 1e-16
    assert rs[center] == pytest.approx(1.0 / N ** 3, rel=1e-12)


def test_apply_matches_exported_matrices():
    p = oracle.Problem(2, 3, coarse_level=2)
    u = np.random.default_rng(0).standard_normal(p.ndof)
    assert np.allclose(p.apply_A(u), p.matrix(3, "A") @ u, rtol=0, atol=1e-13)
    assert np.allclose(p.apply_M(u), p.matrix(3, "M") @ u, rtol=0, atol=1e-16)
    r = p.residual(u, np.ones(p.ndof))
    assert np.allclose(r, 1 - p.matrix(3, "A") @ u, atol=1e-13)
    bc = p.restrict(u)
    assert np.allclose(bc, p.matrix(3, "P").T @ u, atol=1e-14)


def test_closed_form_residual_matches_assembled(oracle_problem):
    """The matrix-free k = 1 residual used at level 8 equals the assembled one."""
    import oracle

    for n_sub, level in ((1, 4), (2, 3)):
        p = oracle_problem(n_sub, level)
        g = np.random.default_rng(3)
        u, b = g.standard_normal(p.ndof), g.standard_normal(p.ndof)
        r = oracle.residual_unit_k(u, b, n_sub, level)
        ref = p.residual(u, b)
        assert np.abs(r - ref).max() <= 1e-13 * np.abs(ref).max()
