"""Pins of the oracle's inhomogeneous Dirichlet data (eq. (1), eliminated into
the right-hand side of eq. (2)) against facts the discretisation fixes:

* P1 elements reproduce linear functions: with g linear the discrete solution
  is g at every interior node, for any mesh;
* constants lie in the kernel of the stiffness matrix for any coefficient, so
  g = 1 gives u = 1 with a log-normal k;
* on this mesh the unit-coefficient stiffness is h times the 7-point Laplacian,
  which differentiates quadratics exactly, so a harmonic quadratic g is also
  reproduced exactly (the data of the recovery-strategy workloads);
* the oracle's multigrid solves the same systems to its tolerance.

A sign error, a missing boundary neighbour, a transposed axis or a wrong scale
in the load moves the solution away from g by O(1)."""
import numpy as np
import pytest
import scipy.sparse.linalg as sla

import oracle
from paper_1506_06185_amd import inputs


def grid(n_sub, level):
    N = n_sub << level
    t = np.arange(N + 1) / N
    z, y, x = np.meshgrid(t, t, t, indexing="ij")
    return N, x, y, z


def interior(a):
    return a[1:-1, 1:-1, 1:-1].ravel()


def direct(p, b):
    return sla.spsolve(p.matrix(p.level, "A").tocsc(), b)


@pytest.mark.parametrize("n_sub,level", [(1, 3), (2, 3)])
def test_linear_data_is_reproduced(n_sub, level):
    N, x, y, z = grid(n_sub, level)
    g = 0.5 + 2.0 * x - 3.0 * y + 0.25 * z
    p = oracle.Problem(n_sub, level)
    b = p.dirichlet_load(g.ravel())
    assert np.abs(b).max() > 0.1 / N
    u = direct(p, b)
    assert np.abs(u - interior(g)).max() < 1e-12
    um, cyc, _ = p.solve(b, rtol=1e-13, max_cycles=40)
    assert cyc > 0 and np.abs(um - interior(g)).max() < 1e-11
    p.close()


def test_constant_data_with_variable_coefficient():
    n_sub, level = 1, 3
    N, x, y, z = grid(n_sub, level)
    k = inputs.lognormal_k(n_sub, level, seed=3)
    p = oracle.Problem(n_sub, level, k=k)
    b = p.dirichlet_load(np.full((N + 1) ** 3, 2.5))
    u = direct(p, b)
    assert np.abs(u - 2.5).max() < 1e-12
    # a linear g is not reproduced with variable k (the flux k grad g has a
    # divergence), which shows the coefficient enters the load
    g = x + 2 * y
    u2 = direct(p, p.dirichlet_load(g.ravel()))
    assert np.abs(u2 - interior(g)).max() > 1e-3
    p.close()


@pytest.mark.parametrize("n_sub,level", [(1, 4), (3, 2)])
def test_harmonic_quadratic_is_reproduced(n_sub, level):
    N, x, y, z = grid(n_sub, level)
    g = inputs.harmonic_boundary(n_sub, level)
    assert np.allclose(g.reshape(N + 1, N + 1, N + 1), 1 + x * x + 2 * y * y - 3 * z * z + x * y)
    p = oracle.Problem(n_sub, level)
    b = p.dirichlet_load(g)
    u = direct(p, b)
    assert np.abs(u - interior(g.reshape(N + 1, N + 1, N + 1))).max() < 1e-12
    # only nodes next to the boundary carry load
    bb = b.reshape(N - 1, N - 1, N - 1)
    assert np.all(bb[1:-1, 1:-1, 1:-1] == 0.0) and np.abs(bb[0]).max() > 0
    p.close()


def test_non_harmonic_data_is_not_reproduced():
    # g = x^2 has Laplacian 2: the solution with its boundary values differs
    n_sub, level = 1, 3
    N, x, y, z = grid(n_sub, level)
    g = x * x
    p = oracle.Problem(n_sub, level)
    u = direct(p, p.dirichlet_load(g.ravel()))
    assert np.abs(u - interior(g)).max() > 1e-2
    p.close()
