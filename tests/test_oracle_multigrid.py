"""Oracle multigrid pins: smoother, coarse PCG, V-cycle and solve against
direct solves, the manufactured solution and the contraction bound."""
import numpy as np
import pytest
import scipy.sparse.linalg as spl

import oracle
from paper_1506_06185_amd import inputs


def colours(N):
    n = N - 1
    i = np.arange(n ** 3)
    x, y, z = i % n + 1, (i // n) % n + 1, i // n ** 2 + 1
    return ((x + y + z) % 2) == 0


def test_gauss_seidel_colour_pass_properties(oracle_problem):
    p = oracle_problem(2, 3)
    red = colours(p.N)
    g = np.random.default_rng(1)
    u0 = g.standard_normal(p.ndof)
    b = g.standard_normal(p.ndof)
    # omega = 1: a red pass zeroes the red residual and leaves black nodes alone
    u1 = p.smooth(u0, b, omega=1.0, colours=1)
    r1 = p.residual(u1, b)
    assert np.abs(r1[red]).max() < 1e-13 * np.abs(b).max()
    assert np.array_equal(u1[~red], u0[~red])
    # ... and is idempotent
    u2 = p.smooth(u1, b, omega=1.0, colours=1)
    assert np.abs(u2 - u1).max() < 1e-14
    # SOR: the red residual is scaled by (1 - omega)
    r0 = p.residual(u0, b)
    us = p.smooth(u0, b, omega=1.25, colours=1)
    rs = p.residual(us, b)
    assert np.allclose(rs[red], -0.25 * r0[red], atol=1e-12)
    # full sweep = red pass then black pass
    uf = p.smooth(u0, b, omega=1.25, colours=3)
    assert np.array_equal(uf, p.smooth(p.smooth(u0, b, 1.25, 1), b, 1.25, 2))


def test_coarse_pcg_matches_dense(oracle_problem):
    p = oracle_problem(2, 3)
    A = p.matrix(2, "A").toarray()
    b = np.random.default_rng(2).standard_normal(A.shape[0])
    x, it = p.coarse_solve(b)
    assert np.abs(x - np.linalg.solve(A, b)).max() < 1e-12 * np.abs(x).max()
    assert 0 < it < 343


@pytest.mark.parametrize("n_sub,level", [(1, 4), (2, 4)])
def test_multigrid_solve_matches_direct(oracle_problem, n_sub, level):
    p = oracle_problem(n_sub, level)
    b = p.apply_M(inputs.sine_source(n_sub, level))
    u, cycles, hist = p.solve(b, rtol=1e-13, max_cycles=60)
    assert cycles > 0
    ud = spl.spsolve(p.matrix(level, "A").tocsc(), b)
    assert np.abs(u - ud).max() / np.abs(ud).max() < 1e-11


def test_manufactured_solution_second_order():
    # P1 on the Kuhn meshes is second order in the nodal max norm for the
    # smooth solution sin(pi x) sin(pi y) sin(pi z).
    errs = []
    for L in (3, 4, 5):
        p = oracle.Problem(1, L)
        b = p.apply_M(inputs.sine_source(1, L))
        u, cycles, _ = p.solve(b, rtol=1e-12)
        errs.append(np.abs(u - inputs.sine_solution(1, L)).max())
        p.close()
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(3.6 < r < 4.4 for r in ratios), (errs, ratios)
    assert errs[-1] < 5e-3


def test_vcycle_contraction_below_0p2(oracle_problem):
    # omega = 1.25, V(2,1): the asymptotic residual contraction is below 0.2.
    p = oracle_problem(2, 5)
    b = inputs.uniform_load(2, 5, seed=0)
    u, cycles, hist = p.solve(b, rtol=1e-13, max_cycles=40)
    rates = hist[1:] / hist[:-1]
    assert rates[-4:].max() < 0.2, rates
    # plain Gauss-Seidel (omega = 1) is slower on this hierarchy
    u1, c1, h1 = p.solve(b, omega=1.0, rtol=1e-10, max_cycles=60)
    assert c1 > 0 and (h1[1:] / h1[:-1])[-3:].max() < 0.35


def test_vcycle_reduces_energy_error(oracle_problem):
    p = oracle_problem(2, 4)
    A = p.matrix(4, "A")
    b = inputs.uniform_load(2, 4, seed=1)
    ud = spl.spsolve(A.tocsc(), b)
    u = np.zeros_like(b)
    e0 = np.sqrt((u - ud) @ (A @ (u - ud)))
    for _ in range(3):
        u, _ = p.vcycle(u, b)
        e1 = np.sqrt((u - ud) @ (A @ (u - ud)))
        assert e1 < 0.5 * e0
        e0 = e1


def test_solve_history_and_reference(oracle_problem):
    p = oracle_problem(2, 4)
    b = p.apply_M(inputs.sine_source(2, 4))
    u, c, hist = p.solve(b, rtol=1e-8)
    assert hist[0] == 1.0 and hist[-1] <= 1e-8 and hist[-2] > 1e-8
    assert np.linalg.norm(p.residual(u, b)) / np.linalg.norm(b) == pytest.approx(hist[-1], rel=1e-10)
