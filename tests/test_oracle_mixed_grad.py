"""Oracle pins for the FP32-inner / FP64-outer refinement loop and for the
adjoint gradients with respect to f and the per-element coefficient k."""
import numpy as np
import pytest
import scipy.sparse.linalg as spl

import oracle
from paper_1506_06185_amd import inputs


@pytest.mark.parametrize("general", [False, True])
def test_mixed_precision_reaches_fp64_accuracy(oracle_problem, general):
    """With general, on a moved mesh (the FP32 cycle takes the 4-class sweep)."""
    p = oracle.Problem(2, 5, vertices=inputs.perturbed_vertices(2, 7)) if general else oracle_problem(2, 5)
    b = inputs.uniform_load(2, 5, seed=0)
    u64, c64, h64 = p.solve(b, rtol=1e-13, max_cycles=60)
    um, cm, hm = p.solve_mixed(b, rtol=1e-12, max_steps=60)
    assert cm > 0
    assert np.linalg.norm(um - u64) / np.linalg.norm(u64) < 1e-9
    # the FP32 inner cycle keeps the FP64 contraction while the residual is large
    assert abs(cm - c64) <= 3
    assert (hm[1:4] / hm[:3]).max() < 0.75


def _grad_problem(n_sub=1, L=3, seed=0):
    k = inputs.lognormal_k(n_sub, L, seed=seed)
    f = inputs.sine_source(n_sub, L)
    uobs = inputs.gaussian_obs(n_sub, L, seed=seed)
    return k, f, uobs


def _solve_direct(p, L, rhs):
    return spl.spsolve(p.matrix(L, "A").tocsc(), rhs)


@pytest.mark.parametrize("general", [False, True])
def test_adjoint_gradients_match_finite_differences(general):
    """With general, on a macro mesh with moved vertices (physical element
    matrices): the derivative is that of the assembled matrix either way."""
    n_sub, L = 1, 3
    k, f, uobs = _grad_problem(n_sub, L)
    V = inputs.perturbed_vertices(n_sub, 5) if general else None
    p = oracle.Problem(n_sub, L, k=k, vertices=V)
    b = p.apply_M(f)
    u, _, _ = p.solve(b, rtol=1e-13, max_cycles=80)
    lam, _, _ = p.solve(u - uobs, rtol=1e-13, max_cycles=80)
    g_f = p.apply_M(lam)
    g_k = p.grad_k(u, lam)
    eps = 1e-6

    def u_of(kk, ff):
        q = oracle.Problem(n_sub, L, coarse_level=1, k=kk, vertices=V)
        x = _solve_direct(q, L, q.apply_M(ff))
        q.close()
        return x

    def dJ(up, um):  # J(u+) - J(u-) without cancellation of the large terms
        return 0.5 * (up - um) @ (up + um - 2 * uobs)

    dirs_f = inputs.fd_directions(len(f), 4, seed=0)
    dirs_k = inputs.fd_directions(len(k), 4, seed=0, offset=20)
    for d in dirs_f:
        fd = dJ(u_of(k, f + eps * d), u_of(k, f - eps * d)) / (2 * eps)
        an = g_f @ d
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-10, (fd, an)
    # J is not quadratic in k: a step of 1e-4 keeps the central difference's
    # truncation near 1e-8 relative, while at 1e-6 the solves' rounding
    # reaches 1e-6 (on a moved mesh)
    eps_k = 1e-4
    for d in dirs_k:
        fd = dJ(u_of(k + eps_k * d, f), u_of(k - eps_k * d, f)) / (2 * eps_k)
        an = g_k @ d
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-10, (fd, an)


@pytest.mark.parametrize("general", [False, True])
def test_coefficient_gradient_homogeneity(general):
    # A(k) is linear in k, so sum_T k_T dJ/dk_T = -lambda^T A u = -lambda^T b.
    n_sub, L = 2, 3
    k, f, uobs = _grad_problem(n_sub, L, seed=4)
    p = oracle.Problem(n_sub, L, k=k, vertices=inputs.perturbed_vertices(n_sub, 6) if general else None)
    b = p.apply_M(f)
    u, _, _ = p.solve(b, rtol=1e-13, max_cycles=80)
    lam, _, _ = p.solve(u - uobs, rtol=1e-13, max_cycles=80)
    g_k = p.grad_k(u, lam)
    assert k @ g_k == pytest.approx(-(lam @ b), rel=1e-10)


def test_rhs_gradient_is_lambda():
    # dJ/db = lambda: central differences on single load entries
    n_sub, L = 1, 3
    p = oracle.Problem(n_sub, L, coarse_level=1)
    uobs = inputs.gaussian_obs(n_sub, L, seed=1)
    b = p.apply_M(inputs.sine_source(n_sub, L))
    A = p.matrix(L, "A").tocsc()
    u = spl.spsolve(A, b)
    lam = spl.spsolve(A, u - uobs)
    for i in (0, 100, 171, 342):
        e = np.zeros_like(b)
        e[i] = 1e-6
        up, um = spl.spsolve(A, b + e), spl.spsolve(A, b - e)
        fd = 0.5 * (up - um) @ (up + um - 2 * uobs) / 2e-6
        assert fd == pytest.approx(lam[i], rel=1e-7, abs=1e-12)
