"""Oracle pins for the fault model (Sec. 2.2), local recovery and the
Dirichlet-Dirichlet intact cycles (Sec. 4, Alg. 1)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spl

import oracle
from paper_1506_06185_amd import inputs


def kappa(k_faulty, k_free, k_F):
    return (k_faulty - k_free) / k_F  # eq. (3)


def test_fault_zeroes_exactly_the_volume_interior(oracle_problem):
    p = oracle_problem(2, 4)
    m = 16
    u = np.random.default_rng(0).uniform(1, 2, p.ndof)
    counts = p.containment_counts()
    for t in (0, 23, 47):
        uf = p.inject_fault(t, u)
        zero = uf == 0
        assert zero.sum() == (m - 1) * (m - 2) * (m - 3) // 6
        assert np.array_equal(zero, p.tet_mask(t))
        iface = counts > 1  # faces, edges, vertex: redundant containers survive
        assert np.array_equal(uf[iface], u[iface])


def test_exact_recovery_invariant(oracle_problem):
    # Converged solution, fault, then the local Dirichlet problem solved
    # accurately gives back exactly the lost values (eq. (4), row 5).
    p = oracle_problem(2, 4)
    b = p.apply_M(inputs.sine_source(2, 4))
    u, _, _ = p.solve(b, rtol=1e-14, max_cycles=60)
    t = inputs.fault_tet(2, seed=0)
    uf = p.inject_fault(t, u)
    mask = p.tet_mask(t)
    # direct solve of A_FF x = b_F - A_FG u_G with scipy
    A = p.matrix(4, "A").tocsr()
    AFF = A[mask][:, mask]
    rhs = b[mask] - A[mask][:, ~mask] @ uf[~mask]
    x = spl.spsolve(AFF.tocsc(), rhs)
    assert np.abs(x - u[mask]).max() < 1e-10 * np.abs(u).max()
    # the oracle's local multigrid converges to the same values
    ur, res = p.recover_local(t, uf, b, n_cycles=25)
    assert np.abs(ur - u).max() < 1e-10 * np.abs(u).max()
    assert res[-1] < 1e-12


def test_local_cycles_contract_like_global(oracle_problem):
    p = oracle_problem(2, 5)
    b = inputs.uniform_load(2, 5, seed=0)
    u, _, _ = p.solve(b, rtol=1e-6)
    uf = p.inject_fault(11, u)
    _, res = p.recover_local(11, uf, b, n_cycles=8)
    rates = res[1:] / res[:-1]
    assert res[0] < 0.5 and rates[-3:].max() < 0.2, res


def test_joint_recovery_of_disjoint_tets_equals_sequential(oracle_problem):
    p = oracle_problem(2, 4)
    b = inputs.uniform_load(2, 4, seed=3)
    u, _, _ = p.solve(b, rtol=1e-5)
    uf = p.inject_fault(5, p.inject_fault(40, u))
    uj, _ = p.recover_local([5, 40], uf, b, n_cycles=3)
    us, _ = p.recover_local([5], uf, b, n_cycles=3)
    us, _ = p.recover_local([40], us, b, n_cycles=3)
    assert np.abs(uj - us).max() < 1e-13


def _cycles_to(p, b, u, r0, rtol=1e-8, cap=80):
    _, c, _ = p.solve(b, u0=u, rtol=rtol, max_cycles=cap, r0=r0)
    assert c >= 0
    return c


def test_fault_pollution_and_recovery_cycle_counts(oracle_problem):
    # Sec. 2.2: a do-nothing job needs about k_F - 1 extra cycles; local
    # recovery with n_F cycles on the faulty tet removes most of that delay.
    n_sub, L, kF = 2, 5, 5
    p = oracle_problem(n_sub, L)
    b = p.apply_M(inputs.sine_source(n_sub, L))
    r0 = np.linalg.norm(b)
    _, k_free, _ = p.solve(b, rtol=1e-8)
    u5, c, _ = p.solve(b, rtol=0.0, max_cycles=kF)
    t = inputs.fault_tet(n_sub, seed=0)
    uf = p.inject_fault(t, u5)
    k_dn = kF + _cycles_to(p, b, uf, r0)
    ur, _ = p.recover_local(t, uf, b, n_cycles=3)
    k_lr = kF + _cycles_to(p, b, ur, r0)
    kap_dn, kap_lr = kappa(k_dn, k_free, kF), kappa(k_lr, k_free, kF)
    assert 0.6 <= kap_dn <= 1.2, (k_free, k_dn)
    assert kap_lr < kap_dn and kap_lr <= 0.4, (k_free, k_dn, k_lr)


def test_dd_intact_cycles_freeze_the_faulty_closure(oracle_problem):
    n_sub, L = 2, 4
    p = oracle_problem(n_sub, L)
    b = p.apply_M(inputs.sine_source(n_sub, L))
    u, _, _ = p.solve(b, rtol=0.0, max_cycles=3)
    t = 19
    uf = p.inject_fault(t, u)
    closed = p.tet_mask(t, closure=True)
    ui = p.dd_intact([t], uf, b, n_cycles=2)
    assert np.array_equal(ui[closed], uf[closed])
    # the intact residual (outside the closure) goes down
    r_before = np.linalg.norm(p.residual(uf, b)[~closed])
    r_after = np.linalg.norm(p.residual(ui, b)[~closed])
    assert r_after < 0.2 * r_before
    # DD (Alg. 1): intact and local solves are independent, the order does not matter
    ul, _ = p.recover_local(t, uf, b, n_cycles=4)
    a = p.recover_local(t, p.dd_intact([t], uf, b, 2), b, n_cycles=4)[0]
    bb = p.dd_intact([t], ul, b, 2)
    assert np.abs(a - bb).max() < 1e-13
    # with enough intact cycles it converges to the solution with frozen interface
    A = p.matrix(L, "A").tocsr()
    free = ~closed
    x = spl.spsolve(A[free][:, free].tocsc(), b[free] - A[free][:, closed] @ uf[closed])
    uc = p.dd_intact([t], uf, b, 30)
    assert np.abs(uc[free] - x).max() < 1e-10 * np.abs(x).max()


def test_dd_recovery_beats_do_nothing(oracle_problem):
    n_sub, L, kF = 2, 5, 5
    p = oracle_problem(n_sub, L)
    b = p.apply_M(inputs.sine_source(n_sub, L))
    r0 = np.linalg.norm(b)
    _, k_free, _ = p.solve(b, rtol=1e-8)
    u5, _, _ = p.solve(b, rtol=0.0, max_cycles=kF)
    t = inputs.fault_tet(n_sub, seed=0)
    uf = p.inject_fault(t, u5)
    k_dn = kF + _cycles_to(p, b, uf, r0)
    n_I, eta = 1, 4
    n_F = int(np.ceil(eta * n_I))
    u = p.dd_intact([t], uf, b, n_I)
    u, _ = p.recover_local(t, u, b, n_cycles=n_F)
    k_dd = kF + n_I + _cycles_to(p, b, u, r0)  # Sec. 4.4: n_I counts towards k_faulty
    assert kappa(k_dd, k_free, kF) < kappa(k_dn, k_free, kF)


def test_side_matrices_split_the_operator(oracle_problem):
    """Sub-stencils of eq. (5): the matrices assembled over the intact and over
    the faulty macro tetrahedra add up to A; the intact one couples no node
    strictly inside a faulty tet, is symmetric and is SPD on the nodes it
    couples; rows of nodes away from the faulty closures equal A's."""
    n_sub, L = 2, 3
    p = oracle_problem(n_sub, L)
    tets = [5, 30]
    A = p.matrix(L, "A").tocsr()
    AI = p.side_matrix(L, tets, "intact").tocsr()
    AF = p.side_matrix(L, tets, "faulty").tocsr()
    assert abs(AI + AF - A).max() <= 1e-15 * abs(A).max()
    assert abs(AI - AI.T).max() <= 1e-15 * abs(A).max()
    inside = np.zeros(p.ndof, bool)
    closed = np.zeros(p.ndof, bool)
    for t in tets:
        inside |= p.tet_mask(t)
        closed |= p.tet_mask(t, closure=True)
    assert abs(AI[inside]).max() == 0.0 and abs(AI[:, inside]).max() == 0.0
    assert abs(AF[~closed]).max() == 0.0
    away = ~closed
    assert abs(AI[away] - A[away]).max() == 0.0
    free = AI.diagonal() > 0
    assert np.array_equal(free, ~inside & (AI.diagonal() > 0))
    np.linalg.cholesky(AI[free][:, free].toarray())


def test_dn_recovery_keeps_the_exact_solution(oracle_problem):
    """At the converged solution the static Neumann data make the intact side
    stationary, and the local Dirichlet cycles restore the faulty interiors."""
    n_sub, L = 2, 4
    p = oracle_problem(n_sub, L)
    b = p.apply_M(inputs.sine_source(n_sub, L))
    u, _, _ = p.solve(b, rtol=1e-14, max_cycles=80)
    tets = [int(t) for t in inputs.batch_faults(2, n_sub, seed=2)]
    uf = u.copy()
    for t in tets:
        uf = p.inject_fault(t, uf)
    ud = p.dn_recover(tets, uf, b, n_intact=3, eta=4)
    inside = np.zeros(p.ndof, bool)
    for t in tets:
        inside |= p.tet_mask(t)
    scale = np.abs(u).max()
    assert np.abs(ud[~inside] - u[~inside]).max() < 1e-12 * scale
    assert np.abs(ud[inside] - u[inside]).max() < 1e-8 * scale


def test_dn_intact_side_is_one_directional(oracle_problem):
    """The intact side never reads u_F: its result does not depend on the
    faulty interiors; the faulty side reads only the interface values of the
    start of each round, so a round with eta = 0 leaves u_F at zero."""
    n_sub, L = 2, 4
    p = oracle_problem(n_sub, L)
    b = inputs.uniform_load(n_sub, L, seed=4)
    u, _, _ = p.solve(b, rtol=0.0, max_cycles=4)
    t = inputs.fault_tet(n_sub, seed=0)
    uf = p.inject_fault(t, u)
    inside = p.tet_mask(t)
    a = p.dn_recover([t], uf, b, n_intact=2, eta=0)
    assert np.all(a[inside] == 0.0)
    c = p.dn_recover([t], uf, b, n_intact=2, eta=3)
    # equal up to the oracle's own run-to-run rounding (OpenMP reduction order)
    assert np.abs(a[~inside] - c[~inside]).max() <= 1e-13 * np.abs(a).max()
    assert np.abs(c[inside]).max() > 0.0


def test_dn_recovery_beats_do_nothing(oracle_problem):
    n_sub, L, kF = 2, 5, 5
    p = oracle_problem(n_sub, L)
    b = p.apply_M(inputs.sine_source(n_sub, L))
    r0 = np.linalg.norm(b)
    _, k_free, _ = p.solve(b, rtol=1e-8)
    u5, _, _ = p.solve(b, rtol=0.0, max_cycles=kF)
    t = inputs.fault_tet(n_sub, seed=0)
    uf = p.inject_fault(t, u5)
    k_nothing = kF + _cycles_to(p, b, uf, r0)
    n_I, eta = 2, 2
    u = p.dn_recover([t], uf, b, n_intact=n_I, eta=eta)
    k_dn = kF + n_I + _cycles_to(p, b, u, r0)  # Sec. 4.4: n_I counts towards k_faulty
    assert kappa(k_dn, k_free, kF) < kappa(k_nothing, k_free, kF)
