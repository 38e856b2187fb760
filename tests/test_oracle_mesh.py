"""Pins of the oracle on general (unstructured) macro meshes, Sec. 3.1: every
macro tetrahedron of a vertex/tetrahedron list refined regularly, P1
elements, Dirichlet boundary on the faces that belong to one tetrahedron.

Each check compares with something fixed outside the oracle: closed-form node
counts of a regular refinement, the exactness of P1 on linear functions
(energy |a|^2 vol, zero interior rows), the volume and first moments of the
domain, the Galerkin identity of nested spaces, the independence of the four
colour classes, a sparse direct solve, O(h^2) nodal convergence to a smooth
solution, and the invariant that a local recovery with exact interface data
returns the exact solution."""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from paper_1506_06185_amd import inputs


def mesh(name):
    if name == "octa8":
        v, t = inputs.octahedron_mesh(True)
        return inputs.perturb_mesh(v, seed=3, amplitude=0.08), t
    if name == "octa4":
        return inputs.octahedron_mesh(False)
    if name == "box211":
        return inputs.box_mesh(2, 1, 1)
    if name == "box222p":
        v, t = inputs.box_mesh(2, 2, 2)
        return inputs.perturb_mesh(v, seed=5, amplitude=0.12), t
    raise KeyError(name)


NAMES = ["octa8", "octa4", "box211", "box222p"]


def tet_volumes(v, t):
    e = v[t[:, 1:]] - v[t[:, :1]]
    return np.abs(np.linalg.det(e)) / 6.0


def primitives(t):
    """Edges, faces (sorted vertex tuples) and which of them are boundary."""
    faces = {}
    for tet in t:
        for f in itertools.combinations(sorted(tet), 3):
            faces[f] = faces.get(f, 0) + 1
    bfaces = [f for f, c in faces.items() if c == 1]
    edges = {e for tet in t for e in itertools.combinations(sorted(tet), 2)}
    bverts = {x for f in bfaces for x in f}
    bedges = {e for f in bfaces for e in itertools.combinations(f, 2)}
    return edges, set(faces), bverts, bedges, set(bfaces)


@pytest.mark.parametrize("name", NAMES)
def test_node_counts_closed_form(name):
    v, t = mesh(name)
    edges, faces, bverts, bedges, bfaces = primitives(t)
    p = oracle.MeshProblem(v, t, 4, 2)
    for l in range(0, 5):
        m = 2 ** l - 1
        per = (m, m * (m - 1) // 2, m * (m - 1) * (m - 2) // 6)
        nn = len(v) + len(edges) * per[0] + len(faces) * per[1] + len(t) * per[2]
        ni = (len(v) - len(bverts)) + (len(edges) - len(bedges)) * per[0] + (len(faces) - len(bfaces)) * per[1] \
            + len(t) * per[2]
        xyz, dof = p.nodes(l)
        assert len(xyz) == nn
        assert int((dof >= 0).sum()) == ni == p.ndof_at(l)
        assert sorted(dof[dof >= 0]) == list(range(ni))


@pytest.mark.parametrize("name", NAMES)
def test_keys_match_positions_and_nodes_are_distinct(name):
    v, t = mesh(name)
    L = 3
    p = oracle.MeshProblem(v, t, L, 2)
    xyz, _ = p.nodes(L)
    k = p.keys(L)
    w = np.where(k[:, :, 0] >= 0, k[:, :, 1], 0)
    assert np.all(w.sum(axis=1) == 2 ** L)
    pos = np.einsum("na,nad->nd", w / 2.0 ** L, v[np.maximum(k[:, :, 0], 0)])
    assert np.abs(pos - xyz).max() < 1e-13
    # every support lies in one macro tetrahedron
    sets = [set(tt) for tt in t]
    for row in k:
        s = {int(a) for a in row[:, 0] if a >= 0}
        assert any(s <= q for q in sets)
    r = np.round(xyz * 2 ** 20).astype(np.int64)
    assert len({tuple(x) for x in r}) == len(r)


def test_user_order_follows_the_documented_primitive_order():
    v, t = mesh("octa8")
    L = 3
    p = oracle.MeshProblem(v, t, L, 2)
    k = p.keys(L)
    _, dof = p.nodes(L)
    order = []
    for n in np.flatnonzero(dof >= 0):
        vs = [int(a) for a in k[n, :, 0] if a >= 0]
        ws = {int(a): int(b) for a, b in k[n] if a >= 0}
        if len(vs) == 4:
            tid = next(i for i, tt in enumerate(t) if set(tt) == set(vs))
            key = (3, (tid,), tuple(ws[int(t[tid][r])] for r in (3, 2, 1)))
        elif len(vs) == 3:
            key = (2, tuple(vs), (ws[vs[2]], ws[vs[1]]))
        elif len(vs) == 2:
            key = (1, tuple(vs), (ws[vs[1]],))
        else:
            key = (0, tuple(vs), ())
        order.append((key, n))
    expect = [n for _, n in sorted(order)]
    got = np.argsort(dof[dof >= 0].astype(np.int64))
    got = np.flatnonzero(dof >= 0)[got]
    assert list(got) == expect
    # the interior macro vertex (the origin) comes first
    assert p.interior_positions(L)[0] == pytest.approx(v[0])


@pytest.mark.parametrize("name", NAMES)
def test_p1_exact_on_linear_functions(name):
    v, t = mesh(name)
    L = 3
    p = oracle.MeshProblem(v, t, L, 2)
    xyz, dof = p.nodes(L)
    A = p.matrix(L, "A", full=True)
    M = p.matrix(L, "M", full=True)
    vol = tet_volumes(v, t)
    assert abs(A - A.T).max() < 1e-14
    assert np.abs(A @ np.ones(len(xyz))).max() < 1e-12
    a = np.array([0.3, -1.1, 0.7])
    f = xyz @ a + 0.25
    assert f @ (A @ f) == pytest.approx(a @ a * vol.sum(), rel=1e-12)
    # zero on the interior rows: a linear function is discrete-harmonic
    assert np.abs((A @ f)[dof >= 0]).max() < 1e-12
    one = np.ones(len(xyz))
    assert one @ (M @ one) == pytest.approx(vol.sum(), rel=1e-12)
    cent = v[t].mean(axis=1)
    assert one @ (M @ xyz) == pytest.approx((vol[:, None] * cent).sum(axis=0), rel=1e-12, abs=1e-14)
    # positive definite on the interior
    Ai = p.matrix(L, "A")
    assert spla.eigsh(Ai, k=1, which="SA", return_eigenvectors=False, tol=1e-8)[0] > 0


@pytest.mark.parametrize("name", NAMES)
def test_prolongation_and_galerkin(name):
    v, t = mesh(name)
    L = 4
    p = oracle.MeshProblem(v, t, L, 2)
    for l in (3, 4):
        Pf = p.matrix(l, "P", full=True)
        xf, _ = p.nodes(l)
        xc, _ = p.nodes(l - 1)
        a = np.array([1.5, 0.2, -0.9])
        assert np.abs(Pf @ (xc @ a) - xf @ a).max() < 1e-13
        P = p.matrix(l, "P")
        Ac = P.T @ p.matrix(l, "A") @ P
        A0 = p.matrix(l - 1, "A")
        assert abs(Ac - A0).max() < 1e-12 * abs(A0).max()
        # transfers of the oracle's cycle are these matrices
        r = np.random.default_rng(l).standard_normal(p.ndof_at(l))
        assert np.abs(p.restrict(r, l) - P.T @ r).max() < 1e-13
        ec = np.random.default_rng(l + 10).standard_normal(p.ndof_at(l - 1))
        assert np.abs(p.prolong_add(ec, np.zeros(p.ndof_at(l)), l) - P @ ec).max() < 1e-14


def colour_classes(p, t, l):
    """(sum over the support of colour x weight) mod 4, colours being the
    vertex positions in the tetrahedra."""
    col = {}
    for tt in t:
        for r, x in enumerate(tt):
            col[int(x)] = r
    k = p.keys(l)
    _, dof = p.nodes(l)
    cls = np.empty(p.ndof_at(l), dtype=np.int64)
    for n in np.flatnonzero(dof >= 0):
        cls[dof[n]] = sum(col[int(a)] * int(b) for a, b in k[n] if a >= 0) % 4
    return cls


@pytest.mark.parametrize("name", NAMES)
def test_colour_classes_decouple_and_class_passes(name):
    v, t = mesh(name)
    L = 3
    p = oracle.MeshProblem(v, t, L, 2)
    A = p.matrix(L, "A").tocsr()
    cls = colour_classes(p, t, L)
    for c in range(4):
        idx = np.flatnonzero(cls == c)
        sub = A[idx][:, idx]
        assert abs(sub - sp.diags(sub.diagonal())).max() == 0.0, c
    g = np.random.default_rng(7)
    u = g.standard_normal(p.ndof)
    b = g.standard_normal(p.ndof)
    d = A.diagonal()
    w = 1.25
    for c in range(4):
        ref = u.copy()
        sel = cls == c
        ref[sel] += w * (b - A @ u)[sel] / d[sel]
        got = p.smooth(u, b, omega=w, colours=1 << c)
        assert np.abs(got - ref).max() < 1e-13
    # a full sweep = the four passes in order
    ref = u.copy()
    for c in range(4):
        sel = cls == c
        ref[sel] += w * (b - A @ ref)[sel] / d[sel]
    assert np.abs(p.smooth(u, b, omega=w, colours=15) - ref).max() < 1e-12


@pytest.mark.parametrize("name", NAMES)
def test_multigrid_matches_direct_solve(name):
    v, t = mesh(name)
    L = 4
    p = oracle.MeshProblem(v, t, L, 2)
    b = np.random.default_rng(11).uniform(-1, 1, p.ndof)
    x = spla.spsolve(p.matrix(L, "A").tocsc(), b)
    u, cycles, hist = p.solve(b, rtol=1e-12, max_cycles=60)
    assert cycles > 0
    assert np.abs(u - x).max() < 1e-9 * np.abs(x).max()
    rho = (hist[-1] / hist[0]) ** (1.0 / (len(hist) - 1))
    assert rho < 0.3, rho


def test_second_order_convergence_on_the_box():
    # u = sin(pi x / 2) sin(pi y) sin(pi z) on [0,2]x[0,1]^2, -lap u = 9/4 pi^2 u
    v, t = inputs.box_mesh(2, 1, 1)
    errs = []
    for L in (3, 4, 5):
        p = oracle.MeshProblem(v, t, L, 1)
        x = p.interior_positions(L)
        ue = np.sin(np.pi * x[:, 0] / 2) * np.sin(np.pi * x[:, 1]) * np.sin(np.pi * x[:, 2])
        xyz, dof = p.nodes(L)
        fe = 2.25 * np.pi ** 2 * np.sin(np.pi * xyz[:, 0] / 2) * np.sin(np.pi * xyz[:, 1]) * np.sin(np.pi * xyz[:, 2])
        b = (p.matrix(L, "M", full=True) @ fe)[np.argsort(np.where(dof >= 0, dof, 1 << 40))[: p.ndof]]
        u, _, _ = p.solve(b, rtol=1e-12, max_cycles=60)
        errs.append(np.abs(u - ue).max())
    r = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(r > 3.4) and r[-1] > r[0], (errs, r)


@pytest.mark.parametrize("name", ["octa8", "box222p"])
def test_local_recovery_with_exact_data_restores_the_solution(name):
    v, t = mesh(name)
    L = 4
    p = oracle.MeshProblem(v, t, L, 2)
    b = np.random.default_rng(13).uniform(-1, 1, p.ndof)
    x = spla.spsolve(p.matrix(L, "A").tocsc(), b)
    tet = inputs.mesh_fault_tet(len(t), seed=1)
    m = 2 ** L - 1
    mask = p.tet_mask(tet)
    assert mask.sum() == m * (m - 1) * (m - 2) // 6
    uf = p.inject_fault(tet, x)
    assert np.all(uf[mask] == 0) and np.all(uf[~mask] == x[~mask])
    ur, res = p.recover_local([tet], uf, b, n_cycles=30)
    assert np.abs(ur - x).max() < 1e-10 * np.abs(x).max()
    assert res[-1] < 1e-12
    # the Dirichlet-Dirichlet intact cycles leave an exact solution exact
    ud = p.dd_intact([tet], x, b, n_cycles=2)
    assert np.abs(ud - x).max() < 1e-12 * np.abs(x).max()


def test_containment_counts_on_a_mesh():
    v, t = mesh("box222p")
    L = 3
    p = oracle.MeshProblem(v, t, L, 2)
    cnt = p.containment_counts(L)
    k = p.keys(L)
    _, dof = p.nodes(L)
    sets = [set(tt) for tt in t]
    ref = np.empty(p.ndof, dtype=np.int64)
    for n in np.flatnonzero(dof >= 0):
        s = {int(a) for a in k[n, :, 0] if a >= 0}
        ref[dof[n]] = sum(s <= q for q in sets)
    assert np.array_equal(cnt, ref)
    closure = sum(p.tet_mask(q, closure=True, level=L).astype(np.int64) for q in range(len(t)))
    assert np.array_equal(closure, ref)


def test_invalid_meshes_are_rejected():
    v, t = inputs.octahedron_mesh(True)
    bad = t.copy()
    bad[0, [2, 3]] = bad[0, [3, 2]]  # colours inconsistent with the other tets
    with pytest.raises(ValueError):
        oracle.MeshProblem(v, bad, 3, 2)
    bad = t.copy()
    bad[1, 0] = len(v)
    with pytest.raises(ValueError):
        oracle.MeshProblem(v, bad, 3, 2)
    flat = v.copy()
    flat[:, 2] = 0.0
    with pytest.raises(ValueError):
        oracle.MeshProblem(flat, t, 3, 2)


def test_dirichlet_neumann_recovery_on_a_mesh():
    # eq. (5): the two one-sided stiffness matrices add up to A; with exact
    # data the DN rounds (Alg. 2) converge to the exact solution
    v, t = mesh("box222p")
    L = 4
    p = oracle.MeshProblem(v, t, L, 2)
    tet = inputs.mesh_fault_tet(len(t), seed=1)
    Ai, Af = p.side_matrix(L, [tet], "intact"), p.side_matrix(L, [tet], "faulty")
    A = p.matrix(L, "A")
    assert abs(Ai + Af - A).max() < 1e-15 * abs(A).max() * 10
    mask = p.tet_mask(tet)
    assert abs(Ai[mask]).max() == 0.0
    b = np.random.default_rng(13).uniform(-1, 1, p.ndof)
    x = spla.spsolve(A.tocsc(), b)
    uf = p.inject_fault(tet, x)
    errs = [np.abs(p.dn_recover([tet], uf, b, n_intact=n, eta=2) - x).max() for n in (1, 3, 6)]
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-12 * np.abs(x).max(), errs


@pytest.mark.parametrize("name", ["octa8", "box222p", "octa4"])
def test_dirichlet_data_linear_reproduction(name):
    """eq. (1): Laplace's equation with the boundary values of a linear
    function has that function as its discrete solution (P1 reproduces
    linear functions), on any mesh; the boundary order lists every
    non-interior node once."""
    v, t = mesh(name)
    L = 4
    p = oracle.MeshProblem(v, t, L, 2)
    xyz, dof = p.nodes(L)
    order = p.boundary_order(L)
    assert sorted(order) == sorted(np.flatnonzero(dof < 0))
    a, c = np.array([0.4, -1.0, 0.7]), 0.3
    b = p.dirichlet_load(xyz[order] @ a + c)
    u, _, _ = p.solve(b, rtol=1e-13, max_cycles=80)
    assert np.abs(u - (p.interior_positions(L) @ a + c)).max() < 1e-11
    # a quadratic is not reproduced
    q = p.dirichlet_load(xyz[order, 0] ** 2)
    uq, _, _ = p.solve(q, rtol=1e-13, max_cycles=80)
    assert np.abs(uq - p.interior_positions(L)[:, 0] ** 2).max() > 1e-3


def layered_k(v, t, k_low, k_high, z0):
    """k per tetrahedron: k_low below the plane z = z0, k_high above it."""
    zc = np.asarray(v)[np.asarray(t)][:, :, 2].mean(axis=1)
    return np.where(zc < z0, k_low, k_high).astype(np.float64)


def test_mesh_coefficient_per_tetrahedron_transmission():
    """eq. (2) with k constant on each macro tetrahedron: two layers of the
    box [0,2]^2 x [0,2] with k = 1 below z = 1 and k = 5 above.  A function
    that is linear on each layer, continuous, with the same x and y slopes
    and the normal fluxes k du/dz equal on z = 1, has zero weak Laplacian;
    P1 elements reproduce it (the layers meet on element faces), so the
    solve from its boundary values returns it at every interior node.  With
    one k the kink is not reproduced."""
    v, t = inputs.box_mesh(2, 2, 2)
    L = 4
    k = layered_k(v, t, 1.0, 5.0, 1.0)
    assert 0 < (k == 5.0).sum() < len(t)
    p = oracle.MeshProblem(v, t, L, 2, k_tet=k)

    def exact(x):
        z = x[:, 2]
        return 0.3 * x[:, 0] - 0.7 * x[:, 1] + np.where(z < 1.0, 2.0 * z, 2.0 + 0.4 * (z - 1.0)) + 0.1

    xyz, dof = p.nodes(L)
    order = p.boundary_order(L)
    u, _, _ = p.solve(p.dirichlet_load(exact(xyz[order])), rtol=1e-13, max_cycles=80)
    xi = p.interior_positions(L)
    assert np.abs(u - exact(xi)).max() < 1e-11
    p1 = oracle.MeshProblem(v, t, L, 2)
    u1, _, _ = p1.solve(p1.dirichlet_load(exact(xyz[order])), rtol=1e-13, max_cycles=80)
    assert np.abs(u1 - exact(xi)).max() > 1e-3


def test_mesh_coefficient_per_tetrahedron_scaling_and_sides():
    """A constant k scales the operator of every level; a piecewise k splits
    it into the one-sided matrices of eq. (5), which keep their k."""
    v, t = mesh("box222p")
    L = 3
    p1 = oracle.MeshProblem(v, t, L, 2)
    pc = oracle.MeshProblem(v, t, L, 2, k_tet=np.full(len(t), 2.5))
    for l in (2, 3):
        A1, Ac = p1.matrix(l, "A"), pc.matrix(l, "A")
        assert abs(Ac - 2.5 * A1).max() <= 1e-14 * abs(Ac).max()
    k = np.random.default_rng(3).uniform(0.5, 4.0, len(t))
    pk = oracle.MeshProblem(v, t, L, 2, k_tet=k)
    tet = inputs.mesh_fault_tet(len(t), seed=2)
    Ai, Af = pk.side_matrix(L, [tet], "intact"), pk.side_matrix(L, [tet], "faulty")
    Ak = pk.matrix(L, "A")
    assert abs(Ai + Af - Ak).max() <= 1e-14 * abs(Ak).max()
    # the faulty side is k of that tetrahedron times its unit-k part
    Af1 = p1.side_matrix(L, [tet], "faulty")
    assert abs(Af - k[tet] * Af1).max() <= 1e-14 * abs(Af).max()
    with pytest.raises(ValueError):
        oracle.MeshProblem(v, t, L, 2, k_tet=np.zeros(len(t)))


def test_mesh_gradient_per_tetrahedron_matches_finite_differences():
    """J(k) = 1/2 |u(k) - u_obs|^2 with A(k) u = b and k constant on each
    macro tetrahedron: the adjoint gradient dJ/dk_t = -lambda^T A_t u
    (A lambda = u - u_obs) against central differences of direct sparse
    solves with k_t moved by +-1e-5."""
    v, t = mesh("octa8")
    L = 3
    k = np.random.default_rng(23).uniform(0.5, 3.0, len(t))
    b = np.random.default_rng(29).uniform(-1, 1, oracle.MeshProblem(v, t, L, 2).ndof)
    u_obs = np.random.default_rng(31).uniform(-0.1, 0.1, b.size)

    def solve(kk):
        A = oracle.MeshProblem(v, t, L, 2, k_tet=kk).matrix(L, "A").tocsc()
        return spla.spsolve(A, b), A

    u, A = solve(k)
    lam = spla.spsolve(A, u - u_obs)
    g = oracle.MeshProblem(v, t, L, 2, k_tet=k).grad_k_tet(u, lam)
    d = 1e-5
    for q in (0, 3, 6):
        kp, km = k.copy(), k.copy()
        kp[q] += d
        km[q] -= d
        jp = 0.5 * np.sum((solve(kp)[0] - u_obs) ** 2)
        jm = 0.5 * np.sum((solve(km)[0] - u_obs) ** 2)
        fd = (jp - jm) / (2 * d)
        assert abs(g[q] - fd) <= 1e-6 * max(abs(fd), 1e-12) + 1e-12, (q, g[q], fd)
    # sum over tetrahedra of k_t dJ/dk_t = -lambda^T A u
    assert abs(np.dot(k, g) + lam @ (A @ u)) <= 1e-12 * abs(lam @ (A @ u))
