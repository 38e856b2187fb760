"""GPU parity on general macro meshes (moved macro vertices, Sec. 3.1's
unstructured macro mesh with regularly refined macro elements): 15-point
operators, the 4-class SOR passes, the coarsest-level solve, V-cycle
iterates, solves, local and Dirichlet-Dirichlet recovery, all through the C
ABI against the oracle assembled in physical coordinates on the same
vertices.  Tolerances as for the cube: per operator and iterate 1e-12
relative, converged solutions 1e-10.  At the benchmark size (2 subcubes per
axis, level 7) the operator is checked on linear functions, which the P1
space reproduces exactly, and a solve must recover the linear function from
its own boundary data."""
import numpy as np
import pytest

import oracle
from paper_1506_06185_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

_PROBLEMS = {}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def hh():
    from paper_1506_06185_amd import hhgr

    hhgr.lib()
    return hhgr


def T(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(dev)


def Nn(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def problem(n_sub, level, seed):
    key = (n_sub, level, seed)
    if key not in _PROBLEMS:
        _PROBLEMS[key] = oracle.Problem(n_sub, level, vertices=inputs.perturbed_vertices(n_sub, seed))
    return _PROBLEMS[key]


def context(hh, dev, n_sub, level, seed, **kw):
    ctx = hh.Context(device=dev, n_sub=n_sub, level=level, general_geometry=True, **kw)
    ctx.set_geometry(inputs.perturbed_vertices(n_sub, seed))
    return ctx


# several workgroups per class list and ragged tails; 1, 2 and 3 subcubes per axis
CASES = [(1, 5, 3), (2, 4, 5), (3, 3, 7)]


@pytest.mark.parametrize("n_sub,level,seed", CASES)
def test_operator_and_class_passes(dev, hh, n_sub, level, seed):
    print(f"\n[general op] n_sub={n_sub} level={level} seed={seed}", flush=True)
    ctx = context(hh, dev, n_sub, level, seed)
    p = problem(n_sub, level, seed)
    g = np.random.default_rng(100 + seed)
    for l in range(2, level + 1):
        nd = p.ndof_at(l)
        u, b = g.standard_normal(nd), g.standard_normal(nd)
        r = Nn(hh.debug_op(ctx, 0, l, T(u, dev), T(b, dev)))
        assert rel(r, p.residual(u, b, level=l)) < 1e-12, l
        for mask in (1, 2, 4, 8, 5, 10, 15):
            us = Nn(hh.debug_op(ctx, 8 + mask, l, T(u, dev), T(b, dev)))
            assert rel(us, p.smooth(u, b, omega=1.25, colours=mask, level=l)) < 1e-12, (l, mask)
        us = Nn(hh.debug_op(ctx, 3, l, T(u, dev), T(b, dev)))
        assert rel(us, p.smooth(u, b, omega=1.25, colours=15, level=l)) < 1e-12, l
        if l > 2:
            # the transfers are those of the cube (index space, affine refinement)
            rc = Nn(hh.debug_op(ctx, 4, l, T(r, dev)))
            assert rel(rc, p.restrict(r, level=l)) < 1e-12, l
    bc = g.standard_normal(p.ndof_at(2))
    uc = Nn(hh.debug_op(ctx, 6, 2, T(bc, dev)))
    uo = p.coarse_solve(bc)
    uo = uo[0] if isinstance(uo, tuple) else uo
    assert rel(uc, uo) < 1e-10
    with pytest.raises(hh.HHGRError):
        hh.debug_op(ctx, 1, level, T(u, dev), T(b, dev))
    ctx.close()


@pytest.mark.parametrize("n_sub,level,seed", CASES)
def test_vcycle_iterates_and_solve(dev, hh, n_sub, level, seed):
    print(f"\n[general solve] n_sub={n_sub} level={level} seed={seed}", flush=True)
    ctx = context(hh, dev, n_sub, level, seed)
    p = problem(n_sub, level, seed)
    b = np.random.default_rng(200 + seed).uniform(0.0, 1.0, p.ndof) / p.ndof
    ctx.set_rhs(T(b, dev))
    for k in (1, 2):
        rr = ctx.vcycle(1)
        uo, _, ho = p.solve(b, rtol=0.0, max_cycles=k)
        assert rel(Nn(ctx.get_solution()), uo) < 1e-12, k
        assert rr == pytest.approx(ho[k], rel=1e-9)
    cyc, rr, hist = ctx.solve(1e-10, 60)
    uo, co, ho = p.solve(b, rtol=1e-10, max_cycles=60)
    print(f"  {cyc + 2} cycles (oracle {co}), rel res {rr:.2e}, rate {hist[-1] / hist[-2]:.3f}", flush=True)
    assert cyc + 2 == co
    assert rel(Nn(ctx.get_solution()), uo) < 1e-10
    ctx.close()


@pytest.mark.parametrize("strategy", ["local", "dd"])
def test_recovery_parity(dev, hh, strategy):
    if strategy == "local":
        n_sub, level, seed = 2, 4, 5
        tets = [inputs.fault_tet(n_sub, seed=3)]
    else:
        n_sub, level, seed = 3, 4, 6
        tets = [inputs.scenario_fault_tet("III")]
        tets.append(inputs.second_fault_tet(n_sub, tets[0]))
    print(f"\n[general recovery] {strategy} tets={tets}", flush=True)
    ctx = context(hh, dev, n_sub, level, seed)
    p = problem(n_sub, level, seed)
    b = np.random.default_rng(300).uniform(0.0, 1.0, p.ndof) / p.ndof
    ctx.set_rhs(T(b, dev))
    ctx.vcycle(3)
    uo, _, _ = p.solve(b, rtol=0.0, max_cycles=3)
    for t in tets:
        ctx.inject_fault(t)
        uo = p.inject_fault(t, uo)
    assert rel(Nn(ctx.get_solution()), uo) < 1e-12
    if strategy == "local":
        ctx.recover_local(tets[0], 3)
        uo, _ = p.recover_local(tets, uo, b, 3)
    else:
        ctx.recover_dd(tets, 2, 4)
        uo = p.dd_intact(tets, uo, b, 2)
        uo, _ = p.recover_local(tets, uo, b, 4)
    assert rel(Nn(ctx.get_solution()), uo) < 1e-12
    ctx.vcycle(2)
    uo, _, _ = p.solve(b, u0=uo, rtol=0.0, max_cycles=2)
    assert rel(Nn(ctx.get_solution()), uo) < 1e-12
    with pytest.raises(hh.HHGRError):
        ctx.recover_dn(tets, 1, 1)
    ctx.close()


def test_geometry_level6_iterates(dev, hh):
    """The oracle at the largest size it runs in seconds (2 subcubes, level 6)."""
    n_sub, level, seed = 2, 6, 9
    print(f"\n[general level 6] n_sub={n_sub} seed={seed}", flush=True)
    ctx = context(hh, dev, n_sub, level, seed)
    p = problem(n_sub, level, seed)
    b = np.random.default_rng(400).uniform(0.0, 1.0, p.ndof) / p.ndof
    ctx.set_rhs(T(b, dev))
    ctx.vcycle(3)
    uo, _, _ = p.solve(b, rtol=0.0, max_cycles=3)
    assert rel(Nn(ctx.get_solution()), uo) < 1e-12
    ctx.close()


def grid_positions(vertices, n_sub, level):
    """Physical positions of the interior grid nodes (vector order), each
    node mapped affinely by the macro tetrahedron holding it (ties on faces,
    edges and vertices give the same point)."""
    m = 1 << level
    N = n_sub * m
    ax = np.arange(1, N)
    z, y, x = np.meshgrid(ax, ax, ax, indexing="ij")
    X = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    cube = np.minimum(X // m, n_sub - 1)
    D = X - m * cube
    order = np.argsort(-D, axis=1, kind="stable")
    Ds = np.take_along_axis(D, order, axis=1)
    ijk = np.stack([Ds[:, 0] - Ds[:, 1], Ds[:, 1] - Ds[:, 2], Ds[:, 2]], axis=1).astype(np.float64) / m
    V = np.asarray(vertices).reshape(n_sub + 1, n_sub + 1, n_sub + 1, 3)  # [z][y][x]
    P = V[cube[:, 2], cube[:, 1], cube[:, 0]]
    out = P.copy()
    corner = cube.copy()
    for s in range(3):
        corner[np.arange(len(X)), order[:, s]] += 1
        Ps = V[corner[:, 2], corner[:, 1], corner[:, 0]]
        out += ijk[:, s:s + 1] * (Ps - P)
    return out


def test_full_size_linear_reproduction(dev, hh):
    """2 subcubes per axis, level 7 (the benchmark size): A u = 0 for a linear
    u away from the boundary, and solving with that u's boundary data
    recovers u on the whole grid."""
    n_sub, level, seed = 2, 7, 5
    print(f"\n[general full size] n_sub={n_sub} level={level}", flush=True)
    V = inputs.perturbed_vertices(n_sub, seed)
    ctx = context(hh, dev, n_sub, level, seed)
    Xp = grid_positions(V, n_sub, level)
    u = 0.3 + Xp @ np.array([1.0, -2.0, 0.5])
    N = n_sub << level
    r = Nn(hh.debug_op(ctx, 0, level, T(u, dev), T(np.zeros_like(u), dev)))
    ax = np.arange(1, N)
    z, y, x = np.meshgrid(ax, ax, ax, indexing="ij")
    far = ((x > 1) & (x < N - 1) & (y > 1) & (y < N - 1) & (z > 1) & (z < N - 1)).ravel()
    scale = np.abs(u).max() / N
    assert np.abs(r[far]).max() < 1e-12 * scale
    assert np.abs(r[~far]).max() > 1e-3 * scale  # boundary data enter next to the boundary
    # b = boundary terms of u (A u restricted to the interior rows is -r)
    ctx.set_rhs(T(-r, dev))
    ctx.set_solution(T(np.zeros_like(u), dev))  # the operator call above left u in the solver
    cyc, rr, hist = ctx.solve(1e-12, 40)
    err = rel(Nn(ctx.get_solution()), u)
    print(f"  {cyc} cycles, rate {hist[-1] / hist[-2]:.3f}, max error {err:.2e}", flush=True)
    assert err < 1e-8
    ctx.close()
