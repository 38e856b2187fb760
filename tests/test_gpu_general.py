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


def context(hh, dev, n_sub, level, seed, k=None, **kw):
    ctx = hh.Context(device=dev, n_sub=n_sub, level=level, general_geometry=True, variable_coeff=k is not None, **kw)
    if k is not None:
        ctx.set_coeff(T(k, dev))
    ctx.set_geometry(inputs.perturbed_vertices(n_sub, seed))
    return ctx


def problem_k(n_sub, level, seed, kseed):
    key = (n_sub, level, seed, "k", kseed)
    if key not in _PROBLEMS:
        _PROBLEMS[key] = oracle.Problem(n_sub, level, k=inputs.lognormal_k(n_sub, level, seed=kseed),
                                        vertices=inputs.perturbed_vertices(n_sub, seed))
    return _PROBLEMS[key]


# several workgroups per class list and ragged tails; 1, 2 and 3 subcubes per axis
CASES = [(1, 5, 3), (2, 4, 5), (3, 3, 7)]
K_CASES = [(1, 4, 3), (2, 4, 5), (3, 3, 7)]


# sweep counts: no post-smoothing, no pre-smoothing, the paper's 3 + 3.  The
# last pre-smoothing class-3 pass writes the residual of its nodes (also in
# a sweep that starts from zero) and the last class-3 pass of a cycle sums
# its squares; the residual launches cover classes 0..2
@pytest.mark.parametrize("vk", [False, True])
@pytest.mark.parametrize("nu_pre,nu_post", [(1, 0), (0, 2), (3, 3)])
def test_sweep_counts(dev, hh, nu_pre, nu_post, vk):
    n_sub, level, seed = 2, 4, 5
    print(f"\n[general sweeps] nu=({nu_pre},{nu_post}) vk={vk}", flush=True)
    k = inputs.lognormal_k(n_sub, level, seed=seed) if vk else None
    ctx = context(hh, dev, n_sub, level, seed, k=k, nu_pre=nu_pre, nu_post=nu_post)
    p = problem_k(n_sub, level, seed, seed) if vk else problem(n_sub, level, seed)
    g = np.random.default_rng(600 + seed)
    b = g.standard_normal(p.ndof)
    u = g.standard_normal(p.ndof)
    ctx.set_rhs(T(b, dev), hh.HHGR_RHS_LOAD)
    ctx.set_solution(T(u, dev))
    for it in range(3):
        relres = ctx.vcycle(1)
        u, rn = p.vcycle(u, b, nu1=nu_pre, nu2=nu_post)
        assert rel(Nn(ctx.get_solution()), u) < 1e-12, it
        assert relres == pytest.approx(rn / np.linalg.norm(b), rel=1e-10)
    ctx.close()


@pytest.mark.parametrize("n_sub,level,seed", K_CASES)
def test_variable_k_operators_and_solve(dev, hh, n_sub, level, seed):
    """Per-element log-normal k on a general macro mesh: per-node stencils on
    every level (coarse k = mean of the 8 children), class passes, the
    coarsest-level rows, iterates and a solve."""
    print(f"\n[general variable k] n_sub={n_sub} level={level} seed={seed}", flush=True)
    k = inputs.lognormal_k(n_sub, level, seed=seed)
    ctx = context(hh, dev, n_sub, level, seed, k=k)
    p = problem_k(n_sub, level, seed, seed)
    g = np.random.default_rng(500 + seed)
    for l in range(2, level + 1):
        nd = p.ndof_at(l)
        u, b = g.standard_normal(nd), g.standard_normal(nd)
        r = Nn(hh.debug_op(ctx, 0, l, T(u, dev), T(b, dev)))
        assert rel(r, p.residual(u, b, level=l)) < 1e-12, l
        for mask in (1, 2, 4, 8, 15):
            us = Nn(hh.debug_op(ctx, 8 + mask, l, T(u, dev), T(b, dev)))
            assert rel(us, p.smooth(u, b, omega=1.25, colours=mask, level=l)) < 1e-12, (l, mask)
    bc = g.standard_normal(p.ndof_at(2))
    uc = Nn(hh.debug_op(ctx, 6, 2, T(bc, dev)))
    uo = p.coarse_solve(bc)
    uo = uo[0] if isinstance(uo, tuple) else uo
    assert rel(uc, uo) < 1e-10
    with pytest.raises(hh.HHGRError) as e:  # per-element k: the coarsest level uses the PCG only
        hh.debug_op(ctx, 7, 2, T(bc, dev))
    assert e.value.code == hh.HHGR_EINVAL
    b = g.uniform(0.0, 1.0, p.ndof) / p.ndof
    ctx.set_rhs(T(b, dev))
    ctx.set_solution(T(np.zeros(p.ndof), dev))  # the operator calls above left their input in u
    ctx.vcycle(2)
    uo, _, _ = p.solve(b, rtol=0.0, max_cycles=2)
    assert rel(Nn(ctx.get_solution()), uo) < 1e-12
    cyc, rr, hist = ctx.solve(1e-10, 80)
    uo, co, _ = p.solve(b, rtol=1e-10, max_cycles=80)
    print(f"  {cyc + 2} cycles (oracle {co}), rate {hist[-1] / hist[-2]:.3f}", flush=True)
    assert cyc + 2 == co
    assert rel(Nn(ctx.get_solution()), uo) < 1e-10
    ctx.close()


@pytest.mark.parametrize("vk", [False, True])
def test_dirichlet_data_and_recovery(dev, hh, vk):
    """Eq. (1) on a general macro mesh: b from boundary values g, iterates,
    a fault with local recovery, and the solve, against the oracle."""
    n_sub, level, seed = 2, 4, 8
    print(f"\n[general Dirichlet] variable_k={vk}", flush=True)
    k = inputs.lognormal_k(n_sub, level, seed=2) if vk else None
    ctx = context(hh, dev, n_sub, level, seed, k=k)
    p = problem_k(n_sub, level, seed, 2) if vk else problem(n_sub, level, seed)
    gb = inputs.harmonic_boundary(n_sub, level)
    b = p.dirichlet_load(gb)
    ctx.set_rhs(T(gb, dev), hh.HHGR_RHS_DIRICHLET)
    rr = ctx.vcycle(3)
    uo, _, ho = p.solve(b, rtol=0.0, max_cycles=3)
    assert rel(Nn(ctx.get_solution()), uo) < 1e-12
    assert rr == pytest.approx(ho[3], rel=1e-9)
    t = inputs.fault_tet(n_sub, seed=4)
    ctx.inject_fault(t)
    ctx.recover_local(t, 2)
    uo = p.inject_fault(t, uo)
    uo, _ = p.recover_local([t], uo, b, 2)
    assert rel(Nn(ctx.get_solution()), uo) < 1e-12
    cyc, rr, _ = ctx.solve(1e-10, 60)
    uo, co, _ = p.solve(b, u0=uo, rtol=1e-10, max_cycles=60, r0=float(np.linalg.norm(b)))
    assert cyc == co
    assert rel(Nn(ctx.get_solution()), uo) < 1e-10
    ctx.close()


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
    if n_sub <= 2:  # k = 1 with at most 512 coarsest unknowns: the dense inverse the cycles use
        assert rel(Nn(hh.debug_op(ctx, 7, 2, T(bc, dev))), uo) < 1e-10
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


@pytest.mark.parametrize("strategy,vk", [("local", False), ("dd", False), ("dn", False), ("dn", True)])
def test_recovery_parity(dev, hh, strategy, vk):
    if strategy == "local":
        n_sub, level, seed = 2, 4, 5
        tets = [inputs.fault_tet(n_sub, seed=3)]
    else:
        n_sub, level, seed = 3, 4, 6
        tets = [inputs.scenario_fault_tet("III")]
        tets.append(inputs.second_fault_tet(n_sub, tets[0]))
    print(f"\n[general recovery] {strategy} variable_k={vk} tets={tets}", flush=True)
    k = inputs.lognormal_k(n_sub, level, seed=4) if vk else None
    ctx = context(hh, dev, n_sub, level, seed, k=k)
    p = problem_k(n_sub, level, seed, 4) if vk else problem(n_sub, level, seed)
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
    elif strategy == "dd":
        ctx.recover_dd(tets, 2, 4)
        uo = p.dd_intact(tets, uo, b, 2)
        uo, _ = p.recover_local(tets, uo, b, 4)
    else:
        # intact side on the sub-stencils of the intact macro tetrahedra, eq. (5)
        ctx.recover_dn(tets, 3, 2)
        uo = p.dn_recover(tets, uo, b, 3, 2)
    assert rel(Nn(ctx.get_solution()), uo) < 1e-12
    ctx.vcycle(2)
    uo, _, _ = p.solve(b, u0=uo, rtol=0.0, max_cycles=2)
    assert rel(Nn(ctx.get_solution()), uo) < 1e-12
    ctx.close()


def test_fault_then_plain_cycles(dev, hh):
    # do-nothing (Sec. 2.2) on a moved mesh: the cycle after the fault reads
    # the faulty closure's ghost copies, which hold the surviving interface
    n_sub, level, seed = 2, 4, 5
    print("\n[general fault + plain cycles]", flush=True)
    p = problem(n_sub, level, seed)
    ctx = context(hh, dev, n_sub, level, seed)
    b = inputs.uniform_load(n_sub, level, seed=4)
    ctx.set_rhs(T(b, dev), hh.HHGR_RHS_LOAD)
    ctx.vcycle(3)
    u, _, _ = p.solve(b, rtol=0.0, max_cycles=3)
    t = inputs.fault_tet(n_sub, seed=0)
    ctx.inject_fault(t)
    u = p.inject_fault(t, u)
    for it in range(2):
        ctx.vcycle(1)
        u, _ = p.vcycle(u, b)
        assert rel(Nn(ctx.get_solution()), u) < 1e-12, it
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


def grid_positions(vertices, n_sub, level, full=False):
    """Physical positions of the interior grid nodes (vector order; with full,
    of all (N+1)^3 nodes, x fastest), each node mapped affinely by the macro
    tetrahedron holding it (ties on faces, edges and vertices give the same
    point)."""
    m = 1 << level
    N = n_sub * m
    ax = np.arange(0, N + 1) if full else np.arange(1, N)
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
    u away from the boundary, and solving with that u's values on the moved
    boundary as Dirichlet data, eq. (1), recovers u on the whole grid."""
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
    # Dirichlet data: the linear function on the boundary nodes
    ug = 0.3 + grid_positions(V, n_sub, level, full=True) @ np.array([1.0, -2.0, 0.5])
    ctx.set_rhs(T(ug, dev), hh.HHGR_RHS_DIRICHLET)
    ctx.set_solution(T(np.zeros_like(u), dev))  # the operator call above left u in the solver
    cyc, rr, hist = ctx.solve(1e-12, 40)
    err = rel(Nn(ctx.get_solution()), u)
    print(f"  {cyc} cycles, rate {hist[-1] / hist[-2]:.3f}, max error {err:.2e}", flush=True)
    assert err < 1e-8
    ctx.close()


def test_full_size_variable_k_symmetry_and_constants(dev, hh):
    """2 subcubes per axis, level 7, per-element log-normal k: the per-node
    stencils give a symmetric operator (x.A y = y.A x for random x, y) whose
    rows annihilate constants away from the boundary."""
    n_sub, level, seed = 2, 7, 5
    print(f"\n[general full size, variable k] n_sub={n_sub} level={level}", flush=True)
    k = inputs.lognormal_k(n_sub, level, seed=1)
    ctx = context(hh, dev, n_sub, level, seed, k=k)
    N = n_sub << level
    nd = (N - 1) ** 3
    g = np.random.default_rng(600)
    x, y = g.standard_normal(nd), g.standard_normal(nd)
    zero = T(np.zeros(nd), dev)
    Ax = -Nn(hh.debug_op(ctx, 0, level, T(x, dev), zero))
    Ay = -Nn(hh.debug_op(ctx, 0, level, T(y, dev), zero))
    xAy, yAx = float(x @ Ay), float(y @ Ax)
    print(f"  x.Ay = {xAy:.15e}, y.Ax = {yAx:.15e}", flush=True)
    assert abs(xAy - yAx) < 1e-11 * np.sqrt(float(x @ Ax) * float(y @ Ay))
    assert float(x @ Ax) > 0 and float(y @ Ay) > 0
    A1 = -Nn(hh.debug_op(ctx, 0, level, T(np.ones(nd), dev), zero))
    ax = np.arange(1, N)
    zz, yy, xx = np.meshgrid(ax, ax, ax, indexing="ij")
    far = ((xx > 1) & (xx < N - 1) & (yy > 1) & (yy < N - 1) & (zz > 1) & (zz < N - 1)).ravel()
    assert np.abs(A1[far]).max() < 1e-12 * np.abs(Ax).max()
    assert np.abs(A1[~far]).min() > 0
    ctx.close()


def test_graphs_and_batches_on_general_meshes(dev, hh):
    """Captured cycles replay the eager ones bitwise, and a batch of a general
    member (with an armed Dirichlet-Dirichlet recovery), a variable-k general
    member and a cube member equals the oracle run member by member."""
    print("\n[general graphs + batch]", flush=True)
    n_sub, level, seed = 2, 4, 5
    b = np.random.default_rng(700).uniform(-1.0, 1.0, (n_sub * 2 ** level - 1) ** 3)
    res = []
    for graph in (False, True):
        ctx = context(hh, dev, n_sub, level, seed)
        ctx.set_graph(graph)
        ctx.set_rhs(T(b, dev))
        for _ in range(4):  # several replays with host reads in between
            ctx.vcycle(1)
        res.append(Nn(ctx.get_solution()))
        ctx.close()
    assert rel(res[1], res[0]) < 1e-14

    k = inputs.lognormal_k(2, 4, seed=6)
    members = [
        dict(ctx=context(hh, dev, 3, 4, 6), p=problem(3, 4, 6), pre=3,
             dd=([inputs.scenario_fault_tet("III"), inputs.second_fault_tet(3, inputs.scenario_fault_tet("III"))], 2, 3)),
        dict(ctx=context(hh, dev, 2, 4, 6, k=k), p=problem_k(2, 4, 6, 6), pre=0, dd=None),
        dict(ctx=hh.Context(device=dev, n_sub=1, level=5), p=oracle.Problem(1, 5), pre=0, dd=None),
    ]
    for q, m in enumerate(members):
        m["b"] = np.random.default_rng(710 + q).uniform(0.0, 1.0, m["p"].ndof) / m["p"].ndof
        m["ctx"].set_rhs(T(m["b"], dev))
        if m["pre"]:
            m["ctx"].vcycle(m["pre"])
        if m["dd"]:
            for t in m["dd"][0]:
                m["ctx"].inject_fault(t)
    batch = hh.Batch([m["ctx"] for m in members])
    for q, m in enumerate(members):
        if m["dd"]:
            batch.arm_dd(q, *m["dd"])
    out = batch.run(1e-10, 80)
    for q, m in enumerate(members):
        p, bb = m["p"], m["b"]
        bn = float(np.linalg.norm(bb))
        u = p.solve(bb, rtol=0.0, max_cycles=m["pre"])[0] if m["pre"] else np.zeros_like(bb)
        done = 0
        if m["dd"]:
            tets, n_i, n_f = m["dd"]
            for t in tets:
                u = p.inject_fault(t, u)
            u = p.dd_intact(tets, u, bb, n_i)
            u, _ = p.recover_local(tets, u, bb, n_f)
            done = n_i
        u, co, _ = p.solve(bb, u0=u, rtol=1e-10, max_cycles=80 - done, r0=bn)
        cyc = out[q][0]
        print(f"  member {q}: cycles {cyc} (oracle {done} + {co})", flush=True)
        assert cyc == done + co
        assert rel(Nn(m["ctx"].get_solution()), u) < 1e-12
    batch.close()
    for m in members:
        m["ctx"].close()


def test_coarse_level_3(dev, hh):
    """A coarser hierarchy ending at level 3 (the 15-point PCG on 343 unknowns)."""
    n_sub, level, seed = 1, 5, 3
    print("\n[general coarse level 3]", flush=True)
    ctx = hh.Context(device=dev, n_sub=n_sub, level=level, coarse_level=3, general_geometry=True)
    ctx.set_geometry(inputs.perturbed_vertices(n_sub, seed))
    p = oracle.Problem(n_sub, level, coarse_level=3, vertices=inputs.perturbed_vertices(n_sub, seed))
    b = np.random.default_rng(720).uniform(0.0, 1.0, p.ndof) / p.ndof
    ctx.set_rhs(T(b, dev))
    ctx.vcycle(3)
    uo, _, _ = p.solve(b, rtol=0.0, max_cycles=3)
    assert rel(Nn(ctx.get_solution()), uo) < 1e-11
    with pytest.raises(hh.HHGRError):
        ctx.recover_local(0, 1)  # local recovery needs coarse level 2
    ctx.close()


def test_mass_source_and_adjoint_gradients(dev, hh):
    """The consistent mass matrix of the moved elements (mass_apply and
    b = M f), and the adjoint gradients dJ/df = M lambda and
    dJ/dk_T = -lambda^T A_T u through the autograd Function, against the
    oracle on the same mesh."""
    n_sub, level, seed = 2, 4, 8
    print("\n[general mass + adjoint]", flush=True)
    k = inputs.lognormal_k(n_sub, level, seed=3)
    f = inputs.sine_source(n_sub, level)
    uobs = inputs.gaussian_obs(n_sub, level, seed=3)
    p = problem_k(n_sub, level, seed, 3)
    ctx = context(hh, dev, n_sub, level, seed, k=k)
    x = np.random.default_rng(800).standard_normal(p.ndof)
    assert rel(Nn(ctx.mass_apply(T(x, dev))), p.apply_M(x)) < 1e-13
    b = p.apply_M(f)
    u, _, _ = p.solve(b, rtol=1e-13, max_cycles=80)
    lam, _, _ = p.solve(u - uobs, rtol=1e-13, max_cycles=80)
    fT = T(f, dev).requires_grad_(True)
    kT = T(k, dev).requires_grad_(True)
    uT = hh.HHGSolve.apply(ctx, fT, kT, 1e-13, 80)
    assert rel(Nn(uT), u) < 1e-10
    J = 0.5 * ((uT - T(uobs, dev)) ** 2).sum()
    J.backward()
    assert rel(Nn(fT.grad), p.apply_M(lam)) < 1e-9
    assert rel(Nn(kT.grad), p.grad_k(u, lam)) < 1e-9
    ctx.close()


def test_autotuned_shapes_give_the_same_iterates(dev, hh):
    """The autotuner's class-pass shape (workgroup size, block order) per
    level leaves the iterates unchanged."""
    n_sub, level, seed = 2, 5, 5
    print("\n[general autotune]", flush=True)
    ctx = context(hh, dev, n_sub, level, seed)
    ctx.autotune()
    print(f"  tuning {ctx.tuning_info()}", flush=True)
    p = problem(n_sub, level, seed)
    b = np.random.default_rng(900).uniform(0.0, 1.0, p.ndof) / p.ndof
    ctx.set_rhs(T(b, dev))
    ctx.vcycle(3)
    uo, _, _ = p.solve(b, rtol=0.0, max_cycles=3)
    assert rel(Nn(ctx.get_solution()), uo) < 1e-12
    ctx.close()


@pytest.mark.parametrize("vk", [False, True])
def test_mixed_precision(dev, hh, vk):
    """FP32 cycles inside FP64 refinement on a general macro mesh: the first
    step equals the oracle's FP32 step to FP32 rounding, the refined solution
    reaches the FP64 oracle solution to 1e-9, and a fault recovered by
    Dirichlet-Dirichlet recovery (intact side in mixed steps) as well."""
    n_sub, level, seed = 2, 5, 5
    print(f"\n[general mixed] variable_k={vk}", flush=True)
    k = inputs.lognormal_k(n_sub, level, seed=9) if vk else None
    p = problem_k(n_sub, level, seed, 9) if vk else problem(n_sub, level, seed)
    b = inputs.uniform_load(n_sub, level, seed=0)
    ctx = context(hh, dev, n_sub, level, seed, k=k, precision="mixed")
    ctx.set_rhs(T(b, dev))
    ctx.vcycle(1)
    u1, _, _ = p.solve_mixed(b, rtol=0.0, max_steps=1)
    assert rel(Nn(ctx.get_solution()), u1) < 1e-5
    cyc, rr, hist = ctx.solve(1e-12, 80)
    u64, _, _ = p.solve(b, rtol=1e-13, max_cycles=80)
    err = np.linalg.norm(Nn(ctx.get_solution()) - u64) / np.linalg.norm(u64)
    print(f"  {cyc + 1} steps, error vs FP64 oracle {err:.2e}", flush=True)
    assert err < 1e-9, err
    tets = [inputs.fault_tet(n_sub, seed=2)]
    ctx.set_solution(T(np.zeros_like(b), dev))
    ctx.vcycle(3)
    ctx.inject_fault(tets[0])
    ctx.recover_dd(tets, 2, 3)
    cyc, rr, hist = ctx.solve(1e-12, 80)
    err = np.linalg.norm(Nn(ctx.get_solution()) - u64) / np.linalg.norm(u64)
    assert err < 1e-9, err
    ctx.close()
