"""GPU parity: the HIP path through the C ABI against the CPU oracle, element
by element on the same seeded inputs.  Tolerances: per operator and per
iterate 1e-12 relative (only summation order differs); converged FP64
solutions 1e-10; mixed precision after refinement 1e-9."""
import numpy as np
import pytest

import oracle
from paper_1506_06185_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


def N(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


# several tiles and ragged chunk tails per plane; n_sub = 1, 2, 3 meshes
OP_CASES = [(1, 5), (2, 4), (3, 3)]


@pytest.mark.parametrize("n_sub,level", OP_CASES)
def test_operator_parity(dev, hh, oracle_problem, n_sub, level):
    print(f"\n[op parity] n_sub={n_sub} level={level}", flush=True)
    ctx = hh.Context(device=dev, n_sub=n_sub, level=level)
    p = oracle_problem(n_sub, level)
    g = np.random.default_rng(10 * n_sub + level)
    nd = p.ndof
    u, b = g.standard_normal(nd), g.standard_normal(nd)
    # residual
    r = N(hh.debug_op(ctx, 0, level, T(u, dev), T(b, dev)))
    assert rel(r, p.residual(u, b)) < 1e-13
    # colour passes and one full sweep
    for op, colours in ((1, 1), (2, 2), (3, 3)):
        us = N(hh.debug_op(ctx, op, level, T(u, dev), T(b, dev)))
        assert rel(us, p.smooth(u, b, omega=1.25, colours=colours)) < 1e-13, op
    # restriction, prolongation on every level pair
    for l in range(level, 2, -1):
        nf, nc = p.ndof_at(l), p.ndof_at(l - 1)
        rf = g.standard_normal(nf)
        bc = N(hh.debug_op(ctx, 4, l, T(rf, dev)))
        assert rel(bc, p.restrict(rf, level=l)) < 1e-14
        ec, uf = g.standard_normal(nc), g.standard_normal(nf)
        up = N(hh.debug_op(ctx, 5, l, T(ec, dev), T(uf, dev)))
        assert rel(up, p.prolong_add(ec, uf, level=l)) < 1e-15
    # coarsest level: PCG, and the dense inverse the cycles use with k = 1
    # (up to 512 unknowns; n_sub = 3 has 1331 and keeps the PCG)
    bc = g.standard_normal(p.ndof_at(2))
    x = N(hh.debug_op(ctx, 6, 2, T(bc, dev)))
    xo, _ = p.coarse_solve(bc)
    assert rel(x, xo) < 1e-12
    if n_sub <= 2:
        xd = N(hh.debug_op(ctx, 7, 2, T(bc, dev)))
        assert rel(xd, xo) < 1e-12
    else:
        with pytest.raises(hh.HHGRError) as e:
            hh.debug_op(ctx, 7, 2, T(bc, dev))
        assert e.value.code == hh.HHGR_EINVAL
    ctx.close()


# fused sweep pairs (one launch per sweep for the volume interiors): two
# sweeps from a random iterate (op 9) and from zero (op 10), against the
# oracle and bitwise against two plain sweeps of two colour passes each;
# the levels give one or several tiles per tetrahedron and ragged ones
@pytest.mark.parametrize("n_sub,level", [(1, 5), (2, 4), (3, 3), (1, 6), (2, 5)])
def test_fused_sweep_pair(dev, hh, oracle_problem, n_sub, level):
    print(f"\n[fused pair] n_sub={n_sub} level={level}", flush=True)
    ctx = hh.Context(device=dev, n_sub=n_sub, level=level)
    p = oracle_problem(n_sub, level)
    g = np.random.default_rng(50 + 10 * n_sub + level)
    for l in range(level, 2, -1):
        nd = p.ndof_at(l)
        u, b = g.standard_normal(nd), g.standard_normal(nd)
        uT, bT = T(u, dev), T(b, dev)
        two = N(hh.debug_op(ctx, 9, l, uT, bT))
        ref = p.smooth(p.smooth(u, b, level=l), b, level=l)
        assert rel(two, ref) < 1e-13, l
        plain = N(hh.debug_op(ctx, 3, l, hh.debug_op(ctx, 3, l, uT, bT), bT))
        assert np.array_equal(two, plain), l
        z = N(hh.debug_op(ctx, 10, l, uT, bT))
        zero = np.zeros(nd)
        refz = p.smooth(p.smooth(zero, b, level=l), b, level=l)
        assert rel(z, refz) < 1e-13, l
    ctx.close()


# launch shapes: (workgroup size, XCD-contiguous block order, nodes per thread)
SHAPES = {"bs256-xcd-1npt": (256, 1, 1), "bs128-hw-4npt": (128, 0, 4), "bs512-xcd-4npt": (512, 1, 4)}


@pytest.mark.parametrize("shape", list(SHAPES))
@pytest.mark.parametrize("n_sub,level", [(1, 4), (2, 4), (2, 5), (3, 3), (1, 6)])
def test_vcycle_iterates(dev, hh, oracle_problem, n_sub, level, shape):
    print(f"\n[vcycle parity] n_sub={n_sub} level={level} shape={shape}", flush=True)
    ctx = hh.Context(device=dev, n_sub=n_sub, level=level)
    ctx.set_tuning(*SHAPES[shape])
    p = oracle_problem(n_sub, level)
    g = np.random.default_rng(7)
    b = g.standard_normal(p.ndof)
    u = g.standard_normal(p.ndof)
    ctx.set_rhs(T(b, dev), hh.HHGR_RHS_LOAD)
    ctx.set_solution(T(u, dev))
    for it in range(3):
        relres = ctx.vcycle(1)
        u, rn = p.vcycle(u, b)
        assert rel(N(ctx.get_solution()), u) < 1e-12, it
        assert relres == pytest.approx(rn / np.linalg.norm(b), rel=1e-10)
    ctx.close()


# smoothing sweep counts and SOR factor: no post-smoothing (the prolongation
# corrects every node), no pre-smoothing with two post sweeps (the red pass
# adds the correction in the first sweep only), the paper's 3 + 3 sweeps,
# and plain Gauss-Seidel
SWEEPS = [(1, 0, 1.25), (0, 2, 1.25), (3, 3, 1.25), (2, 1, 1.0)]


@pytest.mark.parametrize("vk", [False, True])
@pytest.mark.parametrize("nu_pre,nu_post,omega", SWEEPS)
def test_vcycle_sweep_counts(dev, hh, nu_pre, nu_post, omega, vk):
    n_sub, level = 2, 4
    print(f"\n[vcycle sweeps] nu=({nu_pre},{nu_post}) omega={omega} vk={vk}", flush=True)
    k = inputs.lognormal_k(n_sub, level, seed=1) if vk else None
    ctx = hh.Context(device=dev, n_sub=n_sub, level=level, nu_pre=nu_pre, nu_post=nu_post, omega=omega,
                     variable_coeff=vk)
    if vk:
        ctx.set_coeff(T(k, dev))
    p = oracle.Problem(n_sub, level, k=k)
    g = np.random.default_rng(11)
    b = g.standard_normal(p.ndof)
    u = g.standard_normal(p.ndof)
    ctx.set_rhs(T(b, dev), hh.HHGR_RHS_LOAD)
    ctx.set_solution(T(u, dev))
    for it in range(3):
        relres = ctx.vcycle(1)
        u, rn = p.vcycle(u, b, omega=omega, nu1=nu_pre, nu2=nu_post)
        assert rel(N(ctx.get_solution()), u) < 1e-12, it
        assert relres == pytest.approx(rn / np.linalg.norm(b), rel=1e-10)
    ctx.close()
    p.close()


@pytest.mark.parametrize("general", [False, True])
def test_split_norm_equals_full_residual(dev, hh, general):
    """The norm a cycle reports is taken from its last black (class-3) pass
    and a residual over the other nodes; it equals ||b - A u|| of the same
    iterate computed in full by the residual operator."""
    n_sub, level = 2, 5
    print(f"\n[split norm] general={general}", flush=True)
    V = inputs.perturbed_vertices(n_sub, 2) if general else None
    ctx = hh.Context(device=dev, n_sub=n_sub, level=level, general_geometry=general)
    if general:
        ctx.set_geometry(V)
    g = np.random.default_rng(13)
    nd = (n_sub * 2 ** level - 1) ** 3
    b = g.standard_normal(nd)
    ctx.set_rhs(T(b, dev), hh.HHGR_RHS_LOAD)
    ctx.set_solution(None)
    bn = np.linalg.norm(b)
    for it in range(4):
        relres = ctx.vcycle(1)
        u = N(ctx.get_solution())
        r = N(hh.debug_op(ctx, 0, level, T(u, dev), T(b, dev)))
        assert relres == pytest.approx(np.linalg.norm(r) / bn, rel=1e-11), it
    ctx.close()


def test_solve_c1(dev, hh, oracle_problem):
    # 6 macro tets, level 4, sine source, V(2,1) to 1e-8
    n_sub, level = 1, 4
    print("\n[solve C1]", flush=True)
    ctx = hh.Context(device=dev, n_sub=n_sub, level=level)
    f = inputs.sine_source(n_sub, level)
    ctx.set_rhs(T(f, dev), hh.HHGR_RHS_NODAL_F)
    cyc, rr, hist = ctx.solve(1e-8, 50)
    p = oracle_problem(n_sub, level)
    b = p.apply_M(f)
    uo, co, ho = p.solve(b, rtol=1e-8)
    assert cyc == co
    # residual norms are exact up to ~1e-16 ||b|| of rounding in b - A u
    assert np.allclose(hist, ho, rtol=1e-9, atol=1e-13)
    assert rel(N(ctx.get_solution()), uo) < 1e-12
    # converged solutions agree to 1e-10
    ctx.solve(1e-13, 60)
    ut, _, _ = p.solve(b, rtol=1e-13, max_cycles=60)
    assert rel(N(ctx.get_solution()), ut) < 1e-10
    ctx.close()


def test_mass_apply(dev, hh, oracle_problem):
    n_sub, level = 2, 4
    ctx = hh.Context(device=dev, n_sub=n_sub, level=level)
    x = np.random.default_rng(3).standard_normal(oracle_problem(n_sub, level).ndof)
    y = N(ctx.mass_apply(T(x, dev)))
    assert rel(y, oracle_problem(n_sub, level).apply_M(x)) < 1e-14
    ctx.close()


def test_fault_and_local_recovery(dev, hh, oracle_problem):
    n_sub, level, kF = 2, 5, 5
    print("\n[fault + recover_local]", flush=True)
    ctx = hh.Context(device=dev, n_sub=n_sub, level=level)
    p = oracle_problem(n_sub, level)
    f = inputs.sine_source(n_sub, level)
    b = p.apply_M(f)
    ctx.set_rhs(T(f, dev), hh.HHGR_RHS_NODAL_F)
    ctx.vcycle(kF)
    u, _, _ = p.solve(b, rtol=0.0, max_cycles=kF)
    t = inputs.fault_tet(n_sub, seed=0)
    ctx.inject_fault(t)
    u = p.inject_fault(t, u)
    assert rel(N(ctx.get_solution()), u) < 1e-12
    lr = ctx.recover_local(t, 3)
    u, res = p.recover_local(t, u, b, n_cycles=3)
    assert rel(N(ctx.get_solution()), u) < 1e-12
    assert lr == pytest.approx(res[-1], rel=1e-8)
    cyc, rr, hist = ctx.solve(1e-8, 50)
    uo, co, _ = p.solve(b, u0=u, rtol=1e-8, r0=np.linalg.norm(b))
    assert cyc == co
    assert rel(N(ctx.get_solution()), uo) < 1e-11
    ctx.close()


def test_local_recovery_graph_reuse(dev, hh, oracle_problem):
    """The local recovery cycles replay a captured graph kept for one
    (tetrahedron, cycle count): a repeated recovery replays it, another
    tetrahedron or count captures anew, and a Dirichlet-Dirichlet recovery
    in between (another local hierarchy, graphs dropped) leaves the next
    local recovery right; every step against the oracle per iterate."""
    n_sub, level = 2, 4
    print("\n[local recovery graph reuse]", flush=True)
    ctx = hh.Context(device=dev, n_sub=n_sub, level=level)
    p = oracle_problem(n_sub, level)
    b = inputs.uniform_load(n_sub, level, seed=8)
    ctx.set_rhs(T(b, dev), hh.HHGR_RHS_LOAD)
    ctx.vcycle(2)
    u, _, _ = p.solve(b, rtol=0.0, max_cycles=2)
    t1, t2 = 25, 7
    steps = [("lr", t1, 3), ("lr", t1, 3), ("lr", t2, 3), ("lr", t2, 2), ("dd", t1, 2), ("lr", t1, 3), ("lr", t2, 2)]
    for kind, t, n in steps:
        ctx.inject_fault(t)
        u = p.inject_fault(t, u)
        if kind == "lr":
            lr = ctx.recover_local(t, n)
            u, res = p.recover_local(t, u, b, n_cycles=n)
            assert lr == pytest.approx(res[-1], rel=1e-8), (kind, t, n)
        else:
            ctx.recover_dd([t], 1, n)
            u = p.dd_intact([t], u, b, 1)
            u, _ = p.recover_local([t], u, b, n)
        assert rel(N(ctx.get_solution()), u) < 1e-12, (kind, t, n)
        ctx.vcycle(1)
        u, _, _ = p.solve(b, u0=u, rtol=0.0, max_cycles=1)
        assert rel(N(ctx.get_solution()), u) < 1e-12, (kind, t, n)
    ctx.close()


@pytest.mark.parametrize("vk", [False, True])
def test_fault_then_plain_cycles(dev, hh, vk):
    # the do-nothing strategy (Sec. 2.2): cycles continue right after the
    # fault.  The faulty closure's ghost copies must hold the surviving
    # interface values, as the oracle's global vector does.
    n_sub, level = 2, 4
    print(f"\n[fault + plain cycles] vk={vk}", flush=True)
    k = inputs.lognormal_k(n_sub, level, seed=2) if vk else None
    ctx = hh.Context(device=dev, n_sub=n_sub, level=level, variable_coeff=vk)
    if vk:
        ctx.set_coeff(T(k, dev))
    p = oracle.Problem(n_sub, level, k=k)
    b = inputs.uniform_load(n_sub, level, seed=3)
    ctx.set_rhs(T(b, dev), hh.HHGR_RHS_LOAD)
    ctx.vcycle(3)
    u, _, _ = p.solve(b, rtol=0.0, max_cycles=3)
    for t in (inputs.fault_tet(n_sub, seed=0), 0):
        ctx.inject_fault(t)
        u = p.inject_fault(t, u)
        for it in range(2):
            relres = ctx.vcycle(1)
            u, rn = p.vcycle(u, b)
            assert rel(N(ctx.get_solution()), u) < 1e-12, (t, it)
            assert relres == pytest.approx(rn / np.linalg.norm(b), rel=1e-10)
    ctx.close()
    p.close()


@pytest.mark.parametrize("shape", ["bs256-xcd-1npt", "bs128-hw-4npt"])
def test_dirichlet_dirichlet_recovery(dev, hh, oracle_problem, shape):
    n_sub, level = 2, 5
    print(f"\n[recover_dd] shape={shape}", flush=True)
    ctx = hh.Context(device=dev, n_sub=n_sub, level=level)
    ctx.set_tuning(*SHAPES[shape])
    p = oracle_problem(n_sub, level)
    b = inputs.uniform_load(n_sub, level, seed=1)
    ctx.set_rhs(T(b, dev), hh.HHGR_RHS_LOAD)
    ctx.vcycle(4)
    u, _, _ = p.solve(b, rtol=0.0, max_cycles=4)
    tets = inputs.batch_faults(2, n_sub, seed=0)
    for t in tets:
        ctx.inject_fault(int(t))
        u = p.inject_fault(int(t), u)
    ctx.recover_dd([int(t) for t in tets], 2, 4)
    u = p.dd_intact(tets, u, b, 2)
    u, _ = p.recover_local(tets, u, b, n_cycles=4)
    assert rel(N(ctx.get_solution()), u) < 1e-12
    # back to global cycles
    ctx.vcycle(2)
    u, _, _ = p.solve(b, u0=u, rtol=0.0, max_cycles=2)
    assert rel(N(ctx.get_solution()), u) < 1e-12
    ctx.close()


@pytest.mark.parametrize("shape", ["bs256-xcd-1npt", "bs512-xcd-4npt"])
def test_mixed_precision(dev, hh, oracle_problem, shape):
    n_sub, level = 2, 5
    print(f"\n[mixed] shape={shape}", flush=True)
    p = oracle_problem(n_sub, level)
    b = inputs.uniform_load(n_sub, level, seed=0)
    ctx = hh.Context(device=dev, n_sub=n_sub, level=level, precision="mixed")
    ctx.set_tuning(*SHAPES[shape])
    ctx.set_rhs(T(b, dev), hh.HHGR_RHS_LOAD)
    # first refinement step equals the oracle's FP32 step to FP32 rounding
    ctx.vcycle(1)
    u1, _, _ = p.solve_mixed(b, rtol=0.0, max_steps=1)
    assert rel(N(ctx.get_solution()), u1) < 1e-5
    cyc, rr, hist = ctx.solve(1e-12, 60)
    u64, _, _ = p.solve(b, rtol=1e-13, max_cycles=60)
    err = np.linalg.norm(N(ctx.get_solution()) - u64) / np.linalg.norm(u64)
    assert err < 1e-9, err
    ctx.close()


def test_variable_coefficient_parity(dev, hh):
    n_sub, level = 2, 4
    print("\n[variable k]", flush=True)
    k = inputs.lognormal_k(n_sub, level, seed=0)
    p = oracle.Problem(n_sub, level, k=k)
    ctx = hh.Context(device=dev, n_sub=n_sub, level=level, variable_coeff=True)
    ctx.set_coeff(T(k, dev))
    g = np.random.default_rng(5)
    u, b = g.standard_normal(p.ndof), g.standard_normal(p.ndof)
    assert rel(N(hh.debug_op(ctx, 0, level, T(u, dev), T(b, dev))), p.residual(u, b)) < 1e-13
    assert rel(N(hh.debug_op(ctx, 3, level, T(u, dev), T(b, dev))), p.smooth(u, b, 1.25, 3)) < 1e-13
    bc = g.standard_normal(p.ndof_at(2))
    assert rel(N(hh.debug_op(ctx, 6, 2, T(bc, dev))), p.coarse_solve(bc)[0]) < 1e-12
    with pytest.raises(hh.HHGRError) as e:  # per-element k: the coarsest level uses the PCG only
        hh.debug_op(ctx, 7, 2, T(bc, dev))
    assert e.value.code == hh.HHGR_EINVAL
    ctx.close()
    ctx = hh.Context(device=dev, n_sub=n_sub, level=level, variable_coeff=True)
    ctx.set_tuning(*SHAPES["bs128-hw-4npt"])
    ctx.set_coeff(T(k, dev))
    ctx.set_rhs(T(b, dev), hh.HHGR_RHS_LOAD)
    ctx.vcycle(2)
    uo, _, _ = p.solve(b, rtol=0.0, max_cycles=2)
    assert rel(N(ctx.get_solution()), uo) < 1e-12
    ctx.solve(1e-13, 60)
    uo, _, _ = p.solve(b, rtol=1e-13, max_cycles=60)
    assert rel(N(ctx.get_solution()), uo) < 1e-10
    ctx.close()


def test_adjoint_gradients(dev, hh):
    n_sub, level = 1, 4
    print("\n[adjoint]", flush=True)
    k = inputs.lognormal_k(n_sub, level, seed=0)
    f = inputs.sine_source(n_sub, level)
    uobs = inputs.gaussian_obs(n_sub, level, seed=0)
    p = oracle.Problem(n_sub, level, k=k)
    b = p.apply_M(f)
    u, _, _ = p.solve(b, rtol=1e-13, max_cycles=80)
    lam, _, _ = p.solve(u - uobs, rtol=1e-13, max_cycles=80)
    ctx = hh.Context(device=dev, n_sub=n_sub, level=level, variable_coeff=True)
    fT = T(f, dev)
    kT = T(k, dev)
    uT = hh.HHGSolve.apply(ctx, fT.requires_grad_(True), kT.requires_grad_(True), 1e-13, 80)
    assert rel(N(uT), u) < 1e-10
    J = 0.5 * ((uT - T(uobs, dev)) ** 2).sum()
    J.backward()
    assert rel(N(fT.grad), p.apply_M(lam)) < 1e-9
    assert rel(N(kT.grad), p.grad_k(u, lam)) < 1e-9
    ctx.close()


def test_adjoint_after_interleaved_forwards(dev, hh):
    # two forwards on one context before the first backward: each backward
    # must use its own forward's u and k
    n_sub, level = 1, 4
    print("\n[adjoint, interleaved forwards]", flush=True)
    f = inputs.sine_source(n_sub, level)
    uobs = inputs.gaussian_obs(n_sub, level, seed=0)
    ks = [inputs.lognormal_k(n_sub, level, seed=s) for s in (0, 7)]
    ctx = hh.Context(device=dev, n_sub=n_sub, level=level, variable_coeff=True)
    fTs, kTs, Js = [], [], []
    for k in ks:
        fT, kT = T(f, dev).requires_grad_(True), T(k, dev).requires_grad_(True)
        uT = hh.HHGSolve.apply(ctx, fT, kT, 1e-13, 80)
        Js.append(0.5 * ((uT - T(uobs, dev)) ** 2).sum())
        fTs.append(fT)
        kTs.append(kT)
    for q in (0, 1):
        Js[q].backward()
        p = oracle.Problem(n_sub, level, k=ks[q])
        b = p.apply_M(f)
        u, _, _ = p.solve(b, rtol=1e-13, max_cycles=80)
        lam, _, _ = p.solve(u - uobs, rtol=1e-13, max_cycles=80)
        assert rel(N(fTs[q].grad), p.apply_M(lam)) < 1e-9, q
        assert rel(N(kTs[q].grad), p.grad_k(u, lam)) < 1e-9, q
        p.close()
    ctx.close()


def test_batch_matches_sequential(dev, hh, oracle_problem):
    print("\n[batch]", flush=True)
    cases = [(2, 4), (2, 5), (1, 5)]
    ctxs, refs = [], []
    for q, (n_sub, level) in enumerate(cases):
        c = hh.Context(device=dev, n_sub=n_sub, level=level)
        b = inputs.uniform_load(n_sub, level, seed=q)
        c.set_rhs(T(b, dev), hh.HHGR_RHS_LOAD)
        ctxs.append(c)
        refs.append(oracle_problem(n_sub, level).solve(b, rtol=1e-10, max_cycles=60))
    batch = hh.Batch(ctxs)
    out = batch.run(1e-10, 60)
    for c, (cyc, rr, hist), (uo, co, ho) in zip(ctxs, out, refs):
        assert cyc == co
        assert rel(N(c.get_solution()), uo) < 1e-12
    batch.close()
    for c in ctxs:
        c.close()


def test_graph_replay_matches_eager(dev, hh):
    n_sub, level = 2, 5
    print("\n[graph]", flush=True)
    b = inputs.uniform_load(n_sub, level, seed=2)
    res = []
    for graph in (False, True):
        ctx = hh.Context(device=dev, n_sub=n_sub, level=level)
        ctx.set_graph(graph)
        ctx.set_rhs(T(b, dev), hh.HHGR_RHS_LOAD)
        for _ in range(4):  # several replays with host reads in between
            ctx.vcycle(1)
        res.append(N(ctx.get_solution()))
        ctx.close()
    assert rel(res[1], res[0]) < 1e-14


def test_batch_with_dd_recovery(dev, hh, oracle_problem):
    """Faulty members recover by Dirichlet-Dirichlet inside the batch graphs,
    concurrently with the other members; iterates equal the sequential oracle
    (intact cycles, then the local cycles, then global cycles)."""
    print("\n[batch + dd]", flush=True)
    cases = [(2, 5), (2, 4), (1, 5)]
    pre = [4, 0, 3]
    faults = {0: ([int(t) for t in inputs.batch_faults(2, 2, seed=3)], 2, 4), 2: ([int(inputs.fault_tet(1, seed=5))], 0, 3)}
    ctxs, bs = [], []
    for q, (n_sub, level) in enumerate(cases):
        c = hh.Context(device=dev, n_sub=n_sub, level=level)
        b = inputs.uniform_load(n_sub, level, seed=10 + q)
        c.set_rhs(T(b, dev), hh.HHGR_RHS_LOAD)
        if pre[q]:
            c.vcycle(pre[q])
        for t in faults.get(q, ([], 0, 0))[0]:
            c.inject_fault(t)
        ctxs.append(c)
        bs.append(b)
    batch = hh.Batch(ctxs)
    for q, (tets, n_i, n_f) in faults.items():
        batch.arm_dd(q, tets, n_i, n_f)
    out = batch.run(1e-10, 60)
    for q, ((n_sub, level), c, b) in enumerate(zip(cases, ctxs, bs)):
        p = oracle_problem(n_sub, level)
        bn = float(np.linalg.norm(b))
        u, _, _ = p.solve(b, rtol=0.0, max_cycles=pre[q]) if pre[q] else (np.zeros_like(b), 0, None)
        done = 0
        if q in faults:
            tets, n_i, n_f = faults[q]
            for t in tets:
                u = p.inject_fault(t, u)
            if n_i:
                u = p.dd_intact(tets, u, b, n_i)
            u, _ = p.recover_local(tets, u, b, n_cycles=n_f)
            done = n_i
        u, co, _ = p.solve(b, u0=u, rtol=1e-10, max_cycles=60 - done, r0=bn)
        cyc, rr, hist = out[q]
        print(f"  member {q}: cycles {cyc} (oracle {done} + {co}), rel {rr:.3e}", flush=True)
        assert cyc == done + co
        assert rel(N(c.get_solution()), u) < 1e-12
    batch.close()
    for c in ctxs:
        c.close()


@pytest.mark.parametrize("case", ["k1", "variable-k", "mixed-context"])
def test_dirichlet_neumann_recovery(dev, hh, case):
    """Alg. 2 on the GPU (intact Neumann cycles beside local Dirichlet cycles,
    interface refreshed per round) equals the oracle's rounds, then global cycles."""
    n_sub, level = 2, (4 if case == "variable-k" else 5)
    print(f"\n[recover_dn] {case} n_sub={n_sub} level={level}", flush=True)
    k = inputs.lognormal_k(n_sub, level, seed=1) if case == "variable-k" else None
    p = oracle.Problem(n_sub, level, k=k)
    b = inputs.uniform_load(n_sub, level, seed=7)
    ctx = hh.Context(device=dev, n_sub=n_sub, level=level, variable_coeff=k is not None,
                     precision="mixed" if case == "mixed-context" else "fp64")
    if k is not None:
        ctx.set_coeff(T(k, dev))
    ctx.set_rhs(T(b, dev), hh.HHGR_RHS_LOAD)
    u = np.zeros_like(b)
    if case != "mixed-context":
        ctx.vcycle(4)
        u, _, _ = p.solve(b, rtol=0.0, max_cycles=4)
    else:
        ctx.set_solution(T(u, dev))
    tets = [int(t) for t in inputs.batch_faults(2, n_sub, seed=5)]
    for t in tets:
        ctx.inject_fault(t)
        u = p.inject_fault(t, u)
    ctx.recover_dn(tets, 3, 2)
    u = p.dn_recover(tets, u, b, n_intact=3, eta=2)
    assert rel(N(ctx.get_solution()), u) < 1e-12
    if case != "mixed-context":
        ctx.vcycle(2)
        u, _, _ = p.solve(b, u0=u, rtol=0.0, max_cycles=2)
        assert rel(N(ctx.get_solution()), u) < 1e-12
    ctx.close()
    p.close()


@pytest.mark.parametrize("case", ["k1-dd", "vk-dn", "k1-local", "mixed"])
def test_recoveries_level6(dev, hh, case):
    """Faults and recoveries one level above the other small cases (6 tets at
    level 6, 250 k unknowns): iterates equal the oracle's."""
    n_sub, level = 1, 6
    print(f"\n[level 6] {case} n_sub={n_sub} level={level}", flush=True)
    k = inputs.lognormal_k(n_sub, level, seed=2) if case == "vk-dn" else None
    p = oracle.Problem(n_sub, level, k=k)
    b = inputs.uniform_load(n_sub, level, seed=11)
    ctx = hh.Context(device=dev, n_sub=n_sub, level=level, variable_coeff=k is not None,
                     precision="mixed" if case == "mixed" else "fp64")
    if k is not None:
        ctx.set_coeff(T(k, dev))
    ctx.set_rhs(T(b, dev), hh.HHGR_RHS_LOAD)
    if case == "mixed":
        cyc, rr, _ = ctx.solve(1e-12, 60)
        u64, _, _ = p.solve(b, rtol=1e-13, max_cycles=60)
        err = np.linalg.norm(N(ctx.get_solution()) - u64) / np.linalg.norm(u64)
        print(f"  mixed: {cyc} steps, error vs FP64 oracle {err:.2e}", flush=True)
        assert err < 1e-9
        ctx.close()
        p.close()
        return
    ctx.vcycle(3)
    u, _, _ = p.solve(b, rtol=0.0, max_cycles=3)
    assert rel(N(ctx.get_solution()), u) < 1e-12
    tets = [1, 4]
    for t in tets:
        ctx.inject_fault(t)
        u = p.inject_fault(t, u)
    if case == "k1-dd":
        ctx.recover_dd(tets, 2, 3)
        u = p.dd_intact(tets, u, b, 2)
        u, _ = p.recover_local(tets, u, b, n_cycles=3)
    elif case == "vk-dn":
        ctx.recover_dn(tets, 2, 2)
        u = p.dn_recover(tets, u, b, n_intact=2, eta=2)
    else:
        for t in tets:
            ctx.recover_local(t, 3)
        u, _ = p.recover_local(tets, u, b, n_cycles=3)
    d = rel(N(ctx.get_solution()), u)
    print(f"  after recovery: rel diff {d:.2e}", flush=True)
    assert d < 1e-12
    ctx.vcycle(2)
    u, _, _ = p.solve(b, u0=u, rtol=0.0, max_cycles=2)
    assert rel(N(ctx.get_solution()), u) < 1e-12
    ctx.close()
    p.close()
