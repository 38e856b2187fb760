"""GPU edge cases of the hot path against the oracle: every macro tetrahedron
faulty at once (the intact side is empty and the recovery rebuilds the whole
interior from the stored faces, edges and vertices, Sec. 4), the smallest
hierarchy (level 3 over level 2), recovery of a tetrahedron that did not
fault, zero-cycle calls, and rejected arguments."""
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


def Nn(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def make(hh, dev, n_sub, level, general, **kw):
    V = inputs.perturbed_vertices(n_sub, 2) if general else None
    ctx = hh.Context(device=dev, n_sub=n_sub, level=level, general_geometry=general, **kw)
    if general:
        ctx.set_geometry(V)
    return ctx, oracle.Problem(n_sub, level, vertices=V)


@pytest.mark.parametrize("strategy", ["dd", "dn"])
@pytest.mark.parametrize("general", [False, True])
def test_every_tet_faulty(dev, hh, strategy, general):
    n_sub, level = 1, 4
    print(f"\n[all tets faulty] {strategy} general={general}", flush=True)
    ctx, p = make(hh, dev, n_sub, level, general)
    b = inputs.uniform_load(n_sub, level, seed=1)
    ctx.set_rhs(T(b, dev))
    ctx.vcycle(3)
    u, _, _ = p.solve(b, rtol=0.0, max_cycles=3)
    tets = list(range(6 * n_sub ** 3))
    for t in tets:
        ctx.inject_fault(t)
        u = p.inject_fault(t, u)
    # only the 645 interface values (6 faces, 1 edge) survive
    assert np.count_nonzero(Nn(ctx.get_solution())) == np.count_nonzero(u) == 645
    if strategy == "dd":
        ctx.recover_dd(tets, 2, 3)
        u = p.dd_intact(tets, u, b, 2)
        u, _ = p.recover_local(tets, u, b, 3)
    else:
        ctx.recover_dn(tets, 2, 2)
        u = p.dn_recover(tets, u, b, 2, 2)
    assert rel(Nn(ctx.get_solution()), u) < 1e-12
    cyc, rr, _ = ctx.solve(1e-10, 60)
    uo, co, _ = p.solve(b, u0=u, rtol=1e-10, max_cycles=60, r0=float(np.linalg.norm(b)))
    assert cyc == co
    assert rel(Nn(ctx.get_solution()), uo) < 1e-10
    ctx.close()


@pytest.mark.parametrize("general", [False, True])
def test_smallest_hierarchy_and_unfaulted_recovery(dev, hh, general):
    """Level 3 over the level-2 coarse grid (35 interior nodes per
    tetrahedron); local recovery of a tetrahedron that did not fault replaces
    its interior by the local solve, as the oracle does."""
    n_sub, level = 2, 3
    print(f"\n[level 3] general={general}", flush=True)
    ctx, p = make(hh, dev, n_sub, level, general)
    b = inputs.uniform_load(n_sub, level, seed=2)
    ctx.set_rhs(T(b, dev))
    ctx.vcycle(2)
    u, _, _ = p.solve(b, rtol=0.0, max_cycles=2)
    assert rel(Nn(ctx.get_solution()), u) < 1e-12
    ctx.recover_local(11, 2)
    u, _ = p.recover_local([11], u, b, 2)
    assert rel(Nn(ctx.get_solution()), u) < 1e-12
    cyc, rr, _ = ctx.solve(1e-10, 60)
    uo, co, _ = p.solve(b, u0=u, rtol=1e-10, max_cycles=60, r0=float(np.linalg.norm(b)))
    assert cyc == co
    assert rel(Nn(ctx.get_solution()), uo) < 1e-10
    ctx.close()


@pytest.mark.parametrize("general", [False, True])
def test_zero_initial_guess_fill(dev, hh, general):
    """set_solution(None) sets u = 0 by a fill; cycles from it equal cycles
    from a zero vector copied in, bit for bit."""
    n_sub, level = 2, 4
    print(f"\n[zero initial guess] general={general}", flush=True)
    ctx, p = make(hh, dev, n_sub, level, general)
    b = inputs.uniform_load(n_sub, level, seed=4)
    ctx.set_rhs(T(b, dev))
    ctx.set_solution(T(np.ones(p.ndof), dev))
    ctx.set_solution(None)
    assert np.count_nonzero(Nn(ctx.get_solution())) == 0
    r1 = ctx.vcycle(3)
    u1 = Nn(ctx.get_solution())
    ctx.set_solution(T(np.zeros(p.ndof), dev))
    r2 = ctx.vcycle(3)
    assert r1 == r2
    assert np.array_equal(Nn(ctx.get_solution()), u1)
    ctx.close()


def test_zero_cycles_and_rejected_arguments(dev, hh):
    n_sub, level = 1, 4
    ctx = hh.Context(device=dev, n_sub=n_sub, level=level, max_faults=2)
    b = inputs.uniform_load(n_sub, level, seed=3)
    with pytest.raises(hh.HHGRError) as e:
        ctx.vcycle(1)  # no right-hand side yet
    assert e.value.code == hh.HHGR_ESTATE
    ctx.set_rhs(T(b, dev))
    assert ctx.vcycle(0) == pytest.approx(1.0)  # ||b - A 0|| / ||b||
    cyc, rr, hist = ctx.solve(1e-10, 0, raise_on_noconv=False)
    assert cyc == 0 and rr == pytest.approx(1.0) and len(hist) == 1
    with pytest.raises(hh.HHGRError) as e:
        ctx.solve(1e-10, 0)
    assert e.value.code == hh.HHGR_ENOCONV
    for bad in ([0, 0], [0, 1, 2], [6], [-1]):
        with pytest.raises(hh.HHGRError) as e:
            ctx.recover_dd(bad, 1, 1)  # duplicate, more than max_faults, out of range
        assert e.value.code == hh.HHGR_EINVAL
    with pytest.raises(hh.HHGRError):
        ctx.recover_dd([], 1, 1)
    with pytest.raises(hh.HHGRError):
        ctx.inject_fault(6)
    ctx.close()
    c0 = hh.Context(device=dev, n_sub=n_sub, level=level, max_faults=0)
    c0.set_rhs(T(b, dev))
    with pytest.raises(hh.HHGRError) as e:
        c0.recover_local(0, 1)
    assert e.value.code == hh.HHGR_ESTATE
    c0.close()
