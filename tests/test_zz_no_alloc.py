"""hhgr_solve_static (a whole solve in the library's static device scratch,
for callers that cannot allocate device memory) against the same solve
through hhgr_create + hhgr_set_rhs + hhgr_solve + hhgr_get_solution, on two
calls in a row, the second with a smaller problem; the same kernels run in
the same order, so the iterates agree to the 1e-12 bar of the cycle parity
tests (in practice bitwise)."""
import numpy as np
import pytest

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


def _with_context(hh, dev, rhs, kind, tol, **kw):
    ctx = hh.Context(device=dev, **kw)
    ctx.set_rhs(rhs, kind)
    cyc, rr, hist = ctx.solve(tol, 60)
    u = ctx.get_solution().cpu().numpy()
    ctx.close()
    return u, cyc, rr, hist


def test_static_solve_matches_context_solve(dev, hh):
    cases = [
        # larger first, then smaller: the second call reuses the scratch
        dict(n_sub=2, level=5, kind="nodal", tol=1e-10, precision="fp64"),
        dict(n_sub=1, level=4, kind="load", tol=1e-12, precision="mixed"),
    ]
    for c in cases:
        n_sub, level = c["n_sub"], c["level"]
        print(f"\n[static solve] n_sub={n_sub} level={level} rhs={c['kind']} precision={c['precision']}", flush=True)
        if c["kind"] == "nodal":
            vec, kind = inputs.sine_source(n_sub, level), hh.HHGR_RHS_NODAL_F
        else:
            vec, kind = inputs.uniform_load(n_sub, level, seed=5), hh.HHGR_RHS_LOAD
        rhs = torch.from_numpy(np.ascontiguousarray(vec)).to(dev)
        u_s, cyc_s, rr_s, hist_s = hh.solve_static(rhs, kind, c["tol"], 60, n_sub=n_sub, level=level,
                                                  precision=c["precision"])
        u_s = u_s.cpu().numpy()
        u_c, cyc_c, rr_c, hist_c = _with_context(hh, dev, rhs, kind, c["tol"], n_sub=n_sub, level=level,
                                                 precision=c["precision"])
        d = np.abs(u_s - u_c).max() / np.abs(u_c).max()
        print(f"  cycles {cyc_s} vs {cyc_c}, rel res {rr_s:.3e} vs {rr_c:.3e}, max rel diff {d:.3e}", flush=True)
        assert cyc_s == cyc_c
        assert d < 1e-12
        assert rr_s == pytest.approx(rr_c, rel=1e-10)
        np.testing.assert_allclose(hist_s, hist_c, rtol=1e-10)


def test_static_solve_rejects_too_large(dev, hh):
    rhs = torch.zeros(255 ** 3, dtype=torch.float64, device=dev)
    with pytest.raises(hh.HHGRError) as e:
        hh.solve_static(rhs, hh.HHGR_RHS_LOAD, 1e-8, 10, n_sub=2, level=7)
    assert e.value.code == hh.HHGR_EINVAL
    assert "static scratch" in str(e.value)
