"""GPU parity of the inhomogeneous Dirichlet data (eq. (1)) and of the
recovery-strategy comparison (Sec. 4.4, Tables 1 and 2; the fault sequences of
Sec. 5) against the CPU oracle.

The study's jobs are sequenced here a second time with the oracle's
operations (fault-free prefix, fault, LR / DD / DN recovery, cycles to the
stopping rule), and every k_faulty of the GPU driver must equal the oracle's.
Sizes are the three scenarios' meshes (6, 48 and 162 macro tetrahedra, with
the scenarios' fault positions) at levels the oracle finishes in seconds."""
import math

import numpy as np
import pytest

import oracle
from paper_1506_06185_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-13


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


def interior(g, N):
    return g.reshape(N + 1, N + 1, N + 1)[1:-1, 1:-1, 1:-1].ravel()


@pytest.mark.parametrize("n_sub,level,vk", [(1, 4, False), (3, 3, False), (2, 4, True)])
def test_dirichlet_data_parity(dev, hh, n_sub, level, vk):
    print(f"\n[dirichlet data] n_sub={n_sub} level={level} variable_k={vk}", flush=True)
    N = n_sub << level
    g = inputs.harmonic_boundary(n_sub, level)
    k = inputs.lognormal_k(n_sub, level, seed=1) if vk else None
    p = oracle.Problem(n_sub, level, k=k)
    b = p.dirichlet_load(g)
    ctx = hh.Context(device=dev, n_sub=n_sub, level=level, variable_coeff=vk)
    if vk:
        with pytest.raises(hh.HHGRError):
            ctx.set_rhs(T(g, dev), hh.HHGR_RHS_DIRICHLET)  # coefficient not set yet
        ctx.set_coeff(T(k, dev))
    ctx.set_rhs(T(g, dev), hh.HHGR_RHS_DIRICHLET)
    # the first history entry is ||b - A 0|| / ||b|| = 1; iterates follow the oracle's
    rr = ctx.vcycle(2)
    uo, _, ho = p.solve(b, rtol=0.0, max_cycles=2)
    assert rel(Nn(ctx.get_solution()), uo) < 1e-12
    assert rr == pytest.approx(ho[2], rel=1e-9)
    cyc, rr, hist = ctx.solve(TOL, 60)  # continues after the two cycles above
    uo, co, ho = p.solve(b, rtol=TOL, max_cycles=60)
    print(f"  {cyc + 2} cycles (oracle {co}), rel res {rr:.2e}", flush=True)
    assert cyc + 2 == co
    assert rel(Nn(ctx.get_solution()), uo) < 1e-10
    if not vk:
        # a harmonic quadratic is the exact discrete solution on this mesh
        assert rel(Nn(ctx.get_solution()), interior(g, N)) < 1e-10
    ctx.close()
    p.close()


def test_dirichlet_data_rejects_wrong_length(dev, hh):
    ctx = hh.Context(device=dev, n_sub=1, level=3)
    with pytest.raises(hh.HHGRError):
        ctx.set_rhs(torch.zeros(ctx.n_dofs, dtype=torch.float64, device=dev), hh.HHGR_RHS_DIRICHLET)
    ctx.close()


# -- the study's protocol, written again with the oracle's operations ---------
class OracleJobs:
    def __init__(self, p, b):
        self.p, self.b = p, b
        self.bn = float(np.linalg.norm(b))
        self.prefix = {0: np.zeros(p.ndof)}

    def state(self, k):
        if k not in self.prefix:
            self.prefix[k], _, _ = self.p.solve(self.b, rtol=0.0, max_cycles=k, r0=self.bn)
        return self.prefix[k].copy()

    def free(self):
        _, c, _ = self.p.solve(self.b, rtol=TOL, max_cycles=100, r0=self.bn)
        return c

    def faulty(self, events):
        """events: [(after, tet, strategy, n_I, eta)] in time order."""
        p, b = self.p, self.b
        it = events[0][0]
        u = self.state(it)
        for after, tet, strat, n_I, eta in events:
            if after > it:
                u, _, _ = p.solve(b, u0=u, rtol=0.0, max_cycles=after - it, r0=self.bn)
                it = after
            u = p.inject_fault(tet, u)
            n_F = math.ceil(n_I * eta)
            if n_I and strat == "LR":
                u, _ = p.recover_local([tet], u, b, n_F)
            elif n_I and strat == "DD":
                # the intact and the faulty side share no unknowns
                u = p.dd_intact([tet], u, b, n_I)
                u, _ = p.recover_local([tet], u, b, n_F)
            elif n_I and strat == "DN":
                u = p.dn_recover([tet], u, b, n_I, eta)
            it += n_I if strat != "none" else 0
        _, c, h = p.solve(b, u0=u, rtol=TOL, max_cycles=100 - it, r0=self.bn)
        assert c >= 0
        return it + c


SCENARIO_LEVELS = {"I": 5, "II": 4, "III": 4}


@pytest.mark.parametrize("scenario,general", [(s, False) for s in SCENARIO_LEVELS] + [("II", True)])
def test_kappa_tables_match_oracle(dev, hh, scenario, general):
    from paper_1506_06185_amd import study

    n_sub, level = inputs.SCENARIOS[scenario]["n_sub"], SCENARIO_LEVELS[scenario]
    tet = inputs.scenario_fault_tet(scenario)
    V = inputs.perturbed_vertices(n_sub, 0) if general else None
    print(f"\n[kappa tables] scenario {scenario}: n_sub={n_sub} level={level} tet={tet} general={general}", flush=True)
    ctx = study.make_context(n_sub, level, device=dev, tune=False, vertices=V)
    run = study.Runner(ctx, TOL)
    p = oracle.Problem(n_sub, level, vertices=V)
    oj = OracleJobs(p, p.dirichlet_load(inputs.harmonic_boundary(n_sub, level)))
    k_free = oj.free()
    for k_F, n_max in ((5, 4), (11, 6)):
        t = study.kappa_table(run, tet, k_F, (2, 5), range(n_max + 1))
        print(study.format_kappa(t), flush=True)
        assert t["k_free"] == k_free
        for r in t["rows"]:
            ko = oj.faulty([(k_F, tet, r["strategy"] if r["n_I"] else "none", r["n_I"], r["eta"])])
            assert r["k"] == ko, (k_F, r)
    ctx.close()
    p.close()


def test_fault_sequences_match_oracle(dev, hh):
    from paper_1506_06185_amd import study

    n_sub, level = 3, 4
    t1 = inputs.scenario_fault_tet("III")
    t2 = inputs.second_fault_tet(n_sub, t1)
    print(f"\n[fault sequences] n_sub={n_sub} level={level} tets {t1}, {t2}", flush=True)
    ctx = study.make_context(n_sub, level, device=dev, tune=False)
    run = study.Runner(ctx, TOL)
    p = oracle.Problem(n_sub, level)
    oj = OracleJobs(p, p.dirichlet_load(inputs.harmonic_boundary(n_sub, level)))
    single = study.sequence_table(run, [(7, t1)], (1, 4), range(5), repeats=1)
    double = study.sequence_table(run, [(5, t1), (9, t2)], (4,), range(5), strategies=("DD", "DN"), repeats=1)
    for t in (single, double):
        assert t["k_free"] == oj.free()
        for r in t["rows"]:
            s = r["strategy"] if r["n_I"] else "none"
            ev = [(a, tt, s, r["n_I"], r["eta"]) for a, tt in t["events"]]
            ko = oj.faulty(ev)
            print(f"  events {t['events']} {s} eta={r['eta']} n_I={r['n_I']}: k={r['k']} (oracle {ko})", flush=True)
            assert r["k"] == ko
    ctx.close()
    p.close()
