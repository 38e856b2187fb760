"""Benchmark: the fault-tolerant multigrid job on one MI355X.

Headline workload (one step): Poisson -Laplace(u) = f on the unit cube, 2x2x2
subcubes x 6 = 48 macro tetrahedra refined 7 times (257^3 grid, 16,581,375
unknowns), P1, f from u = sin(pi x) sin(pi y) sin(pi z), V(2,1) red-black SOR
(omega 1.25), FP64.  From u = 0: 5 V-cycles, a fault zeroes the interior of
one seeded macro tetrahedron, 3 local Dirichlet V-cycles recover it from the
stored faces/edges/vertex, then global V-cycles continue to ||r|| <= 1e-8 ||b||.

value = unknowns x global V-cycles / step wall time (MDoF/s), so the fault
and the recovery count against it; ms_per_step is the time to 1e-8.
roofline: the finest-level FP64 smoother kernel, timed with HIP events on
the stream it runs on during the timed steps: the red-black colour pass
(12 B per unknown: a sweep reads u and b once and writes u once, 24 B per
unknown, in two passes; the pass's own count, 16 B, is reported beside it),
or the fused sweep kernel where the autotuner chose it (24 B per
volume-interior unknown).  cpu_baseline: the CPU oracle on
the same job (time to 1e-8 on every host thread, a one-thread sample, and the
gradient workload's forward and adjoint solves).

Further legs, each in its own object of the JSON line:
  mixed     the same job in mixed precision (FP32 cycle inside FP64 refinement);
  mixed_l8  level 8 (133,432,831 unknowns), load b ~ U[-1,1]: mixed refinement
            against the FP64 solve of the same problem;
  gradients level 7 with per-element log-normal k: forward solve, adjoint
            gradients dJ/df and dJ/dk of J = 1/2 ||u - u_obs||^2, with an exact
            identity and finite-difference checks;
  batched   the level-7 problem with 2 faulty tetrahedra recovered by
            Dirichlet-Dirichlet, beside 32 independent mixed-precision solves of
            levels 5-7 (6 of them with a faulty tetrahedron recovered locally),
            all as concurrent branches of captured HIP graphs;
  general_mesh  the headline job on a general macro mesh: the 27 macro
            vertices moved (inputs.perturbed_vertices, seed 0), 15-point
            stencils, 4-colour SOR, load b ~ U[-1,1], in FP64 and in mixed
            precision; its roofline is the finest-level FP64 class pass.
  vcycle_rates  plain V-cycle rates at levels 5, 6 and 7, eager and
            graph-replayed, one host read per batch of 20 cycles;
  uninstrumented  the headline steps timed again without kernel events;
  unstructured_mesh  the same job on an unstructured macro mesh from vertex
            and tetrahedron lists (a 3x3x3 box of cubes split into 5
            tetrahedra each, moved vertices, level 7), FP64 and mixed.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fused_sweep_fp64_l7_48tets_traffic.json")
TRAFFIC_FILE_COLOUR = os.path.join(ROOT, "profiles", "colour_pass_fp64_l7_48tets_traffic.json")
TRAFFIC_FILE_GENERAL = os.path.join(ROOT, "profiles", "class_pass15_fp64_l7_48tets_traffic.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash(name: str = "kernels.hip") -> str:
    with open(os.path.join(ROOT, "paper_1506_06185_amd", "csrc", name), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(n_sub: int, level: int, path: str = TRAFFIC_FILE, source: str = "fused.hip"):
    """HBM bytes per launch of the finest-level dominant kernel from the committed
    rocprofv3 counter summary, or None when the summary is not for this workload
    or not for the current kernel source.  The figure is the L2-to-memory read
    and write requests counted in 32-byte units (TCC_EA0_RDREQ_DRAM_32B_sum,
    TCC_EA0_WRREQ_WRITE_DRAM_32B_sum), which read exactly 1 GiB for 1 GiB copies;
    FETCH_SIZE and WRITE_SIZE scaled by the copy kernels serve when those are
    absent (FETCH_SIZE reads 0.5 or 1 GiB for the two 1 GiB copies)."""
    if (n_sub, level) != (2, 7):
        return None
    try:
        with open(path) as f:
            t = json.load(f)
    except OSError:
        return None
    if t.get("kernel_source_sha256_16") != kernel_source_hash(source):
        return None
    if "dram_read_bytes_per_dispatch" in t:
        return round(t["dram_read_bytes_per_dispatch"] + t["dram_write_bytes_per_dispatch"])
    kib = t["fetch_kib_per_dispatch"] * t["fetch_scale"] + t["write_kib_per_dispatch"] * t["write_scale"]
    return round(kib * 1024.0)


def run_job(hh, torch, ctx, f_dev, fault_tet, k_f=5, n_rec=3, rtol=1e-8, max_cycles=60):
    """One step: solve from zero with a fault after k_f cycles and local recovery."""
    ctx.set_rhs(f_dev, hh.HHGR_RHS_NODAL_F)
    ctx.set_solution(None)  # u = 0
    ctx.vcycle(k_f)
    ctx.inject_fault(fault_tet)
    ctx.recover_local(fault_tet, n_rec)
    cyc, rel, _ = ctx.solve(rtol, max_cycles)
    return k_f + cyc, rel


def host_info():
    import platform
    import subprocess

    info = {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "machine": platform.machine()}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)"):
                info["lscpu " + k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return info


def cpu_baseline(n_sub, level, grad=True):
    """The CPU oracle (C + OpenMP, CSR sparse multigrid; a correctness
    baseline, not a tuned CPU stencil code) timed on this host's cores:
    the headline fault job to 1e-8 on every thread, two V-cycles on one
    thread, and the gradient workload's forward + adjoint solve."""
    import numpy as np

    import oracle
    from paper_1506_06185_amd import inputs

    nthr = oracle.threads()
    p = oracle.Problem(n_sub, level)
    b = p.apply_M(inputs.sine_source(n_sub, level))
    t_fault = inputs.fault_tet(n_sub, seed=0)
    # the fault job: 5 cycles, fault, 3 local recovery cycles, solve to 1e-8
    t0 = time.perf_counter()
    u, _, _ = p.solve(b, rtol=0.0, max_cycles=5)
    u = p.inject_fault(t_fault, u)
    u, _ = p.recover_local(t_fault, u, b, n_cycles=3)
    u, cyc, _ = p.solve(b, u0=u, rtol=1e-8, max_cycles=60, r0=np.linalg.norm(b))
    dt = time.perf_counter() - t0
    cycles = 5 + cyc
    # one thread: two V-cycles (a bounded sample of the same job)
    oracle.set_threads(1)
    t1 = time.perf_counter()
    for _ in range(2):
        u, _ = p.vcycle(u, b)
    dt1 = time.perf_counter() - t1
    oracle.set_threads(nthr)
    res = {
        "value": round(p.ndof * cycles / dt / 1e6, 3),
        "unit": "MDoF/s",
        "cores": nthr,
        "kind": "oracle",
        "sample": f"the headline fault job (n_sub={n_sub}, level={level}, {p.ndof} unknowns): 5 V(2,1) cycles, "
                  f"fault in tet {t_fault}, 3 local recovery cycles, cycles to 1e-8 ({cycles} global cycles); "
                  f"CSR sparse multigrid in C/OpenMP on {nthr} threads, assembly ({p.setup_seconds:.1f} s) excluded",
        "time_to_1e8_s": round(dt, 3),
        "one_thread": {"value": round(p.ndof * 2 / dt1 / 1e6, 3), "unit": "MDoF/s", "cores": 1,
                       "sample": "2 V(2,1) cycles of the same problem on one thread",
                       "time_to_1e8_s_estimate": round(dt1 / 2 * cycles, 2)},
        "host": host_info(),
    }
    p.close()
    if grad:
        # the gradient workload: forward and adjoint solves to 1e-11 with
        # per-element log-normal k, dJ/df = M lambda, dJ/dk per element
        k = inputs.lognormal_k(n_sub, level, seed=0)
        uobs = inputs.gaussian_obs(n_sub, level, seed=0)
        pk = oracle.Problem(n_sub, level, k=k)
        bk = pk.apply_M(inputs.sine_source(n_sub, level))
        t2 = time.perf_counter()
        uk, cf, _ = pk.solve(bk, rtol=1e-11, max_cycles=100)
        lam, ca, _ = pk.solve(uk - uobs, rtol=1e-11, max_cycles=100)
        pk.apply_M(lam)
        pk.grad_k(uk, lam)
        dt2 = time.perf_counter() - t2
        res["gradients"] = {"forward_plus_adjoint_s": round(dt2, 3), "forward_cycles": cf, "adjoint_cycles": ca,
                            "cores": nthr,
                            "sample": f"n_sub={n_sub} level={level}, k = exp(0.5 Z): forward and adjoint solves to "
                                      f"1e-11, M lambda and dJ/dk; assembly ({pk.setup_seconds:.1f} s) excluded"}
        pk.close()
    return res


def leg_mixed_job(hh, torch, dev, n_sub, level, f_dev, t_fault, steps, warmup, graph, tune_cache):
    cm = hh.Context(device=dev, n_sub=n_sub, level=level, precision="mixed")
    cm.autotune(tune_cache)
    if graph:
        cm.set_graph(True)
    for _ in range(warmup):
        run_job(hh, torch, cm, f_dev, t_fault)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tot, relm = 0, None
    for _ in range(steps):
        cyc, relm = run_job(hh, torch, cm, f_dev, t_fault)
        tot += cyc
    torch.cuda.synchronize()
    dtm = time.perf_counter() - t0
    um = cm.get_solution()
    cm.close()
    # error against the FP64 solution of the same problem solved to its
    # rounding floor (about 1e-12 relative residual at this size)
    c64 = hh.Context(device=dev, n_sub=n_sub, level=level)
    c64.set_rhs(f_dev, hh.HHGR_RHS_NODAL_F)
    c64.solve(1e-12, 40, raise_on_noconv=False)
    u64 = c64.get_solution()
    c64.close()
    err = float(torch.linalg.norm(um - u64) / torch.linalg.norm(u64))
    return {
        "value": round(um.numel() * tot / dtm / 1e6, 1),
        "unit": "MDoF/s",
        "ms_per_step": round(1e3 * dtm / steps, 3),
        "refinement_steps_per_job": tot // steps,
        "rel_error_vs_fp64_solution": err,
        "rel_res": relm,
    }


def leg_general(hh, torch, dev, n_sub, level, steps, warmup, graph, tune_cache):
    """The headline job (5 cycles, fault, 3 local recovery cycles, solve to
    1e-8) on a general macro mesh; value = unknowns x cycles / time."""
    from paper_1506_06185_amd import inputs

    ctx = hh.Context(device=dev, n_sub=n_sub, level=level, general_geometry=True)
    t0 = time.perf_counter()
    ctx.set_geometry(inputs.perturbed_vertices(n_sub, seed=0))
    t_geom = time.perf_counter() - t0
    ctx.autotune(tune_cache)
    if graph:
        ctx.set_graph(True)
    b = torch.from_numpy(inputs.uniform_load(n_sub, level, seed=0)).to(dev)
    zero = torch.zeros_like(b)
    t_fault = inputs.fault_tet(n_sub, seed=0)

    def job():
        ctx.set_rhs(b)
        ctx.set_solution(zero)
        ctx.vcycle(5)
        ctx.inject_fault(t_fault)
        ctx.recover_local(t_fault, 3)
        cyc, rel, _ = ctx.solve(1e-8, 80)
        return 5 + cyc, rel

    ctx.set_rhs(b)
    k_free, _, hist = ctx.solve(1e-8, 80)
    for _ in range(warmup):
        job()
    if not graph:
        ctx.kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tot, rel = 0, None
    for _ in range(steps):
        cyc, rel = job()
        tot += cyc
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    launches, mean_ms, alg_bytes = ctx.kernel_stats() if not graph else (0, 0.0, 0.0)
    ctx.kernel_timing(False)
    u64 = ctx.get_solution()
    ctx.close()
    # the same job in mixed precision (FP32 class passes inside FP64 refinement)
    cm = hh.Context(device=dev, n_sub=n_sub, level=level, general_geometry=True, precision="mixed")
    cm.set_geometry(inputs.perturbed_vertices(n_sub, seed=0))
    cm.autotune(tune_cache)
    if graph:
        cm.set_graph(True)
    ctx = cm
    for _ in range(warmup):
        job()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    totm, relm = 0, None
    for _ in range(steps):
        cyc, relm = job()
        totm += cyc
    torch.cuda.synchronize()
    dtm = time.perf_counter() - t0
    um = cm.get_solution()
    cm.close()
    mixed = {
        "value": round(b.numel() * totm / dtm / 1e6, 1),
        "unit": "MDoF/s",
        "ms_per_step": round(1e3 * dtm / steps, 3),
        "refinement_steps_per_job": totm // steps,
        "rel_diff_vs_fp64_job": float(torch.linalg.norm(um - u64) / torch.linalg.norm(u64)),
        "rel_res": relm,
    }
    roofline = None
    if launches > 0:
        achieved = alg_bytes / (mean_ms * 1e-3) / 1e9
        roofline = {
            "bound": "hbm",
            "kernel": "k_colour15 (finest-level class pass of the 4-colour SOR, FP64, 15-point)",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(n_sub, level, TRAFFIC_FILE_GENERAL, "kernels.hip"),
            "launches": launches,
            "mean_launch_ms": round(mean_ms, 5),
            "algorithmic_bytes_per_launch": alg_bytes,
        }
    return {
        "value": round(b.numel() * tot / dt / 1e6, 1),
        "unit": "MDoF/s",
        "ms_per_step": round(1e3 * dt / steps, 3),
        "workload": f"general macro mesh n_sub={n_sub} level={level}, macro vertices moved by up to 0.15/n "
                    f"per coordinate (seed 0), load b ~ U[-1,1]; fault in tet {t_fault} after 5 cycles, "
                    f"3 local recovery cycles, solve to 1e-8",
        "cycles_per_job": tot // steps,
        "k_free": k_free,
        "fault_free_rate": round(hist[-1] / hist[-2], 3) if len(hist) > 1 else None,
        "final_rel_res": rel,
        "set_geometry_s": round(t_geom, 3),
        "roofline": roofline,
        "mixed": mixed,
    }


def leg_vcycle_rates(hh, torch, dev, tune_cache, n_sub=2, levels=(5, 6, 7), cycles=20):
    """Plain V(2,1) cycle rates (no fault, one host read at the end of each
    timed batch of cycles), eager and replayed from captured graphs, per
    level: unknowns x cycles / time.  Level 5 (250,047 unknowns, 2 MB per
    vector) stays in the Infinity Cache, level 7 streams from HBM."""
    from paper_1506_06185_amd import inputs

    out = {}
    for level in levels:
        ctx = hh.Context(device=dev, n_sub=n_sub, level=level)
        ctx.autotune(tune_cache)
        ctx.set_rhs(torch.from_numpy(inputs.sine_source(n_sub, level)).to(dev), hh.HHGR_RHS_NODAL_F)
        row = {"unknowns": ctx.n_dofs}
        for mode in ("eager", "graph"):
            ctx.set_graph(mode == "graph")
            ctx.set_solution(None)
            ctx.vcycle(2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.vcycle(cycles)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            row[mode] = {"value": round(ctx.n_dofs * cycles / dt / 1e6, 1), "unit": "MDoF/s",
                         "ms_per_cycle": round(1e3 * dt / cycles, 4)}
        out[str(level)] = row
        ctx.close()
    return out


def leg_recoveries(hh, torch, dev, tune_cache, n_sub=2, level=7, reps=5):
    """Time of one recovery call on the headline problem after 5 cycles
    (nodal sine source), median over reps, each after a fresh fault of the
    same tetrahedra: local recovery (Alg. 1 a), 3 cycles on one
    tetrahedron), Dirichlet-Dirichlet (Alg. 1 b), 1 intact cycle beside 3
    local cycles on two tetrahedra) and Dirichlet-Neumann (Alg. 2, 2 rounds
    of 1 intact cycle beside 2 local ones), with one plain global cycle for
    comparison (DD overlaps its sides, so it costs about max(intact, local)
    plus its set-up)."""
    from paper_1506_06185_amd import inputs

    ctx = hh.Context(device=dev, n_sub=n_sub, level=level)
    ctx.autotune(tune_cache)
    ctx.set_rhs(torch.from_numpy(inputs.sine_source(n_sub, level)).to(dev), hh.HHGR_RHS_NODAL_F)
    ctx.vcycle(5)
    t1 = inputs.fault_tet(n_sub, seed=0)
    t2 = inputs.second_fault_tet(n_sub, t1)
    calls = {
        "global_cycle": ([], lambda: ctx.vcycle(1)),
        "local_3_cycles_1_tet": ([t1], lambda: ctx.recover_local(t1, 3)),
        "dd_1_intact_3_local_2_tets": ([t1, t2], lambda: ctx.recover_dd([t1, t2], 1, 3)),
        "dn_2_rounds_eta_2_2_tets": ([t1, t2], lambda: ctx.recover_dn([t1, t2], 2, 2)),
    }
    out = {"workload": f"n_sub={n_sub} level={level}, nodal sine source, after 5 cycles; faulty tets {t1}, {t2}"}
    for name, (tets, fn) in calls.items():
        ts = []
        for _ in range(reps + 1):
            for t in tets:
                ctx.inject_fault(t)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        out[name] = {"ms": round(1e3 * float(sorted(ts[1:])[len(ts[1:]) // 2]), 3)}
    ctx.close()
    return out


def leg_mesh(hh, torch, dev, steps, warmup, graph, tune_cache, nx=3, level=7):
    """The fault job on an unstructured macro mesh: the box [0, nx]^3 of unit
    cubes split into 5 tetrahedra each (vertices moved by 0.12 U[-1,1]^3,
    seed 0), per-master stencils, 4-colour SOR, load b ~ U[-1,1]: 5 cycles,
    a fault, 3 local recovery cycles, solve to 1e-8, in FP64 and in mixed
    precision; value = unknowns x cycles / time."""
    from paper_1506_06185_amd import inputs

    v, t = inputs.box_mesh(nx, nx, nx)
    v = inputs.perturb_mesh(v, seed=0, amplitude=0.12)
    out = {"workload": f"unstructured macro mesh: box {nx}x{nx}x{nx} of cubes split into 5 tetrahedra each "
                       f"({len(t)} macro tets, vertices moved by 0.12 U[-1,1]^3, seed 0), level {level}, load "
                       f"b ~ U[-1,1]; fault after 5 cycles, 3 local recovery cycles, solve to 1e-8"}
    u64 = None
    for precision in ("fp64", "mixed"):
        t0 = time.perf_counter()
        ctx = hh.Context(device=dev, mesh=(v, t), level=level, precision=precision)
        t_setup = time.perf_counter() - t0
        ctx.autotune(tune_cache)
        if graph:
            ctx.set_graph(True)
        g = torch.Generator().manual_seed(0)
        b = (2.0 * torch.rand(ctx.n_dofs, generator=g, dtype=torch.float64) - 1.0).to(dev)
        t_fault = inputs.mesh_fault_tet(ctx.n_tets, seed=0)

        def job():
            ctx.set_rhs(b)
            ctx.set_solution(None)
            ctx.vcycle(5)
            ctx.inject_fault(t_fault)
            ctx.recover_local(t_fault, 3)
            cyc, rel, _ = ctx.solve(1e-8, 80)
            return 5 + cyc, rel

        ctx.set_rhs(b)
        k_free, _, hist = ctx.solve(1e-8, 80)
        for _ in range(warmup):
            job()
        timing = precision == "fp64" and not graph
        if timing:
            ctx.kernel_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tot, rel = 0, None
        for _ in range(steps):
            cyc, rel = job()
            tot += cyc
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        leg = {
            "value": round(ctx.n_dofs * tot / dt / 1e6, 1),
            "unit": "MDoF/s",
            "ms_per_step": round(1e3 * dt / steps, 3),
            "unknowns": ctx.n_dofs,
            "cycles_per_job": tot // steps,
            "k_free": k_free,
            "fault_free_rate": round(hist[-1] / hist[-2], 3) if len(hist) > 1 else None,
            "final_rel_res": rel,
            "fault_tet": t_fault,
            "setup_s": round(t_setup, 2),
        }
        if timing:
            launches, mean_ms, alg_bytes = ctx.kernel_stats()
            ctx.kernel_timing(False)
            if launches > 0:
                achieved = alg_bytes / (mean_ms * 1e-3) / 1e9
                leg["roofline"] = {
                    "bound": "hbm",
                    "kernel": "k_colour15 (finest-level class pass of the 4-colour SOR on the mesh, FP64)",
                    "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBS,
                    "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "launches": launches,
                    "mean_launch_ms": round(mean_ms, 5),
                    "algorithmic_bytes_per_launch": alg_bytes,
                    "count": "12 B per unknown per class pass (u of the other classes, b and u of its own)",
                }
        if precision == "fp64":
            u64 = ctx.get_solution()
            out.update(leg)
        else:
            leg["rel_diff_vs_fp64_job"] = float(torch.linalg.norm(ctx.get_solution() - u64) / torch.linalg.norm(u64))
            out["mixed"] = leg
        ctx.close()
        torch.cuda.empty_cache()
    return out


def leg_mixed_l8(hh, torch, dev, tune_cache, n_sub=2, level=8):
    """Mixed-precision refinement on 133 M unknowns against the FP64 solve."""
    from paper_1506_06185_amd import inputs

    b = torch.from_numpy(inputs.uniform_load(n_sub, level, seed=0)).to(dev)
    out = {"workload": f"n_sub={n_sub} level={level}, load b ~ U[-1,1] (seed 0)", "unknowns": int(b.numel())}
    sols = {}
    for prec in ("mixed", "fp64"):
        c = hh.Context(device=dev, n_sub=n_sub, level=level, precision=prec)
        c.autotune(tune_cache)
        c.set_rhs(b, hh.HHGR_RHS_LOAD)
        c.vcycle(1)  # warm-up step
        c.set_solution(None)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cyc, _, _ = c.solve(1e-8, 60)
        torch.cuda.synchronize()
        dt8 = time.perf_counter() - t0
        more, rel2, _ = c.solve(1e-12 if prec == "fp64" else 1e-11, 60, raise_on_noconv=False)
        out[prec] = {"time_to_1e8_s": round(dt8, 4), "cycles_to_1e8": cyc,
                     "value": round(b.numel() * cyc / dt8 / 1e6, 1), "unit": "MDoF/s",
                     "final_rel_res": rel2, "cycles_total": cyc + more}
        sols[prec] = c.get_solution()
        c.close()
        log(f"mixed_l8 {prec}: {cyc} cycles to 1e-8 in {dt8:.3f} s")
    um, u64 = sols["mixed"], sols["fp64"]
    out["rel_error_mixed_vs_fp64"] = float(torch.linalg.norm(um - u64) / torch.linalg.norm(u64))
    return out


def leg_gradients(hh, torch, dev, n_sub=2, level=7, n_dirs=2):
    """Forward + adjoint on 100.7 M elements with per-element log-normal k."""
    from paper_1506_06185_amd import inputs

    k = torch.from_numpy(inputs.lognormal_k(n_sub, level, seed=0)).to(dev)
    f = torch.from_numpy(inputs.sine_source(n_sub, level)).to(dev)
    uobs = torch.from_numpy(inputs.gaussian_obs(n_sub, level, seed=0)).to(dev)
    c = hh.Context(device=dev, n_sub=n_sub, level=level, variable_coeff=True)
    c.set_coeff(k)
    c.autotune(None)

    # this variable-coefficient problem reaches a rounding floor near 1.3e-12
    tol = 1e-11

    def forward(ff, kk):
        c.set_coeff(kk)
        c.set_rhs(ff, hh.HHGR_RHS_NODAL_F)
        c.set_solution(None)
        cyc, rr, _ = c.solve(tol, 100, raise_on_noconv=False)
        return c.get_solution(), (cyc, rr)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, (cyc_f, rr_f) = forward(f, k)
    dJdf, dJdk = c.adjoint_grad(u - uobs, rel_tol=tol, max_cycles=100)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # exact identity (A is linear in k): sum_T k_T dJ/dk_T = -lambda^T b = -f . dJ/df
    lhs = float((k * dJdk).sum())
    rhs = -float((f * dJdf).sum())
    fd = []
    df_dirs = inputs.fd_directions(f.numel(), n_dirs, seed=0)
    dk_dirs = inputs.fd_directions(k.numel(), n_dirs, seed=0, offset=20)
    # central differences with steps relative to the parameter's norm: J is
    # quadratic in f (exact for any step), the k step's truncation error is ~1e-6
    for name, dirs, fd_h in (("f", df_dirs, 1e-2), ("k", dk_dirs, 1e-3)):
        step = fd_h * float(torch.linalg.norm(f if name == "f" else k))
        for d in dirs:
            dT = torch.from_numpy(d).to(dev)
            if name == "f":
                up, _ = forward(f + step * dT, k)
                um, _ = forward(f - step * dT, k)
                g = float((dJdf * dT).sum())
            else:
                up, _ = forward(f, k + step * dT)
                um, _ = forward(f, k - step * dT)
                g = float((dJdk * dT).sum())
            # J(+) - J(-) = <u+ - u-, (u+ + u-)/2 - u_obs>, formed without cancellation in J
            fdv = float(((up - um) * (0.5 * (up + um) - uobs)).sum()) / (2 * step)
            fd.append({"param": name, "step_relative": fd_h, "adjoint": g, "finite_difference": fdv,
                       "rel_diff": abs(fdv - g) / max(abs(g), 1e-300)})
    c.close()
    return {"workload": f"n_sub={n_sub} level={level}, {6 * (n_sub << level) ** 3} elements, k = exp(0.5 Z)",
            "forward_cycles": cyc_f, "forward_rel_res": rr_f, "solve_tol": tol,
            "forward_plus_adjoint_s": round(dt, 4),
            "identity": {"sum_k_dJdk": lhs, "minus_f_dot_dJdf": rhs,
                         "rel_err": abs(lhs - rhs) / max(abs(rhs), 1e-300)},
            "fd_checks": fd}


def leg_batched(hh, torch, dev, tune_cache, n_members=32, k_f=5):
    """Global level-7 problem with a Dirichlet-Dirichlet recovery of 2 faulty
    tets beside 32 independent solves (levels 5-7, 6 of them with a local
    recovery), all mixed precision, as concurrent branches of graphs."""
    from paper_1506_06185_amd import inputs

    levels = [7] + [int(x) for x in inputs.batch_levels(n_members, seed=0)]
    ctxs, rhs = [], []
    for q, L in enumerate(levels):
        c = hh.Context(device=dev, n_sub=2, level=L, precision="mixed")
        c.autotune(tune_cache)
        b = torch.from_numpy(inputs.sine_source(2, L) if q == 0 else inputs.uniform_load(2, L, seed=100 + q)).to(dev)
        c.set_rhs(b, hh.HHGR_RHS_NODAL_F if q == 0 else hh.HHGR_RHS_LOAD)
        ctxs.append(c)
        rhs.append(b)
    g_tets = [int(t) for t in inputs.batch_faults(2, 2, seed=0)]
    m_faults = [(m + 1, t) for m, t in inputs.batch_member_faults(n_members, 6, 2, seed=0)]
    batch = hh.Batch(ctxs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pre = batch.run(0.0, k_f, raise_on_noconv=False)  # k_f cycles of every member
    for t in g_tets:
        ctxs[0].inject_fault(t)
    for m, t in m_faults:
        ctxs[m].inject_fault(t)
    batch.arm_dd(0, g_tets, 2, 4)
    for m, t in m_faults:
        batch.arm_dd(m, [t], 0, 3)
    out = batch.run(1e-8, 60)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    dof_cycles = sum(c.n_dofs * (p[0] + o[0]) for c, p, o in zip(ctxs, pre, out))
    res = {
        "members": len(ctxs),
        "levels": {str(L): levels.count(L) for L in sorted(set(levels))},
        "unknowns_total": sum(c.n_dofs for c in ctxs),
        "global_faulty_tets": g_tets, "member_faults": m_faults,
        "wall_s": round(dt, 4),
        "value": round(dof_cycles / dt / 1e6, 1), "unit": "MDoF/s (all members, refinement steps)",
        "global_cycles": pre[0][0] + out[0][0], "all_converged": all(o[1] <= 1e-8 for o in out),
        "max_rel_res": max(o[1] for o in out),
    }
    batch.close()
    for c in ctxs:
        c.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n-sub", type=int, default=2)
    ap.add_argument("--level", type=int, default=7)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the level-8, gradient and batched legs")
    ap.add_argument("--no-general", action="store_true", help="skip the general-macro-mesh leg")
    ap.add_argument("--no-mesh", action="store_true", help="skip the unstructured-macro-mesh leg")
    ap.add_argument("--fused-sweeps", choices=("auto", "on", "off"), default="auto",
                    help="finest-level smoother of the headline job: fused red-black sweep pairs or two colour "
                         "passes per sweep (default: the autotuner's choice)")
    ap.add_argument("--graph", action="store_true", help="replay captured graphs (disables kernel timing)")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file, read before and written after tuning and kept (default: a "
                         "temporary file removed at the end); profiling runs share one so that every run "
                         "launches the same shapes")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run two 1 GiB device copies first (runtime memcpy and an elementwise kernel): "
                         "references of known size for the HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU; --gpus {args.gpus} is not supported "
              f"(sharding the macro tetrahedra over GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1506_06185_amd import hhgr as hh
    from paper_1506_06185_amd import inputs

    dev = torch.device("cuda:0")
    n_sub, level = args.n_sub, args.level
    tune_cache = args.tune_cache or os.path.join(tempfile.gettempdir(), f"hhgr_tune_{os.getpid()}.txt")
    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)                      # runtime copy kernel: reads 1 GiB, writes 1 GiB
        torch.mul(src, 2.0, out=dst)        # elementwise kernel: reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del src, dst
    f_dev = torch.from_numpy(inputs.sine_source(n_sub, level)).to(dev)
    t_fault = inputs.fault_tet(n_sub, seed=0)

    log(f"setup n_sub={n_sub} level={level}")
    ctx = hh.Context(device=dev, n_sub=n_sub, level=level)
    ctx.autotune(tune_cache)
    if args.fused_sweeps != "auto":
        ctx.set_fused_sweeps(level, args.fused_sweeps == "on")
    tuning = ctx.tuning_info()
    log(f"tuning (level: block size, xcd order, nodes per thread) {tuning}")
    if args.graph:
        ctx.set_graph(True)
    # fault-free cycle count for the cycle advantage, eq. (3)
    ctx.set_rhs(f_dev, hh.HHGR_RHS_NODAL_F)
    k_free, _, _ = ctx.solve(1e-8, 60)

    for w in range(args.warmup):
        run_job(hh, torch, ctx, f_dev, t_fault)
        log(f"warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total_cycles = 0
    rel = None
    for s in range(args.steps):
        # HIP events bracket the finest-level colour passes of the last timed
        # step (the roofline's launches); the other steps run without them
        if s == args.steps - 1 and not args.graph:
            ctx.kernel_timing(True)
        cyc, rel = run_job(hh, torch, ctx, f_dev, t_fault)
        total_cycles += cyc
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"timed {args.steps} steps in {dt:.3f} s")
    launches, mean_ms, alg_bytes = ctx.kernel_stats() if not args.graph else (0, 0.0, 0.0)
    ctx.kernel_timing(False)
    # the same steps again without the per-launch events of the roofline
    uninstrumented = None
    if not args.graph:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        cyc_u = 0
        for s in range(args.steps):
            c_u, _ = run_job(hh, torch, ctx, f_dev, t_fault)
            cyc_u += c_u
        torch.cuda.synchronize()
        dt_u = time.perf_counter() - t1
        uninstrumented = {"value": round(ctx.n_dofs * cyc_u / dt_u / 1e6, 1), "unit": "MDoF/s",
                          "ms_per_step": round(1e3 * dt_u / args.steps, 3),
                          "note": "the same steps after the timed ones, with no kernel events in any step"}
    k_faulty = total_cycles // args.steps
    ms_per_step = 1e3 * dt / args.steps
    value = ctx.n_dofs * total_cycles / dt / 1e6

    roofline = None
    if launches > 0:
        t = mean_ms * 1e-3
        pass_bytes = 2.0 * 8.0 * ctx.n_dofs  # a colour pass's own count: u all, b and u of its colour
        if abs(alg_bytes - pass_bytes) > 1.0:
            # the autotuner chose fused sweep pairs on the finest level
            kernel = "k_sweep_fused<double> (finest-level fused red-black SOR sweep of the volume interiors, FP64, k=1)"
            sweep_bytes, own = alg_bytes, None
            traffic = measured_traffic(n_sub, level)
        else:
            # per red-black sweep u and b are read once and u is written once
            # (24 B per unknown in FP64), i.e. 12 B per colour pass; the pass
            # itself reads u of both colours, so its own count is 16 B
            kernel = "k_colour<double> (finest-level red-black SOR colour pass, FP64, k=1)"
            sweep_bytes = 12.0 * ctx.n_dofs
            own = {"algorithmic_bytes_per_launch": pass_bytes, "achieved": round(pass_bytes / t / 1e9, 1),
                   "frac": round(pass_bytes / t / 1e9 / HBM_PEAK_GBS, 4),
                   "count": "16 B per unknown: u of both colours, b and u of the pass's colour"}
            traffic = measured_traffic(n_sub, level, TRAFFIC_FILE_COLOUR, "kernels.hip")
        achieved = sweep_bytes / t / 1e9
        roofline = {
            "bound": "hbm",
            "kernel": kernel,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "launches": launches,
            "mean_launch_ms": round(mean_ms, 5),
            "algorithmic_bytes_per_launch": sweep_bytes,
            "count": "24 B per unknown per red-black sweep (u and b read once, u written once), 12 B per colour pass",
            "pass_own_count": own,
        }
    ctx.close()

    mixed = None
    if not args.no_mixed:
        log("mixed precision leg")
        mixed = leg_mixed_job(hh, torch, dev, n_sub, level, f_dev, t_fault, args.steps, args.warmup, args.graph,
                              tune_cache)
    general = None
    if not args.no_general:
        log("general macro mesh leg")
        general = leg_general(hh, torch, dev, n_sub, level, args.steps, args.warmup, args.graph, tune_cache)
    rates = None
    if not args.no_extra:
        log("V-cycle rates")
        rates = leg_vcycle_rates(hh, torch, dev, tune_cache)
    recoveries = None
    if not args.no_extra:
        log("recovery times")
        recoveries = leg_recoveries(hh, torch, dev, tune_cache)
    mesh = None
    if not args.no_mesh:
        log("unstructured macro mesh leg")
        t1 = time.perf_counter()
        mesh = leg_mesh(hh, torch, dev, args.steps, args.warmup, args.graph, tune_cache)
        log(f"unstructured macro mesh leg done in {time.perf_counter() - t1:.1f} s")
    extra = {}
    if not args.no_extra:
        for name, fn in (("mixed_l8", lambda: leg_mixed_l8(hh, torch, dev, tune_cache)),
                         ("gradients", lambda: leg_gradients(hh, torch, dev)),
                         ("batched", lambda: leg_batched(hh, torch, dev, tune_cache))):
            log(f"{name} leg")
            t1 = time.perf_counter()
            extra[name] = fn()
            torch.cuda.empty_cache()
            log(f"{name} leg done in {time.perf_counter() - t1:.1f} s")

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(n_sub, level)
    if not args.tune_cache:
        try:
            os.remove(tune_cache)
        except OSError:
            pass

    line = {
        "metric": "V-cycle MDoF/s + time-to-1e-8 residual (incl. fault recovery), FP64 vs mixed",
        "value": round(value, 1),
        "unit": "MDoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"poisson-kuhn-cube n_sub={n_sub} ({6 * n_sub ** 3} macro tets) level={level}: "
                        f"fault after 5 V(2,1) cycles, 3 local recovery cycles, solve to 1e-8",
            "unknowns": int(f_dev.numel()),
            "smoother": "red-black SOR omega=1.25, V(2,1), coarse level 2 solved with its dense inverse",
            "fault_tet": t_fault,
            "graph": bool(args.graph),
            "fused_sweeps": args.fused_sweeps,
            "tuning": {str(k): {"block": v[0], "xcd_order": v[1], "nodes_per_thread": v[2]}
                       for k, v in tuning.items()},
        },
        "time_to_1e8_s": round(ms_per_step / 1e3, 5),
        "cycles_per_job": k_faulty,
        "k_free": k_free,
        "kappa": round((k_faulty - k_free) / 5, 3),
        "final_rel_res": rel,
        "roofline": roofline,
        "uninstrumented": uninstrumented,
        "vcycle_rates": rates,
        "recoveries": recoveries,
        "mixed": mixed,
        "general_mesh": general,
        "unstructured_mesh": mesh,
        **extra,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
