"""CPU checks of the C ABI library: it loads, exports every symbol that
include/hhgr.h declares, validates descriptions and sizes workspaces (no GPU
calls), and the host topology/index arithmetic passes its checks."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "hhgr.h")).read()
    return sorted(set(re.findall(r"\b(hhgr_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_1506_06185_amd import hhgr

    L = hhgr.lib()
    syms = header_symbols()
    assert len(syms) >= 20
    missing = [s for s in syms if not hasattr(L, s)]
    assert not missing, missing
    assert set(syms) == set(hhgr.EXPORTED)


def test_workspace_sizing_and_validation():
    from paper_1506_06185_amd import hhgr

    d = hhgr.make_desc(n_sub=2, level=7)
    n7 = hhgr.workspace_bytes(d)
    assert 0.5e9 < n7 < 2e9
    d8 = hhgr.make_desc(n_sub=2, level=8, precision="mixed")
    assert hhgr.workspace_bytes(d8) > 7 * n7
    for bad in (dict(level=2), dict(n_sub=0), dict(omega=2.5), dict(max_faults=9), dict(nu_pre=0, nu_post=0)):
        with pytest.raises(hhgr.HHGRError) as e:
            hhgr.workspace_bytes(hhgr.make_desc(**bad))
        assert e.value.code == hhgr.HHGR_EINVAL


@pytest.mark.parametrize("args", ["1 4", "2 5", "3 4"])
def test_topology_host_checks(args, tmp_path):
    exe = str(tmp_path / "topocheck")
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", exe, os.path.join(ROOT, "tests/host/topology_check.cpp"),
                    os.path.join(ROOT, "paper_1506_06185_amd/csrc/topology.cpp")], check=True)
    out = subprocess.run([exe] + args.split(), capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "ok" in out.stdout


def test_engine_host_logic_under_asan(tmp_path):
    """The engine's host code (set-up, faults, recoveries, batches with armed
    Dirichlet-Dirichlet recoveries, graph bookkeeping, tuning) built with g++
    against a mock HIP runtime and run under AddressSanitizer/UBSan; the
    numerical kernels are skipped."""
    exe = str(tmp_path / "enginecheck")
    h = os.path.join(ROOT, "tests/host")
    subprocess.run(["g++", "-std=c++17", "-O0", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-I" + os.path.join(h, "mock"), "-x", "c++", os.path.join(ROOT, "paper_1506_06185_amd/csrc/engine.hip"),
                    "-x", "none", os.path.join(ROOT, "paper_1506_06185_amd/csrc/topology.cpp"),
                    os.path.join(ROOT, "paper_1506_06185_amd/csrc/mesh.cpp"),
                    os.path.join(ROOT, "paper_1506_06185_amd/csrc/geometry.cpp"),
                    os.path.join(h, "mock/mock_hip.cpp"), os.path.join(h, "mock/mock_kernels.cpp"),
                    os.path.join(h, "engine_host_check.cpp"), "-o", exe], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="halt_on_error=1")
    out = subprocess.run([exe], capture_output=True, text=True, env=env)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "ok" in out.stdout


def test_fused_sweep_kernel_in_cpu_emulation(tmp_path):
    """The fused red-black sweep kernel source (fused.hip) built for the host
    against a device-code emulation (a workgroup = host threads meeting at a
    barrier) and run under AddressSanitizer/UBSan: every slot of one fused
    sweep equals a plain two-colour sweep from the closure layout, bitwise,
    for several meshes, levels and tile shapes (zero start with a NaN source,
    residual tail, FP64 and FP32).  Built with tiles of 8 i values instead of
    64, so that these small levels have several tiles along i as well (the
    seams between tiles are where the halo logic could go wrong)."""
    exe = str(tmp_path / "fusedcheck")
    h = os.path.join(ROOT, "tests/host")
    subprocess.run(["g++", "-std=c++20", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-ffp-contract=off", "-pthread", "-DHHGR_FUSED_TI=8", "-I" + os.path.join(h, "mockdev"), "-x", "c++",
                    os.path.join(ROOT, "paper_1506_06185_amd/csrc/fused.hip"), "-x", "none",
                    os.path.join(h, "fused_check.cpp"), os.path.join(ROOT, "paper_1506_06185_amd/csrc/topology.cpp"),
                    "-o", exe], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="halt_on_error=1")
    out = subprocess.run([exe], capture_output=True, text=True, env=env)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "ok" in out.stdout
