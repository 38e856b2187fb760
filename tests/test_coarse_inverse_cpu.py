"""The dense inverse of the coarsest-level operator that the library
factorises on the host (used for the coarsest solve with k = 1, on the cube
and on general macro meshes) against numpy's inverse of the oracle's own
coarsest-level stiffness matrix, assembled element by element (eq. (2),
level 2: one inner node per macro tetrahedron, Sec. 2.1).  CPU only, no GPU
calls."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1506_06185_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def dump_exe(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("cinv") / "coarse_inverse_dump")
    csrc = os.path.join(ROOT, "paper_1506_06185_amd", "csrc")
    subprocess.run(["g++", "-O2", "-std=c++17", "-pthread", "-o", exe,
                    os.path.join(ROOT, "tests", "host", "coarse_inverse_dump.cpp"), os.path.join(csrc, "topology.cpp"),
                    os.path.join(csrc, "geometry.cpp")], check=True)
    return exe


@pytest.mark.parametrize("general", [False, True])
@pytest.mark.parametrize("n_sub", [1, 2])
def test_coarse_inverse_matches_oracle(dump_exe, tmp_path, n_sub, general):
    V = inputs.perturbed_vertices(n_sub, 0) if general else None
    args = [dump_exe, str(n_sub), str(tmp_path)]
    if general:
        vf = tmp_path / "v.f64"
        np.ascontiguousarray(V, dtype=np.float64).tofile(vf)
        args.append(str(vf))
    r = subprocess.run(args, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    N = 4 * n_sub  # cells per axis at level 2
    n = (N - 1) ** 3
    pos = np.fromfile(tmp_path / "pos.i32", dtype=np.int32).reshape(n, 3)
    inv = np.fromfile(tmp_path / "inv.f64", dtype=np.float64).reshape(n, n)
    # oracle's vector order: (x-1) + (N-1)((y-1) + (N-1)(z-1))
    idx = (pos[:, 0] - 1) + (N - 1) * ((pos[:, 1] - 1) + (N - 1) * (pos[:, 2] - 1))
    assert np.array_equal(np.sort(idx), np.arange(n))
    p = oracle.Problem(n_sub, 3, vertices=V)
    A = p.matrix(2).toarray()
    p.close()
    ref = np.linalg.inv(A)[np.ix_(idx, idx)]
    assert np.abs(inv - ref).max() <= 1e-13 * np.abs(ref).max()
    # symmetric, and the inverse of A in the library's own unknown order
    assert np.abs(inv - inv.T).max() <= 1e-14 * np.abs(ref).max()
    Ap = A[np.ix_(idx, idx)]
    assert np.abs(Ap @ inv - np.eye(n)).max() <= 1e-13
