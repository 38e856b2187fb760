"""CPU check of the unstructured-mesh topology of the GPU path (csrc/mesh.cpp)
against the oracle's independent assembly (Sec. 3.1; eq. (2)).

A small host program (tests/host/mesh_check.cpp) builds the topology, checks
its internal invariants (every user index once, ghost lists, no stencil entry
inside one colour class), and writes, per level, the operator that the
topology's tables define (volume stencils and master rows) and the interface
rows of the transfers, in the user order.  These must equal the oracle's
element-by-element stiffness matrix, mass matrix and prolongation rows."""
import os
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_1506_06185_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def mesh_check(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("mesh") / "mesh_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", exe, os.path.join(ROOT, "tests/host/mesh_check.cpp"),
                    os.path.join(ROOT, "paper_1506_06185_amd/csrc/mesh.cpp"),
                    os.path.join(ROOT, "paper_1506_06185_amd/csrc/topology.cpp")], check=True)
    return exe


def run(exe, tmp_path, v, t, L, Lc, faults=None, k=None):
    mf, of = str(tmp_path / "mesh.txt"), str(tmp_path / "out.txt")
    with open(mf, "w") as fh:
        fh.write(f"{len(v)} {len(t)} {L} {Lc}\n")
        for x in v:
            fh.write("%.17g %.17g %.17g\n" % tuple(x))
        for q in t:
            fh.write("%d %d %d %d\n" % tuple(q))
    extra = [",".join(str(q) for q in faults) if faults else "-"] if faults or k is not None else []
    if k is not None:
        extra.append(",".join("%.17g" % x for x in k))
    out = subprocess.run([exe, mf, of] + extra, capture_output=True, text=True)
    return out, of


def parse(of):
    head = None
    mats = {}
    with open(of) as fh:
        lines = fh.read().split("\n")
    head = lines[0].split()
    i = 1
    while i < len(lines) and lines[i]:
        tag = lines[i].split()
        i += 1
        rows = []
        while lines[i] != "end":
            r, c, v = lines[i].split()
            rows.append((int(r), int(c), float(v)))
            i += 1
        i += 1
        mats[(tag[0], int(tag[1]))] = np.array(rows, dtype=np.float64).reshape(-1, 3)
    return {head[q]: int(head[q + 1]) for q in range(0, len(head), 2)}, mats


def to_csr(trip, shape):
    return sp.coo_matrix((trip[:, 2], (trip[:, 0].astype(int), trip[:, 1].astype(int))), shape=shape).tocsr()


MESHES = {
    "octa8": lambda: (inputs.perturb_mesh(inputs.octahedron_mesh(True)[0], seed=3, amplitude=0.08),
                      inputs.octahedron_mesh(True)[1]),
    "octa4": lambda: inputs.octahedron_mesh(False),
    "box222p": lambda: (inputs.perturb_mesh(inputs.box_mesh(2, 2, 2)[0], seed=5, amplitude=0.12),
                        inputs.box_mesh(2, 2, 2)[1]),
}


@pytest.mark.parametrize("name", sorted(MESHES))
def test_mesh_topology_operator_equals_oracle(name, mesh_check, tmp_path):
    v, t = MESHES[name]()
    L, Lc = 4, 2
    out, of = run(mesh_check, tmp_path, v, t, L, Lc)
    assert out.returncode == 0, out.stdout + out.stderr
    head, mats = parse(of)
    p = oracle.MeshProblem(v, t, L, Lc)
    assert head["n_dofs"] == p.ndof
    for l in range(Lc, L + 1):
        n = p.ndof_at(l)
        A = to_csr(mats[("A", l)], (n, n))
        Ao = p.matrix(l, "A")
        assert abs(A - Ao).max() <= 1e-13 * abs(Ao).max(), (l, abs(A - Ao).max())
    # the consistent mass matrix of the finest level
    M = to_csr(mats[("M", L)], (p.ndof, p.ndof))
    Mo = p.matrix(L, "M")
    assert abs(M - Mo).max() <= 1e-13 * abs(Mo).max(), abs(M - Mo).max()
    # the boundary nodes (order and positions) and the interior-boundary block
    xyz, dof = p.nodes(L)
    order = p.boundary_order(L)
    X = mats[("X", L)]
    assert len(X) == 3 * len(order)
    pos = np.zeros((len(order), 3))
    pos[X[:, 0].astype(int), X[:, 1].astype(int)] = X[:, 2]
    assert np.abs(pos - xyz[order]).max() < 1e-14
    D = to_csr(mats[("D", L)], (p.ndof, len(order)))
    Af = p.matrix(L, "A", full=True).tocsr()
    interior = np.argsort(np.where(dof >= 0, dof, 1 << 40))[: p.ndof]
    Do = Af[interior][:, order]
    assert abs(D - Do).max() <= 1e-13 * abs(Do).max()
    for l in range(Lc + 1, L + 1):
        nf, nc = p.ndof_at(l), p.ndof_at(l - 1)
        P = to_csr(mats[("P", l)], (nf, nc))
        Po = p.matrix(l, "P").tocsr()
        # the masters are the user indices before the tetrahedron interiors
        masters = np.arange(nf - len(t) * ((2 ** l - 1) * (2 ** l - 2) * (2 ** l - 3) // 6))
        assert abs(P[masters] - Po[masters]).max() == 0.0
        R = to_csr(mats[("R", l)], (nc, nf))
        masters_c = np.arange(nc - len(t) * ((2 ** (l - 1) - 1) * (2 ** (l - 1) - 2) * (2 ** (l - 1) - 3) // 6))
        assert abs(R[masters_c] - Po.T.tocsr()[masters_c]).max() == 0.0


def test_mesh_topology_rejects_bad_meshes(mesh_check, tmp_path):
    v, t = inputs.octahedron_mesh(True)
    bad = t.copy()
    bad[0, [2, 3]] = bad[0, [3, 2]]
    out, _ = run(mesh_check, tmp_path, v, bad, 3, 2)
    assert out.returncode == 3 and "4-colouring" in out.stdout
    flat = v.copy()
    flat[:, 2] = 0.0
    out, _ = run(mesh_check, tmp_path, flat, t, 3, 2)
    assert out.returncode == 3 and "flat" in out.stdout


@pytest.mark.parametrize("name,faults", [("box222p", (1,)), ("box222p", (2, 9)), ("octa8", (0, 5)), ("octa4", (3,))])
def test_mesh_intact_side_equals_oracle(name, faults, mesh_check, tmp_path):
    """The intact side of a Dirichlet-Neumann recovery (Sec. 4.3, eq. (5)):
    the master rows summed over the elements of intact tetrahedra only, on
    every level, and the coarsest-level operator built from them, against the
    oracle's assembly over the intact elements."""
    v, t = MESHES[name]()
    L, Lc = 4, 2
    out, of = run(mesh_check, tmp_path, v, t, L, Lc, faults)
    assert out.returncode == 0, out.stdout + out.stderr
    head, mats = parse(of)
    p = oracle.MeshProblem(v, t, L, Lc)
    for l in range(Lc, L + 1):
        n = p.ndof_at(l)
        I = to_csr(mats[("I", l)], (n, n))
        Io = p.side_matrix(l, list(faults), "intact")
        assert abs(I - Io).max() <= 1e-13 * abs(Io).max(), (l, abs(I - Io).max())
    n = p.ndof_at(Lc)
    C = to_csr(mats[("C", Lc)], (n, n))
    Co = p.side_matrix(Lc, list(faults), "intact").tocsr()
    keep = Co.diagonal() > 0
    assert keep.sum() < n
    assert abs(C[keep][:, keep] - Co[keep][:, keep]).max() <= 1e-13 * abs(Co).max()
    assert abs(C[keep][:, ~keep]).max() == 0.0


@pytest.mark.parametrize("name,faults", [("box222p", (1,)), ("octa8", (0, 5)), ("octa4", None)])
def test_mesh_coefficient_per_tetrahedron_equals_oracle(name, faults, mesh_check, tmp_path):
    """eq. (2) with k constant on each macro tetrahedron: the volume
    stencils, master rows, coarsest-level rows and Dirichlet couplings that
    the host builds, and the intact side of a Dirichlet-Neumann recovery
    over the same k (eq. (5)), against the oracle's assembly with that k."""
    v, t = MESHES[name]()
    L, Lc = 4, 2
    k = np.random.default_rng(11).uniform(0.2, 5.0, len(t))
    out, of = run(mesh_check, tmp_path, v, t, L, Lc, faults, k)
    assert out.returncode == 0, out.stdout + out.stderr
    head, mats = parse(of)
    p = oracle.MeshProblem(v, t, L, Lc, k_tet=k)
    for l in range(Lc, L + 1):
        n = p.ndof_at(l)
        W = to_csr(mats[("W", l)], (n, n))
        Wo = p.matrix(l, "A")
        assert abs(W - Wo).max() <= 1e-13 * abs(Wo).max(), (l, abs(W - Wo).max())
    n = p.ndof_at(Lc)
    WC = to_csr(mats[("WC", Lc)], (n, n))
    Wo = p.matrix(Lc, "A")
    assert abs(WC - Wo).max() <= 1e-13 * abs(Wo).max()
    xyz, dof = p.nodes(L)
    order = p.boundary_order(L)
    D = to_csr(mats[("WD", L)], (p.ndof, len(order)))
    Af = p.matrix(L, "A", full=True).tocsr()
    interior = np.argsort(np.where(dof >= 0, dof, 1 << 40))[: p.ndof]
    Do = Af[interior][:, order]
    assert abs(D - Do).max() <= 1e-13 * abs(Do).max()
    if faults:
        for l in range(Lc, L + 1):
            n = p.ndof_at(l)
            I = to_csr(mats[("I", l)], (n, n))
            Io = p.side_matrix(l, list(faults), "intact")
            assert abs(I - Io).max() <= 1e-13 * abs(Io).max(), (l, abs(I - Io).max())
        n = p.ndof_at(Lc)
        C = to_csr(mats[("C", Lc)], (n, n))
        Co = p.side_matrix(Lc, list(faults), "intact").tocsr()
        keep = Co.diagonal() > 0
        assert abs(C[keep][:, keep] - Co[keep][:, keep]).max() <= 1e-13 * abs(Co).max()
