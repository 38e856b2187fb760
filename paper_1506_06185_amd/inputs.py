"""Seeded synthetic inputs for the unit-cube workloads.

This module is shared by the GPU path's callers (tests, benchmark) and by the
oracle-side tests.  It holds no multigrid arithmetic: only random draws,
point evaluations of the source and boundary functions and the macro-mesh
geometry that places a fault, returned in the user-facing orders

* interior nodes: global lexicographic, index = (x-1) + (N-1)*((y-1) + (N-1)*(z-1)),
  x fastest, with N = n_sub * 2**level cells per axis and h = 1/N;
* elements: cell-lexicographic (cx + N*(cy + N*cz)) times 6 Kuhn permutations
  in the order (0,1,2), (0,2,1), (1,0,2), (1,2,0), (2,0,1), (2,1,0).

Every random draw uses ``numpy.random.default_rng([seed, stream])`` with one
stream per quantity, so any input can be rebuilt from (seed, shape) alone.
"""
from __future__ import annotations

import math

import numpy as np

STREAM_FAULT_TET = 1
STREAM_UNIFORM_RHS = 2
STREAM_LOG_K = 3
STREAM_U_OBS = 4
STREAM_FD_DIRS = 5
STREAM_BATCH_SIZES = 6
STREAM_BATCH_FAULTS = 7
STREAM_VERTICES = 8


def rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), int(stream)])


def cells_per_axis(n_sub: int, level: int) -> int:
    return int(n_sub) << int(level)


def n_interior(n_sub: int, level: int) -> int:
    return (cells_per_axis(n_sub, level) - 1) ** 3


def n_macro_tets(n_sub: int) -> int:
    return 6 * n_sub ** 3


def n_elements(n_sub: int, level: int) -> int:
    return 6 * cells_per_axis(n_sub, level) ** 3


def interior_axis(n_sub: int, level: int) -> np.ndarray:
    """Coordinates 1/N .. (N-1)/N of the interior grid lines."""
    N = cells_per_axis(n_sub, level)
    return np.arange(1, N, dtype=np.float64) / N


def sine_source(n_sub: int, level: int) -> np.ndarray:
    """f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z) at the interior nodes (lex order).

    It is the source whose exact solution of -Laplace(u) = f with u = 0 on the
    cube's boundary is u = sin(pi x) sin(pi y) sin(pi z).
    """
    s = np.sin(math.pi * interior_axis(n_sub, level))
    f = (3.0 * math.pi ** 2) * (s[None, None, :] * s[None, :, None] * s[:, None, None])
    return np.ascontiguousarray(f.reshape(-1))


def sine_solution(n_sub: int, level: int) -> np.ndarray:
    """u = sin(pi x) sin(pi y) sin(pi z) at the interior nodes (lex order)."""
    s = np.sin(math.pi * interior_axis(n_sub, level))
    u = s[None, None, :] * s[None, :, None] * s[:, None, None]
    return np.ascontiguousarray(u.reshape(-1))


def uniform_load(n_sub: int, level: int, seed: int = 0) -> np.ndarray:
    """Load vector entries drawn from U[-1, 1] (used directly as b)."""
    return rng(seed, STREAM_UNIFORM_RHS).uniform(-1.0, 1.0, n_interior(n_sub, level))


def lognormal_k(n_sub: int, level: int, seed: int = 0, sigma: float = 0.5) -> np.ndarray:
    """Per-element diffusion coefficient k = exp(sigma * Z), Z ~ N(0, 1)."""
    z = rng(seed, STREAM_LOG_K).standard_normal(n_elements(n_sub, level))
    return np.exp(sigma * z)


def gaussian_obs(n_sub: int, level: int, seed: int = 0) -> np.ndarray:
    """Observation u_obs ~ N(0, 1) per interior node."""
    return rng(seed, STREAM_U_OBS).standard_normal(n_interior(n_sub, level))


def fd_directions(size: int, count: int, seed: int = 0, offset: int = 0) -> np.ndarray:
    """`count` directions of length `size`, N(0,1) entries, each scaled to unit 2-norm.

    ``offset`` skips that many earlier directions of the same stream so that
    the directions for f and for k are distinct draws.
    """
    g = rng(seed, STREAM_FD_DIRS)
    if offset:
        g.standard_normal((offset, size))
    d = g.standard_normal((count, size))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return d


def fault_tet(n_sub: int, seed: int = 0) -> int:
    """Macro tetrahedron that fails (uniform over the 6 n^3 macro-tets)."""
    return int(rng(seed, STREAM_FAULT_TET).integers(n_macro_tets(n_sub)))


def batch_levels(count: int, seed: int = 0, lo: int = 5, hi: int = 7) -> np.ndarray:
    """Refinement levels of a batch of independent n_sub = 2 problems, uniform in [lo, hi]."""
    return rng(seed, STREAM_BATCH_SIZES).integers(lo, hi + 1, size=count)


def batch_faults(n_faults: int, n_sub: int, seed: int = 0) -> np.ndarray:
    """Distinct faulty macro-tets for the concurrent-recovery workload."""
    g = rng(seed, STREAM_BATCH_FAULTS)
    return np.sort(g.choice(n_macro_tets(n_sub), size=n_faults, replace=False))


def batch_member_faults(n_members: int, n_faulty: int, n_sub: int, seed: int = 0):
    """(member, tet) pairs of the faulty batch members: distinct members, one
    faulty macro-tet each (drawn after the global problem's faulty tets of
    ``batch_faults`` in the same stream, so the two plans are independent)."""
    g = rng(seed, STREAM_BATCH_FAULTS)
    g.integers(1 << 30, size=16)
    members = np.sort(g.choice(n_members, size=n_faulty, replace=False))
    tets = g.integers(n_macro_tets(n_sub), size=n_faulty)
    return [(int(m), int(t)) for m, t in zip(members, tets)]


def harmonic_boundary(n_sub: int, level: int) -> np.ndarray:
    """Dirichlet data g = 1 + x^2 + 2 y^2 - 3 z^2 + x y at all (N+1)^3 grid
    vertices, index x + (N+1)*(y + (N+1)*z) with x fastest (the solver reads
    only the boundary entries).  g is harmonic, so it is also the exact
    solution of Laplace's equation with these boundary values."""
    N = cells_per_axis(n_sub, level)
    t = np.arange(N + 1, dtype=np.float64) / N
    z, y, x = t[:, None, None], t[None, :, None], t[None, None, :]
    g = 1.0 + x * x + 2.0 * y * y - 3.0 * z * z + x * y
    return np.ascontiguousarray(g.reshape(-1))


_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def macro_tet_vertices(n_sub: int, tet: int):
    """The 4 vertices of a macro tetrahedron in subcube units: its subcube's
    lowest corner, then one unit step along each axis of its permutation."""
    cube, perm = divmod(int(tet), 6)
    v = [cube % n_sub, (cube // n_sub) % n_sub, cube // (n_sub * n_sub)]
    out = [tuple(v)]
    for a in _PERMS[perm]:
        v[a] += 1
        out.append(tuple(v))
    return out


def boundary_contact(n_sub: int, tet: int):
    """(faces, edges, vertices) of a macro tetrahedron that lie on the cube's
    boundary: a simplex of vertices lies there when they share a coordinate
    equal to 0 or n_sub."""
    from itertools import combinations

    vs = macro_tet_vertices(n_sub, tet)

    def on_boundary(pts):
        return any(all(p[a] == side for p in pts) for a in range(3) for side in (0, n_sub))

    return tuple(sum(on_boundary(c) for c in combinations(vs, k)) for k in (3, 2, 1))


# fault scenarios of the recovery-strategy comparison: mesh size and the
# geometric position of the faulty macro tetrahedron
SCENARIOS = {
    "I": dict(n_sub=1, about="two faces on the boundary"),
    "II": dict(n_sub=2, about="one edge on the boundary, no face"),
    "III": dict(n_sub=3, about="no vertex on the boundary (floating)"),
}


def scenario_fault_tet(name: str) -> int:
    """Lowest-numbered macro tetrahedron matching the scenario's description."""
    n = SCENARIOS[name]["n_sub"]
    want = {"I": lambda f, e, v: f == 2, "II": lambda f, e, v: f == 0 and e == 1,
            "III": lambda f, e, v: v == 0}[name]
    for t in range(n_macro_tets(n)):
        if want(*boundary_contact(n, t)):
            return t
    raise ValueError(f"no macro tetrahedron fits scenario {name}")


def second_fault_tet(n_sub: int, first: int) -> int:
    """Lowest-numbered macro tetrahedron with no face on the boundary that shares
    no vertex with ``first`` (the later fault of a two-fault sequence)."""
    vs = set(macro_tet_vertices(n_sub, first))
    for t in range(n_macro_tets(n_sub)):
        if boundary_contact(n_sub, t)[0] == 0 and not vs & set(macro_tet_vertices(n_sub, t)):
            return t
    raise ValueError("no separated macro tetrahedron")


def perturbed_vertices(n_sub: int, seed: int = 0, amplitude: float = 0.15) -> np.ndarray:
    """Positions ((n+1)^3, 3), x fastest, of the macro vertices of a general
    macro mesh: the grid points (x, y, z) / n, each moved by amplitude / n
    times a U[-1, 1]^3 draw.  Boundary vertices move too, so the domain is a
    perturbed cube.  The connectivity is the Kuhn split's."""
    n = int(n_sub)
    t = np.arange(n + 1, dtype=np.float64) / n
    z, y, x = np.meshgrid(t, t, t, indexing="ij")
    base = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    d = rng(seed, STREAM_VERTICES).uniform(-1.0, 1.0, base.shape)
    return np.ascontiguousarray(base + (amplitude / n) * d)


def macro_tet_corners(vertices: np.ndarray, n_sub: int, tet: int) -> np.ndarray:
    """The 4 corner positions (4, 3) of a macro tetrahedron of a general macro
    mesh, in the order of macro_tet_vertices."""
    n = int(n_sub)
    idx = [v[0] + (n + 1) * (v[1] + (n + 1) * v[2]) for v in macro_tet_vertices(n, tet)]
    return np.asarray(vertices)[idx]


# ---------------------------------------------------------------------------
# Unstructured macro meshes (vertex and tetrahedron lists).  Every tetrahedron
# lists its vertices by a proper 4-colouring of the mesh: a vertex has the
# same position (its colour) in every tetrahedron that contains it.
# ---------------------------------------------------------------------------
STREAM_MESH_VERTICES = 9


def octahedron_mesh(centre: bool = True):
    """The octahedron |x| + |y| + |z| <= 1.  With ``centre``: 8 tetrahedra
    around an interior vertex at the origin (colours: origin 0, poles 1,
    equator vertices 2 and 3 alternately); without: 4 tetrahedra around the
    polar axis (poles 0 and 1, equator 2 and 3).  Returns (vertices (nv, 3),
    tets (nt, 4) int32)."""
    eq = [[1, 0, 0], [0, 1, 0], [-1, 0, 0], [0, -1, 0]]
    if centre:
        v = np.array([[0, 0, 0], [0, 0, 1], [0, 0, -1]] + eq, dtype=np.float64)
        tets = []
        for pole in (1, 2):
            for i in range(4):
                a, b = 3 + i, 3 + (i + 1) % 4
                even, odd = (a, b) if i % 2 == 0 else (b, a)
                tets.append([0, pole, even, odd])
    else:
        v = np.array([[0, 0, 1], [0, 0, -1]] + eq, dtype=np.float64)
        tets = []
        for i in range(4):
            a, b = 2 + i, 2 + (i + 1) % 4
            even, odd = (a, b) if i % 2 == 0 else (b, a)
            tets.append([0, 1, even, odd])
    return v, np.asarray(tets, dtype=np.int32)


# colour of a grid vertex of the 5-tetrahedra box split, by the parities of
# its coordinates (x + 2y + 4z bit pattern): a vertex and its antipode in a
# cube share a colour, the 4 even-parity corners of a cube have 4 colours
_BOX_COLOUR = {0b000: 0, 0b111: 0, 0b011: 1, 0b100: 1, 0b101: 2, 0b010: 2, 0b110: 3, 0b001: 3}


def box_mesh(nx: int, ny: int, nz: int):
    """The box [0, nx] x [0, ny] x [0, nz] of unit cubes, each split into 5
    tetrahedra: the central one on the cube's 4 corners of even coordinate
    sum, and one corner tetrahedron per odd corner with its 3 neighbours.
    Neighbouring cubes then split their common face along the same diagonal.
    Vertex id = x + (nx+1) (y + (ny+1) z); tets ordered cube by cube (x
    fastest), central first, then the corners by ascending vertex id."""
    def vid(x, y, z):
        return x + (nx + 1) * (y + (ny + 1) * z)

    def colour(x, y, z):
        return _BOX_COLOUR[(x & 1) | ((y & 1) << 1) | ((z & 1) << 2)]

    def ordered(vs):
        out = [None] * 4
        for p in vs:
            c = colour(*p)
            assert out[c] is None
            out[c] = vid(*p)
        return out

    tets = []
    for cz in range(nz):
        for cy in range(ny):
            for cx in range(nx):
                corners = [(cx + a, cy + b, cz + c) for c in (0, 1) for b in (0, 1) for a in (0, 1)]
                even = [p for p in corners if sum(p) % 2 == 0]
                odd = sorted((p for p in corners if sum(p) % 2 == 1), key=lambda p: vid(*p))
                tets.append(ordered(even))
                for p in odd:
                    nb = [q for q in even if sum(abs(q[i] - p[i]) for i in range(3)) == 1]
                    tets.append(ordered([p] + nb))
    z, y, x = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    v = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1).astype(np.float64)
    return v, np.asarray(tets, dtype=np.int32)


def perturb_mesh(vertices: np.ndarray, seed: int = 0, amplitude: float = 0.15) -> np.ndarray:
    """Each vertex moved by amplitude times a U[-1, 1]^3 draw (the domain
    changes with it)."""
    v = np.asarray(vertices, dtype=np.float64)
    return np.ascontiguousarray(v + amplitude * rng(seed, STREAM_MESH_VERTICES).uniform(-1.0, 1.0, v.shape))


def mesh_fault_tet(n_tets: int, seed: int = 0) -> int:
    """Macro tetrahedron of an unstructured mesh that fails (uniform)."""
    return int(rng(seed, STREAM_FAULT_TET).integers(0, int(n_tets)))
