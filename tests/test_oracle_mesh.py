"""Oracle mesh pins: macro mesh, Bey refinement, primitive counts and the
sizes printed in the paper (Sec. 2.2, Sec. 4.4, Sec. 5)."""
import json
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def vol_interior(m):  # nodes strictly inside a macro tetrahedron refined to m = 2^L segments per edge
    return (m - 1) * (m - 2) * (m - 3) // 6


def face_interior(m):
    return (m - 1) * (m - 2) // 2


def vol_closure(m):
    return (m + 1) * (m + 2) * (m + 3) // 6


@pytest.mark.parametrize("n_sub,level", [(1, 1), (1, 3), (2, 2), (2, 4), (3, 2)])
def test_bey_refinement_is_freudenthal(n_sub, level):
    # Two independent constructions of the refined mesh must give the same
    # element set: Bey's rule applied level by level, and the Kuhn split of
    # every cell of the N^3 grid.
    p = oracle.Problem(n_sub, level, coarse_level=1)
    assert p.check_freudenthal(level)
    assert p.nelem_at(level) == 6 * (n_sub << level) ** 3


@pytest.mark.parametrize("n_sub,level", [(1, 0), (2, 3), (3, 2)])
def test_volumes_sum_to_one(n_sub, level):
    p = oracle.Problem(n_sub, max(level, 1), coarse_level=1)
    assert abs(p.volume_sum(level) - 1.0) < 1e-12


def test_element_order_is_cell_lex_times_perm():
    p = oracle.Problem(2, 2, coarse_level=1)
    ev, ecl = p.elements(2)
    N = 8
    assert sorted(ecl.tolist()) == list(range(6 * N ** 3))
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    # decode vertices and check cell corner + axis steps
    xyz = np.stack([ev % (N + 1), (ev // (N + 1)) % (N + 1), ev // (N + 1) ** 2], axis=-1)
    for e in range(0, len(ecl), 97):
        cell, q = divmod(int(ecl[e]), 6)
        cx, cy, cz = cell % N, (cell // N) % N, cell // N ** 2
        assert tuple(xyz[e, 0]) == (cx, cy, cz)
        steps = [int(np.argmax(xyz[e, s + 1] - xyz[e, s])) for s in range(3)]
        assert tuple(steps) == perms[q]


@pytest.mark.parametrize("level", [4, 5])
def test_primitive_counts_brute_force(level):
    # Containment counts of every interior node in the 48 macro tetrahedra of
    # the 2x2x2 cube: 1 = volume interior, 2 = face, 24 = the centre vertex,
    # anything else = a macro edge (Sec. 3.1 container classes).
    p = oracle.Problem(2, level, coarse_level=1)
    c = p.containment_counts(level)
    m = 1 << level
    assert (c == 1).sum() == 48 * vol_interior(m)
    assert (c == 2).sum() == 72 * face_interior(m)
    assert (c == 24).sum() == 1
    edge = (c > 2) & (c != 24)
    assert edge.sum() == 26 * (m - 1)
    assert c.min() >= 1
    assert len(c) == (2 * m - 1) ** 3


def test_fault_mask_counts():
    p = oracle.Problem(2, 4, coarse_level=1)
    m = 16
    for t in (0, 17, 47):
        inner = p.tet_mask(t, closure=False)
        closed = p.tet_mask(t, closure=True)
        assert inner.sum() == vol_interior(m)
        assert (closed & ~inner).sum() > 0
        assert np.all(closed[inner])


def test_paper_printed_sizes():
    g = json.load(open(os.path.join(GOLD, "paper_sizes.json")))
    # Fig. 2 setting: 16 million unknowns, 0.3 million lost (Sec. 2.2)
    s = g["fig2_setting"]
    N = s["n_sub"] << s["level"]
    m = 1 << s["level"]
    assert int((N - 1) ** 3 // 10 ** 6) == s["unknowns_millions_printed"]  # "16 million": leading digits
    assert round(vol_interior(m) / 1e6, 1) == s["lost_millions_printed"]
    # Scenarios I-III (Sec. 4.4)
    sc = g["scenarios"]
    for key in ("I", "II", "III"):
        e = sc[key]
        N = e["n_sub"] << sc["level"]
        m = 1 << sc["level"]
        dofs = (N - 1) ** 3
        assert dofs // 10 ** 6 == e["unknowns_millions_printed"]
        share = 100.0 * vol_interior(m) / dofs
        # the paper rounds loosely (Scenario I prints 1/6 = 16.7 %)
        assert abs(share - e["fault_percent_printed"]) < 0.5
    # weak scaling (Sec. 5, Table 3): 6 (2^l+1)^3 tets at refinement level 8
    w = g["weak_scaling"]
    m = 1 << w["level"]
    pts = [n * m + 1 for n in w["n_sub"]]
    assert pts == w["grid_points_per_axis_printed"]
    assert abs(vol_closure(m) - w["points_per_tet_printed"]) / w["points_per_tet_printed"] < 0.05
    largest = (w["n_sub"][-1] * m - 1) ** 3
    assert largest > w["largest_unknowns_printed"]
    ratio_first = 100.0 * vol_interior(m) / (w["n_sub"][0] * m - 1) ** 3
    ratio_last = 100.0 * vol_closure(m) / (w["n_sub"][-1] * m - 1) ** 3
    assert round(ratio_first, 1) == w["ratio_percent_first_printed"]
    assert round(ratio_last, 4) == pytest.approx(w["ratio_percent_last_printed"], rel=0.05)


def test_paper_kappa_denominators():
    # eq. (3): kappa = (k_faulty - k_free) / k_F, so every printed kappa times
    # k_F is (up to the table's rounding) an integer in [0, k_F].
    g = json.load(open(os.path.join(GOLD, "paper_kappa.json")))
    for tab in ("table1", "table2"):
        kF = g[tab]["k_F"]
        for eta in ("eta2", "eta5"):
            v = np.array(g[tab][eta]) * kF
            assert np.all(np.abs(v - np.round(v)) < 0.06 * kF / 10 + 0.06)
            assert v.min() >= -1e-9 and v.max() <= kF + 1e-9
        # n_I = 0 is the do-nothing job: identical for LR, DD and DN
        row0 = np.array(g[tab]["eta2"][0]).reshape(3, 3)
        assert np.all(row0 == row0[:, :1])
