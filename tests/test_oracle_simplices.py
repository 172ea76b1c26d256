"""Pins of the oracle's edge and triangle lists (E, F, I_E, I_F) and of its
VE, VF, EF, ET and FT blocks, against things other than the oracle itself:

* the paper's worked example (Section 4.4, on the mesh of Fig. 4): I_E =
  0, 9, 12, triangle f5 = v0 v3 v4 and FE(f5) = e2, e6, e9 (golden fixture);
* brute force from the set definitions on tiny meshes (pure Python): every
  edge and triangle listed once, in the interval of its owner cluster (the
  smallest cluster among its vertices, Section 4.3), each relation by scanning
  every edge, triangle or tetrahedron for the ones that contain the row;
* closed forms on n^3 Kuhn lattices (|E|, |F| from the Euler characteristic
  of a ball, interior vertex counts) and incidence sums (sum |VE| = 2|E|,
  sum |VF| = sum |EF| = 3|F|, sum |ET| = 6|T|, sum |FT| = 4|T|);
* planted mistakes in the oracle (lexicographic instead of discovery order,
  the largest-cluster owner, a dropped triangle in VF, a dropped term in ET)
  each fail at least one of these.
"""
import os

import numpy as np
import pytest

import meshgen
import oracle
from tests import pinlib

REL_VE, REL_VF, REL_EF, REL_ET, REL_FT = 8, 16, 32, 64, 128
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_example():
    lines = [ln.strip() for ln in open(os.path.join(GOLDEN, "sec44_fe_example.txt")) if ln.strip() and ln[0] != "#"]
    seg = {}
    for ln in lines:
        if ln.startswith("segment"):
            k = int(ln.split()[1])
            for v in ln.split(":")[1].split():
                seg[int(v)] = k
    tets = np.array([[int(x) for x in ln.split()[1:]] for ln in lines if ln.startswith("tet")], np.int32)
    cl = np.array([seg[v] for v in range(len(seg))], np.int32)
    field = lambda key: [int(x) for x in [ln for ln in lines if ln.startswith(key)][0].split(":")[1].split()]
    return tets, cl, field("I_E"), field("F 5"), field("FE 5")


def example_pin(make):
    """Section 4.4's example: the interval array, the sixth triangle and the
    ids of its three edges."""
    tets, cl, ie_exp, f5, fe5 = _read_example()
    o = make(tets, cl, 2)
    e, ie, f, _ = o.simplices()
    if list(ie) != ie_exp or len(f) <= 5 or list(f[5]) != f5:
        return False
    ids = {(int(a), int(b)): i for i, (a, b) in enumerate(e)}
    a, b, c = f5
    return sorted([ids.get((a, b), -1), ids.get((a, c), -1), ids.get((b, c), -1)]) == fe5


def _owner(cluster, q):
    return min(int(cluster[v]) for v in q)


def brute_pin(o, mesh):
    """Every edge / triangle exactly once, in its owner's interval; the five
    relations by scanning all simplices."""
    tets = [tuple(sorted(int(x) for x in t)) for t in mesh.tets]
    cl = mesh.cluster
    edges = {(t[i], t[j]) for t in tets for i in range(4) for j in range(i + 1, 4)}
    faces = {(t[i], t[j], t[k]) for t in tets for i in range(4) for j in range(i + 1, 4) for k in range(j + 1, 4)}
    e, ie, f, if_ = o.simplices()
    el = [tuple(int(x) for x in r) for r in e]
    fl = [tuple(int(x) for x in r) for r in f]
    if sorted(el) != sorted(edges) or len(set(el)) != len(el):
        return False
    if sorted(fl) != sorted(faces) or len(set(fl)) != len(fl):
        return False
    for k in range(mesh.nclusters):
        if any(_owner(cl, el[i]) != k for i in range(ie[k], ie[k + 1])):
            return False
        if any(_owner(cl, fl[i]) != k for i in range(if_[k], if_[k + 1])):
            return False
    for k in range(mesh.nclusters):
        verts = [v for v in range(len(cl)) if cl[v] == k]
        exp = {
            REL_VE: (verts, [[i for i, x in enumerate(el) if v in x] for v in verts]),
            REL_VF: (verts, [[i for i, x in enumerate(fl) if v in x] for v in verts]),
            REL_EF: (list(range(ie[k], ie[k + 1])),
                     [[j for j, y in enumerate(fl) if set(el[i]) <= set(y)] for i in range(ie[k], ie[k + 1])]),
            REL_ET: (list(range(ie[k], ie[k + 1])),
                     [[t for t, y in enumerate(tets) if set(el[i]) <= set(y)] for i in range(ie[k], ie[k + 1])]),
            REL_FT: (list(range(if_[k], if_[k + 1])),
                     [[t for t, y in enumerate(tets) if set(fl[i]) <= set(y)] for i in range(if_[k], if_[k + 1])]),
        }
        for rel, (rows_exp, lists_exp) in exp.items():
            rows, offs, ents = o.block(k, rel)
            if list(rows) != rows_exp or offs[0] != 0 or pinlib.csr_to_lists(offs, ents) != lists_exp:
                return False
    return True


def kuhn_pin(o, mesh, n):
    """Closed forms of the n^3 lattice and the incidence sums."""
    cf = pinlib.kuhn_counts(n)
    V, T, E = n ** 3, 6 * (n - 1) ** 3, cf["E"]
    F = 1 - V + E + T  # chi = V - E + F - T = 1 for a ball
    e, ie, f, if_ = o.simplices()
    if len(e) != E or len(f) != F or ie[-1] != E or if_[-1] != F:
        return False
    sums = {r: 0 for r in (REL_VE, REL_VF, REL_EF, REL_ET, REL_FT)}
    for k in range(mesh.nclusters):
        for r in sums:
            sums[r] += len(o.block(k, r)[2])
    return sums == {REL_VE: 2 * E, REL_VF: 3 * F, REL_EF: 3 * F, REL_ET: 6 * T, REL_FT: 4 * T}


SMALL = [meshgen.random_small(s, n=3 + (s % 2), nclusters=2 + s % 4) for s in range(4)]


def test_section44_example():
    assert example_pin(oracle.Oracle)


def test_lexicographic_order_would_not_give_the_example():
    """The reading matters: sorting each cluster's edges by vertex ids gives
    (v0, v4) the id 3, not the printed e6."""
    tets, cl, _, _, _ = _read_example()
    o = oracle.Oracle(tets, cl, 2)
    e, ie, _, _ = o.simplices()
    lex = sorted(tuple(x) for x in e[ie[0]:ie[1]].tolist())
    assert lex.index((0, 4)) == 3 and [tuple(x) for x in e.tolist()].index((0, 4)) == 6


@pytest.mark.parametrize("idx", range(len(SMALL)))
def test_brute_force_random_small(idx):
    m = SMALL[idx]
    assert brute_pin(oracle.Oracle.of(m), m)


def test_brute_force_cube_fans_and_nonmanifold():
    for m in (meshgen.cube(), meshgen.cube([0, 0, 0, 0, 1, 1, 1, 1]), meshgen.single_tet(), meshgen.fig4_example(),
              meshgen.nonmanifold(n=4, fins=3, dups=2, nclusters=3, seed=2)):
        assert brute_pin(oracle.Oracle.of(m), m)


def test_cube_edge_and_triangle_counts():
    o = oracle.Oracle.of(meshgen.cube())
    e, ie, f, if_ = o.simplices()
    assert len(e) == 19 and len(f) == 18 and list(ie) == [0, 19] and list(if_) == [0, 18]


@pytest.mark.parametrize("n,cap", [(3, 5), (4, 9), (5, 16)])
def test_kuhn_closed_forms(n, cap):
    m = meshgen.grid_mesh(n, cap, seed=n)
    assert kuhn_pin(oracle.Oracle.of(m), m, n)


def test_kuhn_interior_vertex():
    """An interior lattice vertex lies on 14 edges and 36 triangles (each of
    its 24 tetrahedra has three triangles through it, each shared by two)."""
    m = meshgen.grid_mesh(5, 125, seed=0, permute=False)
    o = oracle.Oracle.of(m)
    centre = 2 + 5 * (2 + 5 * 2)
    for rel, want in ((REL_VE, 14), (REL_VF, 36)):
        rows, offs, ents = o.block(0, rel)
        r = list(rows).index(centre)
        assert offs[r + 1] - offs[r] == want


def test_config1_sums():
    m = meshgen.config(1)
    assert kuhn_pin(oracle.Oracle.of(m), m, 32)


MUTATIONS = {
    3: "owner = largest cluster id",
    10: "a cluster's edges in lexicographic order instead of discovery order",
    12: "VF takes two of the three triangles through the vertex",
    13: "ET keeps every tetrahedron of the first vertex",
}


def _make(m):
    def make(tets, cl, ncl):
        o = oracle.Oracle(tets, cl, ncl)
        o.set_mutation(m)
        return o
    return make


def _all_pins(m):
    make = _make(m)
    g = meshgen.grid_mesh(3, 5, seed=1)
    return {
        "example": example_pin(make),
        "brute": all(brute_pin(make(s.tets, s.cluster, s.nclusters), s) for s in SMALL[:2]),
        "kuhn": kuhn_pin(make(g.tets, g.cluster, g.nclusters), g, 3),
    }


def test_pins_pass_on_oracle():
    assert all(_all_pins(0).values())


@pytest.mark.parametrize("m", sorted(MUTATIONS))
def test_planted_mistakes(m):
    res = _all_pins(m)
    assert not all(res.values()), "planted mistake %d (%s) passed every pin" % (m, MUTATIONS[m])
