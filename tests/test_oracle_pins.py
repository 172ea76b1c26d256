"""Pins of the CPU oracle to the paper and to the mathematics (no GPU).

Each check is independent of the oracle's own code: printed values of the
paper's worked examples (tests/golden), brute force from the set definitions,
closed forms of the Kuhn lattice, the Euler characteristic of a ball, and
invariants.  ``test_planted_mistakes`` switches on deliberately wrong variants
of the oracle and shows that at least one pin fails for each.
"""
import os

import numpy as np
import pytest

import meshgen
import oracle
from tests import pinlib
from tests.pinlib import REL_TT, REL_VT, REL_VV

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    lines = []
    with open(os.path.join(GOLDEN, name)) as f:
        for ln in f:
            ln = ln.strip()
            if ln and not ln.startswith("#"):
                lines.append(ln)
    return lines


def _blocks(orc, ncl):
    return pinlib.gather_all(orc.block, ncl)


# ----------------------------------------------------------------------------
# paper's worked examples
# ----------------------------------------------------------------------------

def fig1_pin(orc_factory):
    """Fig. 1(b): VV(v0) = [v1, v2, v3] on the two-tetrahedron complex."""
    lines = _read_golden("fig1_toy.txt")
    tets = np.array([[int(x) for x in ln.split()[1:]] for ln in lines if ln.startswith("tet")], dtype=np.int32)
    vv = [ln for ln in lines if ln.startswith("VV")][0]
    v = int(vv.split()[1])
    expect = [int(x) for x in vv.split(":")[1].split()]
    orc = orc_factory(tets, np.zeros(5, np.int32), 1)
    rows, offs, ents = orc.block(0, REL_VV)
    i = list(rows).index(v)
    return list(ents[offs[i]:offs[i + 1]]) == expect


def fig4_pin(orc_factory):
    """Fig. 4: a tetrahedron with v0 (segment S1) and v4 (segment S2) is a TT
    row of S1 only and appears in S2's VT block (it is external to S2)."""
    lines = _read_golden("fig4_owner.txt")
    seg = {}
    for ln in lines:
        if ln.startswith("segment"):
            k = int(ln.split()[1])
            for v in ln.split(":")[1].split():
                seg[int(v)] = k
    tets = np.array([[int(x) for x in ln.split()[1:]] for ln in lines if ln.startswith("tet")], dtype=np.int32)
    cl = np.array([seg[v] for v in range(len(seg))], dtype=np.int32)
    internal = [ln for ln in lines if ln.startswith("internal")][0]
    t = int(internal.split()[1])
    k_int = int(internal.split(":")[1])
    external = [ln for ln in lines if ln.startswith("external")][0]
    k_ext = int(external.split(":")[1])
    orc = orc_factory(tets, cl, 2)
    rows_int, _, _ = orc.block(k_int, REL_TT)
    rows_ext, _, _ = orc.block(k_ext, REL_TT)
    _, _, vt_ext = orc.block(k_ext, REL_VT)
    return (t in list(rows_int)) and (t not in list(rows_ext)) and (t in list(vt_ext))


def test_fig1_vv_v0():
    assert fig1_pin(oracle.Oracle)


def test_fig4_internal_external():
    assert fig4_pin(oracle.Oracle)


# ----------------------------------------------------------------------------
# brute force on tiny meshes
# ----------------------------------------------------------------------------

def brute_pin(orc, mesh):
    owner = pinlib.brute_owner_lowest_index(mesh.tets, mesh.cluster)
    for k in range(mesh.nclusters):
        for rel in (REL_VT, REL_VV, REL_TT):
            rows, offs, ents = orc.block(k, rel)
            brows, blists = pinlib.brute_block(mesh.tets, mesh.cluster, k, rel, owner)
            if list(rows) != brows:
                return False
            if offs[0] != 0 or pinlib.csr_to_lists(offs, ents) != blists:
                return False
    return True


SMALL = [meshgen.random_small(s, n=3 + (s % 2), nclusters=2 + s % 4) for s in range(6)]


@pytest.mark.parametrize("idx", range(len(SMALL)))
def test_brute_force_random_small(idx):
    m = SMALL[idx]
    orc = oracle.Oracle.of(m)
    assert brute_pin(orc, m)


def test_brute_force_cube_and_specials():
    for m in (meshgen.cube(), meshgen.cube([0, 0, 0, 0, 1, 1, 1, 1]), meshgen.fig1_toy(),
              meshgen.single_tet(), meshgen.fig4_example()):
        assert brute_pin(oracle.Oracle.of(m), m)


def test_cube_split_by_z_owns_no_tt_rows():
    m = meshgen.cube([0, 0, 0, 0, 1, 1, 1, 1])
    orc = oracle.Oracle.of(m)
    rows, offs, ents = orc.block(1, REL_TT)
    assert len(rows) == 0 and list(offs) == [0] and len(ents) == 0
    rows, _, _ = orc.block(0, REL_TT)
    assert list(rows) == list(range(6))


def test_cube_counts_and_cycle():
    """Cube: E = 19, F = 18 with 12 on the boundary, chi = 1, TT a 6-cycle."""
    m = meshgen.cube()
    orc = oracle.Oracle.of(m)
    b = _blocks(orc, 1)
    sums = pinlib.check_invariants(m.tets, m.nv, b)
    E = sums[REL_VV] // 2
    Fb = 4 * m.nt - sums[REL_TT]
    F = (4 * m.nt + Fb) // 2
    assert (E, F, Fb) == (19, 18, 12)
    assert m.nv - E + F - m.nt == 1
    tt = dict(zip(*b[REL_TT]))
    assert all(len(l) == 2 for l in tt.values())
    # walking the adjacency visits all six tetrahedra before returning
    seen, prev, cur = [0], None, 0
    while True:
        nxt = [q for q in tt[cur] if q != prev][0]
        if nxt == 0:
            break
        seen.append(nxt)
        prev, cur = cur, nxt
    assert sorted(seen) == list(range(6))


def test_isolated_vertices_and_empty_clusters():
    m = meshgen.random_small(11, n=3, nclusters=3, isolated=3, empty_clusters=2)
    orc = oracle.Oracle.of(m)
    counts = np.bincount(m.cluster, minlength=m.nclusters)
    for k in range(m.nclusters):
        rows, offs, ents = orc.block(k, REL_VT)
        assert len(rows) == counts[k]
        if counts[k] == 0:
            assert list(offs) == [0] and len(ents) == 0
    assert brute_pin(orc, m)


# ----------------------------------------------------------------------------
# ownership rule (reading of Section 4.3)
# ----------------------------------------------------------------------------

def owner_pin(orc, mesh):
    lit = pinlib.brute_owner_lowest_index(mesh.tets, mesh.cluster)
    return all(orc.owner(t) == lit[t] for t in range(mesh.nt))


def test_owner_equals_lowest_index_rule():
    for m in SMALL + [meshgen.grid_mesh(6, 20, seed=3)]:
        assert owner_pin(oracle.Oracle.of(m), m)


# ----------------------------------------------------------------------------
# closed forms on Kuhn lattices
# ----------------------------------------------------------------------------

def closed_form_pin(orc, mesh, n):
    cf = pinlib.kuhn_counts(n)
    if mesh.nv != cf["V"] or mesh.nt != cf["T"]:
        return False
    try:
        sums = pinlib.check_invariants(mesh.tets, mesh.nv, _blocks(orc, mesh.nclusters))
    except AssertionError:
        return False
    E = sums[REL_VV] // 2
    Fb = 4 * mesh.nt - sums[REL_TT]
    F = (4 * mesh.nt + Fb) // 2
    return (sums[REL_VV] % 2 == 0 and E == cf["E"] and Fb == cf["Fb"] and F == cf["F"]
            and mesh.nv - E + F - mesh.nt == 1)


@pytest.mark.parametrize("n,cap", [(2, 8), (3, 5), (4, 7), (5, 16), (6, 40)])
def test_kuhn_closed_forms(n, cap):
    m = meshgen.grid_mesh(n, cap, seed=n)
    assert closed_form_pin(oracle.Oracle.of(m), m, n)


def test_kuhn_interior_valences():
    """An interior lattice vertex lies in 24 tetrahedra and has 14 neighbours."""
    n = 5
    m = meshgen.grid_mesh(n, 125, seed=1, permute=False)
    orc = oracle.Oracle.of(m)
    rows, offs, ents = orc.block(0, REL_VT)
    rows2, offs2, ents2 = orc.block(0, REL_VV)
    for r, v in enumerate(rows):
        i, j, k = v % n, (v // n) % n, v // (n * n)
        if 0 < i < n - 1 and 0 < j < n - 1 and 0 < k < n - 1:
            assert offs[r + 1] - offs[r] == 24
            assert offs2[r + 1] - offs2[r] == 14


def test_config1_totals():
    """32^3 lattice: sum|VT| = 714,984, sum|VV| = 2E = 434,558,
    sum|TT| = 4T - F_b = 703,452 (E = 217,279, F_b = 11,532)."""
    m = meshgen.config(1)
    cf = pinlib.kuhn_counts(32)
    assert (cf["E"], cf["Fb"]) == (217279, 11532)
    orc = oracle.Oracle.of(m)
    tot = {REL_VT: 0, REL_VV: 0, REL_TT: 0}
    rows_t = 0
    for k in range(m.nclusters):
        for rel in tot:
            rows, offs, ents = orc.block(k, rel)
            tot[rel] += len(ents)
            if rel == REL_TT:
                rows_t += len(rows)
    assert rows_t == m.nt
    assert tot == {REL_VT: 714984, REL_VV: 434558, REL_TT: 703452}


# ----------------------------------------------------------------------------
# metamorphic: relabelling
# ----------------------------------------------------------------------------

def relabel_pin(orc_factory, mesh, seed=7):
    rng = np.random.default_rng(seed)
    vp = rng.permutation(mesh.nv).astype(np.int32)
    tp = rng.permutation(mesh.nt)
    tets2 = np.empty_like(mesh.tets)
    tets2[tp] = vp[mesh.tets]
    cl2 = np.empty_like(mesh.cluster)
    cl2[vp] = mesh.cluster
    a = orc_factory(mesh.tets, mesh.cluster, mesh.nclusters)
    b = orc_factory(tets2, cl2, mesh.nclusters)
    for k in range(mesh.nclusters):
        for rel, mp in ((REL_VT, (vp, tp)), (REL_VV, (vp, vp)), (REL_TT, (tp, tp))):
            r1, o1, e1 = a.block(k, rel)
            r2, o2, e2 = b.block(k, rel)
            m1 = {int(mp[0][r]): sorted(int(mp[1][x]) for x in l)
                  for r, l in zip(r1, pinlib.csr_to_lists(o1, e1))}
            m2 = {int(r): l for r, l in zip(r2, pinlib.csr_to_lists(o2, e2))}
            if m1 != m2 or list(r2) != sorted(r2):
                return False
    return True


def test_relabel_invariance():
    for m in SMALL[:3] + [meshgen.grid_mesh(5, 30, seed=2)]:
        assert relabel_pin(oracle.Oracle, m)


# ----------------------------------------------------------------------------
# validation (O0)
# ----------------------------------------------------------------------------

def test_validation_rejects_bad_input():
    good = np.array([[0, 1, 2, 3]], np.int32)
    cl = np.zeros(4, np.int32)
    assert oracle.validate(good, cl, 1)
    assert not oracle.validate(np.array([[0, 1, 1, 3]], np.int32), cl, 1)
    assert not oracle.validate(np.array([[0, 1, 2, 4]], np.int32), cl, 1)
    assert not oracle.validate(np.array([[0, 1, 2, -1]], np.int32), cl, 1)
    assert not oracle.validate(good, np.array([0, 0, 0, 1], np.int32), 1)
    assert not oracle.validate(good, cl, 0)
    with pytest.raises(ValueError):
        oracle.Oracle(np.array([[0, 1, 1, 3]], np.int32), cl, 1)


# ----------------------------------------------------------------------------
# planted mistakes: each wrong variant fails at least one pin
# ----------------------------------------------------------------------------

MUTATIONS = {
    1: "VV keeps the vertex itself",
    2: "TT keeps the tetrahedron itself",
    3: "owner = largest cluster id",
    4: "VT lists in descending order",
    5: "TT through a shared edge instead of a face",
    6: "VV from one tetrahedron only",
    7: "rows in descending id order",
    8: "VT drops the last tetrahedron of each list",
    9: "TT ignores one face",
}


def _mutated_factory(m):
    def make(tets, cl, ncl):
        o = oracle.Oracle(tets, cl, ncl)
        o.set_mutation(m)
        return o
    return make


def _all_pins(m):
    make = _mutated_factory(m)
    results = {
        "fig1": fig1_pin(make),
        "fig4": fig4_pin(make),
        "brute": all(brute_pin(make(s.tets, s.cluster, s.nclusters), s) for s in SMALL[:3]),
        "closed": all(closed_form_pin(make(g.tets, g.cluster, g.nclusters), g, n)
                      for n, g in ((3, meshgen.grid_mesh(3, 5, seed=1)), (4, meshgen.grid_mesh(4, 9, seed=2)))),
        "owner": all(owner_pin(make(s.tets, s.cluster, s.nclusters), s) for s in SMALL[:3]),
        "relabel": relabel_pin(make, SMALL[0]),
    }
    return results


def test_pins_pass_on_oracle():
    assert all(_all_pins(0).values())


@pytest.mark.parametrize("m", sorted(MUTATIONS))
def test_planted_mistakes(m):
    res = _all_pins(m)
    assert not all(res.values()), "planted mistake %d (%s) passed every pin" % (m, MUTATIONS[m])


def test_fan_closed_forms():
    """Closed fans: the centre of a ring of k lies in 2k tetrahedra and has
    k + 2 neighbours, top and bottom lie in k and have k + 1, a ring vertex lies
    in 4 and has 5; every tetrahedron has exactly 3 face neighbours (its
    fourth face, opposite the centre, is on the boundary)."""
    ks = (3, 16, 33, 70)
    m = meshgen.fans(ks, nclusters=4, seed=5)
    orc = oracle.Oracle.of(m)
    blocks = pinlib.gather_all(orc.block, m.nclusters)
    vt = dict(zip(*blocks[REL_VT]))
    vv = dict(zip(*blocks[REL_VV]))
    tt = dict(zip(*blocks[REL_TT]))
    assert sorted(tt) == list(range(m.nt)) and all(len(l) == 3 for l in tt.values())
    # the valence multiset over all vertices, fan by fan
    exp_vt, exp_vv = [], []
    for k in ks:
        exp_vt += [2 * k, k, k] + [4] * k
        exp_vv += [k + 2, k + 1, k + 1] + [5] * k
    assert sorted(len(l) for l in vt.values()) == sorted(exp_vt)
    assert sorted(len(l) for l in vv.values()) == sorted(exp_vv)
    # each VT list is the set of tetrahedra containing the vertex, ascending
    for v, l in vt.items():
        assert l == sorted(np.nonzero((m.tets == v).any(1))[0].tolist())


@pytest.mark.parametrize("seed", [0, 1])
def test_brute_force_nonmanifold(seed):
    """Fins and duplicated tetrahedra (faces of three or four tetrahedra):
    TT lists every tetrahedron sharing a face, a duplicate once."""
    m = meshgen.nonmanifold(n=4, fins=5, dups=3, nclusters=3, seed=seed)
    orc = oracle.Oracle.of(m)
    assert brute_pin(orc, m)
    blocks = pinlib.gather_all(orc.block, m.nclusters)
    assert max(len(l) for l in blocks[REL_TT][1]) >= 4
