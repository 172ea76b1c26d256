"""Checks that pin relation blocks to things other than the oracle itself.

* brute force straight from the set definitions on tiny meshes (pure Python,
  different computations from the oracle's counting sort and list
  intersections): VT(v) by scanning every tetrahedron, VV(v) from the edges
  (vertex pairs) of every tetrahedron, TT(t) by testing every pair of
  tetrahedra for three shared vertices (Section 2.2: adjacent iff they share a
  (k-1)-simplex);
* the paper's literal "lowest-index vertex" ownership rule on a renumbering in
  which segments are contiguous (Section 4.3);
* closed forms of the n^3 Kuhn lattice (V, T, E and the boundary face count)
  and the Euler characteristic of a ball;
* invariants: symmetry of VV and TT, every vertex and every tetrahedron a row
  exactly once, sorted duplicate-free lists.

Used for the oracle's own pins (``test_oracle_pins.py``) and as property
checks on GPU output at sizes the oracle is too slow for.
"""
from __future__ import annotations

import numpy as np

REL_VT, REL_VV, REL_TT = 1, 2, 4


# ----------------------------------------------------------------------------
# brute force
# ----------------------------------------------------------------------------

def brute_rows_vertices(cluster, k):
    return [v for v in range(len(cluster)) if cluster[v] == k]


def brute_owner_lowest_index(tets, cluster):
    """Owner by the paper's literal rule after renumbering vertices so that
    segments are contiguous (ascending cluster, then ascending id): the segment
    of the tetrahedron's lowest-index vertex."""
    nv = len(cluster)
    order = sorted(range(nv), key=lambda v: (int(cluster[v]), v))
    newid = [0] * nv
    for i, v in enumerate(order):
        newid[v] = i
    old_of_new = order
    out = []
    for q in tets:
        lowest_new = min(newid[int(v)] for v in q)
        out.append(int(cluster[old_of_new[lowest_new]]))
    return out


def brute_block(tets, cluster, k, rel, owner=None):
    """(row_ids, list of entry lists) for cluster k straight from definitions."""
    tets = [tuple(int(x) for x in q) for q in np.asarray(tets).reshape(-1, 4)]
    if rel in (REL_VT, REL_VV):
        rows = brute_rows_vertices(cluster, k)
        out = []
        for v in rows:
            if rel == REL_VT:
                out.append([t for t, q in enumerate(tets) if v in q])
            else:
                nb = set()
                for q in tets:
                    for a in range(4):
                        for b in range(4):
                            if a != b and q[a] == v:
                                nb.add(q[b])
                out.append(sorted(nb))
        return rows, out
    if owner is None:
        owner = brute_owner_lowest_index(tets, cluster)
    rows = [t for t in range(len(tets)) if owner[t] == k]
    out = []
    for t in rows:
        st = set(tets[t])
        # a shared triangle = at least three shared vertices (a duplicate
        # tetrahedron shares all four of its triangles)
        out.append([q for q in range(len(tets)) if q != t and len(st & set(tets[q])) >= 3])
    return rows, out


def csr_to_lists(offsets, entries):
    return [list(map(int, entries[offsets[i]:offsets[i + 1]])) for i in range(len(offsets) - 1)]


# ----------------------------------------------------------------------------
# closed forms
# ----------------------------------------------------------------------------

def kuhn_counts(n: int):
    """Exact counts of the n^3 Kuhn lattice: V, T, E, boundary faces F_b and
    all faces F (from V - E + F - T = 1 for a ball)."""
    V = n ** 3
    T = 6 * (n - 1) ** 3
    # edges: axis edges 3 n^2 (n-1), face diagonals (one per square) 3 n (n-1)^2,
    # cube main diagonals (n-1)^3
    E = 3 * n * n * (n - 1) + 3 * n * (n - 1) ** 2 + (n - 1) ** 3
    Fb = 12 * (n - 1) ** 2  # two triangles per boundary square, 6 (n-1)^2 squares
    F = 1 - V + E + T
    return dict(V=V, T=T, E=E, Fb=Fb, F=F)


# ----------------------------------------------------------------------------
# invariants over all blocks of a mesh
# ----------------------------------------------------------------------------

def gather_all(get_block, ncl):
    """Collect {rel: (row_ids concatenated, lists)} over every cluster."""
    res = {}
    for rel in (REL_VT, REL_VV, REL_TT):
        rows_all, lists_all = [], []
        for k in range(ncl):
            rows, offs, ents = get_block(k, rel)
            rows_all.extend(int(r) for r in rows)
            lists_all.extend(csr_to_lists(offs, ents))
        res[rel] = (rows_all, lists_all)
    return res


def check_invariants(tets, nv, blocks, manifold=True):
    """Raise AssertionError on any violated invariant; return the sums.  On a
    manifold mesh (every triangle in at most two tetrahedra) a TT row has at
    most four entries, one per face."""
    tets = np.asarray(tets).reshape(-1, 4)
    nt = tets.shape[0]
    out = {}
    for rel, nrow in ((REL_VT, nv), (REL_VV, nv), (REL_TT, nt)):
        rows, lists = blocks[rel]
        assert sorted(rows) == list(range(nrow)), "rows of rel %d do not partition the ids" % rel
        for r, l in zip(rows, lists):
            assert all(l[i] < l[i + 1] for i in range(len(l) - 1)), "list not strictly ascending"
            if rel != REL_VT:
                assert r not in l, "self listed"
        out[rel] = sum(len(l) for l in lists)
    vt = dict(zip(*blocks[REL_VT]))
    for v, l in vt.items():
        for t in l:
            assert v in tets[t], "VT lists a tetrahedron without the vertex"
    assert out[REL_VT] == 4 * nt, "sum |VT| != 4 T"
    vv = dict(zip(*blocks[REL_VV]))
    for v, l in vv.items():
        for u in l:
            assert v in vv[u], "VV not symmetric"
    tt = dict(zip(*blocks[REL_TT]))
    for t, l in tt.items():
        if manifold:
            assert len(l) <= 4, "TT row with more than four entries on a manifold mesh"
        for q in l:
            assert t in tt[q], "TT not symmetric"
            assert len(set(tets[t].tolist()) & set(tets[q].tolist())) == 3, "TT pair shares no face"
    return out
