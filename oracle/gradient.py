"""Discrete gradient oracle (DiscreteGradient consumer) -- TEST INFRASTRUCTURE
ONLY: imported by ``tests/`` and never by the library.

The paper's DiscreteGradient workload (Section 5.1) pairs, for every vertex,
the simplices of the vertex's lower star: the vertex with one edge, remaining
edges with triangles, and so on, leaving the unpaired simplices critical.  It
is the lower-star construction of Robins, Wood and Sheppard ("Theory and
algorithms for constructing discrete Morse complexes from grayscale digital
images", IEEE TPAMI 2011, ProcessLowerStars), written here from that
published description on whole-mesh relations, in plain Python (small
meshes only):

* vertex order: u below w iff (f[u], u) < (f[w], w) (ties by id);
* the lower star of v: the simplices containing v whose other vertices are
  all below v;
* a simplex's key: its vertices' (f, id) pairs sorted from the highest down,
  compared lexicographically (a key that is a prefix of another is smaller);
  both priority queues pop the smallest key;
* with an empty lower star v is critical; otherwise v is paired with its
  smallest edge, the other edges go to queue zero, the cofaces of that edge
  with exactly one unclassified facet in the lower star go to queue one, and
  the two queues are drained as the algorithm prescribes (a simplex popped
  from queue one with no unclassified facet moves to queue zero, otherwise it
  is paired with that facet; a simplex popped from queue zero is critical;
  after each classification the cofaces that now have exactly one
  unclassified facet join queue one).

Simplex ids are those of the edge and triangle lists E, F (Section 4.3, as the
oracle numbers them) and the tetrahedron ids of the input.  The result is a
dict with ``pairs`` = set of (dim, lower id, upper id) and ``critical`` = set
of (dim, id).
"""
from __future__ import annotations

import heapq

import numpy as np


def _order(field, v):
    return (float(field[v]), int(v))


def discrete_gradient(tets, field, edges, faces, vertices=None, mutation=0):
    """Pairs and critical simplices of the lower stars of `vertices` (default:
    all).  `edges` (ne x 2) and `faces` (nf x 3) hold ascending vertex ids,
    indexed by edge / triangle id.  mutation != 0 plants a deliberate mistake
    for the pin tests: 1 pairs a vertex with its largest edge, 2 makes every
    queue-one simplex critical instead of pairing it, 3 reverses the vertex
    order (upper stars)."""
    tets = np.asarray(tets)
    field = np.asarray(field, dtype=np.float64)
    if mutation == 3:
        field = -field
    nv = field.shape[0]
    eid = {(int(a), int(b)): i for i, (a, b) in enumerate(np.asarray(edges).tolist())}
    fid = {(int(a), int(b), int(c)): i for i, (a, b, c) in enumerate(np.asarray(faces).tolist())}
    # simplices containing each vertex, by brute force over the tetrahedra
    star_e = [set() for _ in range(nv)]
    star_f = [set() for _ in range(nv)]
    star_t = [set() for _ in range(nv)]
    for t, q in enumerate(tets.tolist()):
        s = sorted(q)
        for i in range(4):
            star_t[s[i]].add(t)
        for i in range(4):
            for j in range(i + 1, 4):
                e = eid[(s[i], s[j])]
                star_e[s[i]].add(e)
                star_e[s[j]].add(e)
                for k in range(j + 1, 4):
                    f = fid[(s[i], s[j], s[k])]
                    for x in (s[i], s[j], s[k]):
                        star_f[x].add(f)

    def verts(dim, i):
        if dim == 1:
            return tuple(int(x) for x in edges[i])
        if dim == 2:
            return tuple(int(x) for x in faces[i])
        return tuple(sorted(int(x) for x in tets[i]))

    def key(dim, i):
        return tuple(sorted((_order(field, x) for x in verts(dim, i)), reverse=True))

    pairs, critical = set(), set()
    for v in (range(nv) if vertices is None else vertices):
        ov = _order(field, v)
        lower = set()
        for dim, st in ((1, star_e[v]), (2, star_f[v]), (3, star_t[v])):
            for i in st:
                if all(_order(field, x) < ov for x in verts(dim, i) if x != v):
                    lower.add((dim, i))
        if not lower:
            critical.add((0, int(v)))
            continue
        vs = {s: set(verts(*s)) for s in lower}
        # facets of a lower-star simplex that lie in the lower star (those containing v)
        facets = {s: [t for t in lower if t[0] == s[0] - 1 and vs[t] <= vs[s]] for s in lower}
        cofaces = {s: [t for t in lower if t[0] == s[0] + 1 and vs[s] <= vs[t]] for s in lower}
        classified = set()

        def unclassified_facets(s):
            return [t for t in facets[s] if t not in classified]

        edges_l = sorted((s for s in lower if s[0] == 1), key=lambda s: key(*s))
        if mutation == 1:
            edges_l = edges_l[::-1]
        delta = edges_l[0]
        pairs.add((0, int(v), int(delta[1])))
        classified.add(delta)
        pq0, pq1 = [], []
        for s in edges_l[1:]:
            heapq.heappush(pq0, (key(*s), s))
        for b in cofaces[delta]:
            if len(unclassified_facets(b)) == 1:
                heapq.heappush(pq1, (key(*b), b))
        while pq1 or pq0:
            while pq1:
                _, a = heapq.heappop(pq1)
                if a in classified:
                    continue
                uf = unclassified_facets(a)
                if not uf or mutation == 2:
                    heapq.heappush(pq0, (key(*a), a))
                    continue
                face = uf[0]
                pairs.add((face[0], int(face[1]), int(a[1])))
                classified.add(face)
                classified.add(a)
                for b in cofaces[a] + cofaces[face]:
                    if b not in classified and len(unclassified_facets(b)) == 1:
                        heapq.heappush(pq1, (key(*b), b))
            while pq0:
                _, g = heapq.heappop(pq0)
                if g in classified:
                    continue
                critical.add((g[0], int(g[1])))
                classified.add(g)
                for b in cofaces[g]:
                    if b not in classified and len(unclassified_facets(b)) == 1:
                        heapq.heappush(pq1, (key(*b), b))
                break
    return {"pairs": pairs, "critical": critical}
