"""Pins of the discrete gradient oracle (oracle/gradient.py) against what the
mathematics fixes, independent of the oracle's own steps:

* a discrete gradient: every vertex, edge, triangle and tetrahedron of the
  mesh is either critical or in exactly one pair; a pair joins a simplex with
  a coface one dimension up; both lie in the lower star of the same vertex;
* the Morse relation: c0 - c1 + c2 - c3 equals the Euler characteristic
  V - E + F - T of the mesh (brute-force counts);
* no closed V-path (gradient paths are acyclic), by depth-first search on the
  directed Hasse diagram with the paired arrows reversed;
* a linear field on a convex lattice (every lower link a disc or a cone) has
  one critical simplex, the global minimum vertex;
* a vertex that is not critical is paired with the edge to its lowest
  neighbour (the smallest edge of its lower star);
* planted mistakes (largest edge, critical instead of paired, upper stars)
  each fail at least one of these.
"""
import numpy as np
import pytest

import meshgen
import oracle
from oracle.gradient import discrete_gradient


def _setup(mesh, field):
    o = oracle.Oracle.of(mesh)
    e, _, f, _ = o.simplices()
    return e, f


def _simplices(mesh, e, f):
    return {0: set(range(mesh.nv)), 1: set(range(len(e))), 2: set(range(len(f))), 3: set(range(mesh.nt))}


def _verts(mesh, e, f, dim, i):
    if dim == 0:
        return {i}
    if dim == 1:
        return set(int(x) for x in e[i])
    if dim == 2:
        return set(int(x) for x in f[i])
    return set(int(x) for x in mesh.tets[i])


def valid_pin(mesh, field, e, f, g):
    seen = {d: {} for d in range(4)}
    for d, i in g["critical"]:
        seen[d][i] = seen[d].get(i, 0) + 1
    order = lambda v: (float(field[v]), v)
    for d, lo, up in g["pairs"]:
        seen[d][lo] = seen[d].get(lo, 0) + 1
        seen[d + 1][up] = seen[d + 1].get(up, 0) + 1
        a, b = _verts(mesh, e, f, d, lo), _verts(mesh, e, f, d + 1, up)
        if not (a < b and len(b) == len(a) + 1):
            return False
        if max(a, key=order) != max(b, key=order):  # one lower star
            return False
    allsx = _simplices(mesh, e, f)
    return all(set(seen[d]) == allsx[d] and all(c == 1 for c in seen[d].values()) for d in range(4))


def euler_pin(mesh, e, f, g):
    c = [0, 0, 0, 0]
    for d, _ in g["critical"]:
        c[d] += 1
    return c[0] - c[1] + c[2] - c[3] == mesh.nv - len(e) + len(f) - mesh.nt


def acyclic_pin(mesh, e, f, g):
    """For each dimension d, the V-paths: from a d-simplex paired with a
    coface c to every other d-facet of c that is itself paired upwards.  A
    discrete gradient has no closed V-path (depth-first search for a cycle)."""
    up_of = {(d, lo): up for d, lo, up in g["pairs"]}
    for d in (0, 1, 2):
        n = {0: mesh.nv, 1: len(e), 2: len(f)}[d]
        index = {frozenset(_verts(mesh, e, f, d, i)): i for i in range(n)}
        succ = {}
        for (dd, lo), up in up_of.items():
            if dd != d:
                continue
            cv = _verts(mesh, e, f, d + 1, up)
            succ[lo] = [index[frozenset(cv - {x})] for x in cv]
        color = {}
        for start in succ:
            if color.get(start):
                continue
            color[start] = 1
            stack = [(start, iter(succ[start]))]
            while stack:
                node, it = stack[-1]
                b = next(it, None)
                if b is None:
                    color[node] = 2
                    stack.pop()
                    continue
                if b == node or b not in succ:
                    continue
                if color.get(b) == 1:
                    return False
                if not color.get(b):
                    color[b] = 1
                    stack.append((b, iter(succ[b])))
    return True


def steepest_pin(mesh, field, e, f, g):
    order = lambda v: (float(field[v]), v)
    nb = {v: set() for v in range(mesh.nv)}
    for a, b in e.tolist():
        nb[a].add(b)
        nb[b].add(a)
    for d, lo, up in g["pairs"]:
        if d == 0:
            lowest = min(nb[lo], key=order)
            if order(lowest) > order(lo) or set(int(x) for x in e[up]) != {lo, lowest}:
                return False
    for d, i in g["critical"]:
        if d == 0 and nb[i] and order(min(nb[i], key=order)) < order(i):
            return False
    return True


def linear_pin(mesh, field, g):
    vmin = min(range(mesh.nv), key=lambda v: (float(field[v]), v))
    return g["critical"] == {(0, vmin)}


def _lattice(n, seed):
    m = meshgen.grid_mesh(n, max(8, n ** 3 // 6), seed=seed)
    return m


def _linear_field(m, seed):
    d = np.random.default_rng(seed).normal(size=3)
    return (m.coords.astype(np.float64) @ d).astype(np.float32)


def _noise_field(m, seed):
    return np.random.default_rng(seed).random(m.nv).astype(np.float32)


CASES = [
    ("lattice5-linear", lambda: _lattice(5, 1), _linear_field),
    ("lattice5-noise", lambda: _lattice(5, 2), _noise_field),
    ("random-noise", lambda: meshgen.random_small(3, n=5, nclusters=4, drop=0.3), _noise_field),
    ("cube-noise", lambda: meshgen.cube(), _noise_field),
]


def _all_pins(mutation):
    res = {}
    for name, mk, fld in CASES:
        m = mk()
        if m.coords is None:
            m.coords = np.random.default_rng(0).random((m.nv, 3)).astype(np.float32)
        field = fld(m, 5)
        e, f = _setup(m, field)
        g = discrete_gradient(m.tets, field, e, f, mutation=mutation)
        res[name + ":valid"] = valid_pin(m, field, e, f, g)
        res[name + ":euler"] = euler_pin(m, e, f, g)
        res[name + ":acyclic"] = acyclic_pin(m, e, f, g)
        res[name + ":steepest"] = steepest_pin(m, field, e, f, g)
        if name.endswith("linear"):
            res[name + ":linear"] = linear_pin(m, field, g)
    return res


def test_pins_pass_on_oracle():
    res = _all_pins(0)
    assert all(res.values()), [k for k, v in res.items() if not v]


@pytest.mark.parametrize("m", [1, 2, 3])
def test_planted_mistakes(m):
    res = _all_pins(m)
    assert not all(res.values()), "planted mistake %d passed every pin" % m


def test_saddle_field_counts():
    """x^2 + y^2 - z^2 on a lattice centred at the origin: Morse relation
    holds and the field has more than the one critical simplex a linear
    field has."""
    m = meshgen.grid_mesh(7, 60, seed=0, permute=False)
    c = m.coords.astype(np.float64) - 3.0
    field = (c[:, 0] ** 2 + c[:, 1] ** 2 - c[:, 2] ** 2 + 1e-3 * np.arange(m.nv) / m.nv).astype(np.float32)
    e, f = _setup(m, field)
    g = discrete_gradient(m.tets, field, e, f)
    assert valid_pin(m, field, e, f, g) and euler_pin(m, e, f, g) and acyclic_pin(m, e, f, g)
    assert len(g["critical"]) > 1
