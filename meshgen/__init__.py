"""Seeded synthetic tetrahedral meshes and vertex clusterings.

This module is the only code shared by the CPU oracle side and the GPU side of
the test-suite and benchmark.  It produces inputs only: vertex coordinates, the
tetrahedron list T (the TV relation, four vertex ids per tetrahedron) and the
vertex -> cluster map S of the paper's input format (Section 4.3, "Input
data").  It contains none of the relation arithmetic (no VT, VV or TT).

Workloads (the paper's datasets, Table 2, are not available; these stand in
for them and bracket their sizes):

* ``grid``: an n x n x n vertex lattice whose cubes are each split into six
  tetrahedra along the main diagonal (Kuhn/Freudenthal split, all cubes with
  the same orientation so the mesh is conforming), coordinates jittered by
  U[-0.2, 0.2] per axis, vertex and tetrahedron ids randomly permuted.
* ``refined``: the same lattice with rounds of 1-to-4 centroid splits applied
  to a seed-chosen fraction of tetrahedra, concentrated inside 8 Gaussian
  blobs, giving vertex valences far above the lattice's.
* clusters are Morton-order runs of vertices, either of a fixed capacity or of
  lognormally distributed capacities (the paper uses PR-octree leaves with a
  vertex capacity, Section 4.3 and Section 5.1; Morton runs are the same kind
  of spatially compact vertex partition).

Every random draw comes from ``numpy.random.default_rng(seed)`` in a fixed
order documented on each function, so a (config, seed) pair names one mesh.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import os

import numpy as np

__all__ = [
    "Mesh", "kuhn_grid", "morton_keys", "clusters_fixed", "clusters_lognormal",
    "refine", "grid_mesh", "refined_mesh", "config", "CONFIGS",
    "cube", "fig1_toy", "fig4_example", "single_tet", "random_small", "fans", "nonmanifold", "loose_tets", "gauss_field",
]


@dataclass
class Mesh:
    """A tetrahedral mesh with a vertex clustering.

    ``tets``    int32 [nt, 4]  vertex ids of each tetrahedron (TV relation)
    ``cluster`` int32 [nv]     cluster id of each vertex, 0-based
    ``coords``  float32 [nv, 3] or None
    ``scalar``  float32 [nv] or None  (per-vertex field for the consumer)
    """
    tets: np.ndarray
    cluster: np.ndarray
    nclusters: int
    coords: np.ndarray | None = None
    scalar: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def nv(self) -> int:
        return int(self.cluster.shape[0])

    @property
    def nt(self) -> int:
        return int(self.tets.shape[0])


# ----------------------------------------------------------------------------
# Lattice and its Kuhn split
# ----------------------------------------------------------------------------

_AXIS_ORDERS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def kuhn_grid(n: int):
    """Vertices and tetrahedra of the n^3 lattice, before jitter/permutation.

    Vertex (i, j, k) has id i + n*(j + n*k).  Cube with corner p0 becomes the
    six tetrahedra {p0, p0+e_a, p0+e_a+e_b, p0+(1,1,1)} for the six axis
    orders (a, b, c); tetrahedron id = 6*cube + order index, cubes in
    x-fastest order.  Returns (coords float64 [n^3,3], tets int32 [6(n-1)^3,4]).
    """
    if n < 2:
        raise ValueError("n must be >= 2")
    ax = np.arange(n, dtype=np.float64)
    k, j, i = np.meshgrid(ax, ax, ax, indexing="ij")
    coords = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)
    m = n - 1
    if n ** 3 >= 2 ** 31:
        raise ValueError("n^3 must stay below 2^31 (int32 vertex ids)")
    c = np.arange(m, dtype=np.int64)
    p0 = (c[None, None, :] + n * (c[None, :, None] + n * c[:, None, None])).ravel().astype(np.int32)
    step = (1, n, n * n)
    off = np.empty((6, 4), dtype=np.int32)
    for o, (a, b, _c) in enumerate(_AXIS_ORDERS):
        off[o] = (0, step[a], step[a] + step[b], 1 + n + n * n)
    tets = (p0[:, None, None] + off[None, :, :]).reshape(-1, 4)
    return coords, tets


# ----------------------------------------------------------------------------
# Morton clustering
# ----------------------------------------------------------------------------

def _spread21(x: np.ndarray) -> np.ndarray:
    x = x.astype(np.uint64) & np.uint64(0x1FFFFF)
    x = (x | (x << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
    x = (x | (x << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
    x = (x | (x << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
    x = (x | (x << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
    x = (x | (x << np.uint64(2))) & np.uint64(0x1249249249249249)
    return x


def morton_keys(coords: np.ndarray) -> np.ndarray:
    """63-bit Morton keys: each axis quantised to 21 bits over the bounding box
    (float64 arithmetic, clamped to 2^21-1), x in bit 3i, y in 3i+1, z in 3i+2."""
    c = np.asarray(coords, dtype=np.float64)
    lo = c.min(axis=0)
    hi = c.max(axis=0)
    span = np.where(hi > lo, hi - lo, 1.0)
    q = np.floor((c - lo) / span * float(1 << 21))
    q = np.clip(q, 0, (1 << 21) - 1).astype(np.uint64)
    return _spread21(q[:, 0]) | (_spread21(q[:, 1]) << np.uint64(1)) | (_spread21(q[:, 2]) << np.uint64(2))


def _morton_order(coords: np.ndarray) -> np.ndarray:
    keys = morton_keys(coords)
    ids = np.arange(keys.shape[0], dtype=np.int64)
    return np.lexsort((ids, keys))  # by key, ties by id


def clusters_fixed(coords: np.ndarray, cap: int):
    """Cut the Morton order into consecutive runs of ``cap`` vertices.
    Cluster ids follow Morton order.  Returns (cluster int32 [nv], nclusters)."""
    order = _morton_order(coords)
    nv = order.shape[0]
    cl = np.empty(nv, dtype=np.int32)
    cl[order] = (np.arange(nv) // cap).astype(np.int32)
    return cl, int((nv + cap - 1) // cap)


def clusters_lognormal(coords: np.ndarray, median: float, sigma: float, lo: int, hi: int,
                       rng: np.random.Generator):
    """Cut the Morton order into runs of lognormal capacity
    c_i = clamp(rint(exp(ln(median) + sigma*z_i)), lo, hi), z_i ~ N(0,1) drawn
    in blocks of 65536 from ``rng`` until the capacities cover every vertex."""
    order = _morton_order(coords)
    nv = order.shape[0]
    caps = []
    total = 0
    while total < nv:
        z = rng.standard_normal(65536)
        c = np.clip(np.rint(np.exp(math.log(median) + sigma * z)), lo, hi).astype(np.int64)
        caps.append(c)
        total += int(c.sum())
    caps = np.concatenate(caps)
    ends = np.cumsum(caps)
    ncl = int(np.searchsorted(ends, nv, side="left")) + 1
    rank = np.arange(nv, dtype=np.int64)
    cid = np.searchsorted(ends[:ncl], rank, side="right").astype(np.int32)
    cl = np.empty(nv, dtype=np.int32)
    cl[order] = cid
    return cl, ncl


# ----------------------------------------------------------------------------
# Refinement by centroid insertion
# ----------------------------------------------------------------------------

def _blob_weights(coords: np.ndarray, tets: np.ndarray, mu: np.ndarray, s: np.ndarray,
                  chunk: int = 1 << 20) -> np.ndarray:
    """w[t] = sum_b exp(-|x_t - mu_b|^2 / (2 s_b^2)) at the centroid x_t of each
    tetrahedron, in chunks over threads (numpy releases the GIL); the same
    operations in the same order as a whole-array evaluation, so the same bits."""
    from concurrent.futures import ThreadPoolExecutor
    nt = tets.shape[0]
    w = np.zeros(nt, dtype=np.float64)

    def work(lo):
        hi = min(nt, lo + chunk)
        t = tets[lo:hi]
        cen = np.zeros((hi - lo, 3), dtype=np.float64)
        for q in range(4):
            cen += coords[t[:, q]]
        cen *= 0.25
        acc = np.zeros(hi - lo, dtype=np.float64)
        for b in range(mu.shape[0]):
            d = cen - mu[b]
            d *= d
            d2 = d[:, 0] + d[:, 1]
            d2 += d[:, 2]
            acc += np.exp(-d2 / (2.0 * s[b] * s[b]))
        w[lo:hi] = acc

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(work, range(0, nt, chunk)))
    return w


def refine(coords: np.ndarray, tets: np.ndarray, n: int, frac: float, rounds: int,
           rng: np.random.Generator, nblobs: int = 8):
    """Rounds of 1-to-4 centroid splits concentrated in Gaussian blobs.

    Draw order: blob centres mu_b ~ U(box) (nblobs x 3), widths
    s_b ~ U(0.04, 0.10)*(n-1) (nblobs); then per round one U(0,1) per current
    tetrahedron.  Each round selects round(frac * T_current) tetrahedra without
    replacement, weighted by w = sum_b exp(-|x - mu_b|^2 / (2 s_b^2)) at the
    centroid x (Efraimidis-Spirakis keys log(u)/w, largest keys win).  A chosen
    (a, b, c, d) with centroid vertex m becomes (m,b,c,d) in place plus
    (a,m,c,d), (a,b,m,d), (a,b,c,m) appended in that order.
    """
    coords = np.asarray(coords, dtype=np.float64)
    tets = np.asarray(tets, dtype=np.int32)
    box = float(n - 1)
    mu = rng.uniform(0.0, box, size=(nblobs, 3))
    s = rng.uniform(0.04, 0.10, size=nblobs) * box
    for _ in range(rounds):
        nt = tets.shape[0]
        u = rng.uniform(0.0, 1.0, size=nt)
        k = int(round(frac * nt))
        w = _blob_weights(coords, tets, mu, s)
        with np.errstate(divide="ignore"):
            key = np.log(np.maximum(u, 1e-300)) / np.maximum(w, 1e-300)
        sel = np.argpartition(-key, k - 1)[:k] if k > 0 else np.empty(0, dtype=np.int64)
        sel = np.sort(sel)
        nv = coords.shape[0]
        m = np.arange(nv, nv + k, dtype=np.int64).astype(np.int32)
        old = tets[sel].copy()
        newc = coords[old].mean(axis=1)
        coords = np.concatenate([coords, newc], axis=0)
        a, b, c, d = old[:, 0], old[:, 1], old[:, 2], old[:, 3]
        tets[sel] = np.stack([m, b, c, d], axis=1)
        extra = np.empty((k, 3, 4), dtype=np.int32)
        extra[:, 0] = np.stack([a, m, c, d], axis=1)
        extra[:, 1] = np.stack([a, b, m, d], axis=1)
        extra[:, 2] = np.stack([a, b, c, m], axis=1)
        tets = np.concatenate([tets, extra.reshape(-1, 4)], axis=0)
    return coords, tets


# ----------------------------------------------------------------------------
# Permutation of ids
# ----------------------------------------------------------------------------

def _permute(rng: np.random.Generator, tets, cluster, coords, scalar):
    """Relabel vertices by vperm (old v -> vperm[v]) then tetrahedra by tperm
    (old t -> tperm[t]); vperm is drawn before tperm."""
    nv = cluster.shape[0]
    nt = tets.shape[0]
    vperm = rng.permutation(nv).astype(np.int32)
    tperm = rng.permutation(nt)
    new_tets = np.empty_like(tets)
    # new_tets[tperm] = vperm[tets], in chunks over threads
    from concurrent.futures import ThreadPoolExecutor
    chunk = 1 << 21

    def work(lo):
        hi = min(nt, lo + chunk)
        new_tets[tperm[lo:hi]] = vperm[tets[lo:hi]]

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(work, range(0, nt, chunk)))
    new_cl = np.empty_like(cluster)
    new_cl[vperm] = cluster
    new_coords = None
    if coords is not None:
        new_coords = np.empty_like(coords)
        new_coords[vperm] = coords
    new_scalar = None
    if scalar is not None:
        new_scalar = np.empty_like(scalar)
        new_scalar[vperm] = scalar
    return new_tets, new_cl, new_coords, new_scalar


def gauss_field(coords: np.ndarray, n: int, rng: np.random.Generator, ng: int = 16) -> np.ndarray:
    """f = sum_g a_g exp(-|x-mu_g|^2/(2 s_g^2)) + 1e-3 U[0,1); draw order a (16),
    s (16), mu (16x3), then the noise (one per vertex).  float32."""
    box = float(n - 1)
    a = rng.uniform(-1.0, 1.0, size=ng)
    s = rng.uniform(0.05, 0.2, size=ng) * box
    mu = rng.uniform(0.0, box, size=(ng, 3))
    f = np.zeros(coords.shape[0], dtype=np.float64)
    for g in range(ng):
        d2 = ((coords - mu[g]) ** 2).sum(axis=1)
        f += a[g] * np.exp(-d2 / (2.0 * s[g] * s[g]))
    f += 1e-3 * rng.uniform(0.0, 1.0, size=coords.shape[0])
    return f.astype(np.float32)


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

def grid_mesh(n: int, cap: int, seed: int = 0, permute: bool = True) -> Mesh:
    """Jittered, permuted Kuhn lattice with fixed-capacity Morton clusters.
    Draw order: jitter (nv x 3 uniforms), vperm, tperm."""
    rng = np.random.default_rng(seed)
    coords, tets = kuhn_grid(n)
    coords = coords + rng.uniform(-0.2, 0.2, size=coords.shape)
    cluster, ncl = clusters_fixed(coords, cap)
    coords32 = coords.astype(np.float32)
    scalar = None
    if permute:
        tets, cluster, coords32, scalar = _permute(rng, tets, cluster, coords32, scalar)
    return Mesh(tets=np.ascontiguousarray(tets, dtype=np.int32), cluster=cluster.astype(np.int32),
                nclusters=ncl, coords=coords32, scalar=scalar,
                meta={"kind": "grid", "n": n, "cap": cap, "seed": seed})


def refined_mesh(n: int, frac: float, rounds: int, median: float, sigma: float, seed: int = 0,
                 lo: int = 64, hi: int = 8192, with_scalar: bool = False) -> Mesh:
    """Jittered Kuhn lattice, refined in blobs, lognormal Morton clusters,
    optional scalar field, permuted.  Draw order: jitter, blobs and refinement
    rounds, cluster capacities, scalar field (if any), vperm, tperm."""
    rng = np.random.default_rng(seed)
    coords, tets = kuhn_grid(n)
    coords = coords + rng.uniform(-0.2, 0.2, size=coords.shape)
    coords, tets = refine(coords, tets, n, frac, rounds, rng)
    cluster, ncl = clusters_lognormal(coords, median, sigma, lo, hi, rng)
    scalar = gauss_field(coords, n, rng) if with_scalar else None
    coords32 = coords.astype(np.float32)
    tets, cluster, coords32, scalar = _permute(rng, tets, cluster, coords32, scalar)
    return Mesh(tets=np.ascontiguousarray(tets, dtype=np.int32), cluster=cluster.astype(np.int32),
                nclusters=ncl, coords=coords32, scalar=scalar,
                meta={"kind": "refined", "n": n, "frac": frac, "rounds": rounds,
                      "median": median, "sigma": sigma, "seed": seed})


CONFIGS = {
    1: dict(kind="grid", n=32, cap=512),
    2: dict(kind="grid", n=128, cap=1024),
    3: dict(kind="refined", n=256, frac=0.05, rounds=3, median=512, sigma=1.0),
    4: dict(kind="refined", n=256, frac=0.05, rounds=3, median=512, sigma=1.0, scalar=True),
    5: dict(kind="refined", n=384, frac=0.03, rounds=2, median=1024, sigma=1.2),
}


def config(cfg: int, seed: int = 0) -> Mesh:
    """The five named workloads: 1 = 32^3 lattice, clusters of 512; 2 = 128^3,
    clusters of 1024; 3 = 256^3 refined (5%, 3 rounds), lognormal clusters
    (median 512, sigma 1.0, clamp 64..8192); 4 = config 3 plus a scalar field;
    5 = 384^3 refined (3%, 2 rounds), lognormal (median 1024, sigma 1.2)."""
    c = CONFIGS[cfg]
    if c["kind"] == "grid":
        m = grid_mesh(c["n"], c["cap"], seed)
    else:
        m = refined_mesh(c["n"], c["frac"], c["rounds"], c["median"], c["sigma"], seed,
                         with_scalar=bool(c.get("scalar", False)))
    m.meta["config"] = cfg
    return m


# ----------------------------------------------------------------------------
# Hand-built small cases
# ----------------------------------------------------------------------------

def cube(cluster=None) -> Mesh:
    """One unit cube, vertex id x + 2y + 4z, split into the six Kuhn
    tetrahedra around the diagonal 0-7."""
    tets = np.array([[0, 1, 3, 7], [0, 1, 5, 7], [0, 2, 3, 7],
                     [0, 2, 6, 7], [0, 4, 5, 7], [0, 4, 6, 7]], dtype=np.int32)
    cl = np.zeros(8, dtype=np.int32) if cluster is None else np.asarray(cluster, dtype=np.int32)
    coords = np.array([[x, y, z] for z in (0, 1) for y in (0, 1) for x in (0, 1)], dtype=np.float32)
    return Mesh(tets=tets, cluster=cl, nclusters=int(cl.max()) + 1, coords=coords,
                meta={"kind": "cube"})


def fig1_toy() -> Mesh:
    """Two tetrahedra sharing one triangle (the complex of Fig. 1)."""
    tets = np.array([[0, 1, 2, 3], [1, 2, 3, 4]], dtype=np.int32)
    return Mesh(tets=tets, cluster=np.zeros(5, dtype=np.int32), nclusters=1, meta={"kind": "fig1"})


def fig4_example() -> Mesh:
    """Six vertices in two segments {0,1,2} and {3,4,5} (0-based ids of the
    segments S1, S2 of Fig. 4) and three tetrahedra; tetrahedron 1 contains
    v0 and v4."""
    tets = np.array([[0, 1, 2, 3], [0, 2, 3, 4], [2, 3, 4, 5]], dtype=np.int32)
    cl = np.array([0, 0, 0, 1, 1, 1], dtype=np.int32)
    return Mesh(tets=tets, cluster=cl, nclusters=2, meta={"kind": "fig4"})


def single_tet() -> Mesh:
    return Mesh(tets=np.array([[0, 1, 2, 3]], dtype=np.int32),
                cluster=np.zeros(4, dtype=np.int32), nclusters=1, meta={"kind": "single"})


def fans(ks=(16, 32, 33, 64, 65, 128, 129, 200, 300, 520), nclusters: int = 6, seed: int = 0) -> Mesh:
    """High-valence vertices: one closed fan per k, each a centre vertex, a
    top and a bottom vertex and a ring of k vertices, with tetrahedra
    (centre, top, r_i, r_i+1) and (centre, bottom, r_i, r_i+1) around the
    ring.  The centre lies in 2k tetrahedra, top and bottom in k, ring
    vertices in 4; every triangle is shared by at most two tetrahedra.
    Random cluster labels, then random vertex and tetrahedron ids.  Draw
    order: cluster labels, vperm, tperm."""
    rng = np.random.default_rng(seed)
    tets, base = [], 0
    for k in ks:
        c, top, bot = base, base + 1, base + 2
        ring = base + 3 + np.arange(k)
        nxt = np.roll(ring, -1)
        for apex in (top, bot):
            tets.append(np.stack([np.full(k, c), np.full(k, apex), ring, nxt], axis=1))
        base += k + 3
    tets = np.concatenate(tets).astype(np.int32)
    cluster = rng.integers(0, nclusters, size=base).astype(np.int32)
    tets, cluster, _, _ = _permute(rng, tets, cluster, None, None)
    return Mesh(tets=np.ascontiguousarray(tets), cluster=cluster, nclusters=nclusters,
                meta={"kind": "fans", "ks": list(ks), "seed": seed})


def nonmanifold(n: int = 5, fins: int = 6, dups: int = 3, nclusters: int = 3, seed: int = 0) -> Mesh:
    """Faces shared by more than two tetrahedra: the n^3 Kuhn lattice plus
    `fins` tetrahedra (a, b, c, x), each on a face (a, b, c) of a random
    lattice tetrahedron with a new vertex x, and `dups` copies of random
    lattice tetrahedra (same four vertices, new ids).  Random cluster labels,
    then random vertex and tetrahedron ids.  Draw order: fin tetrahedra, fin
    faces, duplicated tetrahedra, cluster labels, vperm, tperm."""
    rng = np.random.default_rng(seed)
    _, tets = kuhn_grid(n)
    nv0 = n ** 3
    ft = rng.choice(tets.shape[0], size=fins, replace=False)
    fk = rng.integers(0, 4, size=fins)
    extra = []
    for i, (t, k) in enumerate(zip(ft, fk)):
        face = [int(v) for j, v in enumerate(tets[t]) if j != k]
        extra.append(face + [nv0 + i])
    dt = rng.choice(tets.shape[0], size=dups, replace=False)
    extra += [[int(v) for v in tets[t]] for t in dt]
    tets = np.concatenate([tets, np.array(extra, dtype=np.int32).reshape(-1, 4)]).astype(np.int32)
    nv = nv0 + fins
    cluster = rng.integers(0, nclusters, size=nv).astype(np.int32)
    tets, cluster, _, _ = _permute(rng, tets, cluster, None, None)
    return Mesh(tets=np.ascontiguousarray(tets), cluster=cluster, nclusters=nclusters,
                meta={"kind": "nonmanifold", "n": n, "fins": fins, "dups": dups, "seed": seed})


def loose_tets(singles: int = 800, pairs: int = 100, seed: int = 0) -> Mesh:
    """Tetrahedra sharing almost no faces: `singles` tetrahedra on vertices of
    their own and `pairs` pairs sharing one triangle, all in one cluster
    (3.9 distinct faces per tetrahedron for the defaults, more than a closed
    region's 2 plus boundary).  Random vertex and tetrahedron ids.  Draw order:
    vperm, tperm."""
    rng = np.random.default_rng(seed)
    tets, v = [], 0
    for _ in range(singles):
        tets.append([v, v + 1, v + 2, v + 3])
        v += 4
    for _ in range(pairs):
        tets.append([v, v + 1, v + 2, v + 3])
        tets.append([v, v + 1, v + 2, v + 4])
        v += 5
    tets = np.array(tets, dtype=np.int32)
    cluster = np.zeros(v, dtype=np.int32)
    tets, cluster, _, _ = _permute(rng, tets, cluster, None, None)
    return Mesh(tets=np.ascontiguousarray(tets), cluster=cluster, nclusters=1,
                meta={"kind": "loose_tets", "singles": singles, "pairs": pairs, "seed": seed})


def random_small(seed: int, n: int = 4, nclusters: int = 5, drop: float = 0.3,
                 isolated: int = 2, empty_clusters: int = 1) -> Mesh:
    """A small irregular mesh: the n^3 Kuhn lattice with a random fraction of
    tetrahedra removed (leaving pockets, boundary faces and possibly
    disconnected pieces), a few isolated vertices appended, random cluster
    labels (some cluster ids unused), random vertex and tetrahedron ids.
    Draw order: drop mask, cluster labels, vperm, tperm."""
    rng = np.random.default_rng(seed)
    coords, tets = kuhn_grid(n)
    keep = rng.uniform(size=tets.shape[0]) >= drop
    tets = tets[keep]
    nv = coords.shape[0] + isolated
    used = nclusters + empty_clusters
    lab = rng.integers(0, nclusters, size=nv).astype(np.int32)
    # leave ids nclusters..used-1 empty, and shuffle which ids are used
    remap = rng.permutation(used).astype(np.int32)
    cluster = remap[lab]
    tets, cluster, _, _ = _permute(rng, tets.astype(np.int32), cluster, None, None)
    return Mesh(tets=np.ascontiguousarray(tets), cluster=cluster, nclusters=used,
                meta={"kind": "random_small", "seed": seed, "n": n})
