"""CPU checks of the host consumer (critical points by lower/upper links) on
blocks from the oracle: against a brute-force classification written from the
definition, and against facts of PL Morse theory."""
import numpy as np
import pytest

import meshgen
import oracle

REL_VT, REL_VV = 1, 2


def _gale():
    from paper_2507_15230_amd import gale
    return gale


def brute_labels(tets, field, vertices):
    """Links found by scanning every tetrahedron; components by breadth-first
    search; same (f, id) order."""
    def below(a, b):
        return (field[a], a) < (field[b], b)
    out = []
    for v in vertices:
        adj = {}
        for t in tets:
            if v in t:
                o = [int(u) for u in t if u != v]
                for u in o:
                    adj.setdefault(u, set())
                for i in range(3):
                    for j in range(i + 1, 3):
                        adj[o[i]].add(o[j])
                        adj[o[j]].add(o[i])
        low = {u for u in adj if below(u, v)}
        up = set(adj) - low

        def comps(part):
            seen, n = set(), 0
            for s in part:
                if s in seen:
                    continue
                n += 1
                stack = [s]
                seen.add(s)
                while stack:
                    x = stack.pop()
                    for y in adj[x]:
                        if y in part and y not in seen:
                            seen.add(y)
                            stack.append(y)
            return n
        if not low:
            out.append(1)
        elif not up:
            out.append(2)
        elif comps(low) > 1 or comps(up) > 1:
            out.append(3)
        else:
            out.append(0)
    return np.array(out, np.int32)


def classify_all(m, field):
    gale = _gale()
    orc = oracle.Oracle.of(m)
    labels = {}
    for k in range(m.nclusters):
        vt = orc.block(k, REL_VT)
        vv = orc.block(k, REL_VV)
        lab = gale.lowerstar_classify(vt[0], vt, vv, m.tets, field)
        for v, l in zip(vt[0], lab):
            labels[int(v)] = int(l)
    return labels


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_matches_brute_force(seed):
    m = meshgen.random_small(seed, n=5, nclusters=5, drop=0.2, isolated=2)
    rng = np.random.default_rng(seed)
    field = rng.integers(0, 6, size=m.nv).astype(np.float32)  # many ties: the id breaks them
    got = classify_all(m, field)
    verts = sorted(got)
    exp = brute_labels(m.tets, field, verts)
    assert [got[v] for v in verts] == exp.tolist()


def test_linear_field_on_a_ball_has_one_minimum_and_one_maximum():
    n = 5
    m = meshgen.grid_mesh(n, 32, seed=3)
    f = (m.coords[:, 0] + 1.1 * m.coords[:, 1] + 1.3 * m.coords[:, 2]).astype(np.float32)
    labels = np.array(list(classify_all(m, f).values()))
    assert (labels == 1).sum() == 1
    assert (labels == 2).sum() == 1
    assert (labels == 3).sum() == 0


def test_saddle_at_the_centre():
    n = 5
    coords, tets = meshgen.kuhn_grid(n)
    m = meshgen.Mesh(tets=tets, cluster=np.zeros(coords.shape[0], np.int32), nclusters=1, coords=coords)
    c = coords.astype(np.float64) - 2.0
    # x^2 + y^2 - z^2: the lower set near the origin is the two cones along
    # +z and -z, so the lower link has two components (a small linear term
    # separates neighbours of equal value)
    f = (c[:, 0] ** 2 + c[:, 1] ** 2 - c[:, 2] ** 2 + 1e-3 * (c[:, 0] + 2 * c[:, 1] + 3 * c[:, 2]))
    f = f.astype(np.float32)
    labels = classify_all(m, f)
    centre = int(np.nonzero((np.abs(c) < 1e-9).all(1))[0][0])
    assert labels[centre] == 3
    assert brute_labels(m.tets, f, [centre]).tolist() == [3]


def test_rejects_inconsistent_blocks():
    gale = _gale()
    m = meshgen.cube()
    orc = oracle.Oracle.of(m)
    vt = orc.block(0, REL_VT)
    vv = orc.block(0, REL_VV)
    field = np.arange(m.nv, dtype=np.float32)
    bad = (vt[0], vt[1], (vt[2] + 1) % m.nt)  # a tetrahedron that misses its row vertex
    with pytest.raises(gale.GaleError):
        gale.lowerstar_classify(vt[0], bad, vv, m.tets, field)
