"""The DiscreteGradient consumer on blocks built on the GPU: VE, VF and VT
requested through the C ABI, the gradient computed by the library's consumer
(gale_gradient_cluster), every record equal to the oracle's discrete gradient
(oracle/gradient.py); and the threaded workload (gale_gradient_run) counting
the same critical simplices and pairs as the oracle."""
import sys

import numpy as np
import pytest

import meshgen
import oracle
from oracle.gradient import discrete_gradient

pytestmark = pytest.mark.gpu


def _say(*a):
    from tests.conftest import say
    say(*a)


def _field(m, seed):
    f = meshgen.gauss_field(m.coords.astype(np.float64), int(round(m.nv ** (1 / 3))), np.random.default_rng(seed))
    return np.asarray(f, dtype=np.float32)  # the consumer's precision, on both sides


@pytest.mark.parametrize("kind", ["lattice", "refined"])
def test_gradient_from_gpu_blocks_equals_oracle(kind):
    from paper_2507_15230_amd import gale
    m = meshgen.grid_mesh(10, 120, seed=3) if kind == "lattice" else meshgen.refined_mesh(10, 0.1, 2, 96, 1.0, seed=6)
    field = _field(m, 2)
    orc = oracle.Oracle.of(m)
    e, _, f, _ = orc.simplices()
    g = discrete_gradient(m.tets, field, e, f)
    _say(kind, m.nv, "vertices", len(g["critical"]), "critical")
    pairs, crit = set(), set()
    with gale.Context(form="batched", simplex_lists=True) as ctx:
        ctx.load(m.tets, m.cluster, m.nclusters)
        le, _, lf, _ = ctx.simplices()
        ids = np.arange(m.nclusters, dtype=np.int32)
        tk = ctx.submit(ids, gale.REL_VT | gale.REL_VE | gale.REL_VF)
        for k in range(m.nclusters):
            rec = gale.gradient_cluster(ctx.block(tk, k, gale.REL_VE), ctx.block(tk, k, gale.REL_VF),
                                        ctx.block(tk, k, gale.REL_VT), le, lf, m.tets, field)
            for d, lo, up in rec.tolist():
                if up < 0:
                    crit.add((d, lo))
                else:
                    pairs.add((d, lo, up))
        ctx.release(tk)
    assert pairs == g["pairs"] and crit == g["critical"]


def test_gradient_workload_counts():
    from paper_2507_15230_amd import gale
    m = meshgen.grid_mesh(12, 100, seed=5)
    field = _field(m, 4)
    orc = oracle.Oracle.of(m)
    e, _, f, _ = orc.simplices()
    g = discrete_gradient(m.tets, field, e, f)
    crit = [0, 0, 0, 0]
    for d, _ in g["critical"]:
        crit[d] += 1
    pairs = [0, 0, 0]
    for d, _, _ in g["pairs"]:
        pairs[d] += 1
    with gale.Context(form="batched", simplex_lists=True) as ctx:
        ctx.load(m.tets, m.cluster, m.nclusters)
        res = gale.gradient_run(ctx, m.tets, field, np.arange(m.nclusters, dtype=np.int32), threads=8)
    _say("workload", res["critical"], res["pairs"], "p50 %.0f us" % res["lat_p50_us"])
    assert res["errors"] == 0 and res["clusters"] == m.nclusters
    assert res["critical"] == crit and res["pairs"] == pairs
