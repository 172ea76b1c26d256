"""gale_build_static (no device allocation, static scratch) against
gale_build's blocks on the same context: every (cluster, relation) block
equal, on two calls in a row, the second with a smaller request, with the
LDS path and the hybrid global path (whose workspace sits in the scratch)."""
import sys

import numpy as np
import pytest

import meshgen

pytestmark = pytest.mark.gpu

REL = (1, 2, 4)


def _say(*a):
    from tests.conftest import say
    say(*a)


def _d2h(ptr, n):
    import ctypes as C
    out = np.empty(n, np.int32)
    if n:
        hip = C.CDLL("libamdhip64.so")
        st = hip.hipMemcpy(C.c_void_p(out.ctypes.data), C.cast(ptr, C.c_void_p), C.c_size_t(4 * n), 2)
        assert st == 0
    return out


def _static_block(words, base, rel):
    """(row ids, offsets, entries) of relation rel from a block at word
    `base` of the host copy `words`, by the layout gale.h documents."""
    h = words[base:base + 8]
    nV, nT, nvt, nvv, ntt, cap_vv, cap_tt = (int(x) for x in h[1:8])
    al = lambda w: (w + 31) // 32 * 32
    w = al(8)
    mask = 7
    vrows = w
    w = al(w + nV)
    vt_off = w
    w = al(w + nV + 1)
    vt_ent = w
    w = al(w + nvt)
    trows = w
    w = al(w + nT)
    tt_off = w
    w = al(w + nT + 1)
    tt_ent = w
    w = al(w + cap_tt)
    vv_off = w
    w = al(w + nV + 1)
    vv_ent = w
    assert mask == 7
    b = base
    if rel == 1:
        return words[b + vrows:b + vrows + nV], words[b + vt_off:b + vt_off + nV + 1], words[b + vt_ent:b + vt_ent + nvt]
    if rel == 2:
        return words[b + vrows:b + vrows + nV], words[b + vv_off:b + vv_off + nV + 1], words[b + vv_ent:b + vv_ent + nvv]
    return words[b + trows:b + trows + nT], words[b + tt_off:b + tt_off + nT + 1], words[b + tt_ent:b + tt_ent + ntt]


def _run(ctx, ids, torch):
    gale = __import__("paper_2507_15230_amd.gale", fromlist=["gale"])
    st, bw = ctx.build_static(ids, 7, 0, 0)
    assert st == gale.ENOMEM and bw[-1] > 0          # size query: nothing built
    out = torch.full((int(bw[-1]),), -7, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    st, bw2 = ctx.build_static(ids, 7, out.data_ptr(), out.numel())
    assert st == gale.OK, gale.strerror(st)
    assert np.array_equal(bw, bw2)
    words = out.cpu().numpy()
    tk = ctx.build(ids, 7, "batched")
    ctx.poll(tk)
    bad = []
    for i, k in enumerate(ids):
        for rel in REL:
            v = ctx.block_device(tk, int(k), rel)
            ref = (_d2h(v.row_ids, v.nrows), _d2h(v.offsets, v.nrows + 1), _d2h(v.entries, v.nnz))
            got = _static_block(words, int(bw2[i]), rel)
            if not all(g.shape == r.shape and np.array_equal(g, r) for g, r in zip(got, ref)):
                bad.append((int(k), rel))
    ctx.release(tk)
    return bad


@pytest.mark.parametrize("lds", [0, 12288])
def test_build_static_equals_build(lds):
    import torch
    from paper_2507_15230_amd import gale
    m = meshgen.refined_mesh(24, 0.05, 2, 256, 1.0, seed=3)
    _say("build_static: refined 24^3,", m.nt, "tetrahedra,", m.nclusters, "clusters, lds", lds)
    with gale.Context(form="batched", lds_bytes=lds) as ctx:
        ctx.load(m.tets, m.cluster, m.nclusters)
        ids = np.random.default_rng(1).permutation(m.nclusters).astype(np.int32)
        bad = _run(ctx, ids, torch)
        assert not bad, bad[:10]
        g0 = ctx.stats()["global_path_blocks"]
        if lds:
            assert g0 > 0
        small = ids[: max(1, len(ids) // 5)]
        bad = _run(ctx, small, torch)
        assert not bad, bad[:10]


def test_build_static_errors():
    import torch  # noqa: F401
    from paper_2507_15230_amd import gale
    m = meshgen.grid_mesh(8, 64, seed=0)
    with gale.Context(form="batched") as ctx:
        ctx.load(m.tets, m.cluster, m.nclusters)
        with pytest.raises(gale.GaleError) as e:
            ctx.build_static([0, 0], 7, 0, 0)
        assert e.value.status == gale.EINVAL
        with pytest.raises(gale.GaleError) as e:
            ctx.build_static([m.nclusters], 7, 0, 0)
        assert e.value.status == gale.EINVAL
    with gale.Context(mode="serve") as sctx:
        sctx.load(m.tets, m.cluster, m.nclusters)
        with pytest.raises(gale.GaleError) as e:
            sctx.build_static([0], 7, 0, 0)
        assert e.value.status == gale.ESTATE
