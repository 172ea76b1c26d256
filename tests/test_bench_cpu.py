"""CPU checks of bench.py's host logic: the algorithmic bytes of a step, and
the rocprofv3 summaries (traffic scaled by the copy calibration, the record
read back only while the kernel sources are unchanged)."""
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


class _Ctx:
    def __init__(self, infos):
        self.infos = infos

    def cluster_info(self, k):
        return self.infos[k]


def test_alg_bytes_counts_each_term():
    ctx = _Ctx([{"ns": 10, "nh": 2, "nV": 5, "nT": 7}, {"ns": 3, "nh": 0, "nV": 1, "nT": 1}])
    b, parts = bench.alg_bytes(ctx, 2, entries=100)
    # 20 B per star or halo tetrahedron, 4 B per entry, offsets (2 nV + nT + 3 per cluster), row ids
    assert b == 20 * 15 + 4 * 100 + 4 * (2 * 6 + 8 + 6) + 4 * (6 + 8)
    assert parts == {"star_tets": 13, "halo_tets": 2, "vertex_rows": 6, "tet_rows": 8}


def _write_csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        f.write(",".join('"%s"' % h for h in header) + "\n")
        for r in rows:
            f.write(",".join('"%s"' % x for x in r) + "\n")


def test_traffic_record_follows_the_kernel_sources(tmp_path, monkeypatch):
    kt, fe, wr = tmp_path / "kt", tmp_path / "fetch", tmp_path / "write"
    _write_csv(str(kt / "kt_kernel_stats.csv"), ["Name", "Calls", "TotalDurationNs", "AverageNs", "MinNs", "MaxNs"],
               [["gale::gale_persistent_kernel<1024, true>", 2, 2000000, 1000000, 900000, 1100000]])
    _write_csv(str(kt / "kt_kernel_trace.csv"), ["Kernel_Name", "Start_Timestamp", "End_Timestamp"],
               [["gale::gale_zero_kernel", 0, 10], ["gale::gale_persistent_kernel<1024, true>", 20, 1000020]])
    copy = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel>"
    cols = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    mib = bench.COPY_BYTES / 1024.0
    _write_csv(str(fe / "f_counter_collection.csv"), cols,
               [[copy, "FETCH_SIZE", mib / 2], ["gale::gale_persistent_kernel<1024, true>", "FETCH_SIZE", 1000]])
    _write_csv(str(wr / "w_counter_collection.csv"), cols,
               [[copy, "WRITE_SIZE", mib], ["gale::gale_persistent_kernel<1024, true>", "WRITE_SIZE", 3000]])
    prof = tmp_path / "profiles"
    prof.mkdir()
    out_md = prof / "k_traffic_case.md"
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    sha = {"v": "abc"}
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: sha["v"])
    bench.summarize_profile(str(out_md), "t", "cmd", str(kt), "cf", str(fe), "cw", str(wr), kernel_ms=1.0,
                            config_index=7, alg_bytes=4.0e6)
    rec = json.load(open(str(prof / "k_traffic_case_traffic.json")))
    # fetch counted at half the copy's bytes: scaled by 2; write by 1
    assert rec["fetch_factor"] == pytest.approx(2.0) and rec["write_factor"] == pytest.approx(1.0)
    assert rec["traffic_bytes_per_step"] == pytest.approx((2 * 1000 + 3000) * 1024.0)
    assert "traffic / algorithmic" in out_md.read_text()
    t, src = bench.committed_traffic(7)
    assert t == pytest.approx(5000 * 1024.0) and src.endswith("k_traffic_case_traffic.json")
    assert bench.committed_traffic(3) == (None, None)
    sha["v"] = "changed"
    assert bench.committed_traffic(7) == (None, None)
