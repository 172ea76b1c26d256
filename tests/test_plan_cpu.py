"""CPU checks of the working-array plans (paper_2507_15230_amd/csrc/gale_layout.h)
that the host and the kernels share: for many cluster shapes, relation masks,
budgets and workgroup sizes, every plan the host accepts keeps each array
inside the LDS budget or the workspace slice, in order and without overlap.
Region sizes are written out here from what each array holds, not taken from
the plan functions."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2507_15230_amd", "csrc")

HARNESS = r"""
#include <cstdio>
#include <cstdlib>
#include <random>
#include "gale_layout.h"
using namespace gale;

static int64_t a16(int64_t b) { return (b + 15) / 16 * 16; }
static int fails = 0;
#define CHECK(c, what) do { if (!(c)) { if (fails++ < 10) std::printf("FAIL %s: %s ns=%d nT=%d L=%d nV=%d nnz=%d mask=%u budget=%lld B=%d\n", \
    kind, what, m.ns, m.nT, m.L, m.nV, m.nnzVT, mask, (long long)budget, B); } } while (0)

int main() {
    std::mt19937_64 rng(12345);
    long n_lds = 0, n_hyb = 0, n_ws = 0;
    const int Bs[3] = {256, 512, 1024};
    for (int iter = 0; iter < 200000; ++iter) {
        ClusterMeta m{};
        // shapes from tiny to large: vertices, star and halo, local table
        const int scale = 1 << (rng() % 15);
        m.nV = (int)(rng() % (scale + 1));
        m.nT = (int)(rng() % (6 * m.nV + 2));
        m.ns = m.nT + (int)(rng() % (4 * m.nV + 2));
        m.nh = (int)(rng() % (m.nT / 4 + 2));
        m.L = m.nV + (int)(rng() % (3 * m.nV + 5));
        m.nnzVT = (int)(rng() % (40 * m.nV + 2));
        m.cap_vv = m.nnzVT;
        const uint32_t mask = 1 + (uint32_t)(rng() % 7);
        const int B = Bs[rng() % 3];
        const int64_t budget = 4096 + (int64_t)(rng() % 160000);
        const bool tt = mask & kRelTT, v = mask & (kRelVT | kRelVV), vv = mask & kRelVV;
        const int64_t W = (m.L + 31) / 32, SW = (W + 31) / 32;
        {
            const char *kind = "lds";
            const Plan p = lds_plan(m, mask, budget, B);
            if (p.ok) {
                ++n_lds;
                CHECK(m.L <= 65535 && (int64_t)m.ns + m.nh <= 65535, "narrow ids");
                if (tt) {
                    CHECK(p.win >= (int64_t)m.nT * 8, "internal stream before the partner cells");
                    CHECK(p.lowb >= p.win + (int64_t)m.nT * 8, "partner cells before the lower bits");
                    CHECK(p.ht >= p.lowb + W * 4, "lower bits before the table");
                    CHECK(p.ht + 2 * (int64_t)p.H <= budget, "table within the budget");
                    CHECK(p.H >= 64 && p.H % 2 == 0, "table cells");
                    CHECK(p.P >= 1 && p.P <= kLdsFacePasses, "passes");
                }
                if (v) {
                    CHECK(p.rix >= (int64_t)m.ns * 8, "V arrays after the star stream");
                    CHECK(p.rowl >= p.rix + (int64_t)m.L * 2, "rix");
                    CHECK(p.cnt >= p.rowl + (int64_t)m.nV * 2, "rowl");
                    CHECK(p.lvt >= p.cnt + ((int64_t)m.nV + 1) * 4, "cnt");
                    CHECK(p.wbm >= p.lvt + (int64_t)m.nnzVT * 2, "lvt");
                    int64_t end = p.wbm;
                    if (vv) {
                        CHECK(p.G == 8 || p.G == 16 || p.G == 32, "group size");
                        CHECK(p.G != 8 || W <= 64, "8-lane groups keep their words in registers");
                        CHECK(p.lvl >= p.wbm + (int64_t)(B / p.G) * (W + SW) * 4, "bitmaps and summaries");
                        end = p.lvl + (int64_t)m.L * 4;
                    }
                    CHECK(end <= budget, "V arrays within the budget");
                }
            }
        }
        {
            const char *kind = "hybrid";
            const Plan p = hyb_plan(m, mask, budget, B);
            if (p.ok) {
                ++n_hyb;
                if (tt) {
                    CHECK(p.ht >= W * 4, "lower bits before the table");
                    CHECK(p.ht + 8 * (int64_t)p.H <= budget, "table within the budget");
                    CHECK(p.H >= 64 && p.P >= 1 && p.P <= kHybFacePasses, "table cells and passes");
                    CHECK(m.L <= 32767 && (int64_t)m.ns + m.nh < (1 << 17) - 1, "face key and position bits");
                    CHECK(p.ws_bytes >= (int64_t)m.nT * 32, "partner counters in the workspace");
                }
                if (v) {
                    CHECK(m.L <= 65535, "16-bit row index");
                    CHECK(p.rowl >= p.rix + (int64_t)m.L * 2, "rix");
                    CHECK(p.cnt >= p.rowl + (int64_t)m.nV * 2, "rowl");
                    CHECK(p.wbm >= p.cnt + ((int64_t)m.nV + 1) * 4, "cnt");
                    int64_t end = p.wbm;
                    if (vv) {
                        CHECK(p.G == 16 || p.G == 32, "group size");
                        end = p.wbm + (int64_t)(B / p.G) * (W + SW) * 4;
                        if (p.lvl >= 0) {
                            CHECK(p.lvl >= end, "lverts copy after the bitmaps");
                            end = p.lvl + (int64_t)m.L * 4;
                        }
                    }
                    CHECK(end <= budget, "V arrays within the budget");
                    CHECK(p.lv4 >= (int64_t)m.nnzVT * 4, "entry ids before the entry tetrahedra");
                    CHECK(p.ws_bytes >= p.lv4 + (int64_t)m.nnzVT * 8, "entry tetrahedra in the workspace");
                }
            }
        }
        {
            const char *kind = "global";
            const Plan p = ws_plan(m, mask, B);
            ++n_ws;
            if (tt) {
                CHECK(p.lowb >= (int64_t)m.nT * 16, "partner cells");
                CHECK(p.ht >= p.lowb + W * 4, "lower bits");
                CHECK(p.bytes >= p.ht + 4 * (int64_t)p.H && p.H >= 6 * (int64_t)m.nT, "table");
            }
            if (v) {
                int64_t end = p.rix + (int64_t)m.L * 4 + (int64_t)m.nV * 4 + ((int64_t)m.nV + 1) * 4 + (int64_t)m.nnzVT * 4;
                CHECK(p.wbm >= end, "V arrays in order");
                if (vv) CHECK(p.bytes >= p.wbm + (int64_t)(B / 32) * (W + SW) * 4, "bitmaps");
            }
        }
    }
    std::printf("plans lds %ld hybrid %ld global %ld fails %d\n", n_lds, n_hyb, n_ws, fails);
    return fails ? 1 : 0;
}
"""


def test_plans_keep_arrays_inside_their_memory(tmp_path):
    src = tmp_path / "plans.cpp"
    src.write_text(HARNESS)
    exe = tmp_path / "plans"
    r = subprocess.run(["g++", "-std=c++17", "-O2", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + CSRC,
                        str(src), "-o", str(exe)], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("host compiler cannot build the layout header here: " + r.stderr[-400:])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    print(out.stdout)
    assert out.returncode == 0, out.stdout
    counts = dict(zip(("lds", "hybrid", "global"), [int(x) for x in out.stdout.split("plans")[1].split()[1:6:2]]))
    assert counts["lds"] > 1000 and counts["hybrid"] > 1000
