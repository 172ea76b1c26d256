"""The C-ABI library on a machine without a GPU: it loads, exports every
function include/gale.h declares, its structs have the layout the binding
assumes, and calls that need a device fail cleanly."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def _declared():
    names = set()
    for h in HEADERS:
        txt = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(gale_[a-z_]+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    from paper_2507_15230_amd import gale
    lib = gale.load_library()
    names = _declared()
    assert len(names) >= 16
    for n in names:
        assert hasattr(lib, n), "libgale.so does not export " + n
    out = subprocess.run(["nm", "-D", "--defined-only", gale.LIB_PATH], capture_output=True, text=True).stdout
    for n in names:
        assert re.search(r"\bT " + n + r"\b", out), n + " is not a defined text symbol"


def test_struct_layout_matches_binding(tmp_path):
    from paper_2507_15230_amd import gale
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "gale.h"\n#include "gale_lowerstar.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(gale_config),'
                   ' sizeof(gale_csr), sizeof(gale_stats), offsetof(gale_csr, entries),'
                   ' offsetof(gale_stats, kernel_ms_total), sizeof(gale_consumer_cfg), sizeof(gale_consumer_result),'
                   ' offsetof(gale_consumer_cfg, nv), offsetof(gale_consumer_result, first_error));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert got == [C.sizeof(gale.GaleConfig), C.sizeof(gale.GaleCsr), C.sizeof(gale.GaleStats),
                   gale.GaleCsr.entries.offset, gale.GaleStats.kernel_ms_total.offset,
                   C.sizeof(gale.GaleConsumerCfg), C.sizeof(gale.GaleConsumerResult),
                   gale.GaleConsumerCfg.nv.offset, gale.GaleConsumerResult.first_error.offset]


def test_strerror_and_last_error():
    from paper_2507_15230_amd import gale
    lib = gale.load_library()
    assert lib.gale_strerror(0) == b"ok"
    assert lib.gale_strerror(-1) == b"invalid argument"
    assert lib.gale_strerror(-6) == b"device error"
    assert isinstance(lib.gale_last_error(), bytes)


def test_null_arguments_rejected():
    from paper_2507_15230_amd import gale
    lib = gale.load_library()
    assert lib.gale_create(None, None) == gale.EINVAL
    assert lib.gale_poll(None, 1, 0) == gale.EINVAL
    assert lib.gale_release(None, 1) == gale.EINVAL
    lib.gale_destroy(None)


def test_create_rejects_bad_config_before_the_device():
    from paper_2507_15230_amd import gale
    for kw in ({"block_threads": 100}, {"global_cu_share": 1.5}, {"global_cu_share": -0.1}):
        with pytest.raises(gale.GaleError) as ei:
            gale.Context(**kw)
        assert ei.value.status == gale.EINVAL


def test_create_without_device_is_edevice():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    from paper_2507_15230_amd import gale
    with pytest.raises(gale.GaleError) as ei:
        gale.Context()
    assert ei.value.status == gale.EDEVICE


def test_binding_refuses_missing_library(tmp_path):
    """In a fresh interpreter (nothing loaded yet) the binding raises when the
    library file is absent: there is no fallback path."""
    import subprocess
    import sys
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_2507_15230_amd import gale\n"
        "try:\n"
        "    gale.load_library(%r)\n"
        "except RuntimeError as e:\n"
        "    print('refused', e)\n"
        "    sys.exit(0)\n"
        "sys.exit(3)\n" % (ROOT, str(tmp_path / "missing.so")))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "refused" in r.stdout
