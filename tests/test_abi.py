"""Host-side checks of the C-ABI library (no GPU needed).

The library must load and export every function the public header declares;
the pure host function qrng_output_bits must agree with the oracle's rule;
argument errors must be reported before any device work.
"""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qrng.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2011_04130_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2011_04130_amd import build
        build.build()
    return _lib.load_library()


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(qrng_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_three_core_calls():
    names = declared_functions()
    for core in ("qrng_minentropy", "qrng_toeplitz_hash", "qrng_toeplitz_hash_batched"):
        assert core in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2011_04130_amd import _lib
    names = declared_functions()
    assert sorted(names) == sorted(_lib.EXPORTS)
    for name in names:
        assert hasattr(lib, name), name


def test_version(lib):
    assert b"gfx950" in lib.qrng_version()


@pytest.mark.parametrize("n", [1, 63, 64, 1000, 131072, 1 << 23, (1 << 40) + 17])
@pytest.mark.parametrize("h", [-1.0, 0.0, 0.3, 1.0, 4.999999, 5.0, 5.57, 7.9, 8.0, 9.5])
@pytest.mark.parametrize("eps", [0.0, 0.5, 10.0, 64.0])
def test_output_bits_matches_oracle(lib, n, h, eps):
    from paper_2011_04130_amd import output_bits
    assert output_bits(n, 8, h, eps) == oracle.output_bits(n, 8, h, eps)


def test_output_bits_other_widths(lib):
    from paper_2011_04130_amd import output_bits
    for N in (1, 3, 5, 8, 12, 16):
        for h in np.linspace(-1, N + 1, 23):
            for n in (1, 7, 1000, 999983):
                assert output_bits(n, N, float(h), 3.0) == oracle.output_bits(n, N, float(h), 3.0)


def test_output_bits_rejects_bad_arguments(lib):
    out = ctypes.c_uint64()
    assert lib.qrng_output_bits(10, 0, 5.0, 0.0, ctypes.byref(out)) == -1
    assert lib.qrng_output_bits(10, 8, float("nan"), 0.0, ctypes.byref(out)) == -1
    assert lib.qrng_output_bits(10, 8, 5.0, -1.0, ctypes.byref(out)) == -1
    assert lib.qrng_output_bits(10, 8, 5.0, 0.0, None) == -1
    assert b"null" in lib.qrng_last_error()


def test_null_context_is_rejected_without_device_work(lib):
    buf = (ctypes.c_uint64 * 4)()
    p = ctypes.cast(buf, ctypes.c_void_p)
    assert lib.qrng_toeplitz_hash(None, p, 64, p, 32, p, 0, None) == -1
    assert lib.qrng_toeplitz_hash_seeded(None, p, 64, 1, 32, p, 0, None) == -1
    assert lib.qrng_toeplitz_hash_batched(None, p, 1, p, None, p, 0, None) == -1
    assert lib.qrng_toeplitz_hash_batched_host(None, None, 1, p, p, 0, None) == -1
    assert lib.qrng_toeplitz_hash_batched_rejected(None, None, None) == -1
    assert lib.qrng_seed_register(None, p, 64, None, None) == -1
    assert lib.qrng_minentropy(None, p, 8, None, None, None, None) == -1
    lib.qrng_destroy(None)  # no-op


def test_create_without_gpu_reports_device_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    st = lib.qrng_create(ctypes.byref(h), 0)
    assert st in (-3, -1) and not h.value


def test_new_entry_points_reject_null_handles(lib):
    """Plans, tuning table and server calls fail cleanly without a context
    or handle (no device work is attempted)."""
    from paper_2011_04130_amd._lib import Block, MeOpts, PlanInfo, Served, ServerCfg, ServerStats
    buf = (ctypes.c_uint64 * 8)()
    p = ctypes.cast(buf, ctypes.c_void_p)
    h = ctypes.c_void_p()
    blk = (Block * 1)()
    assert lib.qrng_plan_create(None, blk, 1, p, p, None, None, None, 0.0, 0, 0, None,
                                ctypes.byref(h)) == -1 and not h.value
    assert lib.qrng_plan_create(None, blk, 1, p, p, None, None, None, 0.0, 0, 0, None,
                                None) == -1
    assert lib.qrng_plan_execute(None, None) == -1
    assert lib.qrng_plan_query(None, ctypes.byref(PlanInfo())) == -1
    lib.qrng_plan_destroy(None)  # no-op
    n = ctypes.c_uint64()
    assert lib.qrng_tune_export(None, None, 0, ctypes.byref(n)) == -1
    assert lib.qrng_tune_import(None, b"ntt 20 10 27\n") == -1
    cfg = ServerCfg()
    assert lib.qrng_server_create(None, ctypes.byref(cfg), ctypes.byref(h)) == -1
    assert lib.qrng_server_create(None, ctypes.byref(cfg), None) == -1
    rid = ctypes.c_uint64()
    cnt = ctypes.c_uint32()
    assert lib.qrng_server_submit(None, 10, ctypes.byref(rid)) == -1
    assert lib.qrng_server_submit_many(None, p, 1, p, ctypes.byref(cnt)) == -1
    assert lib.qrng_server_step(None, None) == -1
    assert lib.qrng_server_poll(None, (Served * 1)(), 1, ctypes.byref(cnt)) == -1
    assert lib.qrng_server_release(None, 1) == -1
    assert lib.qrng_server_release_many(None, p, 1) == -1
    assert lib.qrng_server_read(None, 1, p, None) == -1
    assert lib.qrng_server_query(None, ctypes.byref(ServerStats())) == -1
    assert lib.qrng_server_feed(None, p, None) == -1
    lib.qrng_server_destroy(None)  # no-op
    assert lib.qrng_extract(None, p, 8, ctypes.byref(MeOpts(8, 0, 0.0, 0.0, 0, 0)), 0.0, 1, 8,
                            p, None, None, 0, None) == -1
    assert lib.qrng_toeplitz_hash_strided(None, p, 64, 1, 1, 32, p, 1, 1, 0, None) == -1


def test_struct_layouts_match_header(lib, tmp_path):
    """ctypes mirrors of the header's structs have the sizes and field
    offsets a C compiler gives them."""
    import subprocess
    from paper_2011_04130_amd import _lib as L
    structs = {"qrng_me_opts": L.MeOpts, "qrng_me_result": L.MeResult, "qrng_block": L.Block,
               "qrng_plan_info": L.PlanInfo, "qrng_server_cfg": L.ServerCfg,
               "qrng_served": L.Served, "qrng_server_stats": L.ServerStats}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "qrng.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines += ['return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src),
                           "-o", str(exe)])
    got = dict(l.rsplit(" ", 1) for l in subprocess.check_output([str(exe)]).decode().splitlines())
    for cname, py in structs.items():
        assert int(got["%s size" % cname]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got["%s %s" % (cname, f)]) == getattr(py, f).offset, (cname, f)
