"""The C ABI without a GPU: the library loads, exports every function the
header declares, its structs have the layout the binding assumes, and
argument checks that need no device reject bad calls."""

import ctypes
import os
import re
import subprocess

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "pulscan.h")


@pytest.fixture(scope="module")
def L():
    import paper_2406_15186_amd as pk
    if not os.path.exists(pk.LIB_PATH):
        from paper_2406_15186_amd import build
        build.build()
    return pk.lib()


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pulscan_\w+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    names = header_functions()
    for must in ("pulscan_search", "pulscan_search_ex", "pulscan_search_batched",
                 "pulscan_ctx_create", "pulscan_ctx_destroy", "pulscan_strerror",
                 "pulscan_debug_tables", "pulscan_debug_bank_from_power"):
        assert must in names


def test_every_declared_function_is_exported(L):
    import paper_2406_15186_amd as pk
    names = header_functions()
    assert sorted(pk.SIGNATURES) == names
    out = subprocess.run(["nm", "-D", "--defined-only", pk.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    for n in names:
        assert n in exported, n
        assert hasattr(L, n)


def test_struct_layout_matches_binding(tmp_path):
    import paper_2406_15186_amd as pk
    src = tmp_path / "probe.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "pulscan.h"
int main(void) {
  printf("%zu %zu %zu\\n", sizeof(pulscan_candidate), sizeof(pulscan_candidates), sizeof(pulscan_opts));
  printf("%zu %zu %zu %zu %zu %zu %zu\\n", offsetof(pulscan_candidate, spectrum), offsetof(pulscan_candidate, bin),
         offsetof(pulscan_candidate, width), offsetof(pulscan_candidate, power),
         offsetof(pulscan_candidate, sigma), offsetof(pulscan_candidate, chunk),
         offsetof(pulscan_candidate, harmonics));
  printf("%zu %zu %zu %zu %zu\\n", offsetof(pulscan_candidates, capacity), offsetof(pulscan_candidates, count),
         offsetof(pulscan_candidates, on_device), offsetof(pulscan_candidates, count_device), sizeof(pulscan_complex));
  printf("%zu %zu %zu %zu\\n", sizeof(pulscan_server_config), offsetof(pulscan_server_config, opts),
         sizeof(pulscan_result), offsetof(pulscan_result, candidates));
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", offsetof(pulscan_opts, norm), offsetof(pulscan_opts, norm_block),
         offsetof(pulscan_opts, ntrials), offsetof(pulscan_opts, width_search),
         offsetof(pulscan_opts, async), offsetof(pulscan_opts, stream), offsetof(pulscan_opts, dense),
         offsetof(pulscan_opts, numharm), offsetof(pulscan_opts, best_per_chunk),
         offsetof(pulscan_opts, rblock), offsetof(pulscan_opts, graph), offsetof(pulscan_opts, power_fp16));
  return 0;
}
""")
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    lines = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    sizes = [int(v) for v in lines[0].split()]
    assert sizes == [ctypes.sizeof(pk.pulscan_candidate), ctypes.sizeof(pk.pulscan_candidates),
                     ctypes.sizeof(pk.pulscan_opts)]
    C = pk.pulscan_candidate
    assert [int(v) for v in lines[1].split()] == [C.spectrum.offset, C.bin.offset, C.width.offset,
                                                  C.power.offset, C.sigma.offset, C.chunk.offset,
                                                  C.harmonics.offset]
    S = pk.pulscan_candidates
    assert [int(v) for v in lines[2].split()] == [S.capacity.offset, S.count.offset,
                                                  S.on_device.offset, S.count_device.offset, 8]
    assert [int(v) for v in lines[3].split()] == [
        ctypes.sizeof(pk.pulscan_server_config), pk.pulscan_server_config.opts.offset,
        ctypes.sizeof(pk.pulscan_result), pk.pulscan_result.candidates.offset]
    O = pk.pulscan_opts
    assert [int(v) for v in lines[4].split()] == [O.norm.offset, O.norm_block.offset,
                                                  O.ntrials.offset, O.width_search.offset,
                                                  O.async_.offset, O.stream.offset, O.dense.offset,
                                                  O.numharm.offset, O.best_per_chunk.offset,
                                                  O.rblock.offset, O.graph.offset,
                                                  O.power_fp16.offset]
    assert [d[0] for d in pk.CANDIDATE_DTYPE.descr] == [f[0] for f in C._fields_]


def test_strerror_and_default_options(L):
    import paper_2406_15186_amd as pk
    assert pk.pulscan_strerror(0) == "ok"
    assert "invalid" in pk.pulscan_strerror(-1)
    assert "capacity" in pk.pulscan_strerror(-3)
    assert pk.pulscan_strerror(12345) == "unknown status"
    o = pk.pulscan_opts_default()
    assert (o.norm, o.norm_block, o.ntrials, o.width_search, o.async_, o.stream, o.dense,
            o.numharm, o.best_per_chunk, o.rblock, o.graph, o.power_fp16) == \
        (pk.PULSCAN_NORM_MOM, 0, 0.0, pk.PULSCAN_W_ALL, 0, None, 0, 1, 0, 0, 0, 0)


def test_null_arguments_are_rejected_without_a_device(L):
    import paper_2406_15186_amd as pk
    EINVAL = pk.PULSCAN_EINVAL
    out = pk.pulscan_candidates()
    o = pk.pulscan_opts_default()
    assert L.pulscan_search_ex(None, None, 1024, 10, 256, 6.0, ctypes.byref(o), ctypes.byref(out)) == EINVAL
    assert L.pulscan_search_batched(None, 1, None, None, None, 256, 6.0, ctypes.byref(o),
                                    ctypes.byref(out), None) == EINVAL
    assert L.pulscan_debug_tables(None, None, 1024, 10, 256, None, None, None, None, None) == EINVAL
    assert L.pulscan_debug_bank_from_power(None, None, 1024, 10, 256, None, None) == EINVAL
    T = (ctypes.c_float * 4)()
    assert L.pulscan_threshold_table(None, 4, 6.0, 100.0, 0, T) == EINVAL
    assert L.pulscan_ctx_set_timing(None, 1) == EINVAL
    ms, k = ctypes.c_double(), ctypes.c_uint64()
    assert L.pulscan_ctx_kernel_time(None, ctypes.byref(ms), ctypes.byref(k)) == EINVAL
    assert L.pulscan_ctx_create(None, 0) == EINVAL
    L.pulscan_ctx_destroy(None)   # a no-op
    cfg = pk.pulscan_server_config()
    L.pulscan_server_config_default(ctypes.byref(cfg))
    assert (cfg.hbm_budget, cfg.max_batch, cfg.chunk, cfg.sigma_thresh, cfg.max_candidates) == \
        (4 << 30, 256, 1024, 6.0, 1 << 20)
    assert L.pulscan_server_create(None, 0, ctypes.byref(cfg)) == EINVAL
    assert L.pulscan_server_submit(None, None, 4096, 10, 1) == EINVAL
    assert L.pulscan_server_poll(None, None, 0, 0) == EINVAL
    assert L.pulscan_server_stats(None, None, None, None, None) == EINVAL
    assert L.pulscan_host_alloc(None, 64) == EINVAL
    L.pulscan_server_destroy(None)   # a no-op
    L.pulscan_host_free(None)        # a no-op


def test_binding_fails_loudly_without_library(monkeypatch):
    import paper_2406_15186_amd as pk
    monkeypatch.setattr(pk, "_lib", None)
    monkeypatch.setattr(pk, "LIB_PATH", "/nonexistent/libpulscan.so")
    with pytest.raises(ImportError):
        pk.lib()
