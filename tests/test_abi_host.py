"""The C-ABI library on a machine without a GPU: it loads, exports every
symbol include/bcd.h declares, and every check that happens before the
device is touched behaves as documented."""
import ctypes as C
import os
import re
import subprocess
import sys

import numpy as np
import pytest

from paper_1708_08739_amd import bcd
from paper_1708_08739_amd import graphgen as gg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(bcd_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def _lib():
    # a fresh checkout holds no built library: build it (hipcc cross-compiles
    # for gfx950 without a GPU), as the oracle fixture builds the oracle
    from paper_1708_08739_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    return bcd.load()


@pytest.fixture(scope="module")
def lib():
    return _lib()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert "bcd_bc_exact" in names and "bcd_rv" in names and "bcd_bc_sampled" in names
    for name in names:
        assert hasattr(lib, name), name
    for name in bcd.SIGNATURES:
        assert name in names, name


def test_status_strings(lib):
    for code in range(10):
        s = lib.bcd_status_string(code).decode()
        assert s and s != "unknown status"
    assert lib.bcd_status_string(99).decode() == "unknown status"


def test_sample_count_eq8(lib):
    # Eq.(8) values worked by hand in tests/golden/sample_count_eq8.txt
    rows = [l.split() for l in open(os.path.join(ROOT, "tests", "golden", "sample_count_eq8.txt"))
            if l.strip() and not l.startswith("#")]
    for eps, delta, K, rv, T in rows:
        assert bcd.bcd_sample_count(float(eps), float(delta), float(K), int(rv)) == int(T)
    assert bcd.bcd_sample_count(1e-9, 0.1, 1e6, 10 ** 7) == 2 ** 63 - 1
    for bad in [(0.0, 0.1, 1, 1), (1.0, 0.0, 1, 1), (1.0, 1.0, 1, 1), (1.0, 0.5, -1, 1), (1.0, 0.5, 1, -1)]:
        with pytest.raises(bcd.BcdError) as e:
            bcd.bcd_sample_count(*bad)
        assert e.value.code == bcd.BCD_ERR_INVALID_ARG


def _load(n, m, rp, col, w=None):
    L = _lib()
    h = C.c_void_p()
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    w = None if w is None else np.ascontiguousarray(w, dtype=np.uint32)
    rc = L.bcd_graph_load_csr(n, m, rp.ctypes.data, col.ctypes.data if col.size else None,
                              None if w is None else w.ctypes.data, C.byref(h))
    return rc, h


@pytest.mark.parametrize("case,expect", [
    ("rp0", bcd.BCD_ERR_BAD_GRAPH), ("rpn", bcd.BCD_ERR_BAD_GRAPH), ("decreasing", bcd.BCD_ERR_BAD_GRAPH),
    ("col_range", bcd.BCD_ERR_BAD_GRAPH), ("self_loop", bcd.BCD_ERR_BAD_GRAPH),
    ("repeat", bcd.BCD_ERR_BAD_GRAPH), ("unsorted", bcd.BCD_ERR_BAD_GRAPH),
    ("zero_weight", bcd.BCD_ERR_BAD_GRAPH), ("n0", bcd.BCD_ERR_INVALID_ARG),
    ("neg_m", bcd.BCD_ERR_INVALID_ARG),
])
def test_graph_validation_before_device(case, expect):
    """Malformed CSR is rejected on the host, before any device call."""
    n, rp, col, w = 3, [0, 2, 3, 3], [1, 2, 0], None
    m = 3
    if case == "rp0":
        rp = [1, 2, 3, 3]
    elif case == "rpn":
        rp = [0, 2, 3, 2]
    elif case == "decreasing":
        rp = [0, 2, 1, 3]
    elif case == "col_range":
        col = [1, 3, 0]
    elif case == "self_loop":
        col = [0, 2, 0]
    elif case == "repeat":
        col = [2, 2, 0]
    elif case == "unsorted":
        col = [2, 1, 0]
    elif case == "zero_weight":
        w = [1, 0, 1]
    elif case == "n0":
        n = 0
    elif case == "neg_m":
        m = -1
    rc, h = _load(n, m, rp, col, w)
    assert rc == expect, (case, rc, bcd.last_error())
    assert h.value is None


def test_null_arguments(lib):
    assert lib.bcd_graph_load_csr(3, 0, None, None, None, None) == bcd.BCD_ERR_INVALID_ARG
    assert lib.bcd_bc_exact(None, 0, None, None) == bcd.BCD_ERR_INVALID_ARG
    assert lib.bcd_rv(None, 0, None, 0, None) == bcd.BCD_ERR_INVALID_ARG
    assert lib.bcd_graph_free(None) == bcd.BCD_OK
    assert lib.bcd_sample_count(1.0, 0.5, 1.0, 1, None) == bcd.BCD_ERR_INVALID_ARG
    assert bcd.last_error()


def test_valid_graph_without_device_reports_device_error():
    """With no GPU, a well-formed graph fails with BCD_ERR_DEVICE (never a
    silent CPU path)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    g = gg.directed_path(5)
    rc, h = _load(g.n, g.m, g.row_ptr, g.col)
    assert rc == bcd.BCD_ERR_DEVICE


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits with a message before
    touching a device."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_bench_roofline_uses_busy_time():
    """The benchmark's roofline divides algorithmic bytes by the union of the
    launch intervals (overlapping launches on two streams count once), keeps
    the per-launch average beside it, and names the weighted forward by its
    three kernels."""
    sys.path.insert(0, ROOT)
    import bench

    class Stub:
        def __init__(self, weighted):
            self.w = weighted

        def info(self):
            return 10, 20, self.w

        def config(self):
            return bcd.Config(engine=bcd.BCD_ENGINE_BATCHED, groups=2, block=256, grid_mult=32, items=2,
                              bottom_up=0)

    fwd = {"launches": 4, "total_ms": 8.0, "union_ms": 5.0, "alg_bytes": 4e10, "vertex_pairs": 300, "items": 100}
    bwd = {"launches": 4, "total_ms": 2.0, "union_ms": 1.5, "alg_bytes": 1e10, "vertex_pairs": 0, "items": 0}
    r = bench.roofline_from_profile(Stub(False), fwd, bwd, "batched", "no-such-workload")
    assert r["kernel"] == "k_fwd_level" and r["traffic"] is None
    assert r["achieved"] == pytest.approx(4e10 / 5e-3 / 1e9)
    assert r["per_launch_achieved"] == pytest.approx(4e10 / 8e-3 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, abs=1e-4)
    assert r["avg_launch_us"] == pytest.approx(2000.0) and r["lanes_per_item"] == pytest.approx(3.0)
    w = bench.roofline_from_profile(Stub(True), fwd, bwd, "batched", "no-such-workload")
    assert w["kernel"] == "k_w_relax+k_w_count+k_w_sigma"
    # the backward dominates when its launches took longer
    b = bench.roofline_from_profile(Stub(False), bwd, fwd, "batched", "no-such-workload")
    assert b["kernel"] == "k_bwd_level"
    assert bench.roofline_from_profile(Stub(False), dict(fwd, launches=0), bwd, "batched", "x") is None


def test_bench_traffic_records_follow_their_kernel_sources(tmp_path, monkeypatch):
    """A counter-measured traffic record counts only while the sources of its
    kernel family hash to the recorded value, and only at its own workload
    and width; the weighted and unweighted families hash different files."""
    sys.path.insert(0, ROOT)
    import bench

    assert bench.kernel_sources_sha256("k_w_relax+k_w_count+k_w_sigma") != bench.kernel_sources_sha256("k_fwd_level")
    sha = bench.kernel_sources_sha256("k_fwd_level")
    prof = tmp_path / "p.md"
    prof.write_text("text\n"
                    f"traffic: kernel=k_fwd_level workload=w1 batch_width=64 bytes_per_launch=1234 sources_sha256={sha}\n"
                    "traffic: kernel=k_fwd_level workload=w2 batch_width=64 bytes_per_launch=99 sources_sha256=00\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "TRAFFIC_FILES", {"k_fwd_level": ["p.md"]})
    monkeypatch.setattr(bench, "kernel_sources_sha256", lambda kernel="k_fwd_level": sha)
    assert bench.measured_traffic("k_fwd_level", "w1", 64) == 1234.0
    assert bench.measured_traffic("k_fwd_level", "w1", 128) is None  # another width
    assert bench.measured_traffic("k_fwd_level", "w2", 64) is None   # stale sources
    assert bench.measured_traffic("k_bu_level", "w1", 64) is None    # no file for the kernel


def test_ctypes_structs_match_the_header(tmp_path):
    """Every struct the binding mirrors has the header's size and, field by
    field, the header's offsets (a C program built from include/bcd.h with
    gcc prints them)."""
    import shutil
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    pairs = {"bcd_stats": bcd.Stats, "bcd_config": bcd.Config, "bcd_sample_params": bcd.SampleParams,
             "bcd_kernel_profile": bcd.KernelProfile, "bcd_server_config": bcd.ServerConfig,
             "bcd_query": bcd.Query, "bcd_result": bcd.Result, "bcd_server_stats": bcd.ServerStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "bcd.h"', "int main(void) {"]
    for cname, py in pairs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True, timeout=120)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True, timeout=60).stdout.split("\n")
    got = {}
    for ln in out:
        if ln.strip():
            a, b, c = ln.split()
            got[(a, b)] = int(c)
    for cname, py in pairs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_serving_width_fits_budget_and_splits_evenly():
    """The serving benchmark's batch width: the widest that fits 85 % of the
    budget and is at most 8 or a multiple of 8 (R-MAT 22: 5.5 GB per group)."""
    sys.path.insert(0, ROOT)
    import bench
    per_group = 1312 * (1 << 22)  # bytes per (group, vertex) x n at R-MAT 22

    def width(workers, budget_gib, start=16):
        return bench.serving_width(lambda g: g * per_group * workers, start, budget_gib << 30)

    assert [width(w, 240) for w in (1, 2, 3, 4, 6, 8)] == [16, 16, 8, 8, 6, 4]
    assert width(6, 64) == 1 and width(2, 64) == 5  # 2 x 5 x 5.5 GB <= 0.85 x 64 GiB
    for w in range(1, 17):
        for budget in (16, 64, 128, 240, 288):
            g = width(w, budget, start=96)
            assert g >= 1 and (g <= 8 or g % 8 == 0)
            assert g == 1 or g * per_group * w <= (budget << 30) * 85 // 100
