"""Host logic of bench.py that needs no GPU.

* The committed HBM-traffic record is used only while the kernel's source is
  byte-for-byte the one the counters were taken with: with the repository's
  own files the dominant kernel's record is returned, and a copy of the tree
  whose kernel source differs by one byte gets None.
* The algorithmic byte counts per site follow the formulas the bench states
  (compulsory links, spinors, clover records, FP16 scales).
* --gpus N with N > 1 is refused with a message, before anything touches a GPU.
"""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_traffic_record_follows_the_source(tmp_path, monkeypatch):
    import hashlib
    name = "k_coarse_gcr_site<float>"
    src = open(os.path.join(ROOT, "paper_1011_2775_amd", "csrc", "coarse_persist.hip"), "rb").read()
    # the repository's own record: used exactly when its hash matches the source
    rec = json.load(open(os.path.join(ROOT, "profiles", "hbm_traffic.json")))["kernels"]
    if name in rec:
        fresh = hashlib.sha256(src).hexdigest() == rec[name]["source_sha256"]
        assert bench.measured_traffic(name) == (rec[name]["bytes_per_launch"] if fresh else None)
    # a tree with a record taken on this source, then the source changed by one byte
    (tmp_path / "profiles").mkdir()
    record = {"kernels": {name: {"bytes_per_launch": 12345, "source_sha256": hashlib.sha256(src).hexdigest(),
                                 "sources": ["coarse_persist.hip"]}}}
    (tmp_path / "profiles" / "hbm_traffic.json").write_text(json.dumps(record))
    csrc = tmp_path / "paper_1011_2775_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "coarse_persist.hip").write_bytes(src)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic(name) == 12345
    (csrc / "coarse_persist.hip").write_bytes(src + b"\n")
    assert bench.measured_traffic(name) is None
    assert bench.measured_traffic("no_such_kernel") is None


def test_algorithmic_bytes_per_site():
    # FP64 DIAG = 1 hop: neighbour spinor, links, output, diagonal input
    assert bench.dslash_bytes_per_site(0, 1, False) == (24 + 144 + 24 + 24) * 8
    # FP32 POSTINV hop: plus the 72-real clover inverse record
    assert bench.dslash_bytes_per_site(1, 0, True) == (24 + 144 + 24 + 72) * 4
    # FP16 DIAG = 2 hop: halves, plus one FP32 scale per spinor read or written
    assert bench.dslash_bytes_per_site(2, 2, False) == (24 + 144 + 24 + 24 + 72) * 2 + 4 * 3
    # D_r per even site: 5 spinor passes, 16 links, 2 clover records; fields shared by the batch
    assert [bench.dr_compulsory_bytes(p) for p in (0, 1, 2)] == [4416, 2208, 1104 + 20]
    assert bench.dr_compulsory_bytes(1, 12) == 1728 / 12 + 480
    assert bench.clover_bytes_per_site(0) == 120 * 8
    # a persistent coarse GCR step: both half hops and ten vector passes
    assert bench.coarse_step_bytes(256, 48) == 256 * (2 * 8 * 48 * 48 + 10 * 48) * 8


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode != 0
    assert "single GPU" in p.stderr and "--gpus 2" in p.stderr


def test_kernel_table_names_the_launched_hop_variant():
    """The hop rows name the kernel the library launches at that volume: the
    unpinned small-grid variant at 16^3x32, the pinned one at 24^3x64."""
    class Ctx:
        def timer_read(self, kid):
            return (4, 0.1) if kid in (7, 8) else (0, 0.0)
    small = bench.kernel_table([Ctx()], 16 ** 3 * 32 // 2, 256, 48)
    large = bench.kernel_table([Ctx()], 24 ** 3 * 64 // 2, 256, 48)
    assert {r["kernel"] for r in small} == {"dslash_kernel_wide<float,0,true>", "dslash_kernel_wide<float,1,false>"}
    assert {r["kernel"] for r in large} == {"dslash_kernel<float,0,true>", "dslash_kernel<float,1,false>"}
