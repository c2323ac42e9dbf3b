"""Host logic of bench.py, on the CPU: the one-GPU guard and the rule that the
committed counter summary is reported only for the sources it was taken on."""
from __future__ import annotations

import hashlib
import json
import os
import subprocess
import sys

import bench

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def _fake_root(tmp_path, sources, summary):
    csrc = tmp_path / "paper_2401_13185_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name, text in sources.items():
        (csrc / name).write_text(text)
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "gram_hbm_traffic.txt").write_text(summary)


def test_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    sources = {"gram.hip": "g", "api.hip": "a", "internal.h": "i"}
    digest = hashlib.sha256(b"g" + b"a" + b"i").hexdigest()
    summary = ("# comment: ignored\n"
               "kernel: gram_kernel<0, 128>\n"
               "workload: spectra N=100000 K=512 M=8 P=10 fp64\n"
               "fetch_bytes_scaled: 1000\n"
               "write_bytes_scaled: 234\n"
               f"source_sha256: {digest}\n")
    _fake_root(tmp_path, sources, summary)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.source_digest() == digest
    wl = "spectra N=100000 K=512 M=8 P=10 fp64"
    assert bench.profiled_traffic("gram_kernel<0, 128>", wl) == 1234.0
    # another kernel or workload than the one measured: nothing to report
    assert bench.profiled_traffic("gram_kernel<0, 64>", wl) is None
    assert bench.profiled_traffic("gram_kernel<0, 128>", "offset N=1000000") is None
    # the sources changed after the counters were taken: stale, not reported
    (tmp_path / "paper_2401_13185_amd" / "csrc" / "api.hip").write_text("a2")
    assert bench.profiled_traffic("gram_kernel<0, 128>", wl) is None


def test_committed_summary_names_its_sources():
    # the committed summary carries a hash of the three sources it covers
    kv = {}
    with open(os.path.join(ROOT, "profiles", "gram_fp64_large_hbm_traffic.txt")) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    assert len(kv["source_sha256"]) == 64
    assert float(kv["fetch_bytes_scaled"]) > 0 and float(kv["write_bytes_scaled"]) > 0
