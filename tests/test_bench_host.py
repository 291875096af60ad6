"""Host-side logic of bench.py, CPU only: the traffic look-up keyed to the
kernel sources and the launch shape, the bounded CPU-baseline sample, and the
one-GPU guard (no device is touched)."""
import hashlib
import json
import os
import shutil
import subprocess
import sys

import pytest

import bench
from paper_2310_07002_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _copy_tree(tmp_path):
    """profiles/ and the kernel sources under a scratch root."""
    shutil.copytree(os.path.join(ROOT, "profiles"), tmp_path / "profiles")
    shutil.copytree(os.path.join(ROOT, "paper_2310_07002_amd", "csrc"), tmp_path / "paper_2310_07002_amd" / "csrc")
    return tmp_path


def _source_hash(root, kernel):
    h = hashlib.sha256()
    for f in ("k_mfma.hip" if kernel == "k_mfma" else "k_valu.hip", "pcv_internal.h"):
        with open(os.path.join(root, "paper_2310_07002_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


@pytest.mark.parametrize("name,prec,kernel", [("c5", "bf16x3", "k_mfma"), ("c4", "bf16x3", "k_mfma"),
                                              ("c3", "fp64", "k_valu_part"), ("c2", "fp32", "k_valu_part")])
def test_traffic_follows_sources_and_launch_shape(tmp_path, monkeypatch, name, prec, kernel):
    """A counter summary keyed to the current sources gives its bytes at its
    own shape and at the other shapes it holds, nothing at a shape it does
    not hold, and nothing once the kernel's sources change."""
    w = W.make(name)
    root = _copy_tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(root))
    t = {"kernel_source_sha256_16": _source_hash(root, kernel), "launch_config": 13, "bytes_per_launch": 1.5e9,
         "other_launch_configs": {"11": {"bytes_per_launch": 1.3e9}}}
    with open(root / "profiles" / f"traffic_{w.name}_{prec}.json", "w") as f:
        json.dump(t, f)
    assert bench.traffic_from_profiles(w, prec, kernel, 13) == 1.5e9
    assert bench.traffic_from_profiles(w, prec, kernel, 11) == 1.3e9
    assert bench.traffic_from_profiles(w, prec, kernel, 99999) is None
    src = root / "paper_2310_07002_amd" / "csrc" / ("k_mfma.hip" if kernel == "k_mfma" else "k_valu.hip")
    src.write_text(src.read_text() + "\n// edited\n")
    assert bench.traffic_from_profiles(w, prec, kernel, 13) is None
    hdr = root / "paper_2310_07002_amd" / "csrc" / "pcv_internal.h"
    t["kernel_source_sha256_16"] = _source_hash(root, kernel)
    with open(root / "profiles" / f"traffic_{w.name}_{prec}.json", "w") as f:
        json.dump(t, f)
    assert bench.traffic_from_profiles(w, prec, kernel, 13) == 1.5e9
    hdr.write_text(hdr.read_text() + "\n// edited\n")
    assert bench.traffic_from_profiles(w, prec, kernel, 13) is None


def test_traffic_missing_summary_is_none(tmp_path, monkeypatch):
    root = _copy_tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(root))
    assert bench.traffic_from_profiles(W.make("c1"), "fp64", "k_valu_iter", 8) is None


def test_cpu_baseline_sample_sizes():
    """Every fold of the small workloads; 200 chains of the two GLMs."""
    for name in ("c1", "c2", "c3"):
        w = W.make(name)
        assert bench.baseline_folds(w) == w.K
    assert bench.baseline_folds(W.make("c4")) * W.make("c4").L == 200
    assert bench.baseline_folds(W.make("c5")) * W.make("c5").L == 200


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
