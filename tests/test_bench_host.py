"""Host-side checks of bench.py (no GPU): the one-GPU guard, and the HBM
traffic summaries under profiles/ that the JSON line's roofline entry reads.

Each summary holds the raw FETCH_SIZE / WRITE_SIZE counters (KiB per
dispatch), the factors a copy of known size gave in the same runs, the bytes
derived from them and the hash of the kernel source they were taken on;
bench.py reports the bytes only while that hash matches the source."""
import glob
import hashlib
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _summaries():
    out = []
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.txt"))):
        vals = {}
        for line in open(path):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
        tag = os.path.basename(path)[len("traffic_"):-len(".txt")]
        out.append((tag, vals))
    return out


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("tag_vals", _summaries(), ids=[t for t, _ in _summaries()])
def test_traffic_summary_is_consistent(tag_vals):
    """Bytes = raw KiB x 1024 x the copy factor, read + write = total, the
    ratio to the algorithmic bytes as stated; the copy factors are the ones
    this memory system shows (FETCH_SIZE counts half the bytes a copy moves,
    WRITE_SIZE all of them)."""
    tag, v = tag_vals
    fs, ws = float(v["fetch_scale"]), float(v["write_scale"])
    assert abs(fs - 2.0) < 1e-3 and abs(ws - 1.0) < 1e-3
    rb, wb = int(v["read_bytes_per_launch"]), int(v["write_bytes_per_launch"])
    # the factors are printed to 5 decimals: a relative 5e-6 of slack
    assert abs(rb - float(v["fetch_size_kib_raw"]) * 1024 * fs) <= 5e-6 * rb + 1024
    assert abs(wb - float(v["write_size_kib_raw"]) * 1024 * ws) <= 5e-6 * wb + 1024
    assert int(v["hbm_bytes_per_launch"]) == rb + wb
    ratio = (rb + wb) / int(v["algorithmic_bytes_per_launch"])
    assert abs(ratio - float(v["ratio_measured_to_algorithmic"])) < 1e-4
    assert 1.0 <= ratio < 2.0
    assert len(v["kernel_source_sha256_16"]) == 16


def test_traffic_is_reported_only_for_the_source_it_was_taken_on(tmp_path, monkeypatch):
    """_traffic_from_profile returns the summary's bytes while the hash matches
    the kernel source, and None once the source differs from it."""
    sys.path.insert(0, ROOT)
    import bench
    copy = tmp_path / "repo"
    (copy / "profiles").mkdir(parents=True)
    (copy / "paper_1507_06767_amd" / "csrc").mkdir(parents=True)
    tag, v = next((t, v) for t, v in _summaries() if not t.startswith("refined256"))
    src = os.path.join(ROOT, "paper_1507_06767_amd", "csrc", "step_kernel.hpp")
    dst_src = copy / "paper_1507_06767_amd" / "csrc" / "step_kernel.hpp"
    shutil.copy(src, dst_src)
    text = open(os.path.join(ROOT, "profiles", f"traffic_{tag}.txt")).read()
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    text = "\n".join(f"kernel_source_sha256_16: {sha}" if ln.startswith("kernel_source_sha256_16:") else ln
                     for ln in text.splitlines())
    (copy / "profiles" / f"traffic_{tag}.txt").write_text(text + "\n")
    monkeypatch.setattr(bench, "ROOT", str(copy))
    assert bench._traffic_from_profile(tag) == float(v["hbm_bytes_per_launch"])
    with open(dst_src, "a") as fh:
        fh.write("\n// changed\n")
    assert bench._traffic_from_profile(tag) is None
