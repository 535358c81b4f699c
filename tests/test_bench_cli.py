"""Host-side checks of bench.py (no GPU): the multi-GPU refusal and the
stored-counter lookup."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_stored_counters_follow_the_code_digest(tmp_path, monkeypatch):
    digest = "a" * 16
    # an entry recorded for other device code is never reported
    fake = {"k1_local_merge@w": {"bytes_per_launch": 1, "code_digest": "0" * 16}}
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "counters.json").write_text(json.dumps(fake))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "device_code_digest", lambda: digest)
    assert bench.stored_counters("k1_local_merge", "w") is None
    fake["k1_local_merge@w"]["code_digest"] = digest
    (prof / "counters.json").write_text(json.dumps(fake))
    assert bench.stored_counters("k1_local_merge", "w")["bytes_per_launch"] == 1


def test_device_code_digest_reads_the_fatbin_section():
    import hashlib

    lib = os.path.join(ROOT, "paper_1708_08180_amd", "libccl.so")
    fat = bench.elf_section(lib, ".hip_fatbin")
    assert len(fat) > 4096
    assert bench.device_code_digest() == hashlib.sha256(fat).hexdigest()[:16]
