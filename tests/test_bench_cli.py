"""bench.py's command-line contract that needs no GPU: one GPU only."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_recorded_traffic_only_for_the_profiled_sources(tmp_path, monkeypatch):
    """roofline.traffic comes from rocprofv3 counter runs recorded with the
    SHA-1 of the kernel and runtime sources they measured: it is reported only
    while those files are unchanged, and is null otherwise."""
    import hashlib
    import json
    import shutil
    sys.path.insert(0, ROOT)
    import bench
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic_k_step3d_fwd_layered304.json")))
    assert rec["traffic_bytes_per_launch"] == (rec["fetch_bytes_per_launch"]
                                               + rec["write_bytes_per_launch"])
    assert rec.get("measured_commit")
    # the committed record names the sources it measured: it is reported
    # exactly when the tree's sources still hash to those values
    same = all(hashlib.sha1(open(os.path.join(ROOT, src), "rb").read()).hexdigest() == h
               for src, h in rec["sources_sha1"].items())
    assert bench.recorded_traffic() == (rec["traffic_bytes_per_launch"] if same else None)
    # a tree whose sources match the record, then one byte changed
    fake = tmp_path / "repo"
    os.makedirs(fake / "profiles")
    fake_rec = dict(rec, sources_sha1={})
    for src in rec["sources_sha1"]:
        os.makedirs(fake / os.path.dirname(src), exist_ok=True)
        shutil.copy(os.path.join(ROOT, src), fake / src)
        fake_rec["sources_sha1"][src] = hashlib.sha1(open(fake / src, "rb").read()).hexdigest()
    json.dump(fake_rec, open(fake / "profiles" / "traffic_k_step3d_fwd_layered304.json", "w"))
    monkeypatch.setattr(bench, "ROOT", str(fake))
    assert bench.recorded_traffic() == rec["traffic_bytes_per_launch"]
    first = next(iter(rec["sources_sha1"]))
    with open(fake / first, "a") as f:
        f.write("\n")
    assert bench.recorded_traffic() is None
