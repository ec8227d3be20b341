"""bench.py's command-line contract on the CPU: more than one GPU and a batch
that the streams do not divide are refused with a message and exit code 2,
before any GPU work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_batch_must_split_over_streams():
    r = _run("--batch", "16", "--streams", "3")
    assert r.returncode == 2
    assert "--streams" in r.stderr
    assert r.stdout == ""


def test_committed_traffic_profile_matches_kernel_sources():
    """The HBM-traffic record the bench reports was taken on the committed
    sources of the sweep kernel (else the bench reports traffic as null)."""
    import hashlib
    import json
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    rec = json.load(open(os.path.join(root, "profiles", "sgm_sweep_kernel_traffic.json")))
    h = hashlib.sha256()
    for src in rec["sources"]:
        h.update(open(os.path.join(root, src), "rb").read())
    assert rec["source_sha256"] == h.hexdigest()
    assert rec["frames_per_launch"] == 128
    # the summary it names exists and quotes the same total
    summ = open(os.path.join(root, "profiles", rec["summary"])).read()
    assert f"{rec['traffic_bytes_per_launch'] / 1e9:.2f} GB per launch" in summ
