"""Host-side logic of bench.py (no GPU): the one-GPU guard, the kernel-source
hash that ties committed counter data to the sources it was taken on, and
the lookup of that data."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _fake_tree(tmp_path, body):
    csrc = tmp_path / "paper_2603_20889_amd" / "csrc"
    csrc.mkdir(parents=True, exist_ok=True)
    (csrc / "tsqr_k.hip").write_text(body)
    (csrc / "api.hip").write_text("int entry() { return 0; }\n")
    (tmp_path / "profiles").mkdir(exist_ok=True)
    return tmp_path


def test_source_hash_ignores_comments_and_spacing(tmp_path, monkeypatch):
    root = _fake_tree(tmp_path, "int f(int a) { return a + 1; }  // one\n")
    csrc = root / "paper_2603_20889_amd" / "csrc"
    monkeypatch.setattr(bench, "ROOT", str(root))
    h0 = bench.kernel_source_hash()
    (csrc / "tsqr_k.hip").write_text("/* reworded */\nint f(int a)   {\n  return a + 1;  // two\n}\n")
    assert bench.kernel_source_hash() == h0
    # entry-point glue is not a profiled source
    (csrc / "api.hip").write_text("int entry() { return 1; }\n")
    assert bench.kernel_source_hash() == h0
    (csrc / "tsqr_k.hip").write_text("int f(int a) { return a + 2; }\n")
    assert bench.kernel_source_hash() != h0
    h1 = bench.kernel_source_hash()
    (csrc / "gram.hip").write_text("int g() { return 0; }\n")
    assert bench.kernel_source_hash() != h1


def test_traffic_is_used_only_for_the_sources_it_was_taken_on(tmp_path, monkeypatch):
    root = _fake_tree(tmp_path, "int g() { return 0; }\n")
    monkeypatch.setattr(bench, "ROOT", str(root))
    rec = {"workload": "w", "kernel_hash": bench.kernel_source_hash(), "traffic_bytes_per_launch": 1234}
    (root / "profiles" / "tsqr_stage1_traffic.json").write_text(json.dumps(rec))
    assert bench.load_traffic("w") == 1234
    assert bench.load_traffic("other workload") is None
    (root / "paper_2603_20889_amd" / "csrc" / "tsqr_k.hip").write_text("int g() { return 1; }\n")
    assert bench.load_traffic("w") is None


def test_committed_traffic_record_is_consistent():
    """The committed record scales its counters as it says: FETCH_SIZE and
    WRITE_SIZE (KiB) times the copy-kernel factors give the bytes."""
    d = json.load(open(os.path.join(ROOT, "profiles", "tsqr_stage1_traffic.json")))
    c = d["calibration"]
    rd = d["fetch_size_kib_per_dispatch"] * 1024 * c["fetch_factor"]
    wr = d["write_size_kib_per_dispatch"] * 1024 * c["write_factor"]
    assert abs(rd - d["read_bytes_per_launch"]) <= 1e-5 * rd
    assert abs(rd + wr - d["traffic_bytes_per_launch"]) <= 1e-5 * (rd + wr)
    assert abs(c["fetch_factor"] - 1048576 / c["fetch_size_kib"]) < 1e-5
    assert d["traffic_bytes_per_launch"] >= d["algorithmic_bytes_per_launch"]


def test_committed_profiles_name_the_current_kernel_sources():
    """Every committed rocprofv3 summary, and the tuning table, was taken on
    the kernel sources as they are: a change to a profiled kernel has to come
    with new profiles."""
    import re
    h = bench.kernel_source_hash()
    prof = os.path.join(ROOT, "profiles")
    named = 0
    for fn in sorted(os.listdir(prof)):
        text = open(os.path.join(prof, fn)).read()
        for found in re.findall(r"Kernel sources hash \(bench\.py `kernel_hash`[^)]*\): ([0-9a-f]{16})", text):
            assert found == h, "%s was taken on %s, the sources are now %s" % (fn, found, h)
            named += 1
    assert named >= 6
    assert json.load(open(os.path.join(prof, "tsqr_stage1_traffic.json")))["kernel_hash"] == h
    table = json.load(open(os.path.join(ROOT, "paper_2603_20889_amd", "tuning_gfx950.json")))
    assert table["kernel_hash"] == h


def test_host_threads_follows_affinity_and_omp_cap(monkeypatch):
    avail = len(os.sched_getaffinity(0))
    monkeypatch.delenv("OMP_NUM_THREADS", raising=False)
    assert bench.host_threads() == (avail, avail)
    monkeypatch.setenv("OMP_NUM_THREADS", "1")
    assert bench.host_threads() == (1, avail)
    monkeypatch.setenv("OMP_NUM_THREADS", str(avail + 5))
    assert bench.host_threads() == (avail, avail)
    monkeypatch.setenv("OMP_NUM_THREADS", "junk")
    assert bench.host_threads() == (avail, avail)
