"""Host logic of bench.py (no GPU): the one-GPU guard, the workload it times,
and the lookup of committed HBM-traffic records."""
import os
import subprocess
import sys

import numpy as np

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_workload_is_the_two_day_grid():
    w, x, nodes = bench.workload()
    assert (w.n, w.nfft, w.dt, w.days) == (344656, 1 << 20, 0.5, 2)
    assert x.shape == (344656,) and np.all(np.isfinite(x))
    assert len(nodes) == 16384
    # 1024 sky positions, each with the same 16 spindowns in [-1e-9, 0]
    assert len(np.unique(nodes["alpha"])) == 1024
    assert np.allclose(nodes["fdot"].reshape(1024, 16), np.linspace(-1e-9, 0.0, 16)[None, :], rtol=0, atol=1e-24)
    assert np.all(nodes["alpha"].reshape(1024, 16) == nodes["alpha"][::16, None])
    assert np.all(nodes["seg"] == 0) and np.all(nodes["bin_offset"] == 0)


def test_traffic_record_lookup(tmp_path, monkeypatch):
    # a record is used only for its kernel, FFT length, output kind, schedule
    # and the digest of the current kernel sources
    digest = bench.kernel_digest()
    assert len(digest) == 16 and int(digest, 16) >= 0
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "passes_traffic.md").write_text(
        "# traffic\n\n"
        "`record: kernel=k_pass1 nfft=1048576 interbin=0 schedule=C4096,batch128 digest=%s bytes_per_launch=123`\n"
        "`record: kernel=k_pass2 nfft=524288 interbin=1 schedule=C4096,batch128 digest=%s bytes_per_launch=456`\n"
        "`record: kernel=k_pass2 nfft=1048576 interbin=0 schedule=C4096,batch128 digest=0000000000000000 "
        "bytes_per_launch=789`\n" % (digest, digest))
    (prof / "other_stats.md").write_text(
        "`record: kernel=k_pass1 nfft=1048576 interbin=0 schedule=C2048,batch64 digest=%s bytes_per_launch=1`\n"
        % digest)
    monkeypatch.setattr(bench, "PROFILES", str(prof))
    sched = {"C": 4096, "batch": 128}
    assert bench.traffic_record("k_pass1", sched, 1 << 20, False) == 123.0
    assert bench.traffic_record("k_pass2", sched, 1 << 19, True) == 456.0
    # stale digest, other output kind, other schedule, other file name: no record
    assert bench.traffic_record("k_pass2", sched, 1 << 20, False) is None
    assert bench.traffic_record("k_pass1", sched, 1 << 20, True) is None
    assert bench.traffic_record("k_pass1", {"C": 2048, "batch": 64}, 1 << 20, False) is None
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path / "missing"))
    assert bench.traffic_record("k_pass1", sched, 1 << 20, False) is None
