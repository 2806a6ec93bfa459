"""Host-side checks of the benchmark driver (no GPU needed)."""

import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), (["--gpus", "8"], {}), ([], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_is_refused_before_any_device_work(argv, env):
    """A request for several GPUs ends with a message and exit status 2
    before torch or the library is imported."""
    e = dict(os.environ, **env)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], capture_output=True, text=True,
                       env=e, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_traffic_summary_is_tied_to_the_sources(tmp_path, monkeypatch):
    """The committed counter summary is used only while the hash of the
    kernel sources and build flags matches; a summary taken on other sources
    reads as missing, and so does one after any source byte changes."""
    import shutil
    name = "sweep_d3q19_trt_256_f64_traffic.txt"
    path = os.path.join(ROOT, "profiles", name)
    if os.path.exists(path):
        kv = dict(l.strip().split("=", 1) for l in open(path) if "=" in l and not l.startswith("#"))
        assert set(kv) >= {"source_sha", "hbm_bytes_per_launch"}
    pkg = tmp_path / "paper_2001_11806_amd"
    shutil.copytree(os.path.join(ROOT, "paper_2001_11806_amd", "csrc"), pkg / "csrc")
    shutil.copy(os.path.join(ROOT, "paper_2001_11806_amd", "build.py"), pkg / "build.py")
    (tmp_path / "profiles").mkdir()
    prof = tmp_path / "profiles" / name
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    sha = bench.source_hash()
    prof.write_text("source_sha=0000000000000000\nhbm_bytes_per_launch=123.0\n")
    assert bench.read_traffic(name) is None
    prof.write_text("source_sha=%s\nhbm_bytes_per_launch=123.0\n" % sha)
    assert bench.read_traffic(name) == 123.0
    with open(pkg / "build.py", "a") as f:
        f.write("\n")
    assert bench.read_traffic(name) is None


def test_attach_lines_relates_each_workload_to_its_lines(monkeypatch):
    """Each workload is divided by the copy and pull-stream lines of its own
    launch shape, and the AA workload also by the AA pattern's line."""
    monkeypatch.setattr(bench, "read_traffic", lambda name: None)
    extras = {k: {"GBps": 1000.0 + i} for i, k in enumerate(bench.LINES)}
    for w in bench.MATCH:
        extras[w] = {"achieved_GBps": 900.0}
    bench.attach_lines(extras)
    for w, (line, sline, _) in bench.MATCH.items():
        r = extras[w]
        if line is None:    # the adjoint workload: counters only, no line of its own
            assert "copy_line" not in r and "stream_line" not in r and r["traffic"] is None
            continue
        assert line in bench.LINES and sline in bench.LINES
        assert r["copy_line"] == line and r["frac_of_copy_line"] == pytest.approx(900.0 / extras[line]["GBps"])
        assert r["stream_line"] == sline
        assert r["frac_of_stream_line"] == pytest.approx(900.0 / extras[sline]["GBps"])
        assert bench.LINES[line][0] == "copy" and bench.LINES[sline][0] == "stream"
        assert bench.LINES[line][5:] == bench.LINES[sline][5:]     # same waves per CU and block
        aline = bench.AA_LINE.get(w)
        if aline:
            assert bench.LINES[aline][0] == "aa" and bench.LINES[aline][5:] == bench.LINES[sline][5:]
            assert r["frac_of_aa_line"] == pytest.approx(900.0 / extras[aline]["GBps"])
        else:
            assert "frac_of_aa_line" not in r
        assert r["traffic"] is None
