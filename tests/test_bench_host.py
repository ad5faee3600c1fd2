"""Host logic of bench.py, no GPU: the one-GPU guard, and the rule that the HBM traffic recorded
under profiles/ is reported only while the kernel's sources and build flags are the ones it was
measured with."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def run_bench(args, **env):
    e = dict(os.environ, **env)
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, env=e)


def test_more_than_one_gpu_is_refused():
    r = run_bench(["--gpus", "2"])
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_a_multi_rank_launch_is_refused():
    r = run_bench([], WORLD_SIZE="2")
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_recorded_traffic_follows_the_kernel_sources(tmp_path, monkeypatch):
    name, files = bench.TRAFFIC_RECORDS["pair_integral_adjoint"]
    sha = bench.kernel_sources_sha256(files)
    (tmp_path / "profiles").mkdir()
    rec = tmp_path / "profiles" / name
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))

    rec.write_text(f"fetch_bytes_per_launch: 123\nwrite_bytes_per_launch: 45\nsource_sha256: {sha}\n")
    assert bench.recorded_traffic("pair_integral_adjoint", 128) == (123.0, 45.0, "profiles/" + name)
    # measured at G=128 only
    assert bench.recorded_traffic("pair_integral_adjoint", 64) is None
    # a record taken from other sources (one hex digit changed) is stale
    other = ("0" if sha[0] != "0" else "1") + sha[1:]
    rec.write_text(f"fetch_bytes_per_launch: 123\nwrite_bytes_per_launch: 45\nsource_sha256: {other}\n")
    assert bench.recorded_traffic("pair_integral_adjoint", 128) is None
    # incomplete records and unknown kernels give nothing
    rec.write_text(f"fetch_bytes_per_launch: 123\nsource_sha256: {sha}\n")
    assert bench.recorded_traffic("pair_integral_adjoint", 128) is None
    assert bench.recorded_traffic("no_such_kernel", 128) is None


def test_the_hash_covers_the_build_flags():
    for _, files in bench.TRAFFIC_RECORDS.values():
        assert "../build.py" in files
        assert all(os.path.exists(os.path.join(bench.CSRC, f)) for f in files)
