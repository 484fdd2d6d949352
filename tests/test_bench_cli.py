"""bench.py's contract that needs no GPU: more than one GPU is refused with a
message and exit status 2, before anything touches a device; the roofline's
traffic figure is taken from a committed PMC summary only while that summary
matches the kernel source."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _bench():
    sys.path.insert(0, ROOT)
    import bench
    return bench


def test_traffic_figure_only_for_the_current_kernel_source(tmp_path):
    """The bench line's roofline.traffic comes from a committed PMC summary only
    while the summary's source hash is that of the kernel source it covers."""
    bench = _bench()
    src = tmp_path / "kernel.hpp"
    src.write_text("// kernel source\n")
    summ = tmp_path / "summary.txt"
    summ.write_text(f"# kernel_source_sha256_16: {bench.kernel_hash(str(src))}\n"
                    "hbm_bytes_per_launch: 4.896474e+09\n")
    assert bench.read_traffic(str(summ), (str(src),)) == 4.896474e9
    src.write_text("// kernel source, edited\n")
    assert bench.read_traffic(str(summ), (str(src),)) is None
    assert bench.read_traffic(str(tmp_path / "missing.txt"), (str(src),)) is None
    summ.write_text(f"# kernel_source_sha256_16: {bench.kernel_hash(str(src))}\n")
    assert bench.read_traffic(str(summ), (str(src),)) is None

