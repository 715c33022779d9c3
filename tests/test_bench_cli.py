"""bench.py on the CPU: the benchmark measures one GPU, and asking for more
exits with a message before anything touches a device; the HBM traffic it
reports comes only from counter summaries taken on the current kernel
source."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_only_from_the_current_kernel_source(tmp_path, monkeypatch):
    # roofline.traffic comes from a committed counter summary only while the
    # kernel source it was taken on is unchanged; otherwise it is null
    sys.path.insert(0, ROOT)
    import bench
    src = tmp_path / "k.hip"
    src.write_text("// kernel v1\n")
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "KERNEL_SRC", str(src))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h = bench.kernel_hash()
    (tmp_path / "profiles" / "traffic_adaptive_c2.txt").write_text(
        f"# counters\nkernel_source_sha256_16: {h}\nhbm_bytes_per_launch: 2.5e9\n")
    assert bench.read_traffic("adaptive", "c2") == 2.5e9
    assert bench.read_traffic("adaptive", "c4") is None          # no summary for that workload
    src.write_text("// kernel v2\n")
    assert bench.read_traffic("adaptive", "c2") is None          # taken on another source


def test_committed_traffic_summaries_are_well_formed():
    import re
    d = os.path.join(ROOT, "profiles")
    names = [f for f in os.listdir(d) if f.startswith("traffic_")]
    assert names
    for f in names:
        text = open(os.path.join(d, f)).read()
        assert re.search(r"kernel_source_sha256_16:\s*[0-9a-f]{16}\b", text), f
        m = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
        assert m and float(m.group(1)) > 0, f
