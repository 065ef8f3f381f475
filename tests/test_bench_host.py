"""Host-side logic of bench.py (no GPU): the graph size of the timed region,
the code digests that keep recorded HBM counters attached to the kernels they
measured, and the refusal to run on more than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("steps,every", [(2000, 64), (20, 64), (7, 4), (1, 64), (100, 50), (97, 64)])
def test_graph_size_divides_the_timed_region(steps, every):
    g = bench.graph_size(steps, every)
    assert 1 <= g <= min(steps, every) and steps % g == 0
    # the largest such divisor
    assert all(steps % d for d in range(g + 1, min(steps, every) + 1))


def test_source_digest_ignores_comments_and_blank_lines(tmp_path):
    a, b, c = tmp_path / "a.hip", tmp_path / "b.hip", tmp_path / "c.hip"
    a.write_text("int f(int x) {\n  return x + 1;\n}\n")
    b.write_text("// header\n/* block\n comment */\nint f(int x) {  // trailing\n\n  return x + 1;\n}\n")
    c.write_text("int f(int x) {\n  return x + 2;\n}\n")
    assert bench.source_digest(a) == bench.source_digest(b)
    assert bench.source_digest(a) != bench.source_digest(c)


def _summary(path, digests, workload="64x64 float32", traffic=123456):
    lines = ["# a comment", f"workload {workload}", f"sweep_traffic_bytes {traffic}"]
    lines += [f"source_digest {rel} {h}" for rel, h in digests.items()]
    path.write_text("\n".join(lines) + "\n")


def test_pmc_traffic_only_while_the_sources_match(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel body\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    summ = tmp_path / "profiles" / "sweep_aux_f32_64x64.txt"
    _summary(summ, {"k.hip": bench.source_digest(src)})
    assert bench.pmc_traffic(64, 64) == 123456.0
    assert bench.pmc_traffic(128, 128) is None                 # no summary for this size
    src.write_text("kernel body changed\n")
    assert bench.pmc_traffic(64, 64) is None                   # the kernel changed since
    _summary(summ, {"k.hip": bench.source_digest(src)}, workload="64x64 float64")
    assert bench.pmc_traffic(64, 64) is None                   # another workload
    _summary(summ, {})
    assert bench.pmc_traffic(64, 64) is None                   # no digests recorded


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""
