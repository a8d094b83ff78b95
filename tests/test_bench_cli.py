"""bench.py on the CPU: more than one GPU is refused with a message before
anything touches a device, and the oracle's baseline leg leaves the CPU
affinity mask as it found it."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)
    assert r.stdout.strip() == "" or not r.stdout.strip().startswith("{")


def test_cpu_baseline_restores_the_affinity_mask():
    # the oracle's leg pins the process to one core; threads started later
    # (the library's host threads, the server's workers) inherit the mask,
    # so the leg must leave it as it found it
    sys.path.insert(0, ROOT)
    import bench
    from paper_2111_12493_amd import graphgen as gg

    before = os.sched_getaffinity(0)
    r = bench.cpu_baseline(gg.rmat_graph(10, 4000, n_types=4, n_labels=4, seed=1), 4)
    assert os.sched_getaffinity(0) == before
    assert r["cores"] == 1 and r["value"] > 0
