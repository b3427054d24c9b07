"""bench.py's command-line contract and its roofline table, on the CPU (no
GPU run: only argument handling and static tables)."""
import glob
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402  (defines tables; main() runs only as a script)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout == ""   # no JSON line for a run that did not happen


def _kernels_in_sources():
    names = set()
    for path in glob.glob(os.path.join(ROOT, "paper_2106_00449_amd", "csrc", "*.hip")):
        names.update(re.findall(r"__global__(?:\s+__launch_bounds__\([^)]*\))?\s+void\s+(k_\w+)\s*\(",
                                open(path).read()))
    return names


def test_every_workload_names_an_existing_dominant_kernel():
    src = open(os.path.join(ROOT, "bench.py")).read()
    m = re.search(r'"--workload", default="rods32768", choices=\[([^\]]*)\]', src)
    assert m, "workload choices not found"
    choices = re.findall(r'"(\w+)"', m.group(1))
    kernels = _kernels_in_sources()
    assert set(bench.DOMINANT) == set(choices)
    for w, (family, kernel, nbytes) in bench.DOMINANT.items():
        assert kernel in kernels, (w, kernel)
        assert family.startswith("fft_") or family in ("spread", "interp")
        # the grid term of every dominant pass: 24 bytes per grid point
        assert nbytes(128 ** 3, 10_000) == 24 * 128 ** 3


def test_traffic_figures_belong_to_the_measured_kernels():
    # each measured traffic figure is quoted against its workload's dominant
    # kernel and must be within a factor 2 of that kernel's algorithmic bytes
    grids = {"rods1000": 128, "mixed4096": 256, "rods32768": 384}
    assert set(bench.TRAFFIC_BYTES) <= set(bench.DOMINANT)
    for w, t in bench.TRAFFIC_BYTES.items():
        if t is None:
            continue
        alg = bench.DOMINANT[w][2](grids[w] ** 3, 0)
        assert 0.5 < t / alg < 2.0, (w, t, alg)


def test_early_exit_launches_are_not_averaged():
    # one launch per solve returns at the done flag: it must not lower the
    # average that the roofline divides the algorithmic bytes by
    each = [370.0, 5.0, 372.0, 368.0, 5.5, 371.0]
    n, ms, early = bench.working_launches([x * 1e-3 for x in each])
    assert (n, early) == (4, 2)
    assert abs(ms - 1.481) < 1e-12
    assert bench.working_launches([]) == (0, 0.0, 0)
