"""Host-side logic that needs no GPU: the served stream's request recipe
(cutoff, splitting parameter, neighbour-list skin that the cell allows),
Poisson arrivals, and the benchmark's refusal of several GPUs."""
import math
import os
import subprocess
import sys

import numpy as np

from paper_2110_14362_amd import serve, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_list_skin_fits_the_cell():
    # the kernels need every side >= 2.5 (rc + skin); the recipe keeps 2.6
    for L, rc, want in ((66.88, 10.0, 2.0), (31.0, 10.0, 1.0), (22.0, 6.6, 1.0),
                        (17.0, 6.5, 0.0)):
        s = workloads.list_skin((L, L, 1.25 * L), rc, want)
        assert 0.0 <= s <= want
        if s > 0.0:
            assert L >= 2.6 * (rc + s) - 1e-12
            assert s >= 0.1
        else:
            assert L / 2.6 - rc < 0.1


def test_served_requests_keep_erfc_at_the_cutoff():
    reqs = serve.make_requests(16, seed=123, nmin=1000, nmax=60000, kinds=("ions", "water"),
                               skin=1.0)
    g0, rc0 = 0.3, 10.0
    for r in reqs:
        s = r.sysd
        box = np.asarray(s["box"])
        assert s["rc"] <= rc0 + 1e-12 and box.min() >= 3.3 * s["rc"] - 1e-9
        # erfc(g rc) unchanged where the cutoff had to shrink
        assert abs(math.sqrt(s["alpha"]) * s["rc"] - g0 * rc0) < 1e-12
        assert abs(float(np.sum(s["q"]))) < 1e-9
        skin = r.md.get("skin", 0.0)
        assert box.min() >= 2.6 * (s["rc"] + skin) - 1e-9
        assert r.desc.skin == skin and r.desc.n == len(s["q"])
        if s["kind"] == "water":
            assert r.n % 3 == 0 and r.desc.rigid_count == r.n // 3


def test_poisson_arrivals_rate():
    t = serve.poisson_arrivals(20000, rate=250.0, seed=5)
    assert np.all(np.diff(t) > 0)
    assert abs(len(t) / t[-1] / 250.0 - 1.0) < 0.03


def test_bench_refuses_several_gpus():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr
