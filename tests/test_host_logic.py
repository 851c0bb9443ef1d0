"""Host-side logic that needs no GPU: the served stream's request recipe
(cutoff, splitting parameter, neighbour-list skin that the cell allows),
Poisson arrivals, the benchmark's refusal of several GPUs, and the generated
erfcx polynomial that the pair kernels evaluate."""
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


def _header_array(text, name):
    body = text.split(name + "[")[1].split("{", 1)[1].split("}", 1)[0]
    return [float(v.strip().rstrip("f")) for v in body.split(",") if v.strip()]


def test_erfcx_polynomial_of_the_pair_kernels():
    # the pair kernels' erfc(x) = exp(-x^2) erfcx(x) takes erfcx from the
    # generated polynomial in t = (x - K)/(x + K); checked here against
    # scipy's erfcx (an independent implementation) over the range the
    # kernels reach (x = g r up to g rc ~ 3-6) and beyond
    from scipy.special import erfcx
    text = open(os.path.join(ROOT, "paper_2110_14362_amd", "csrc", "erfcx_poly.h")).read()
    K = float(text.split("kErfcxK =")[1].split(";")[0])
    c64 = np.array(_header_array(text, "kErfcxPoly"), dtype=np.float64)
    c32 = np.array(_header_array(text, "kErfcxPoly32"), dtype=np.float32)
    assert len(c64) == int(text.split("kErfcxTerms =")[1].split(";")[0])
    assert len(c32) == int(text.split("kErfcxTerms32 =")[1].split(";")[0])
    x = np.concatenate([np.linspace(0.0, 12.0, 20001), np.geomspace(1e-8, 1.0, 2001)])
    ref = erfcx(x)
    t = (x - K) / (x + K)
    y = np.full_like(x, c64[-1])
    for c in c64[-2::-1]:
        y = y * t + c
    assert np.max(np.abs(y / ref - 1.0)) < 4e-15
    t32 = ((x.astype(np.float32) - np.float32(K)) / (x.astype(np.float32) + np.float32(K))).astype(np.float32)
    y32 = np.full_like(t32, c32[-1])
    for c in c32[-2::-1]:
        y32 = (y32 * t32 + c).astype(np.float32)
    assert np.max(np.abs(y32.astype(np.float64) / erfcx(x.astype(np.float32).astype(np.float64)) - 1.0)) < 2e-6
    # the bounded-range series (0 <= x <= XS, in u = (A x - K)/(x + K)) that
    # the FP64 kernels take when g rc <= XS
    XS = float(text.split("kErfcxShortX =")[1].split(";")[0])
    A = float(text.split("kErfcxShortA =")[1].split(";")[0])
    s64 = np.array(_header_array(text, "kErfcxPolyS"), dtype=np.float64)
    assert len(s64) == int(text.split("kErfcxTermsS =")[1].split(";")[0]) < len(c64)
    x = np.concatenate([np.linspace(0.0, XS, 40001), np.geomspace(1e-8, 1.0, 2001)])
    u = (A * x - K) / (x + K)
    assert u.min() >= -1.0 and u.max() <= 1.0 + 1e-15
    y = np.full_like(x, s64[-1])
    for c in s64[-2::-1]:
        y = y * u + c
    assert np.max(np.abs(y / erfcx(x) - 1.0)) < 4e-15


def test_exponential_table_of_the_pair_kernels():
    # the FP64 pair kernels take exp(-alpha r^2) from a table-driven
    # exponential (2^(j/64) table, ln2/64 split in two); its steps, with each
    # fused multiply-add rounded once (mpmath at 200 bits, then to FP64),
    # reproduce mpmath's exp within 2 ulp over [-745, 0]
    import math
    import random
    import mpmath as mp
    text = open(os.path.join(ROOT, "paper_2110_14362_amd", "csrc", "exp_table.h")).read()
    const = lambda name: float(text.split(name + " =")[1].split(";")[0])
    inv, hi, lo = const("kExpInvL"), const("kExpLhi"), const("kExpLlo")
    tab = _header_array(text, "kExpTab")
    assert len(tab) == 64 and tab[0] == 1.0
    mant = int(float.hex(hi).split("p")[0].split(".")[1], 16)
    assert (mant & -mant).bit_length() - 1 >= 20             # short head: n * hi exact
    mp.mp.prec = 200
    fma = lambda a, b, c: float(mp.mpf(a) * mp.mpf(b) + mp.mpf(c))

    def exp_nonpos(x):
        n = float(round(x * inv))                 # rint: ties never occur here
        r = fma(-n, lo, fma(-n, hi, x))
        ni = int(n)
        p = fma(r, 1.0 / 720.0, 1.0 / 120.0)
        for c in (1.0 / 24.0, 1.0 / 6.0, 0.5, 1.0):
            p = fma(p, r, c)
        t = tab[ni & 63]
        return math.ldexp(fma(t, p * r, t), ni >> 6)

    rng = random.Random(7)
    xs = [0.0, -1e-300, -1e-12, -0.5, -math.log(2) / 128, -10.9, -700.0, -708.3]
    xs += [-rng.uniform(0.0, 12.0) for _ in range(3000)] + [-rng.uniform(0.0, 708.0) for _ in range(1000)]
    worst = 0.0
    for x in xs:
        ref = mp.exp(mp.mpf(x))
        got = exp_nonpos(x)
        worst = max(worst, float(abs(mp.mpf(got) - ref) / (mp.mpf(2) ** (mp.floor(mp.log(ref, 2)) - 52))))
    assert worst < 2.0
    assert exp_nonpos(-800.0) == 0.0
