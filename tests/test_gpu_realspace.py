"""Real-space pair kernels vs the FP64 brute-force oracle (nearest image,
cutoff), with and without the Lennard-Jones term.  Tolerance 1e-10 relative
for FP64 pair arithmetic (differences are rounding order only); 2e-5 for the
FP32 option (single-precision erfc, exp and 1/sqrt, a few ulp each; FP32 sums
over one particle's pairs)."""
import math

import numpy as np
import pytest

from oracle import realspace as orsp
from paper_2110_14362_amd import workloads

pytestmark = pytest.mark.gpu

# SPC/E oxygen-oxygen Lennard-Jones (sigma 3.166 A, epsilon 0.1553 kcal/mol)
SIG_O, EPS_O = 3.166, 0.1553


def lj_table_water():
    c12 = np.zeros((2, 2)); c6 = np.zeros((2, 2))
    c12[0, 0] = 4 * EPS_O * SIG_O ** 12
    c6[0, 0] = 4 * EPS_O * SIG_O ** 6
    return c12, c6


def water_types(n):
    return (np.arange(n) % 3 != 0).astype(np.int32)      # O = 0, H = 1


TOLR = {"fp64": 1e-10, "fp32": 2e-5}


def make_ctx(s, dev, rc, lj=None, types=None, precision="fp64", skin=0.0):
    import torch
    from paper_2110_14362_amd.rbe import RealSpace
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    lj_arr = None if lj is None else np.stack(lj, axis=-1)
    tt = None if types is None else torch.tensor(types, dtype=torch.int32, device=dev)
    ctx = RealSpace(t(s["q"]), s["box"], s["alpha"], rc, coulomb=s.get("coulomb", 1.0),
                    types=tt, lj=lj_arr, precision=precision)
    if skin > 0.0:
        ctx.set_skin(skin)
    return ctx


def evaluate(ctx, dev, pos, accumulate=False, f0=None):
    import torch
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    x, y, z = (t(pos[:, a]) for a in range(3))
    f = [t(f0[:, a]) if f0 is not None else torch.zeros_like(x) for a in range(3)]
    vir = torch.zeros(6, dtype=torch.float64, device=dev)
    en = torch.zeros(1, dtype=torch.float64, device=dev)
    ctx.forces(x, y, z, *f, accumulate=accumulate, virial6=vir, energy=en)
    ctx.check()
    W6 = vir.cpu().numpy()
    W = np.array([[W6[0], W6[3], W6[4]], [W6[3], W6[1], W6[5]], [W6[4], W6[5], W6[2]]])
    return dict(forces=np.stack([a.cpu().numpy() for a in f], 1), virial=W,
                energy=float(en.cpu()[0]))


def run_gpu(s, dev, rc, lj=None, types=None, accumulate=False, f0=None, shift=None,
            precision="fp64", skin=0.0):
    pos = s["pos"] if shift is None else s["pos"] + shift
    ctx = make_ctx(s, dev, rc, lj=lj, types=types, precision=precision, skin=skin)
    out = evaluate(ctx, dev, pos, accumulate=accumulate, f0=f0)
    ctx.close()
    return out


def oracle(s, rc, lj=None, types=None, rows=None):
    o = orsp.realspace_nearest(s["pos"], s["q"], s["box"], s["alpha"], rc,
                               coulomb=s.get("coulomb", 1.0), rows=rows)
    if lj is not None:
        l = orsp.lj_nearest(s["pos"], types, s["box"], lj[0], lj[1], rc, rows=rows)
        o["forces"] = o["forces"] + l["forces"]
        if rows is None:
            o["energy"] += l["energy"]
            o["virial"] = o["virial"] + l["virial"]
    return o


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_electrolyte_coulomb(gpu, precision):
    s = workloads.make("electrolyte_1k")
    g = run_gpu(s, gpu, 6.0, precision=precision)
    o = oracle(s, 6.0)
    print("electrolyte real space %s: force %.2e virial %.2e energy %.2e" %
          (precision, rel(g["forces"], o["forces"]), rel(g["virial"], o["virial"]),
           abs(g["energy"] - o["energy"]) / abs(o["energy"])))
    tol = TOLR[precision]
    assert rel(g["forces"], o["forces"]) < tol
    assert rel(g["virial"], o["virial"]) < tol
    assert abs(g["energy"] - o["energy"]) < tol * abs(o["energy"])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("skin", [0.0, 1.0])
def test_wide_splitting_takes_the_full_erfcx_series(gpu, precision, skin):
    # sqrt(alpha) rc = 5.4 lies beyond the bounded-range erfcx series (x <= 4)
    # that the other cases take: the cell and list kernels then evaluate the
    # series over all x >= 0
    s = dict(workloads.make("electrolyte_1k"))
    s["alpha"] = 0.81
    g = run_gpu(s, gpu, 6.0, precision=precision, skin=skin)
    o = oracle(s, 6.0)
    print("wide splitting %s skin %.1f: force %.2e virial %.2e energy %.2e" %
          (precision, skin, rel(g["forces"], o["forces"]), rel(g["virial"], o["virial"]),
           abs(g["energy"] - o["energy"]) / abs(o["energy"])))
    tol = TOLR[precision]
    assert rel(g["forces"], o["forces"]) < tol
    assert rel(g["virial"], o["virial"]) < tol
    assert abs(g["energy"] - o["energy"]) < tol * abs(o["energy"])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_splitting_at_the_bounded_series_range_end(gpu, precision):
    # sqrt(alpha) rc = 4 exactly (rc = 8 = 2 L / 5, alpha = 0.25): the FP64
    # kernels take the bounded-range erfcx series up to the end of its range
    s = dict(workloads.make("electrolyte_1k"))
    s["alpha"] = 0.25
    assert np.sqrt(s["alpha"]) * 8.0 == 4.0
    g = run_gpu(s, gpu, 8.0, precision=precision)
    o = oracle(s, 8.0)
    print("g rc = 4 %s: force %.2e virial %.2e energy %.2e" %
          (precision, rel(g["forces"], o["forces"]), rel(g["virial"], o["virial"]),
           abs(g["energy"] - o["energy"]) / abs(o["energy"])))
    tol = TOLR[precision]
    assert rel(g["forces"], o["forces"]) < tol
    assert rel(g["virial"], o["virial"]) < tol
    assert abs(g["energy"] - o["energy"]) < tol * abs(o["energy"])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_water_with_lj(gpu, precision):
    s = workloads.water(1000, seed=7)
    s.update(alpha=0.09, coulomb=332.0637)
    types = water_types(len(s["q"]))
    lj = lj_table_water()
    g = run_gpu(s, gpu, 10.0, lj=lj, types=types, precision=precision)
    o = oracle(s, 10.0, lj=lj, types=types)
    print("water real space %s: force %.2e virial %.2e energy %.2e" %
          (precision, rel(g["forces"], o["forces"]), rel(g["virial"], o["virial"]),
           abs(g["energy"] - o["energy"]) / abs(o["energy"])))
    tol = TOLR[precision]
    assert rel(g["forces"], o["forces"]) < tol
    assert rel(g["virial"], o["virial"]) < tol
    assert abs(g["energy"] - o["energy"]) < tol * abs(o["energy"])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_water_30k_sampled_rows(gpu, precision):
    s = workloads.make("water_30k")
    types = water_types(len(s["q"]))
    lj = lj_table_water()
    g = run_gpu(s, gpu, 10.0, lj=lj, types=types, precision=precision)
    rows = np.random.default_rng(1).choice(len(s["q"]), 3000, replace=False)
    o = oracle(s, 10.0, lj=lj, types=types, rows=rows)
    assert rel(g["forces"][rows], o["forces"]) < TOLR[precision]
    # Newton's third law over the whole system
    tol3 = 1e-9 if precision == "fp64" else 1e-5
    assert np.abs(g["forces"].sum(0)).max() < tol3 * np.sqrt((g["forces"] ** 2).sum())


def test_unwrapped_accumulate_and_reproducible(gpu):
    s = workloads.make("electrolyte_1k")
    base = run_gpu(s, gpu, 6.0)
    shift = np.random.default_rng(2).integers(-2, 3, size=s["pos"].shape) * s["box"]
    moved = run_gpu(s, gpu, 6.0, shift=shift)
    assert rel(moved["forces"], base["forces"]) < 1e-12
    again = run_gpu(s, gpu, 6.0)
    assert np.array_equal(again["forces"], base["forces"])
    assert np.array_equal(again["virial"], base["virial"])
    f0 = np.random.default_rng(3).standard_normal(s["pos"].shape)
    acc = run_gpu(s, gpu, 6.0, accumulate=True, f0=f0)
    assert np.allclose(acc["forces"] - f0, base["forces"], rtol=1e-12, atol=1e-12)


def test_rejects_cutoff_above_two_fifths_of_box(gpu):
    # the cell grid needs at least five cells of width >= rc/2 per axis
    import torch
    from paper_2110_14362_amd.rbe import RealSpace, RBEError
    q = torch.tensor([1.0, -1.0], dtype=torch.float64, device=gpu)
    with pytest.raises(RBEError):
        RealSpace(q, (10.0, 10.0, 10.0), 0.3, 4.5)


# ---------------------------------------------------------------------------
# neighbour lists (a skin): the lists are built at the first evaluation and
# rebuilt only when 2 max|displacement| + sqrt(3) max|box change| reaches the
# skin; every evaluation must still equal the brute-force sum at rc.

def moved(pos, rng, step):
    """pos with every particle moved by exactly `step` in a random direction."""
    d = rng.standard_normal(pos.shape)
    return pos + step * d / np.linalg.norm(d, axis=1, keepdims=True)


def check_frame(g, o, tol, what):
    print("%s: force %.2e virial %.2e energy %.2e" %
          (what, rel(g["forces"], o["forces"]), rel(g["virial"], o["virial"]),
           abs(g["energy"] - o["energy"]) / abs(o["energy"])), flush=True)
    assert rel(g["forces"], o["forces"]) < tol
    assert rel(g["virial"], o["virial"]) < tol
    assert abs(g["energy"] - o["energy"]) < tol * abs(o["energy"])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_lists_follow_moves_and_box_changes(gpu, precision):
    s = workloads.make("electrolyte_1k")          # L = 20, rc = 6: skin up to 2
    rc, skin = 6.0, 1.5
    rng = np.random.default_rng(41)
    box0 = np.asarray(s["box"], dtype=np.float64)
    p0 = s["pos"]
    p1 = moved(p0, rng, 0.2 * skin)               # 2 x 0.3 < 1.5: lists kept
    p2 = moved(p0, rng, 0.6 * skin)               # 2 x 0.9 >= 1.5: rebuilt
    box3 = box0 * 1.003                           # scaled cell and positions: kept
    p3 = p2 * 1.003
    shift = rng.integers(-1, 2, size=p0.shape) * box3
    p4 = p3 + shift                               # images of p3: rebuilt, same forces
    frames = [(p0, box0, "first build"), (p1, box0, "lists kept"), (p2, box0, "rebuilt"),
              (p3, box3, "scaled cell, lists kept"), (p4, box3, "whole-box jumps")]
    ctx = make_ctx(s, gpu, rc, precision=precision, skin=skin)
    tol = TOLR[precision]
    for pos, box, what in frames:
        if box is not box0:
            ctx.set_box(box)
        g = evaluate(ctx, gpu, pos)
        o = orsp.realspace_nearest(pos, s["q"], box, s["alpha"], rc, coulomb=s["coulomb"])
        check_frame(g, o, tol, "%s %s" % (precision, what))
    assert ctx.list_stats() == (5, 3)
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_lists_water_with_lj(gpu, precision):
    s = workloads.water(1000, seed=7)
    s.update(alpha=0.09, coulomb=332.0637)
    types = water_types(len(s["q"]))
    lj = lj_table_water()
    rc, skin = 10.0, 2.0                          # L = 31.0: 2.5 (rc + skin) fits
    ctx = make_ctx(s, gpu, rc, lj=lj, types=types, precision=precision, skin=skin)
    rng = np.random.default_rng(43)
    for k, step in enumerate((0.0, 0.3 * skin, 0.45 * skin)):
        pos = moved(s["pos"], rng, step) if step > 0 else s["pos"]
        g = evaluate(ctx, gpu, pos)
        sk = dict(s, pos=pos)
        check_frame(g, oracle(sk, rc, lj=lj, types=types), TOLR[precision],
                    "water lists %s frame %d" % (precision, k))
    assert ctx.list_stats() == (3, 1)
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_lists_water_30k_sampled_rows(gpu, precision):
    s = workloads.make("water_30k")
    types = water_types(len(s["q"]))
    lj = lj_table_water()
    cells = run_gpu(s, gpu, 10.0, lj=lj, types=types, precision=precision)
    g = run_gpu(s, gpu, 10.0, lj=lj, types=types, precision=precision, skin=2.0)
    rows = np.random.default_rng(5).choice(len(s["q"]), 3000, replace=False)
    o = oracle(s, 10.0, lj=lj, types=types, rows=rows)
    assert rel(g["forces"][rows], o["forces"]) < TOLR[precision]
    # the same pairs as the cell path's
    assert rel(g["forces"], cells["forces"]) < TOLR[precision]
    assert rel(g["virial"], cells["virial"]) < TOLR[precision]


def test_list_overflow_is_flagged(gpu):
    # 300 particles packed in a 3 A ball: far more neighbours than the
    # capacity sized from the mean density; the host check reports it
    from paper_2110_14362_amd.rbe import RBEError
    rng = np.random.default_rng(47)
    n = 300
    d = rng.standard_normal((n, 3))
    pos = 10.0 + 3.0 * d / np.linalg.norm(d, axis=1, keepdims=True) * rng.random((n, 1))
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    s = dict(pos=pos, q=q, box=np.array([20.0, 20.0, 20.0]), alpha=0.09, coulomb=1.0)
    ctx = make_ctx(s, gpu, 6.0, skin=1.0)
    with pytest.raises(RBEError):
        evaluate(ctx, gpu, pos)
    ctx.close()


def test_skin_rejected_when_box_too_small(gpu):
    import torch
    from paper_2110_14362_amd.rbe import RealSpace, RBEError
    q = torch.tensor([1.0, -1.0], dtype=torch.float64, device=gpu)
    ctx = RealSpace(q, (20.0, 20.0, 20.0), 0.3, 6.0)
    with pytest.raises(RBEError):
        ctx.set_skin(2.5)                         # 2.5 x 8.5 > 20
    ctx.close()
