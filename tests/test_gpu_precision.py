"""Precision at scale: the 10^6-charge water (333,333 rigid-geometry
molecules, L = 215.24 A, g = 0.3/A) at P = 100, 500 and 2000, both device
paths (FP64 throughout; FP64 phase reduction + FP32 trig + compensated rho +
FP64 virial) against the FP64 oracle on the same drawn batch of P
frequencies (i.i.d. draws of the sampler, not repeated).  The oracle sums
rho over all N particles for every frequency; forces are compared particle
by particle on a seeded sample of 10,000 particles; the virial tensor, the
isotropic pressure P2* = tr W/(3V) and the energy in full.  Tolerances:
1e-5 relative on the FP64 path, 1e-4 on the FP32 path (also for the worst
particle, see gpu_cases.errors)."""
import os

import numpy as np
import pytest

from oracle import ewald as oew
from oracle import sampler as osamp
from paper_2110_14362_amd import workloads
from tests.gpu_cases import TOL, assert_parity, errors, to_dev

pytestmark = pytest.mark.gpu

ROWS = 10000


@pytest.fixture(scope="module")
def water_1m():
    s = workloads.make("water_1m")
    s["rows"] = np.random.default_rng(2110143627).choice(len(s["q"]), ROWS, replace=False)
    return s


@pytest.mark.parametrize("P", [100, 500, 2000])
def test_precision_water_1m(gpu, water_1m, P):
    import torch
    from paper_2110_14362_amd.rbe import RBE
    s = water_1m
    N, rows, box = len(s["q"]), s["rows"], s["box"]
    m = osamp.sample_k(s["alpha"], box, P, seed=2110143628, system_id=0, step=P)
    distinct = len(np.unique(m, axis=0))
    S = osamp.box_tables(s["alpha"], box)["S"]
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    o = oew.kspace_weighted(s["pos"], s["q"], np.diag(box), s["alpha"], m, S / P,
                            coulomb=s["coulomb"], force_rows=rows, threads=threads)
    o["energy"] += oew.self_energy(s["q"], s["alpha"], s["coulomb"])
    V = float(np.prod(box))
    P2o = np.trace(o["virial"]) / (3.0 * V)
    x, y, z = (to_dev(s["pos"][:, a], gpu) for a in range(3))
    q = to_dev(s["q"], gpu)
    for prec in ("fp64", "fp32"):
        ctx = RBE(q, box, P, s["alpha"], coulomb=s["coulomb"], precision=prec, box_mode="iso",
                  seed=1, system_id=0)
        ctx.set_k(m)
        f = [torch.zeros(N, dtype=torch.float64, device=gpu) for _ in range(3)]
        vir = torch.zeros(6, dtype=torch.float64, device=gpu)
        en = torch.zeros(1, dtype=torch.float64, device=gpu)
        ctx.forces_pressure(x, y, z, *f, virial6=vir, energy=en)
        torch.cuda.synchronize()
        W6 = vir.cpu().numpy()
        W = np.array([[W6[0], W6[3], W6[4]], [W6[3], W6[1], W6[5]], [W6[4], W6[5], W6[2]]])
        F = np.stack([a.cpu().numpy() for a in f], 1)
        g = dict(forces=F[rows], virial=W, energy=float(en.cpu()[0]), rho=ctx.get_rho())
        ctx.check()
        ctx.close()
        e = errors(g, o, s["q"])
        pr = abs(np.trace(W) / (3.0 * V) - P2o) / abs(P2o)
        print("water_1m P=%d (%d distinct) %s: force %.2e (worst particle %.2e) pressure %.2e "
              "virial %.2e rho %.2e energy %.2e" % (P, distinct, prec, e["force"], e["force_max"],
                                                     pr, e["virial"], e["rho"], e["energy"]),
              flush=True)
        assert_parity(e, prec, P)
        assert pr < TOL[prec], (P, prec, pr)
        if prec == "fp64":
            assert e["force"] < 1e-10 and e["virial"] < 1e-10
        # the total force vanishes for any batch (Im |rho|^2 = 0), to rounding
        # (FP32: per-particle errors of ~1e-6 add up over 10^6 particles)
        tol = 1e-10 if prec == "fp64" else TOL[prec]
        assert np.abs(F.sum(axis=0)).max() < tol * np.sqrt((F ** 2).sum())
