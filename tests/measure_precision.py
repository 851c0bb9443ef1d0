"""Precision sweep of the Fourier-space path at scale (a measurement, not a
test: `python -m tests.measure_precision` on a GPU prints one JSON line).

The 10^6-charge water (333,333 molecules, L = 215.24 A, g = 0.3/A) for
P = 100, 500, 2000: both device paths (FP64; FP32 trig with the exact phase
reduction and compensated sums) against the FP64 oracle on the same drawn
batch.  Lives under tests/ because it runs the oracle."""
import json
import sys
import time

import numpy as np


def note(msg):
    print("[precision] " + msg, file=sys.stderr, flush=True)


def precision_sweep(torch):
    """Errors of both device paths against the FP64 oracle on the 10^6-charge
    water (333,333 molecules, L = 215.24 A, g = 0.3/A) for P = 100, 500, 2000:
    the same drawn batch on both sides; the oracle's rho over all N, forces on a
    seeded 10,000-particle subsample."""
    from oracle import ewald as oew
    from oracle import sampler as osamp
    from paper_2110_14362_amd import workloads
    from paper_2110_14362_amd.rbe import RBE
    dev = torch.device("cuda:0")
    s = workloads.make("water_1m")
    N = len(s["q"])
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    x, y, z, q = t(s["pos"][:, 0]), t(s["pos"][:, 1]), t(s["pos"][:, 2]), t(s["q"])
    rows = np.random.default_rng(2110143627).choice(N, 10000, replace=False)
    h = np.diag(s["box"])
    S = osamp.box_tables(s["alpha"], s["box"])["S"]
    V = float(np.prod(s["box"]))
    out = []
    for P in (100, 500, 2000):
        m = osamp.sample_k(s["alpha"], s["box"], P, seed=2110143628, system_id=0, step=P)
        t0 = time.perf_counter()
        o = oew.kspace_weighted(s["pos"], s["q"], h, s["alpha"], m, S / P, coulomb=s["coulomb"],
                                force_rows=rows)
        t_or = time.perf_counter() - t0
        Fo = o["forces"]
        Po = np.trace(o["virial"]) / (3.0 * V)
        for prec in ("fp64", "fp32"):
            ctx = RBE(q, s["box"], P, s["alpha"], coulomb=s["coulomb"], precision=prec,
                      box_mode="iso", seed=1, system_id=0)
            ctx.set_k(m)
            f = [torch.zeros(N, dtype=torch.float64, device=dev) for _ in range(3)]
            vir = torch.zeros(6, dtype=torch.float64, device=dev)
            en = torch.zeros(1, dtype=torch.float64, device=dev)
            ctx.forces_pressure(x, y, z, *f, accumulate=False, virial6=vir, energy=en)
            torch.cuda.synchronize()
            Fg = np.stack([a.cpu().numpy() for a in f], 1)[rows]
            W6 = vir.cpu().numpy()
            Wg = np.array([[W6[0], W6[3], W6[4]], [W6[3], W6[1], W6[5]], [W6[4], W6[5], W6[2]]])
            rho = ctx.get_rho()
            ctx.close()
            out.append({
                "p": P, "precision": prec,
                "force_rms_rel": float(np.sqrt(((Fg - Fo) ** 2).sum() / (Fo ** 2).sum())),
                "pressure_rel": float(abs(np.trace(Wg) / (3.0 * V) - Po) / abs(Po)),
                "virial_rel": float(np.linalg.norm(Wg - o["virial"]) / np.linalg.norm(o["virial"])),
                "rho_max_rel": float(np.abs(rho - o["rho"]).max() / np.sqrt((s["q"] ** 2).sum())),
                "oracle_seconds": t_or})
            note("sweep P=%d %s: force %.2e pressure %.2e" % (P, prec, out[-1]["force_rms_rel"],
                                                               out[-1]["pressure_rel"]))
    return {"workload": "water_1m: N = %d, L = %.2f A, g = 0.3/A" % (N, s["box"][0]),
            "sample": "forces on 10,000 seeded particles; rho and virial over all N",
            "results": out}


if __name__ == "__main__":
    import torch
    print(json.dumps({"precision_sweep": precision_sweep(torch)}), flush=True)
