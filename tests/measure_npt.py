"""Long-run NPT statistics on the device (a measurement, not a test:
`python -m tests.measure_npt` on a GPU prints one JSON line).

Section 3 (the pressure identities of the Langevin NPT dynamics): the time
average of the instantaneous pressure equals the imposed pressure, and
<P_ins V> = P <V> - k_B T.  This runs the full device step (random batch
Fourier part, real-space pairs with a repulsive core, BAOAB integrator with
the isotropic Langevin barostat) on a 1000-ion primitive electrolyte in
reduced units and reports the averages with block-average standard errors."""
import json
import sys

import numpy as np


def note(msg):
    print("[npt] " + msg, file=sys.stderr, flush=True)


def electrolyte_core(n=1000, L=20.0, seed=5):
    """n ions (+1 / -1) on a jittered cubic lattice in an L^3 cell, unit
    masses, pure r^-12 core (c12 = 4, sigma 1), reduced units (C = 1)."""
    g = np.random.default_rng(seed)
    k = int(round(n ** (1.0 / 3.0)))
    assert k ** 3 == n
    idx = np.stack(np.meshgrid(*[np.arange(k)] * 3, indexing="ij"), -1).reshape(-1, 3)
    a = L / k
    pos = np.mod((idx + 0.5) * a + g.uniform(-0.2, 0.2, (n, 3)), L)
    q = np.where(g.permutation(n) < n // 2, 1.0, -1.0)
    s = dict(pos=pos, q=q, mass=np.ones(n), box=np.array([L, L, L]), alpha=0.3 ** 2, p=100,
             coulomb=1.0)
    md = dict(dt=0.005, kT=1.0, p_ext=0.1, gamma_p=1.0, gamma_cell=1.0,
              mass_cell=1.0 / (8.0 * 8000.0), ftm=1.0, box_mode="iso", rc=6.0,
              types=np.zeros(n, dtype=np.int32), lj=np.array([[[4.0, 0.0]]]))
    mom = g.normal(0.0, 1.0, (n, 3))
    return s, md, mom


def block_mean(x, nblocks=20):
    x = np.asarray(x)
    b = len(x) // nblocks
    m = x[:b * nblocks].reshape(nblocks, b).mean(axis=1)
    return float(m.mean()), float(m.std(ddof=1) / np.sqrt(nblocks))


def run(equil=4000, prod=20000, every=4, precision="fp32", sampler="exact", seed=11):
    from paper_2110_14362_amd.md import NPTSystem
    s, md, mom = electrolyte_core()
    if sampler != "exact":
        md["sampler"] = sampler
    sysg = NPTSystem(s, md, precision=precision, seed=seed, system_id=1, momenta=mom)
    sysg.step(equil)
    sysg.check()
    P, V, T = [], [], []
    n = len(s["q"])
    for _ in range(prod // every):
        sysg.step(every)
        st = sysg.integ.state()
        P.append(np.trace(st["pressure"]) / 3.0)
        V.append(st["volume"])
        T.append(np.trace(st["kinetic"]) / (3.0 * n))
    sysg.check()
    P, V, T = np.array(P), np.array(V), np.array(T)
    pm, pse = block_mean(P)
    vm, vse = block_mean(V)
    tm, tse = block_mean(T)
    pv, pvse = block_mean(P * V - md["p_ext"] * V)
    return dict(p_ext=md["p_ext"], kT=md["kT"], steps=prod, dt=md["dt"], precision=precision,
                sampler=sampler, p_mean=pm, p_se=pse, v_mean=vm, v_se=vse, t_mean=tm, t_se=tse,
                pv_minus_p_v=pv, pv_minus_p_v_se=pvse)


if __name__ == "__main__":
    out = []
    for prec in ("fp32", "fp64"):
        r = run(precision=prec)
        note("%s: <P_ins> = %.5f +- %.5f (P = %.3f), <V> = %.1f +- %.1f, <T> = %.4f +- %.4f, "
             "<P_ins V> - P <V> = %.4f +- %.4f (-kT = %.3f)"
             % (prec, r["p_mean"], r["p_se"], r["p_ext"], r["v_mean"], r["v_se"], r["t_mean"],
                r["t_se"], r["pv_minus_p_v"], r["pv_minus_p_v_se"], -r["kT"]))
        out.append(r)
    print(json.dumps({"npt_statistics": out}), flush=True)
