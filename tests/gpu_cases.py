"""Shared helpers of the GPU parity tests: run a system through the C ABI and
through the oracle on the same batch, and measure the differences."""
import numpy as np

from oracle import rbe as orbe
from oracle import sampler as osamp


def to_dev(a, dev):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)


def gpu_eval(sysd, dev, precision, p=None, m=None, step=None, seed=11, system_id=0,
             box_mode="iso", accumulate=False, f0=None, shift=None, p_pressure=0, fused=None):
    import torch
    from paper_2110_14362_amd.rbe import RBE
    pos = sysd["pos"] if shift is None else sysd["pos"] + shift
    p = int(p if p is not None else (len(m) if m is not None else sysd["p"]))
    q = to_dev(sysd["q"], dev)
    ctx = RBE(q, sysd["box"], p, sysd["alpha"], coulomb=sysd.get("coulomb", 1.0),
              precision=precision, box_mode=box_mode, seed=seed, system_id=system_id,
              p_pressure=p_pressure)
    if fused is not None:
        ctx.set_fused(fused)
    if m is not None:
        ctx.set_k(m)
    else:
        ctx.sample_k(step)
    x, y, z = (to_dev(pos[:, a], dev) for a in range(3))
    if f0 is None:
        f = [torch.zeros_like(x) for _ in range(3)]
    else:
        f = [to_dev(f0[:, a], dev) for a in range(3)]
    vir = torch.zeros(6, dtype=torch.float64, device=dev)
    en = torch.zeros(1, dtype=torch.float64, device=dev)
    ctx.forces_pressure(x, y, z, f[0], f[1], f[2], accumulate=accumulate, virial6=vir, energy=en)
    torch.cuda.synchronize()
    W6 = vir.cpu().numpy()
    W = np.array([[W6[0], W6[3], W6[4]], [W6[3], W6[1], W6[5]], [W6[4], W6[5], W6[2]]])
    out = dict(rho=ctx.get_rho(), forces=np.stack([t.cpu().numpy() for t in f], 1),
               virial=W, energy=float(en.cpu().numpy()[0]), m=ctx.get_k().astype(np.int64),
               info=ctx.get_box_info())
    ctx.close()
    return out


def oracle_eval(sysd, m):
    S = osamp.box_tables(sysd["alpha"], sysd["box"])["S"]
    return orbe.rbe_kspace(sysd["pos"], sysd["q"], sysd["box"], sysd["alpha"], m, S,
                           coulomb=sysd.get("coulomb", 1.0))


def errors(g, o, q):
    """Relative differences of the HIP path (g) from the oracle (o) on the
    same batch.  force: RMS over particles, sqrt(sum |dF_i|^2 / sum |F_i|^2);
    force_max: the worst particle, max_i |dF_i| / sqrt(sum |F_i|^2 / N), so a
    mistake confined to a few particles (a chunk edge, a lane group) cannot
    hide in the mean; virial: Frobenius norm; rho: worst frequency over
    sqrt(sum q^2); energy: relative."""
    dF = g["forces"] - o["forces"]
    fr = np.sqrt((dF ** 2).sum() / max((o["forces"] ** 2).sum(), 1e-300))
    frms = np.sqrt(max((o["forces"] ** 2).sum(), 1e-300) / len(o["forces"]))
    fmax = np.sqrt((dF ** 2).sum(axis=1)).max() / frms
    wr = np.linalg.norm(g["virial"] - o["virial"]) / max(np.linalg.norm(o["virial"]), 1e-300)
    rr = np.abs(g["rho"] - o["rho"]).max() / np.sqrt((np.asarray(q) ** 2).sum())
    er = abs(g["energy"] - o["energy"]) / max(abs(o["energy"]), 1e-300)
    return dict(force=fr, force_max=fmax, virial=wr, rho=rr, energy=er)


# Parity tolerances (relative): 1e-5 on the FP64 path, 1e-4 on the FP32 path,
# applied to every key of errors(), the per-particle force bound included.
TOL = {"fp64": 1e-5, "fp32": 1e-4}
KEYS = ("force", "force_max", "virial", "rho", "energy")


def assert_parity(e, precision, tag=""):
    for key in KEYS:
        assert e[key] < TOL[precision], (tag, key, e)
