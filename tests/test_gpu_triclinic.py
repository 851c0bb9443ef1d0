"""Triclinic cells (appendix C) on the device against the FP64 oracle: the
cell values (S from the device's Poisson-summed form against the oracle's
direct lattice sum), the rejection sampler's batches (identical integers to
the oracle's draws over several steps and cells), and forces, full virial
tensor, energy and rho on the same batch, for both launch forms and both
precisions, with a new skewed cell every step; the calls a triclinic cell
does not support fail cleanly."""
import numpy as np
import pytest

from oracle import triclinic as tri
from paper_2110_14362_amd import workloads
from tests.gpu_cases import TOL, assert_parity, errors, to_dev

pytestmark = pytest.mark.gpu

CELLS = [(20.0, 20.0, 20.0, 4.0, -3.0, 2.5),          # sheared cube
         (18.0, 21.0, 24.0, -6.0, 5.0, -7.0),         # strongly skewed
         (31.0, 31.0, 31.0, 0.0, 0.0, 0.0)]           # no tilt


def skewed(sysd, h6):
    """The system's reduced coordinates placed in the cell h6."""
    box = np.asarray(sysd["box"], dtype=np.float64)
    h = tri.cell_matrix(*h6)
    return (sysd["pos"] / box) @ h.T


def test_cell_values_and_draws_match_the_oracle(gpu):
    import torch
    from paper_2110_14362_amd.rbe import RBE
    q = torch.tensor([1.0, -1.0], dtype=torch.float64, device=gpu)
    alpha, P = 0.09, 700
    for h6 in CELLS:
        ctx = RBE(q, h6, P, alpha, box_mode="triclinic", seed=2110, system_id=9)
        info = ctx.get_box_info()
        h = tri.cell_matrix(*h6)
        S = tri.normaliser(alpha, h)
        assert abs(info["S"] - S) < 1e-12 * S, (h6, info["S"], S)
        assert abs(info["V"] - np.linalg.det(h)) < 1e-12 * np.linalg.det(h)
        for step in (0, 1, 2**40 + 7):
            ctx.sample_k(step)
            g = ctx.get_k().astype(np.int64)
            o, tries = tri.sample_k_cell(alpha, h, P, 2110, 9, step)
            bad = np.where(np.any(g != o, axis=1))[0]
            assert len(bad) == 0, (h6, step, bad[:5], g[bad[:5]], o[bad[:5]])
        print("cell %s: S %.10g, draws identical to the oracle, mean attempts %.2f"
              % (h6, S, tries.mean()), flush=True)
        ctx.check()
        ctx.close()


def _run(s, pos, h6s, dev, precision, fused, p, steps):
    import torch
    from paper_2110_14362_amd.rbe import RBE
    ctx = RBE(to_dev(s["q"], dev), h6s[0], p, s["alpha"], coulomb=s["coulomb"],
              precision=precision, box_mode="triclinic", seed=77, system_id=5)
    ctx.set_fused(fused)
    out = []
    for step, h6 in zip(steps, h6s):
        x, y, z = (to_dev(pos[step][:, a], dev) for a in range(3))
        f = [torch.zeros_like(x) for _ in range(3)]
        vir = torch.zeros(6, dtype=torch.float64, device=dev)
        en = torch.zeros(1, dtype=torch.float64, device=dev)
        ctx.rescale_box(h6)
        ctx.sample_k(step)
        ctx.forces_pressure(x, y, z, *f, virial6=vir, energy=en)
        torch.cuda.synchronize()
        W6 = vir.cpu().numpy()
        W = np.array([[W6[0], W6[3], W6[4]], [W6[3], W6[1], W6[5]], [W6[4], W6[5], W6[2]]])
        out.append(dict(forces=np.stack([t.cpu().numpy() for t in f], 1), virial=W,
                        energy=float(en.cpu()[0]), rho=ctx.get_rho(),
                        m=ctx.get_k().astype(np.int64)))
    plan = ctx.plan()
    ctx.check()
    ctx.close()
    return plan, out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("fused", [1, 0])
@pytest.mark.parametrize("case", ["water_3k", "electrolyte_1k"])
def test_triclinic_parity(gpu, case, precision, fused):
    # three steps, each with its own skewed cell (the particles follow the
    # cell at fixed reduced coordinates, with some moved by whole cell
    # vectors: reduced coordinates wrap), the batch drawn on the device
    if case == "water_3k":
        s = workloads.water(1000, seed=5)
        s.update(alpha=0.09, coulomb=332.0637)
        base = (31.04, 31.04, 31.04)
    else:
        s = workloads.make("electrolyte_1k")
        base = (20.0, 20.0, 20.0)
    h6s = [base + (0.1 * base[0], -0.05 * base[0], 0.08 * base[1]),
           base + (0.12 * base[0], -0.04 * base[0], 0.07 * base[1]),
           tuple(1.01 * b for b in base) + (-0.2 * base[0], 0.15 * base[0], -0.1 * base[1])]
    steps = (0, 1, 2)
    rng = np.random.default_rng(8)
    pos = {}
    for step, h6 in zip(steps, h6s):
        h = tri.cell_matrix(*h6)
        shift = rng.integers(-2, 3, size=s["pos"].shape) * (rng.random(s["pos"].shape) < 0.1)
        pos[step] = skewed(s, h6) + shift @ h.T
    plan, out = _run(s, pos, h6s, gpu, precision, fused, 100, steps)
    assert plan["fused"] == fused
    for step, h6, g in zip(steps, h6s, out):
        h = tri.cell_matrix(*h6)
        m_o, _ = tri.sample_k_cell(s["alpha"], h, 100, 77, 5, step)
        assert np.array_equal(g["m"], m_o), step
        o = tri.rbe_kspace_cell(pos[step], s["q"], h, s["alpha"], m_o,
                                tri.normaliser(s["alpha"], h), coulomb=s["coulomb"])
        e = errors(g, o, s["q"])
        print("%s triclinic step %d %s fused=%d: force %.2e (worst %.2e) virial %.2e rho %.2e "
              "energy %.2e" % (case, step, precision, fused, e["force"], e["force_max"],
                               e["virial"], e["rho"], e["energy"]), flush=True)
        assert_parity(e, precision, step)
        # the off-diagonal virial components of a skewed cell are compared
        # element by element too
        off = [(0, 1), (0, 2), (1, 2)]
        scale = np.linalg.norm(o["virial"])
        for a, b in off:
            assert abs(g["virial"][a, b] - o["virial"][a, b]) < TOL[precision] * scale


def test_triclinic_unsupported_calls(gpu):
    import torch
    from paper_2110_14362_amd.rbe import RBE, RBEError
    q = torch.tensor([1.0, -1.0], dtype=torch.float64, device=gpu)
    ctx = RBE(q, CELLS[0], 16, 0.09, box_mode="triclinic")
    dbox = torch.tensor(CELLS[0][:3], dtype=torch.float64, device=gpu)
    for call in (lambda: ctx.rescale_box_dev(dbox), lambda: ctx.set_sampler("mh", 1),
                 lambda: ctx.set_sample_reuse(4),
                 lambda: ctx.rescale_box((20.0, 20.0, 20.0, 25.0, 0.0, 0.0))):
        with pytest.raises(RBEError) as ei:
            call()
        assert ei.value.status == 1
    with pytest.raises(RBEError) as ei:                 # beyond the table capacity
        ctx.rescale_box((45.0, 45.0, 45.0, 0.0, 0.0, 0.0))
    assert ei.value.status == 6
    ctx.check()
    ctx.close()
