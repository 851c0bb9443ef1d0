"""rbe_forces_pressure_noalloc (the entry point for callers that cannot
allocate device memory) against the context entry point rbe_forces_pressure
on the same configuration, cell and step: identical bits, on two calls in a
row, the second with a smaller system (the shared static scratch keeps the
first call's contents, which the second must not see)."""
import numpy as np
import pytest

from paper_2110_14362_amd import workloads
from tests.gpu_cases import to_dev

pytestmark = pytest.mark.gpu


def _context_step(s, dev, precision, step, p, seed, system_id):
    import torch
    from paper_2110_14362_amd.rbe import RBE
    ctx = RBE(to_dev(s["q"], dev), s["box"], p, s["alpha"], coulomb=s["coulomb"],
              precision=precision, seed=seed, system_id=system_id)
    ctx.set_fused(1)                  # the launch form the no-allocation call uses
    assert ctx.plan()["fused"] == 1
    x, y, z = (to_dev(s["pos"][:, a], dev) for a in range(3))
    f = [torch.zeros_like(x) for _ in range(3)]
    vir = torch.zeros(6, dtype=torch.float64, device=dev)
    en = torch.zeros(1, dtype=torch.float64, device=dev)
    ctx.rescale_box(s["box"])
    ctx.sample_k(step)
    ctx.forces_pressure(x, y, z, *f, virial6=vir, energy=en)
    torch.cuda.synchronize()
    out = dict(F=np.stack([t.cpu().numpy() for t in f], 1), W=vir.cpu().numpy(),
               U=en.cpu().numpy(), rho=ctx.get_rho())
    ctx.check()
    ctx.close()
    return out


def _noalloc_step(s, dev, precision, step, p, seed, system_id):
    import torch
    from paper_2110_14362_amd.rbe import forces_pressure_noalloc
    x, y, z = (to_dev(s["pos"][:, a], dev) for a in range(3))
    f = [torch.full_like(x, 7.0) for _ in range(3)]          # overwritten
    vir = torch.zeros(6, dtype=torch.float64, device=dev)
    en = torch.zeros(1, dtype=torch.float64, device=dev)
    rho = torch.zeros(2 * p, dtype=torch.float64, device=dev)
    forces_pressure_noalloc(to_dev(s["q"], dev), s["box"], p, s["alpha"], step, x, y, z, *f,
                            coulomb=s["coulomb"], precision=precision, seed=seed,
                            system_id=system_id, virial6=vir, energy=en, rho=rho)
    torch.cuda.synchronize()
    r = rho.cpu().numpy()
    return dict(F=np.stack([t.cpu().numpy() for t in f], 1), W=vir.cpu().numpy(),
                U=en.cpu().numpy(), rho=r[0::2] + 1j * r[1::2])


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_noalloc_equals_context_entry_point(gpu, precision):
    big = workloads.make("water_30k")                 # 30,000 charges, P = 100
    small = workloads.make("electrolyte_1k")          # 1,000 charges, P = 64 below
    for s, p, step in ((big, 100, 12345), (small, 64, 7)):
        a = _noalloc_step(s, gpu, precision, step, p, 2110, 3)
        b = _context_step(s, gpu, precision, step, p, 2110, 3)
        for key in ("F", "W", "U", "rho"):
            np.testing.assert_array_equal(a[key], b[key], err_msg="%s N=%d" % (key, len(s["q"])))
        print("noalloc %s N=%d P=%d: identical to the context entry point"
              % (precision, len(s["q"]), p), flush=True)


def test_noalloc_rejects_beyond_its_limits(gpu):
    import torch
    from paper_2110_14362_amd.rbe import RBEError, forces_pressure_noalloc
    s = workloads.make("electrolyte_1k")
    x = to_dev(s["pos"][:, 0], gpu)
    f = [torch.zeros_like(x) for _ in range(3)]
    with pytest.raises(RBEError) as ei:               # p~ beyond the single-launch batch
        forces_pressure_noalloc(to_dev(s["q"], gpu), s["box"], 600, s["alpha"], 0, x, x, x, *f)
    assert ei.value.status == 6
