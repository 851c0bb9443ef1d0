"""Device NPT trajectories vs the oracle's: same initial state, same batch
and noise streams, FP64 path.  10 steps of the primitive electrolyte (cubic,
isotropic) and of small rectangular systems (semi-isotropic, anisotropic)."""
import numpy as np
import pytest

from paper_2110_14362_amd import workloads
from tests.md_cases import oracle_trajectory

pytestmark = pytest.mark.gpu


def o_kin(o_state, mom, md, s):
    # molecular kinetic tensor of the device momenta (centre-of-mass part)
    from oracle import constraints as cons
    rg = md["rigid"]
    mol = cons.molecules(rg["first"], rg["count"])
    return cons.molecular_kinetic(mom, np.asarray(s["mass"]), mol) / md["ftm"]


def electrolyte_setup():
    s = workloads.make("electrolyte_1k")
    md = dict(dt=0.005, kT=1.0, p_ext=0.1, gamma_p=1.0, gamma_cell=1.0,
              mass_cell=1.0 / (8.0 * 8000.0), ftm=1.0, box_mode="iso", rc=6.0)
    mom = np.random.default_rng(17).normal(0.0, 1.0, s["pos"].shape)     # m = kT = 1
    return s, md, mom


def slab_setup():
    s = workloads.random_neutral(600, (14.0, 14.0, 18.0), seed=23)
    s.update(alpha=0.5 ** 2, p=64, coulomb=1.0)
    md = dict(dt=0.004, kT=1.0, p_ext=0.2, gamma_p=1.0, gamma_cell=2.0,
              mass_cell=2e-3, mass_cell_z=1e-2, ftm=1.0, box_mode="semiiso", rc=4.5)
    mom = np.random.default_rng(18).normal(0.0, 1.0, s["pos"].shape)
    return s, md, mom


def aspect_setup():
    # isotropic coupling of a 1:1:1.25 cell (the aspect ratio is kept)
    s = workloads.random_neutral(500, (13.0, 13.0, 16.25), seed=29)
    s.update(alpha=0.5 ** 2, p=48, coulomb=1.0)
    md = dict(dt=0.004, kT=1.0, p_ext=0.3, gamma_p=1.0, gamma_cell=1.5,
              mass_cell=3e-3, ftm=1.0, box_mode="iso", rc=4.2)
    mom = np.random.default_rng(19).normal(0.0, 1.0, s["pos"].shape)
    return s, md, mom


def aniso_setup():
    # rectangular cell, every side length with its own momentum
    s = workloads.random_neutral(560, (13.0, 14.0, 15.5), seed=37)
    s.update(alpha=0.5 ** 2, p=48, coulomb=1.0)
    md = dict(dt=0.004, kT=1.0, p_ext=0.3, gamma_p=1.0, gamma_cell=1.5,
              mass_cell=2e-3, mass_cell_z=4e-3, ftm=1.0, box_mode="aniso", rc=4.2)
    mom = np.random.default_rng(20).normal(0.0, 1.0, s["pos"].shape)
    return s, md, mom


def rigid_water_setup():
    # rigid SPC/E-shaped water (150 molecules), O-O Lennard-Jones, real units
    s = workloads.rigid_water(150, seed=31)
    rc = float(s["box"].min()) / 3.2
    g = 3.0 / rc
    s.update(alpha=g * g, p=100, coulomb=workloads.COULOMB_REAL)
    md = workloads.npt_real(s["box"], rc=rc)
    md.update(types=s["types"], lj=s["lj"], rigid=s["rigid"])
    mom = None
    return s, md, mom


def electrolyte_lists_setup():
    # real-space neighbour lists (skin 1.5): the trajectory is unchanged
    s, md, mom = electrolyte_setup()
    md["skin"] = 1.5
    return s, md, mom


def rigid_water_lists_setup():
    s, md, mom = rigid_water_setup()
    md["skin"] = workloads.list_skin(s["box"], md["rc"], 1.0)
    assert md["skin"] > 0.5
    return s, md, mom


@pytest.mark.parametrize("setup", [electrolyte_setup, slab_setup, aspect_setup, aniso_setup,
                                   rigid_water_setup, electrolyte_lists_setup,
                                   rigid_water_lists_setup])
def test_npt_trajectory_matches_oracle(gpu, setup):
    from paper_2110_14362_amd.md import NPTSystem
    s, md, mom = setup()
    if mom is None:
        mom = np.zeros_like(s["pos"])
    steps = 10
    sysg = NPTSystem(s, md, precision="fp64", seed=99, system_id=5, momenta=mom)
    sysg.step(steps)
    sysg.check()
    g = sysg.state()
    o = oracle_trajectory(s, md, mom, steps, seed=99, system_id=5)
    dpos = np.abs(g["pos"] - o["pos"]).max()
    dmom = np.abs(g["mom"] - o["mom"]).max() / np.abs(o["mom"]).max()
    dbox = np.abs(g["box"] - o["box"]).max() / o["box"].max()
    print("%s: max |dr| %.2e, rel |dp| %.2e, rel |dl| %.2e, box %s" %
          (setup.__name__, dpos, dmom, dbox, g["box"]), flush=True)
    assert dpos < 1e-8 and dmom < 1e-8 and dbox < 1e-10
    # the cell moved: the barostat is live
    assert np.abs(o["box"] - np.asarray(s["box"])).max() > 1e-8
    if md.get("rigid"):
        x = g["pos"]
        rg = md["rigid"]
        o, h1, h2 = x[0::3], x[1::3], x[2::3]
        for a, b, d in ((o, h1, rg["d_oh"]), (o, h2, rg["d_oh"]), (h1, h2, rg["d_hh"])):
            assert np.abs(np.linalg.norm(a - b, axis=1) - d).max() < 1e-12
        np.testing.assert_allclose(g["kinetic"], o_kin(o_state=o, mom=g["mom"], md=md, s=s),
                                   rtol=1e-8, atol=1e-12)
    if md["box_mode"] == "semiiso":
        assert g["box"][0] == g["box"][1]
    elif md["box_mode"] == "aniso":
        # the three sides move independently
        rel = g["box"] / np.asarray(s["box"])
        assert abs(rel[0] - rel[1]) > 1e-9 and abs(rel[1] - rel[2]) > 1e-9
    else:
        b0 = np.asarray(s["box"], dtype=np.float64)
        np.testing.assert_allclose(g["box"] / g["box"][0], b0 / b0[0], rtol=1e-14)


def test_long_run_pressure_and_temperature_averages(gpu):
    # section 3: the Langevin NPT dynamics holds the time-averaged
    # instantaneous pressure at the imposed one and the kinetic temperature at
    # kT; 1000 ions with a repulsive core in reduced units, full device step
    # (random batch Fourier part, pairs, integrator), 4000 + 12000 steps
    from tests.measure_npt import run
    r = run(equil=4000, prod=12000, every=4, precision="fp32")
    print("<P_ins> = %.5f +- %.5f (P = %.3f), <T> = %.4f +- %.4f, <V> = %.1f"
          % (r["p_mean"], r["p_se"], r["p_ext"], r["t_mean"], r["t_se"], r["v_mean"]), flush=True)
    assert abs(r["p_mean"] - r["p_ext"]) < 4.0 * r["p_se"] + 0.02 * r["p_ext"]
    assert abs(r["t_mean"] - r["kT"]) < 4.0 * r["t_se"] + 0.01
    assert r["p_se"] < 0.05 * r["p_ext"]
