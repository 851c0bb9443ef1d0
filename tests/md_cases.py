"""Oracle-side NPT trajectories matching paper_2110_14362_amd.md.NPTSystem
(same step order, same noise and batch streams)."""
import numpy as np

from oracle import integrator as oint
from oracle import rbe as orbe
from oracle import realspace as orsp
from oracle import sampler as osamp

INIT_STEP = 2 ** 63       # batch stream step used for the forces before step 0


def oracle_forces(sysd, md, pos, box, step, seed, system_id, draw=None):
    if draw is None:
        m = osamp.sample_k(sysd["alpha"], box, sysd["p"], seed=seed, system_id=system_id,
                           step=step)
    else:
        m = draw(box, step)
    S = osamp.box_tables(sysd["alpha"], box)["S"]
    k = orbe.rbe_kspace(pos, sysd["q"], box, sysd["alpha"], m, S, coulomb=sysd["coulomb"])
    r = orsp.realspace_nearest(pos, sysd["q"], box, sysd["alpha"], md["rc"], coulomb=sysd["coulomb"])
    F = k["forces"] + r["forces"]
    W = k["virial"] + r["virial"]
    if md.get("lj") is not None:
        lj = np.asarray(md["lj"])
        l = orsp.lj_nearest(pos, md["types"], box, lj[..., 0], lj[..., 1], md["rc"])
        F = F + l["forces"]
        W = W + l["virial"]
    return F, W


def oracle_trajectory(sysd, md, momenta, steps, seed, system_id, draw=None):
    """draw(box, step) -> batch: the frequency sampler (default: the exact
    draw of that step and cell)."""
    mode = {"iso": "iso", "semiiso": "semi", "aniso": "aniso"}[md.get("box_mode", "iso")]
    masses = (md["mass_cell"], md.get("mass_cell_z", 0.0))
    if mode == "aniso":                  # M_x = M_y = mass_cell, M_z = mass_cell_z
        masses = (md["mass_cell"], md["mass_cell"], md["mass_cell_z"])
    st = oint.NPTState(mode, sysd["box"], masses)
    integ = oint.LangevinNPT(mode, None, md["dt"], md["kT"], md["p_ext"], md["gamma_p"],
                             md["gamma_cell"], md["ftm"], seed, system_id,
                             rigid=md.get("rigid"))
    m = np.asarray(sysd["mass"], dtype=np.float64)
    r = np.asarray(sysd["pos"], dtype=np.float64).copy()
    p = np.asarray(momenta, dtype=np.float64).copy()
    F, W = oracle_forces(sysd, md, r, st.box(), INIT_STEP, seed, system_id, draw)
    p = integ.project(r, p, m)
    st.P_ins = integ.pressure(st, p, m, W, r, F)
    for s in range(steps):
        r, p = integ.first_half(st, r, p, m, F, s)
        F, W = oracle_forces(sysd, md, r, st.box(), s, seed, system_id, draw)
        p = integ.second_half(st, p, m, F, W, r)
    return dict(pos=r, mom=p, box=st.box(), state=st)
