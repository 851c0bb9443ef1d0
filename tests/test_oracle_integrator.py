"""Pins of the integrator oracle: exact Ornstein-Uhlenbeck variance, energy
conservation of the frictionless splitting, and the ideal-gas NPT volume."""
import math

import numpy as np
import pytest

from oracle import ewald
from oracle import integrator as oint
from paper_2110_14362_amd import workloads


def test_noise_is_standard_normal():
    from scipy import stats
    z = np.concatenate([oint.particle_noise(11, 2, s, 500).ravel() for s in range(4)])
    assert abs(z.mean()) < 4 / math.sqrt(len(z))
    assert abs(z.var() - 1) < 0.05
    assert stats.kstest(z, "norm").pvalue > 1e-4


def test_ou_step_variance_closed_form():
    # F = 0, cell frozen: Var p(t) = m kT (1 - e^{-2 g t}) + e^{-2 g t} Var p(0)
    n, m_, kT, g, dt = 6000, 2.0, 1.5, 0.7, 0.3
    integ = oint.LangevinNPT("iso", None, dt, kT, 0.0, g, 0.0, 1.0, seed=5, system_id=1)
    p0 = np.random.default_rng(1).normal(0, 0.5, (n, 3))
    p = integ.O_particles(p0, np.full(n, m_), step=0)
    c = math.exp(-2 * g * dt)
    expect = m_ * kT * (1 - c) + c * 0.25
    assert abs(p.var() / expect - 1) < 0.05
    # and the mean decays by e^{-g dt}
    assert np.allclose((p - math.exp(-g * dt) * p0).mean(), 0.0, atol=0.05)


BOXES = {"iso": (6.0, 6.0, 6.0), "semi": (6.0, 6.0, 7.0), "aniso": (6.0, 6.5, 7.0)}


def _energy_drift(with_potential, mode):
    n = 16 if with_potential else 12
    s = workloads.random_neutral(n, BOXES[mode], seed=3)
    m = np.ones(n)
    M, P, dt = 0.05, 0.02, 0.002
    masses = {"iso": (M, 0.0), "semi": (M, 1.5 * M), "aniso": (M, 1.3 * M, 0.8 * M)}[mode]
    st = oint.NPTState(mode, s["box"], masses)
    integ = oint.LangevinNPT(mode, None, dt, 1.0, P, 0.0, 0.0, 1.0, seed=0, system_id=0)
    r = s["pos"].copy()
    p = np.random.default_rng(2).normal(0, 1.0, (n, 3))
    alpha, rc = 0.8 ** 2, 2.9

    def forces(r, box):
        if not with_potential:
            return np.zeros_like(r), np.zeros((3, 3)), 0.0
        res = ewald.ewald_total(r, s["q"], np.diag(box), alpha, rc, ktol=1e-14)
        return res["forces"], res["virial"], res["energy"]

    def cell_kinetic(st):
        # the Hamiltonian's cell part for each cell parametrisation
        if mode == "iso":
            return 0.5 * st.pV ** 2 / st.M
        if mode == "semi":
            return 0.5 * st.pA ** 2 / st.MA + 0.5 * st.pL ** 2 / st.ML
        return 0.5 * float((st.pl ** 2 / st.Ml).sum())

    def H(st, p, U):
        return 0.5 * (p * p).sum() + U + P * st.volume() + cell_kinetic(st)

    F, W, U = forces(r, st.box())
    st.P_ins = integ.pressure(st, p, m, W)
    H0 = H(st, p, U)
    Hs, boxes = [], []
    for k in range(200 if with_potential else 2000):
        r, p = integ.first_half(st, r, p, m, F, k)
        F, W, U = forces(r, st.box())
        p = integ.second_half(st, p, m, F, W)
        Hs.append(H(st, p, U))
        boxes.append(st.box())
    return H0, np.array(Hs), np.array(boxes)


@pytest.mark.parametrize("mode", ["iso", "semi", "aniso"])
@pytest.mark.parametrize("with_potential", [False, True])
def test_frictionless_step_conserves_extended_energy(with_potential, mode):
    # gamma = 0: the splitting is symplectic for H = K + U + P V + (cell
    # momenta)^2 / 2 (cell masses), in each cell parametrisation
    H0, Hs, boxes = _energy_drift(with_potential, mode)
    scale = max(1.0, abs(H0))
    assert np.abs(Hs - H0).max() < 2e-3 * scale
    # no secular drift: late fluctuations are as small as early ones
    k = len(Hs) // 4
    assert abs(Hs[-k:].mean() - Hs[:k].mean()) < 1e-3 * scale
    # the cell moved, with the freedom of its parametrisation
    rel = boxes / boxes[0]
    assert np.ptp(boxes, axis=0).min() > 1e-4
    if mode == "iso":
        assert np.abs(rel - rel[:, :1]).max() < 1e-12
    elif mode == "semi":
        assert np.abs(boxes[:, 0] - boxes[:, 1]).max() < 1e-12
        assert np.abs(rel[:, 2] - rel[:, 0]).max() > 1e-4
    else:
        assert min(np.abs(rel[:, 0] - rel[:, 1]).max(), np.abs(rel[:, 1] - rel[:, 2]).max()) > 1e-4


@pytest.mark.slow
def test_ideal_gas_npt_mean_volume():
    # U = 0: the invariant measure exp(-beta H) dV dr dp has <V> = (N + 1) kT / P
    n, kT, P = 8, 1.0, 0.5
    st = oint.NPTState("iso", (3.0, 3.0, 3.0), (0.2, 0.0))
    integ = oint.LangevinNPT("iso", None, 0.02, kT, P, 1.0, 2.0, 1.0, seed=9, system_id=4)
    m = np.ones(n)
    r = np.random.default_rng(0).random((n, 3)) * 3.0
    p = np.random.default_rng(1).normal(0, 1.0, (n, 3))
    F = np.zeros((n, 3)); W = np.zeros((3, 3))
    st.P_ins = integ.pressure(st, p, m, W)
    vols = []
    for k in range(30000):
        r, p = integ.first_half(st, r, p, m, F, k)
        p = integ.second_half(st, p, m, F, W)
        if k >= 2000:
            vols.append(st.volume())
    expect = (n + 1) * kT / P
    assert abs(np.mean(vols) / expect - 1) < 0.06, (np.mean(vols), expect)
