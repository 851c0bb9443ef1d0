"""Pins of the rigid-molecule oracle (constraints.py and the constrained
integrator): SHAKE and RATTLE against the properties that define them,
exact rigid-body motions (free rotation, a uniform force field), energy
conservation of the frictionless constrained step, and the molecular virial
against a finite difference of the full Ewald energy under rigid
centre-of-mass scaling."""
import math

import numpy as np
import pytest

from oracle import constraints as cons
from oracle import ewald
from oracle import integrator as oint
from paper_2110_14362_amd import workloads

M3 = np.array([workloads.M_O, workloads.M_H, workloads.M_H])
D_OH, D_HH = workloads.D_OH, workloads.D_HH


def rigid_waters(k, seed, spacing=4.0):
    g = np.random.default_rng(seed)
    ref = np.array([[0.0, 0.0, 0.0],
                    [D_HH / 2, 0.0, math.sqrt(D_OH ** 2 - D_HH ** 2 / 4)],
                    [-D_HH / 2, 0.0, math.sqrt(D_OH ** 2 - D_HH ** 2 / 4)]])
    R = workloads._random_rotations(g, k)
    centres = spacing * np.arange(k)[:, None] * np.array([1.0, 0.3, 0.2])
    r = (centres[:, None, :] + np.einsum("kab,sb->ksa", R, ref)).reshape(-1, 3)
    return r, np.tile(M3, k), cons.molecules(0, k)


def bond_lengths(r, mol):
    x = r[mol]
    return np.stack([np.linalg.norm(x[:, 0] - x[:, 1], axis=1),
                     np.linalg.norm(x[:, 0] - x[:, 2], axis=1),
                     np.linalg.norm(x[:, 1] - x[:, 2], axis=1)], 1)


def test_shake_satisfies_its_definition():
    r0, m, mol = rigid_waters(20, 1)
    g = np.random.default_rng(2)
    r1 = r0 + g.normal(0, 0.04, r0.shape) + 0.02 * (r0 - r0.mean(0))
    r = cons.shake(r0, r1, m, mol, D_OH, D_HH)
    assert np.abs(bond_lengths(r, mol) - [D_OH, D_OH, D_HH]).max() < 1e-13
    # positions reach |r| ~ 80 here: rounding of an update is ~1e-14 absolute
    tol = 1e-14 * np.abs(r0).max() * M3.sum()
    for idx in mol:
        mm = m[idx]
        d = r[idx] - r1[idx]
        # centre of mass unchanged
        assert np.abs(mm @ d).max() < tol
        # m_a d_a is a combination of the OLD bond vectors (forces along them)
        s01 = r0[idx[0]] - r0[idx[1]]
        s02 = r0[idx[0]] - r0[idx[2]]
        s12 = r0[idx[1]] - r0[idx[2]]
        G = np.zeros((9, 3))
        G[0:3, 0], G[3:6, 0] = s01, -s01
        G[0:3, 1], G[6:9, 1] = s02, -s02
        G[3:6, 2], G[6:9, 2] = s12, -s12
        md = (mm[:, None] * d).ravel()
        lam, *_ = np.linalg.lstsq(G, md, rcond=None)
        assert np.abs(G @ lam - md).max() < tol


def test_shake_keeps_a_rigid_motion():
    r0, m, mol = rigid_waters(5, 3)
    R = workloads._random_rotations(np.random.default_rng(4), 1)[0]
    small = np.eye(3) + 0.0 * R
    # a small rotation about each molecule's centre plus a shift satisfies the
    # constraints already: SHAKE must leave it alone
    th = 0.03
    Rz = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    r1 = r0.copy()
    for idx in mol:
        c = M3 @ r0[idx] / M3.sum()
        r1[idx] = c + 0.1 + (r0[idx] - c) @ (Rz @ small).T
    r = cons.shake(r0, r1, m, mol, D_OH, D_HH)
    assert np.abs(r - r1).max() < 1e-13


def test_rattle_projects_onto_rigid_motions():
    r, m, mol = rigid_waters(12, 5)
    p = np.random.default_rng(6).normal(0, 1.0, r.shape)
    q = cons.rattle_momenta(r, p, m, mol, D_OH, D_HH)
    for idx in mol:
        x, mm = r[idx], m[idx]
        v = q[idx] / mm[:, None]
        for a, b in ((0, 1), (0, 2), (1, 2)):
            assert abs((x[a] - x[b]) @ (v[a] - v[b])) < 1e-12 * np.abs(p[idx] / mm[:, None]).max()
        # linear and angular momentum unchanged (the removed part is internal)
        c = mm @ x / mm.sum()
        assert np.abs(q[idx].sum(0) - p[idx].sum(0)).max() < 1e-13
        L0 = np.cross(x - c, p[idx]).sum(0)
        L1 = np.cross(x - c, q[idx]).sum(0)
        assert np.abs(L1 - L0).max() < 1e-12
    # idempotent
    assert np.abs(cons.rattle_momenta(r, q, m, mol, D_OH, D_HH) - q).max() < 1e-13 * np.abs(q).max() * 10


def _frozen_integrator(dt, rigid):
    # gamma = 0 and a cell too heavy to move: plain constrained dynamics
    return oint.LangevinNPT("iso", None, dt, 1.0, 0.0, 0.0, 0.0, 1.0, seed=1, system_id=1,
                            rigid=rigid)


def _run(r, p, m, dt, steps, force=None):
    k = len(m) // 3
    rigid = dict(first=0, count=k, d_oh=D_OH, d_hh=D_HH)
    integ = _frozen_integrator(dt, rigid)
    st = oint.NPTState("iso", (1e4, 1e4, 1e4), (1e30, 0.0))
    F = np.zeros_like(r) if force is None else force(r)
    W = np.zeros((3, 3))
    p = integ.project(r, p, m)
    st.P_ins = integ.pressure(st, p, m, W, r, F)
    for s in range(steps):
        r, p = integ.first_half(st, r, p, m, F, s)
        if force is not None:
            F = force(r)
        p = integ.second_half(st, p, m, F, W, r)
    return r, p


def test_free_rigid_rotation():
    # no forces: bonds, momentum, angular momentum and the kinetic energy are
    # invariants (the last one of the splitting as well, to rounding here)
    r0, m, mol = rigid_waters(1, 7)
    p0 = np.cross(np.array([0.3, -0.7, 1.1]), r0 - M3 @ r0 / M3.sum()) * m[:, None]
    p0 += m[:, None] * np.array([0.05, 0.0, -0.02])
    p0 = cons.rattle_momenta(r0, p0, m, mol, D_OH, D_HH)
    K0 = 0.5 * (p0 * p0 / m[:, None]).sum()
    errs = []
    for dt, n in ((0.02, 100), (0.01, 200)):
        r, p = _run(r0.copy(), p0.copy(), m, dt, n)
        assert np.abs(bond_lengths(r, mol) - [D_OH, D_OH, D_HH]).max() < 1e-13
        assert np.abs(p.sum(0) - p0.sum(0)).max() < 1e-10       # rounding only
        c0, c = M3 @ r0 / M3.sum(), M3 @ r / M3.sum()
        L0 = np.cross(r0 - c0, p0).sum(0)
        L = np.cross(r - c, p).sum(0)
        assert np.abs(L - L0).max() < 1e-10
        errs.append(abs(0.5 * (p * p / m[:, None]).sum() - K0) / K0)
        # and it did turn: the H-H axis moved by a finite angle
        u0 = r0[2] - r0[1]
        u = r[2] - r[1]
        assert np.arccos(u0 @ u / (u0 @ u0)) > 0.5
    assert max(errs) < 1e-10


def test_uniform_field_moves_the_centre_of_mass_exactly():
    r0, m, mol = rigid_waters(3, 8)
    gvec = np.array([0.2, -0.1, 0.4])
    p0 = np.zeros_like(r0)
    dt, n = 0.05, 40
    r, p = _run(r0.copy(), p0, m, dt, n, force=lambda r: m[:, None] * gvec)
    T = dt * n
    for idx in mol:
        c0 = m[idx] @ r0[idx] / m[idx].sum()
        c = m[idx] @ r[idx] / m[idx].sum()
        assert np.abs(c - (c0 + 0.5 * gvec * T * T)).max() < 1e-12
        assert np.abs(p[idx].sum(0) - m[idx].sum() * gvec * T).max() < 1e-12


def _water_system(n_mol, seed, qscale=1.0):
    s = workloads.water(n_mol, seed=seed)
    first = 0
    pos = workloads.whole_molecules(s["pos"], s["box"], first, n_mol)
    return pos, s["q"] * qscale, s["mass"], s["box"]


def test_constrained_step_conserves_energy():
    # soft charges (0.4 e scale): frictionless, frozen cell, full Ewald forces
    n_mol = 8
    r, q, m, box = _water_system(n_mol, 4, qscale=0.4)
    alpha, rc = 1.0, 3.0
    ftm = workloads.FTM_REAL
    rigid = dict(first=0, count=n_mol, d_oh=D_OH, d_hh=D_HH)

    def forces(r):
        e = ewald.ewald_total(r, q, np.diag(box), alpha, rc, ktol=1e-14,
                              coulomb=workloads.COULOMB_REAL)
        return e["forces"], e["virial"], e["energy"]

    integ = oint.LangevinNPT("iso", None, 0.5, 0.6, 0.0, 0.0, 0.0, ftm, seed=1, system_id=1,
                             rigid=rigid)
    st = oint.NPTState("iso", box, (1e30, 0.0))
    p = np.random.default_rng(3).normal(0, 1, r.shape) * np.sqrt(m * 0.6 * ftm)[:, None]
    F, W, U = forces(r)
    p = integ.project(r, p, m)
    st.P_ins = integ.pressure(st, p, m, W, r, F)
    H = lambda p, U: 0.5 * (p * p / m[:, None]).sum() + ftm * U
    H0, K0 = H(p, U), 0.5 * (p * p / m[:, None]).sum()
    dev = 0.0
    for s in range(40):
        r, p = integ.first_half(st, r, p, m, F, s)
        F, W, U = forces(r)
        p = integ.second_half(st, p, m, F, W, r)
        dev = max(dev, abs(H(p, U) - H0))
    assert dev < 2e-3 * K0, dev / K0


@pytest.mark.parametrize("axis", [0, 2])
def test_molecular_virial_is_the_rigid_scaling_derivative(axis):
    # U(s): centres of mass and the cell side along `axis` scaled by s, each
    # molecule rigid.  -dU/ds at s = 1 equals W_mol[axis, axis] = W - C.
    n_mol = 6
    r, q, m, box = _water_system(n_mol, 9)
    mol = cons.molecules(0, n_mol)
    alpha, rc = 1.1, 2.9

    def energy(s):
        b = box.copy()
        b[axis] *= s
        x = r.copy()
        for idx in mol:
            c = m[idx] @ r[idx] / m[idx].sum()
            shift = np.zeros(3)
            shift[axis] = (s - 1.0) * c[axis]
            x[idx] += shift
        return ewald.ewald_total(x, q, np.diag(b), alpha, rc, ktol=1e-15)

    e0 = energy(1.0)
    C = cons.molecular_correction(r, e0["forces"], m, mol)
    Wmol = e0["virial"] - C
    h = 1e-5
    dU = (energy(1 + h)["energy"] - energy(1 - h)["energy"]) / (2 * h)
    assert abs(-dU - Wmol[axis, axis]) < 1e-7 * max(1.0, abs(dU)), (-dU, Wmol[axis, axis])
