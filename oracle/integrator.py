"""Langevin NPT integrator in FP64 (reference).

TEST INFRASTRUCTURE ONLY (FP64 CPU oracle; imported by tests, the smoke check
and the benchmark's CPU-baseline leg, never by the product path).

Equations of motion: section 3.2 eq. (24) for a cubic cell (V, p^V),
appendix A eq. (99999) for the semi-isotropic cell (A, p^A, L, p^L) and the
appendix's rectangular cell with anisotropic fluctuation (side lengths l_j,
momenta p^l_j, masses M_j; its pressure eq. (e:instrectangular)):

    r' = p/m + D r,         p' = F - D p - gamma p + sqrt(2 kT m gamma) W'
    iso:  D = (V'/3V) I,    V' = p^V/M,  p^V' = P_ins - P - gamma_c p^V + noise
    semi: D = diag(A'/2A, A'/2A, L'/L),
          p^A' = L (P_A - P) - ...,  P_A = (P_xx + P_yy)/2 + gamma0/L (gamma0 = 0),
          p^L' = A (P_zz - P) - ...
    aniso: D = diag(l_j'/l_j),  l_j' = p^l_j/M_j,
          p^l_j' = V (P_jj - P)/l_j - gamma_c p^l_j + noise

Time step (section 3.3): the palindromic Trotter order
    B_V(h) B_R(h) A_V(h) A_R(h) O^p(dt) O(dt) A_R(h) A_V(h) [forces, pressure] B_R(h) B_V(h),
h = dt/2.  Sub-flows, each solved exactly with the other variables frozen
(reading of the cited exact solutions): with the per-axis rate a = D_aa,
    A_R:  r <- r e^{a h} + (p/m) (e^{a h} - 1)/a
    B_R:  p <- p e^{-a h} + F (1 - e^{-a h})/a
    A_V:  V <- V + h p^V/M   (A, L, l_j likewise)
    B_V:  p^V <- p^V + h (P_ins - P)   (semi: h L (P_A - P), h A (P_zz - P);
          aniso: h V (P_jj - P)/l_j)
    O:    p <- e^{-g dt} p + sqrt(kT m (1 - e^{-2 g dt})) R   (exact OU, section 3.3)
The instantaneous pressure tensor is (sum_i p_i p_i^T/m_i + W)/V, W the
virial tensor of the forces (eq. pressuretensorflexible); its trace/3 is the
scalar P_ins of eq. (pressurecubic).  The B_V that opens a step uses the
pressure from the end of the previous step (same momenta and virial).

Units: forces and virials enter multiplied by `ftm` (force unit -> mass x
length / time^2); kT and P are given in energy units and multiplied by ftm.

Rigid molecules (optional; constraints.py): every sub-flow that moves
positions (A_R) is followed by SHAKE against the positions before it, with
the momentum change that the A_R map gives the position change,
    p <- p + m (r_shake - r_unconstrained) a / (e^{a h} - 1)   (per axis),
and every sub-flow that changes momenta (B_R, O) by the RATTLE velocity
stage.  The pressure then takes the molecular form of constraints.py.

Noise: Philox4x64-10 keyed (seed, system_id); particle i at step s uses
counter (s, i, TAG_NOISE, 0): uniforms u0..u3 give three normals by Box-Muller,
z0 = sqrt(-2 ln(1-u0)) cos(2 pi u1), z1 = ... sin(2 pi u1),
z2 = sqrt(-2 ln(1-u2)) cos(2 pi u3).  The cell uses counter (s, 0, TAG_CELL, 0):
z0 for V (or A, or l_x), z1 for L (or l_y), z2 for l_z.
"""

import math
import numpy as np

from . import constraints as cons
from .philox import philox4x64, u01

TAG_NOISE = 0x6E6F6973   # 'nois'
TAG_CELL = 0x63656C6C    # 'cell'


def normals3(seed, system_id, step, index, tag):
    r = philox4x64((step, index, tag, 0), (seed, system_id))
    u = [u01(x) for x in r]
    a = math.sqrt(-2.0 * math.log(1.0 - u[0]))
    b = math.sqrt(-2.0 * math.log(1.0 - u[2]))
    return (a * math.cos(2.0 * math.pi * u[1]), a * math.sin(2.0 * math.pi * u[1]),
            b * math.cos(2.0 * math.pi * u[3]))


def particle_noise(seed, system_id, step, n):
    return np.array([normals3(seed, system_id, step, i, TAG_NOISE) for i in range(n)])


def _expm1_over(a, h):
    """(e^{a h} - 1)/a, with its limit h at a = 0."""
    return h if a == 0.0 else math.expm1(a * h) / a


class NPTState:
    """Cell and barostat state.  mode 'iso': V, pV, M; 'semi': A, pA, MA, L, pL, ML;
    'aniso': l[3], pl[3], Ml[3] (masses (M_x, M_y, M_z))."""

    def __init__(self, mode, box, masses):
        self.mode = mode
        box = [float(b) for b in box]
        if mode == "iso":
            self.V = box[0] * box[1] * box[2]
            self.pV = 0.0
            self.M = float(masses[0])
            # D = (V'/3V) I scales every side by the same factor, so the
            # initial aspect ratio is kept (1:1:1 for a cube)
            if box[0] == box[1] == box[2]:
                self.asp = np.ones(3)
            else:
                self.asp = np.array(box) / self.V ** (1.0 / 3.0)
        elif mode == "aniso":
            self.l = np.array(box)
            self.pl = np.zeros(3)
            self.Ml = np.array([float(v) for v in masses], dtype=np.float64)
        else:
            self.A = box[0] * box[1]
            self.L = box[2]
            self.pA = 0.0
            self.pL = 0.0
            self.MA = float(masses[0])
            self.ML = float(masses[1])
        self.P_ins = np.zeros((3, 3))

    def box(self):
        if self.mode == "iso":
            return self.asp * self.V ** (1.0 / 3.0)
        if self.mode == "aniso":
            return self.l.copy()
        s = math.sqrt(self.A)
        return np.array([s, s, self.L])

    def volume(self):
        if self.mode == "aniso":
            return float(self.l[0] * self.l[1] * self.l[2])
        return self.V if self.mode == "iso" else self.A * self.L

    def rates(self):
        """Per-axis scaling rate D_aa of eq. (24) / eq. (99999)."""
        if self.mode == "iso":
            a = self.pV / (3.0 * self.M * self.V)
            return np.array([a, a, a])
        if self.mode == "aniso":
            return self.pl / (self.Ml * self.l)
        axy = self.pA / (2.0 * self.MA * self.A)
        return np.array([axy, axy, self.pL / (self.ML * self.L)])


class LangevinNPT:
    """One BAOAB step of the Langevin NPT equations (see the module docstring)."""

    def __init__(self, mode, masses_cell, dt, kT, P, gamma_p, gamma_c, ftm, seed, system_id,
                 rigid=None):
        """rigid: None or dict(first, count, d_oh, d_hh) (rigid 3-site molecules)."""
        self.mode = mode
        self.rigid = rigid
        self.mol = cons.molecules(rigid["first"], rigid["count"]) if rigid else None
        self.masses_cell = masses_cell
        self.dt, self.kT, self.P = dt, kT, P
        self.gp, self.gc, self.ftm = gamma_p, gamma_c, ftm
        self.seed, self.sysid = seed, system_id

    def pressure(self, st, p, m, W, r=None, F=None):
        """Instantaneous pressure tensor (internal units): (sum p p^T/m + ftm W)/V,
        or with rigid molecules (K_mol + ftm (W - C))/V (constraints.py)."""
        if self.rigid is None:
            K = np.einsum("ia,ib->ab", p, p / m[:, None])
            return (K + self.ftm * np.asarray(W)) / st.volume()
        K = cons.molecular_kinetic(p, m, self.mol)
        C = cons.molecular_correction(r, np.asarray(F), m, self.mol)
        return (K + self.ftm * (np.asarray(W) - C)) / st.volume()

    def project(self, r, p, m):
        """RATTLE velocity stage (identity without rigid molecules)."""
        if self.rigid is None:
            return p
        rg = self.rigid
        return cons.rattle_momenta(r, p, m, self.mol, rg["d_oh"], rg["d_hh"])

    def drift(self, st, r, p, m, h):
        """A_R, then SHAKE and the matching momentum change (rigid molecules)."""
        r1 = self.A_R(st, r, p, m, h)
        if self.rigid is None:
            return r1, p
        rg = self.rigid
        rs = cons.shake(r, r1, m, self.mol, rg["d_oh"], rg["d_hh"])
        a = st.rates()
        phi = np.array([_expm1_over(a[ax], h) for ax in range(3)])
        p = p + m[:, None] * (rs - r1) / phi[None, :]
        return rs, p

    def B_V(self, st, h):
        P = self.ftm * self.P
        Pt = st.P_ins
        if st.mode == "iso":
            st.pV += h * (np.trace(Pt) / 3.0 - P)
        elif st.mode == "aniso":
            V = st.volume()
            for j in range(3):
                st.pl[j] += h * V * (Pt[j, j] - P) / st.l[j]
        else:
            st.pA += h * st.L * (0.5 * (Pt[0, 0] + Pt[1, 1]) - P)
            st.pL += h * st.A * (Pt[2, 2] - P)

    def A_V(self, st, h):
        if st.mode == "iso":
            st.V += h * st.pV / st.M
        elif st.mode == "aniso":
            st.l = st.l + h * st.pl / st.Ml
        else:
            st.A += h * st.pA / st.MA
            st.L += h * st.pL / st.ML

    def B_R(self, st, p, F, h):
        a = st.rates()
        out = p.copy()
        for ax in range(3):
            e = math.exp(-a[ax] * h)
            out[:, ax] = p[:, ax] * e + self.ftm * F[:, ax] * _expm1_over(-a[ax], h)
        return out

    def A_R(self, st, r, p, m, h):
        a = st.rates()
        out = r.copy()
        for ax in range(3):
            out[:, ax] = r[:, ax] * math.exp(a[ax] * h) + (p[:, ax] / m) * _expm1_over(a[ax], h)
        return out

    def O_cell(self, st, step):
        z = normals3(self.seed, self.sysid, step, 0, TAG_CELL)
        c1 = math.exp(-self.gc * self.dt)
        if st.mode == "iso":
            st.pV = c1 * st.pV + math.sqrt(self.ftm * self.kT * st.M * (1.0 - c1 * c1)) * z[0]
        elif st.mode == "aniso":
            for j in range(3):
                st.pl[j] = (c1 * st.pl[j]
                            + math.sqrt(self.ftm * self.kT * st.Ml[j] * (1.0 - c1 * c1)) * z[j])
        else:
            st.pA = c1 * st.pA + math.sqrt(self.ftm * self.kT * st.MA * (1.0 - c1 * c1)) * z[0]
            st.pL = c1 * st.pL + math.sqrt(self.ftm * self.kT * st.ML * (1.0 - c1 * c1)) * z[1]

    def O_particles(self, p, m, step):
        z = particle_noise(self.seed, self.sysid, step, p.shape[0])
        c1 = math.exp(-self.gp * self.dt)
        return c1 * p + np.sqrt(self.ftm * self.kT * m * (1.0 - c1 * c1))[:, None] * z

    def first_half(self, st, r, p, m, F, step):
        h = 0.5 * self.dt
        self.B_V(st, h)
        p = self.project(r, self.B_R(st, p, F, h), m)
        self.A_V(st, h)
        r, p = self.drift(st, r, p, m, h)
        self.O_cell(st, step)
        p = self.project(r, self.O_particles(p, m, step), m)
        r, p = self.drift(st, r, p, m, h)
        self.A_V(st, h)
        return r, p

    def second_half(self, st, p, m, F, W, r=None):
        h = 0.5 * self.dt
        p = self.project(r, self.B_R(st, p, F, h), m)
        st.P_ins = self.pressure(st, p, m, W, r, F)
        self.B_V(st, h)
        return p
