"""Rigid 3-site molecules for the NPT integrator (reference).

TEST INFRASTRUCTURE ONLY (FP64 CPU oracle; imported by tests, the smoke check
and the benchmark's CPU-baseline leg, never by the product path).

The paper runs rigid water with bond constraints (SHAKE, section 5).  The
reference takes the two classical iterative constraint solvers:

* positions: SHAKE (Ryckaert, Ciccotti and Berendsen, J. Comput. Phys. 23,
  327 (1977)).  Given positions r0 that satisfy the constraints and
  unconstrained new positions r1, find r = r1 + M^-1 sum_c lambda_c grad g_c(r0)
  with |r_a - r_b| = d_ab for every bond; each bond is corrected in turn along
  its old direction until all hold to a relative 1e-13 (in d^2).
* momenta: the velocity stage of RATTLE (Andersen, J. Comput. Phys. 52, 24
  (1983)): p <- p + sum_c mu_c grad g_c(r) such that every bond's relative
  velocity along the bond vanishes; again bond by bond until converged.

A molecule k of a rigid set (first, count) holds atoms first + 3k (O),
first + 3k + 1 and first + 3k + 2 (H), bonds O-H, O-H (d_oh) and H-H (d_hh).

Pressure with rigid molecules (reading): the molecular form
    P V = sum_free p p^T/m + sum_mol P_mol P_mol^T / M_mol + W - C,
    C = sum_mol sum_{a in mol} sym((r_a - R_mol) (x) F_a),
W the atomic virial of the forces, R_mol and P_mol the molecule's centre of
mass and total momentum, sym(X) = (X + X^T)/2.  It equals the atomic
pressure with the constraint forces' virial up to the time derivative of a
bounded quantity, so both have the same average; it needs no constraint
multipliers.
"""

import numpy as np

_TOL = 1e-13
_MAX_SWEEPS = 500


def molecules(first, count):
    """(count, 3) atom indices of the rigid molecules."""
    base = first + 3 * np.arange(count)
    return np.stack([base, base + 1, base + 2], 1)


def _bonds(d_oh, d_hh):
    return ((0, 1, d_oh), (0, 2, d_oh), (1, 2, d_hh))


def shake(r0, r1, m, mol, d_oh, d_hh):
    """SHAKE: constrained positions from old r0 and unconstrained r1 (N, 3)."""
    r = r1.copy()
    for idx in mol:
        ro = r0[idx]
        mm = m[idx]
        x = r[idx].copy()
        for _ in range(_MAX_SWEEPS):
            worst = 0.0
            for a, b, d in _bonds(d_oh, d_hh):
                s = x[a] - x[b]
                s0 = ro[a] - ro[b]
                diff = d * d - s @ s
                worst = max(worst, abs(diff) / (d * d))
                g = diff / (2.0 * (1.0 / mm[a] + 1.0 / mm[b]) * (s @ s0))
                x[a] += g * s0 / mm[a]
                x[b] -= g * s0 / mm[b]
            if worst < _TOL:
                break
        else:
            raise RuntimeError("SHAKE did not converge")
        r[idx] = x
    return r


def rattle_momenta(r, p, m, mol, d_oh, d_hh):
    """RATTLE velocity stage: momenta with no relative velocity along any bond."""
    out = p.copy()
    for idx in mol:
        x = r[idx]
        mm = m[idx]
        q = out[idx].copy()
        vscale = max(np.abs(q / mm[:, None]).max(), 1e-300)
        for _ in range(_MAX_SWEEPS):
            worst = 0.0
            for a, b, _d in _bonds(d_oh, d_hh):
                s = x[a] - x[b]
                dv = q[a] / mm[a] - q[b] / mm[b]
                sv = s @ dv
                worst = max(worst, abs(sv) / np.sqrt(s @ s) / vscale)
                k = sv / ((s @ s) * (1.0 / mm[a] + 1.0 / mm[b]))
                q[a] -= k * s
                q[b] += k * s
            if worst < _TOL:
                break
        else:
            raise RuntimeError("RATTLE did not converge")
        out[idx] = q
    return out


def _sym(X):
    return 0.5 * (X + X.T)


def molecular_kinetic(p, m, mol):
    """sum over free atoms of p p^T/m plus sum over molecules of P P^T/M."""
    free = np.ones(len(m), dtype=bool)
    free[mol.ravel()] = False
    K = np.einsum("ia,ib->ab", p[free], p[free] / m[free, None])
    for idx in mol:
        P = p[idx].sum(0)
        K += np.outer(P, P) / m[idx].sum()
    return K


def molecular_correction(r, F, m, mol):
    """C = sum_mol sum_a sym((r_a - R_mol) (x) F_a)."""
    C = np.zeros((3, 3))
    for idx in mol:
        R = m[idx] @ r[idx] / m[idx].sum()
        C += np.einsum("ia,ib->ab", r[idx] - R, F[idx])
    return _sym(C)
