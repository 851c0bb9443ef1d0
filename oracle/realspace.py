"""Nearest-image real-space Ewald sum with a cutoff (FP64 reference).

TEST INFRASTRUCTURE ONLY (FP64 CPU oracle; imported by tests, the smoke check
and the benchmark's CPU-baseline leg, never by the product path).

Section 4.2 computes the short-range force F_i2 and pressure term P3 of
eq. (force) and (pressurecubic) with the nearest image only, every pair
closer than the cutoff r_c (requires r_c <= min(l)/2).  For x the nearest-image
vector from i to j:

    U2 = (C/2) sum_{i != j, |x| < rc} q_i q_j erfc(sqrt(alpha)|x|)/|x|
    F_i2 = -C q_i sum_{j, |x| < rc} q_j G(|x|) x/|x|
    W2 = +(C/2) sum_{i != j, |x| < rc} q_i q_j G(|x|) x x^T/|x|

(sign of W2: the reading explained in oracle/ewald.py).  Brute force over all
pairs, in row blocks to bound memory.
"""

import math
import numpy as np
from scipy.special import erfc


def realspace_nearest(r, q, box, alpha, rc, coulomb=1.0, rows=None, block=512):
    """Energy, forces and virial of the cutoff real-space sum.

    rows: optional index array; forces are then returned only for these
    particles (energy and virial are still over all pairs unless rows is
    given, in which case they are None).
    """
    r = np.asarray(r, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    if rc > 0.5 * box.min() + 1e-12:
        raise ValueError("nearest-image sum needs rc <= min(box)/2")
    N = r.shape[0]
    sel = np.arange(N) if rows is None else np.asarray(rows)
    sa = math.sqrt(alpha)
    energy = 0.0
    virial = np.zeros((3, 3))
    forces = np.zeros((len(sel), 3))
    for b0 in range(0, len(sel), block):
        ii = sel[b0:b0 + block]
        x = r[None, :, :] - r[ii, None, :]                 # x[a, j] = r_j - r_i
        x -= box * np.rint(x / box)
        d = np.sqrt((x * x).sum(axis=2))
        mask = (d < rc) & (ii[:, None] != np.arange(N)[None, :])
        dm = np.where(mask, d, 1.0)
        qq = q[ii][:, None] * q[None, :]
        phi = np.where(mask, erfc(sa * dm) / dm, 0.0)
        G = np.where(mask, erfc(sa * dm) / dm ** 2
                     + 2.0 * sa * np.exp(-alpha * dm * dm) / (math.sqrt(math.pi) * dm), 0.0)
        fr = qq * G / dm
        forces[b0:b0 + block] = -np.einsum("ij,ija->ia", fr, x)
        if rows is None:
            energy += 0.5 * float(np.sum(qq * phi))
            virial += 0.5 * np.einsum("ij,ija,ijb->ab", fr, x, x)
    if rows is not None:
        return dict(energy=None, forces=coulomb * forces, virial=None)
    return dict(energy=coulomb * energy, forces=coulomb * forces, virial=coulomb * virial)


def lj_nearest(r, types, box, c12, c6, rc, rows=None, block=512):
    """Truncated Lennard-Jones pair sum, nearest image, every pair closer than rc.

    Not part of the paper's method (which treats Coulomb only); the water-
    and membrane-shaped systems need a short-range repulsion.  Pair energy
    U(r) = c12[ti,tj]/r^12 - c6[ti,tj]/r^6 (no shift), force on i
    F_i = sum_j U'(r) x/r with x = r_j - r_i, virial
    W = (1/2) sum_{i != j} (-U'(r)) x x^T / r.
    """
    r = np.asarray(r, dtype=np.float64)
    types = np.asarray(types)
    box = np.asarray(box, dtype=np.float64)
    c12 = np.asarray(c12, dtype=np.float64)
    c6 = np.asarray(c6, dtype=np.float64)
    if rc > 0.5 * box.min() + 1e-12:
        raise ValueError("nearest-image sum needs rc <= min(box)/2")
    N = r.shape[0]
    sel = np.arange(N) if rows is None else np.asarray(rows)
    energy = 0.0
    virial = np.zeros((3, 3))
    forces = np.zeros((len(sel), 3))
    for b0 in range(0, len(sel), block):
        ii = sel[b0:b0 + block]
        x = r[None, :, :] - r[ii, None, :]
        x -= box * np.rint(x / box)
        d = np.sqrt((x * x).sum(axis=2))
        mask = (d < rc) & (ii[:, None] != np.arange(N)[None, :])
        dm = np.where(mask, d, 1.0)
        a12 = c12[types[ii][:, None], types[None, :]]
        a6 = c6[types[ii][:, None], types[None, :]]
        inv6 = dm ** -6
        U = np.where(mask, a12 * inv6 * inv6 - a6 * inv6, 0.0)
        dU = np.where(mask, (-12.0 * a12 * inv6 * inv6 + 6.0 * a6 * inv6) / dm, 0.0)
        forces[b0:b0 + block] = np.einsum("ij,ija->ia", dU / dm, x)
        if rows is None:
            energy += 0.5 * float(np.sum(U))
            virial += 0.5 * np.einsum("ij,ija,ijb->ab", -dU / dm, x, x)
    if rows is not None:
        return dict(energy=None, forces=forces, virial=None)
    return dict(energy=energy, forces=forces, virial=virial)
