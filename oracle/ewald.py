"""Classical Ewald summation in FP64, for a general (triclinic) cell.

TEST INFRASTRUCTURE ONLY (FP64 CPU oracle; imported by tests, the smoke check
and the benchmark's CPU-baseline leg, never by the product path).

Conventions
* h is the 3x3 cell matrix whose COLUMNS are the cell vectors; r = h s with s
  the reduced coordinates (section 2, the relation between r_i and s_i);
  V = det h.  Reciprocal vectors k = 2 pi h^-T m, m integer (appendix C).
* C is the Coulomb constant (1 in reduced units); the paper writes C = 1.
* The splitting parameter alpha is the paper's: the kernel splits as
  erf(sqrt(alpha) r)/r + erfc(sqrt(alpha) r)/r (section 4.1), so alpha has
  units of length^-2.

Formulas (section 4.1 and appendix C):
* U = U1 + U2 with the self term inside U1 (eq. U1fourier, eq. U2):
    U1 = (2 pi C / V) sum_{k != 0} exp(-k^2/(4 alpha)) |rho(k)|^2 / k^2
         - C sum_i q_i^2 sqrt(alpha/pi),      rho(k) = sum_j q_j exp(i k.r_j)
    U2 = (C/2) sum'_n sum_ij q_i q_j erfc(sqrt(alpha) |x|)/|x|,
         x = r_j - r_i + h n  (reading: r_ij = r_j - r_i, as the force
         formula states)
* F_i = F_i1 + F_i2 (eq. force):
    F_i1 = -C sum_k (4 pi q_i k / (V k^2)) exp(-k^2/(4 alpha)) Im(exp(-i k.r_i) rho(k))
    F_i2 = -C q_i sum'_{j,n} q_j G(|x|) x/|x|,
    G(r) = erfc(sqrt(alpha) r)/r^2 + 2 sqrt(alpha) exp(-alpha r^2)/(sqrt(pi) r)
* Virial tensor W (energy units; the pressure tensor is (W + kinetic)/V),
  eq. pressuretensorflexible and pressurerect:
    W1 = (2 pi C / V) sum_k exp(-k^2/(4 alpha)) |rho|^2/k^2
          [I - 2 (1/k^2 + 1/(4 alpha)) k k^T]
    W2 = +(C/2) sum' q_i q_j G(|x|) x x^T / |x|
  Reading (sign): the paper prints W2 with a minus sign (it writes the
  pairwise term as F_ij (x) x with F_ij = -q_i q_j G x/|x|).  Differentiating
  U2 in the cell at fixed s gives the plus sign used here; the finite-
  difference tests pin it.
"""

import math
import numpy as np
from scipy.special import erfc


def cell_volume(h):
    return float(np.linalg.det(h))


def recip(h):
    """Matrix whose columns are the reciprocal vectors b_i = 2 pi h^-T e_i."""
    return 2.0 * math.pi * np.linalg.inv(h).T


def kvectors(h, m):
    """k = 2 pi h^-T m for integer rows m (K x 3) -> (K x 3) float64."""
    return np.asarray(m, dtype=np.float64) @ recip(h).T


def reduced(r, h):
    """s = h^-1 r."""
    return np.linalg.solve(h, np.asarray(r, dtype=np.float64).T).T


def _row_blocks(N, K, budget=2_000_000):
    """Particle row ranges keeping N x K temporaries near `budget` elements."""
    step = max(1, budget // max(K, 1))
    return [(a, min(N, a + step)) for a in range(0, N, step)]


def structure_factor(r, q, h, m, threads=1):
    """rho(k_l) = sum_j q_j exp(i k_l . r_j) for each row of m (complex128).

    The particle sum runs over row blocks only to bound memory; with
    threads > 1 the blocks are evaluated by a thread pool (numpy releases
    the interpreter lock inside its array operations) and their sums are
    added in block order."""
    s = reduced(r, h)
    mf = np.asarray(m, dtype=np.float64)

    def block(ab):
        a, b = ab
        phase = 2.0 * math.pi * (s[a:b] @ mf.T)
        return (q[a:b, None] * np.exp(1j * phase)).sum(axis=0)

    blocks = _row_blocks(s.shape[0], mf.shape[0])
    if threads > 1 and len(blocks) > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(threads) as ex:
            parts = list(ex.map(block, blocks))
    else:
        parts = [block(ab) for ab in blocks]
    rho = np.zeros(mf.shape[0], dtype=np.complex128)
    for part in parts:
        rho += part
    return rho


def kspace_weighted(r, q, h, alpha, m, weight, coulomb=1.0, force_rows=None, threads=1):
    """Fourier-space sum over the modes m with per-mode weights.

    With weight_l = exp(-k_l^2/(4 alpha)) over all nonzero m in a converged
    range this is the Ewald U1 (without self term), F_i1 and W1.  With the
    random batch weight S/p over a sampled batch it is the RBE estimator.
    force_rows: optional particle indices; forces are then returned for those
    rows only.  threads: thread pool size of the structure-factor sum.

    Returns dict(rho, energy, forces, virial, k, k2) -- energy excludes the
    self term.
    """
    r = np.asarray(r, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    m = np.asarray(m, dtype=np.int64).reshape(-1, 3)
    w = np.broadcast_to(np.asarray(weight, dtype=np.float64), (m.shape[0],))
    V = cell_volume(h)
    k = kvectors(h, m)
    k2 = (k * k).sum(axis=1)
    rho = structure_factor(r, q, h, m, threads)
    A, B = rho.real, rho.imag
    rho2 = A * A + B * B
    energy = coulomb * (2.0 * math.pi / V) * float(np.sum(w * rho2 / k2))
    # F_i = -C q_i sum_l w_l 4 pi k_l/(V k_l^2) Im(exp(-i k_l.r_i) rho_l),
    # Im(exp(-i theta) rho) = cos(theta) B - sin(theta) A
    coef = w * 4.0 * math.pi / (V * k2)
    rows = np.arange(r.shape[0]) if force_rows is None else np.asarray(force_rows)
    s = reduced(r[rows], h)
    mf = m.astype(np.float64)
    forces = np.zeros((len(rows), 3))
    for a, b in _row_blocks(len(rows), m.shape[0]):
        phase = 2.0 * math.pi * (s[a:b] @ mf.T)
        im = np.cos(phase) * B[None, :] - np.sin(phase) * A[None, :]
        forces[a:b] = -coulomb * q[rows[a:b], None] * ((im * coef[None, :]) @ k)
    fac = w * rho2 / k2
    beta = 2.0 * (1.0 / k2 + 1.0 / (4.0 * alpha))
    virial = coulomb * (2.0 * math.pi / V) * (
        np.eye(3) * fac.sum()
        - np.einsum("l,la,lb->ab", fac * beta, k, k))
    return dict(rho=rho, energy=energy, forces=forces, virial=virial, k=k, k2=k2)


def self_energy(q, alpha, coulomb=1.0):
    return -coulomb * float(np.sum(np.asarray(q, dtype=np.float64) ** 2)) * math.sqrt(alpha / math.pi)


def ewald_modes(h, alpha, tol=1e-16):
    """All m != 0 with exp(-k^2/(4 alpha)) >= tol (k = 2 pi h^-T m)."""
    k2max = -4.0 * alpha * math.log(tol)
    kmax = math.sqrt(k2max)
    # |m_i| <= kmax * |h_i| / (2 pi): m_i = k . h_i / (2 pi)
    lens = np.linalg.norm(h, axis=0)
    mm = [int(math.ceil(kmax * lens[i] / (2.0 * math.pi))) for i in range(3)]
    g = np.stack(np.meshgrid(np.arange(-mm[0], mm[0] + 1),
                             np.arange(-mm[1], mm[1] + 1),
                             np.arange(-mm[2], mm[2] + 1), indexing="ij"), -1).reshape(-1, 3)
    g = g[np.any(g != 0, axis=1)]
    k = kvectors(h, g)
    k2 = (k * k).sum(axis=1)
    keep = k2 <= k2max
    return g[keep], np.exp(-k2[keep] / (4.0 * alpha))


def G_radial(rr, alpha):
    """G(r) of eq. force: -(d/dr) [erfc(sqrt(alpha) r)/r]."""
    sa = math.sqrt(alpha)
    return erfc(sa * rr) / rr ** 2 + 2.0 * sa * np.exp(-alpha * rr * rr) / (math.sqrt(math.pi) * rr)


def realspace_images(r, q, h, alpha, rc, coulomb=1.0):
    """Real-space Ewald sum over all periodic images with |x| < rc.

    Every pair (i, j) and every lattice shift n are visited (n = 0 skipped
    for i = j), so rc may exceed half the cell.  Returns energy, forces, virial.
    """
    r = np.asarray(r, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    N = r.shape[0]
    b = recip(h)
    # distance between lattice planes along each cell vector: 2 pi / |b_i|
    dplane = 2.0 * math.pi / np.linalg.norm(b, axis=0)
    s = np.linalg.solve(h, r.T).T
    spread = s.max(axis=0) - s.min(axis=0)
    nmax = [int(math.ceil(rc / dplane[i] + spread[i])) + 1 for i in range(3)]
    d0 = r[None, :, :] - r[:, None, :]          # d0[i, j] = r_j - r_i
    qq = q[:, None] * q[None, :]
    eye = np.eye(N, dtype=bool)
    energy = 0.0
    forces = np.zeros((N, 3))
    virial = np.zeros((3, 3))
    for n0 in range(-nmax[0], nmax[0] + 1):
        for n1 in range(-nmax[1], nmax[1] + 1):
            for n2 in range(-nmax[2], nmax[2] + 1):
                shift = h @ np.array([n0, n1, n2], dtype=np.float64)
                x = d0 + shift
                d = np.sqrt((x * x).sum(axis=2))
                mask = d < rc
                if n0 == 0 and n1 == 0 and n2 == 0:
                    mask &= ~eye
                if not mask.any():
                    continue
                dm = np.where(mask, d, 1.0)
                phi = np.where(mask, erfc(math.sqrt(alpha) * dm) / dm, 0.0)
                g = np.where(mask, G_radial(dm, alpha), 0.0)
                energy += 0.5 * float(np.sum(qq * phi))
                fr = qq * g / dm                   # q_i q_j G / |x|
                forces += -np.einsum("ij,ija->ia", fr, x)
                virial += 0.5 * np.einsum("ij,ija,ijb->ab", fr, x, x)
    return dict(energy=coulomb * energy, forces=coulomb * forces, virial=coulomb * virial)


def ewald_total(r, q, h, alpha, rc, ktol=1e-16, coulomb=1.0):
    """Full Ewald: energy, forces and virial (no kinetic part)."""
    h = np.asarray(h, dtype=np.float64)
    m, w = ewald_modes(h, alpha, ktol)
    ks = kspace_weighted(r, q, h, alpha, m, w, coulomb)
    rs = realspace_images(r, q, h, alpha, rc, coulomb)
    es = self_energy(q, alpha, coulomb)
    return dict(energy=ks["energy"] + rs["energy"] + es,
                forces=ks["forces"] + rs["forces"],
                virial=ks["virial"] + rs["virial"],
                k_energy=ks["energy"] + es, k_forces=ks["forces"], k_virial=ks["virial"],
                r_energy=rs["energy"], r_forces=rs["forces"], r_virial=rs["virial"])
