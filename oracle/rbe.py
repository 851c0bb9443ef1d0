"""Random batch Ewald Fourier-space estimator (FP64 reference).

TEST INFRASTRUCTURE ONLY (FP64 CPU oracle; imported by tests, the smoke check
and the benchmark's CPU-baseline leg, never by the product path).

For an orthorhombic cell h = diag(l1, l2, l3) and a batch of p nonzero integer
vectors m_l (k_l = 2 pi m_l / l componentwise), section 4.2 replaces the Ewald
Fourier sums by sample means with weight S/p:

* force, eq. (appforce):
    F*_i = -C sum_l (S/p) (4 pi q_i k_l / (V k_l^2)) Im(exp(-i k_l.r_i) rho(k_l))
* pressure, eq. (apppress), and its tensor form (eq. pressuretensorflexible /
  pressurerect with exp(-k^2/(4 alpha)) replaced by S/p over the batch):
    W* = (2 pi C / V) sum_l (S/p) |rho_l|^2/k_l^2 [I - 2(1/k_l^2 + 1/(4 alpha)) k_l k_l^T]
    P2* = tr(W*)/(3V)   (remark after eq. pressurerect)
* energy (reading: the paper gives no batch energy; this is the batch mean of
  the U1 summand, a diagnostic whose gradient is exactly F*):
    U1* = (2 pi C / V) sum_l (S/p) |rho_l|^2/k_l^2 - C sum_i q_i^2 sqrt(alpha/pi)

Reading: one batch serves force and pressure (p = p~, as in all of section 5)
in `rbe_kspace`; `rbe_kspace_split` takes a pressure batch of p~ >= p draws
whose first p serve the forces (the remark after eq. (apppress)).
Proposition 1 (eq. EE, ForceExp, PressExp) gives the mean and variance of the
per-batch deviations; `force_variance` and `pressure_variance` evaluate them.
"""

import math
import numpy as np

from .ewald import kspace_weighted, self_energy, ewald_modes


def rbe_kspace(r, q, box, alpha, m, S, coulomb=1.0):
    """RBE estimator on an explicit batch m (p x 3 ints) for box = (l1, l2, l3).

    Returns dict(rho (complex p), forces (N x 3), virial (3 x 3), energy
    (U1* including the self term), pressure2 (P2*)).
    """
    m = np.asarray(m, dtype=np.int64).reshape(-1, 3)
    p = m.shape[0]
    h = np.diag(np.asarray(box, dtype=np.float64))
    V = float(np.prod(box))
    res = kspace_weighted(r, q, h, alpha, m, S / p, coulomb)
    res["energy"] = res["energy"] + self_energy(q, alpha, coulomb)
    res["pressure2"] = float(np.trace(res["virial"])) / (3.0 * V)
    return res


def rbe_kspace_split(r, q, box, alpha, m, S, p_force, coulomb=1.0):
    """Separate force and pressure batches (the remark after eq. (apppress):
    the pressure batch size p~ may differ from the force batch size p).
    Reading: one batch of p~ = len(m) >= p i.i.d. draws; the force estimator
    of eq. (appforce) takes its first p draws with weight S/p, the pressure
    (virial tensor) and the energy take all p~ draws with weight S/p~.  Each
    estimator is the batch mean of i.i.d. draws, so each is unbiased with the
    variance of Proposition 1 at its own batch size.

    Returns dict(rho (complex, all p~), forces, virial, energy (with the self
    term), pressure2)."""
    m = np.asarray(m, dtype=np.int64).reshape(-1, 3)
    pp = m.shape[0]
    if not 1 <= p_force <= pp:
        raise ValueError("need 1 <= p_force <= len(m)")
    h = np.diag(np.asarray(box, dtype=np.float64))
    V = float(np.prod(box))
    press = kspace_weighted(r, q, h, alpha, m, S / pp, coulomb)
    force = kspace_weighted(r, q, h, alpha, m[:p_force], S / p_force, coulomb)
    return dict(rho=press["rho"], forces=force["forces"], virial=press["virial"],
                energy=press["energy"] + self_energy(q, alpha, coulomb),
                pressure2=float(np.trace(press["virial"])) / (3.0 * V))


def mode_sums(r, q, box, alpha, tol=1e-16, threads=1):
    """The Ewald modes m != 0 with weight e = exp(-k^2/(4 alpha)) >= tol and
    their structure factors: (m, e, rho), shared by the closed forms below."""
    from .ewald import structure_factor
    h = np.diag(np.asarray(box, dtype=np.float64))
    m, e = ewald_modes(h, alpha, tol)
    return m, e, structure_factor(r, q, h, m, threads)


def force_variance(r, q, box, alpha, S, p, coulomb=1.0, tol=1e-16, rows=None, threads=1,
                   sums=None):
    """Prop. 1, eq. (ForceExp): E|chi_i|^2 for every particle (length N), or
    for the particles `rows`; returns it with the Ewald force F_1 of those
    particles.  The mode sums run over particle blocks (memory) with
    `threads` threads for rho; `sums` = mode_sums(...) if already formed."""
    from .ewald import _row_blocks
    r = np.asarray(r, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    V = float(np.prod(box))
    m, e, rho = sums if sums is not None else mode_sums(r, q, box, alpha, tol, threads)
    mf = m.astype(np.float64)
    k = 2.0 * math.pi * mf / box[None, :]
    k2 = (k * k).sum(axis=1)
    rows = np.arange(r.shape[0]) if rows is None else np.asarray(rows)
    s = r[rows] / box
    second = np.zeros(len(rows))
    F1 = np.zeros((len(rows), 3))
    coef = 4.0 * math.pi * coulomb / (V * k2)
    for a, b in _row_blocks(len(rows), m.shape[0]):
        phase = 2.0 * math.pi * (s[a:b] @ mf.T)
        im = np.cos(phase) * rho.imag[None, :] - np.sin(phase) * rho.real[None, :]
        qa = q[rows[a:b], None]
        # F_1 (eq. force, Fourier part) and the second moment of one draw
        F1[a:b] = -qa * ((im * (e * coef)[None, :]) @ k)
        second[a:b] = ((qa * coef[None, :]) ** 2 * S * k2[None, :] * e[None, :] * im * im).sum(axis=1)
    return (second - (F1 * F1).sum(axis=1)) / p, F1


def pressure_variance(r, q, box, alpha, S, p, coulomb=1.0, tol=1e-16, threads=1, sums=None):
    """Prop. 1, eq. (PressExp): E|chi~|^2 of the isotropic P2*, and P2."""
    box = np.asarray(box, dtype=np.float64)
    V = float(np.prod(box))
    m, e, rho = sums if sums is not None else mode_sums(r, q, box, alpha, tol, threads)
    k = 2.0 * math.pi * m.astype(np.float64) / box[None, :]
    k2 = (k * k).sum(axis=1)
    rho2 = np.abs(rho) ** 2
    fac = (1.0 / 3.0 - k2 / (6.0 * alpha))
    P2 = coulomb * (2.0 * math.pi / V ** 2) * float(np.sum(e * rho2 / k2 * fac))
    second = float(np.sum(4.0 * math.pi ** 2 * coulomb ** 2 * rho2 ** 2 * S
                          / (V ** 4 * k2 ** 2) * e * fac ** 2))
    return (second - P2 * P2) / p, P2


def reuse_expected(r, q, box_now, box_frozen, alpha, coulomb=1.0, tol=1e-16):
    """Expectation of the RBE estimator (forces, virial, energy without the
    self term) at cell box_now when the batch is drawn from the law of cell
    box_frozen (sample reuse, section 4.3): the estimator weights every drawn
    mode by S_now/p (eq. (appforce), (apppress)) while mode m is drawn with
    probability w_frozen(m)/S_frozen, so the expectation is the mode sum with
    weights S_now w_frozen(m)/S_frozen, w(m) = exp(-|k|^2/(4 alpha)) of the
    respective cell (eq. (probexpression)).  With box_frozen = box_now the
    weights are w_now(m): the Ewald sum, which makes the estimator unbiased
    (section 4.2).  The modes are those of the larger cell within `tol`."""
    box_now = np.asarray(box_now, dtype=np.float64)
    box_frozen = np.asarray(box_frozen, dtype=np.float64)
    big = np.maximum(box_now, box_frozen)
    m, _ = ewald_modes(np.diag(big), alpha, tol)
    mf = m.astype(np.float64)

    def weights(box):
        k2 = (((2.0 * math.pi) * mf / box[None, :]) ** 2).sum(axis=1)
        return np.exp(-k2 / (4.0 * alpha))

    from .sampler import box_tables
    S_now = box_tables(alpha, tuple(box_now))["S"]
    S_fr = box_tables(alpha, tuple(box_frozen))["S"]
    w = S_now * weights(box_frozen) / S_fr
    return kspace_weighted(r, q, np.diag(box_now), alpha, m, w, coulomb)
