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

Reading: one batch serves force and pressure (p = p~, as in all of section 5).
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


def force_variance(r, q, box, alpha, S, p, coulomb=1.0, tol=1e-16):
    """Prop. 1, eq. (ForceExp): E|chi_i|^2 for every particle (length N)."""
    r = np.asarray(r, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    V = float(np.prod(box))
    h = np.diag(box)
    m, e = ewald_modes(h, alpha, tol)
    full = kspace_weighted(r, q, h, alpha, m, e, coulomb)
    k2 = full["k2"]
    rho = full["rho"]
    s = r / box
    phase = 2.0 * math.pi * (s @ m.T.astype(np.float64))
    im = np.cos(phase) * rho.imag[None, :] - np.sin(phase) * rho.real[None, :]
    second = ((4.0 * math.pi * coulomb * q[:, None]) ** 2 * S / (V * V * k2[None, :])
              * e[None, :] * im * im).sum(axis=1)
    F1 = full["forces"]
    return (second - (F1 * F1).sum(axis=1)) / p, F1


def pressure_variance(r, q, box, alpha, S, p, coulomb=1.0, tol=1e-16):
    """Prop. 1, eq. (PressExp): E|chi~|^2 of the isotropic P2*, and P2."""
    box = np.asarray(box, dtype=np.float64)
    V = float(np.prod(box))
    h = np.diag(box)
    m, e = ewald_modes(h, alpha, tol)
    full = kspace_weighted(r, q, h, alpha, m, e, coulomb)
    k2 = full["k2"]
    rho2 = np.abs(full["rho"]) ** 2
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
