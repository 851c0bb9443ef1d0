"""Random batch Ewald in a triclinic cell (appendix C): normaliser, sampler
and estimator for a general cell matrix h (FP64 reference).

TEST INFRASTRUCTURE ONLY (FP64 CPU oracle; imported by tests, the smoke check
and the benchmark's CPU-baseline leg, never by the product path).

What it follows:
* Appendix C: for a cell h whose columns are the cell vectors, r = h s, the
  reciprocal vectors are k = 2 pi h^-T m (m integer) and V = det h.
* Section 4.2 eq. (probexpression), (S): the sampling law is
  exp(-|k|^2/(4 alpha))/S over m != 0, S the sum of the same weights.  With
  Q(m) = |k|^2/(4 alpha) = m^T A m, A = (pi^2/alpha) h^-1 h^-T, the weight is
  exp(-Q(m)); for a non-rectangular cell A has off-diagonal entries and the
  law does not factorise over the three components of m.
* Eq. (appforce), (apppress) and appendix C eq. (pressuretensorflexible) with
  exp(-k^2/(4 alpha)) replaced by S/p: `rbe_kspace_cell`.

Readings:
* Normaliser: S + 1 = sum over all m of exp(-Q(m)), summed directly over the
  ellipsoid Q(m) <= 53 ln 2 + 8 (the tail is below 2^-53 of the m = 0 term).
  The Poisson-summed form (eq. (psf) for a general lattice),
  S + 1 = (alpha/pi)^(3/2) V sum_n exp(-alpha |h n|^2), pins it.
* Sampler (exact draws by rejection; the paper's chain, section 4.3, leaves
  this open): the separable envelope D = t diag(A), t = (1 - 1e-9) times the
  smallest eigenvalue of diag(A)^-1/2 A diag(A)^-1/2 (exactly t = 1 for a
  rectangular cell), makes A - D positive semidefinite, so
  Q(m) >= m^T D m.  A proposal from exp(-m^T D m) on m != 0 (three
  independent one-axis discrete Gaussians, w_j(m) = exp(-d_j m^2), the
  nonzero event split by its first nonzero axis exactly as in sampler.py)
  accepted with probability exp(-(Q(m) - m^T D m)) has the law
  exp(-Q(m))/S.
  Stream: attempt a of sample l at step s takes its proposal uniforms from
  the Philox4x64-10 counter (s, l, 'ksam', a) (the rectangular draw is
  attempt 0 with every proposal accepted) and its acceptance uniform from
  the first output of (s, l, 'kacc', a); after 256 rejected attempts the
  last proposal is kept (probability (1 - acceptance)^256).
"""

import math
import numpy as np

from .ewald import kspace_weighted, self_energy
from .philox import philox4x64, u01
from .sampler import TAG_KSAMPLE, TAIL_LN

TAG_KACCEPT = 0x6B616363   # 'kacc': acceptance uniforms of the triclinic draws
MAX_ATTEMPTS = 256


def cell_matrix(lx, ly, lz, xy=0.0, xz=0.0, yz=0.0):
    """Upper-triangular h: a = (lx, 0, 0), b = (xy, ly, 0), c = (xz, yz, lz)."""
    return np.array([[lx, xy, xz], [0.0, ly, yz], [0.0, 0.0, lz]], dtype=np.float64)


def quad_matrix(alpha, h):
    """A with Q(m) = |2 pi h^-T m|^2/(4 alpha) = m^T A m."""
    hi = np.linalg.inv(np.asarray(h, dtype=np.float64))
    return (math.pi ** 2 / alpha) * (hi @ hi.T)


def envelope(alpha, h):
    """Per-axis coefficients d of the separable envelope exp(-sum d_j m_j^2)."""
    A = quad_matrix(alpha, h)
    dg = np.diag(A)
    if np.all(A - np.diag(dg) == 0.0):
        return dg.copy()
    s = 1.0 / np.sqrt(dg)
    t = np.linalg.eigvalsh(A * s[:, None] * s[None, :]).min() * (1.0 - 1e-9)
    return t * dg


def ellipsoid_modes(A, c):
    """All integer m with m^T A m <= c (m = 0 included)."""
    Ai = np.linalg.inv(A)
    mm = [int(math.floor(math.sqrt(c * Ai[j, j]))) for j in range(3)]
    g = np.stack(np.meshgrid(*[np.arange(-b, b + 1) for b in mm], indexing="ij"), -1).reshape(-1, 3)
    Q = np.einsum("ia,ab,ib->i", g, A, g)
    keep = Q <= c
    return g[keep], Q[keep]


def normaliser(alpha, h):
    """S: the direct sum of exp(-Q(m)) over m != 0 within the ellipsoid."""
    m, Q = ellipsoid_modes(quad_matrix(alpha, h), TAIL_LN + 8.0)
    nz = np.any(m != 0, axis=1)
    return float(np.sum(np.exp(-Q[nz])))


def normaliser_poisson(alpha, h):
    """S from the Poisson-summed lattice sum over real-space cell vectors n."""
    h = np.asarray(h, dtype=np.float64)
    V = abs(float(np.linalg.det(h)))
    n, Qr = ellipsoid_modes(alpha * (h.T @ h), 60.0)
    return (alpha / math.pi) ** 1.5 * V * float(np.sum(np.exp(-Qr))) - 1.0


def law(alpha, h):
    """(modes m != 0, probabilities exp(-Q(m))/S) over the ellipsoid."""
    m, Q = ellipsoid_modes(quad_matrix(alpha, h), TAIL_LN + 8.0)
    nz = np.any(m != 0, axis=1)
    w = np.exp(-Q[nz])
    return m[nz], w / w.sum()


def proposal_tables(d):
    """One-axis tables of the envelope: for each axis the m values and the
    running sums of w(m) = exp(-d m^2), |m| <= ceil(sqrt(53 ln 2 / d)), over
    all m and over m != 0, and the first-nonzero-axis case weights."""
    axes = []
    for dj in d:
        mc = int(math.ceil(math.sqrt(TAIL_LN / dj)))
        m = np.arange(-mc, mc + 1, dtype=np.int64)
        w = np.exp(-(dj * (m.astype(np.float64) ** 2)))
        nz = m != 0
        axes.append(dict(m_full=m, c_full=np.cumsum(w), m_nz=m[nz], c_nz=np.cumsum(w[nz]),
                         T=float(np.cumsum(w[nz])[-1])))
    Tx, Ty, Tz = (a["T"] for a in axes)
    case_w = (Tx * (1.0 + Ty) * (1.0 + Tz), Ty * (1.0 + Tz), Tz)
    return dict(axes=axes, case_w=case_w, Sprop=case_w[0] + case_w[1] + case_w[2])


def _table_draw(m_vals, cum, u):
    target = u * cum[-1]
    i = int(np.searchsorted(cum, target, side="right"))   # first running sum > target
    return int(m_vals[min(i, len(cum) - 1)])


def propose(tab, u):
    """The envelope draw from four uniforms (as sampler.sample_k)."""
    wx, wy, _ = tab["case_w"]
    t = u[0] * tab["Sprop"]
    pivot = 0 if t < wx else (1 if t < wx + wy else 2)
    m = [0, 0, 0]
    for j in range(3):
        ax = tab["axes"][j]
        if j == pivot:
            m[j] = _table_draw(ax["m_nz"], ax["c_nz"], u[j + 1])
        elif j > pivot:
            m[j] = _table_draw(ax["m_full"], ax["c_full"], u[j + 1])
    return m


def sample_k_cell(alpha, h, P, seed, system_id, step):
    """P nonzero integer vectors (P x 3 int64) with law exp(-Q(m))/S, and the
    number of attempts each took."""
    A = quad_matrix(alpha, h)
    d = envelope(alpha, h)
    tab = proposal_tables(d)
    key = (seed, system_id)
    out = np.zeros((P, 3), dtype=np.int64)
    tries = np.zeros(P, dtype=np.int64)
    for l in range(P):
        for a in range(MAX_ATTEMPTS):
            u = [u01(x) for x in philox4x64((step, l, TAG_KSAMPLE, a), key)]
            m = propose(tab, u)
            mv = np.array(m, dtype=np.float64)
            excess = float(mv @ A @ mv) - float(np.sum(d * mv * mv))
            ua = u01(philox4x64((step, l, TAG_KACCEPT, a), key)[0])
            if ua < math.exp(-excess) or a == MAX_ATTEMPTS - 1:
                break
        out[l] = m
        tries[l] = a + 1
    return out, tries


def rbe_kspace_cell(r, q, h, alpha, m, S, coulomb=1.0):
    """RBE estimator on an explicit batch for a general cell h (weights S/p):
    dict(rho, forces, virial (full tensor), energy (with the self term),
    pressure2)."""
    m = np.asarray(m, dtype=np.int64).reshape(-1, 3)
    h = np.asarray(h, dtype=np.float64)
    res = kspace_weighted(r, q, h, alpha, m, S / m.shape[0], coulomb)
    res["energy"] = res["energy"] + self_energy(q, alpha, coulomb)
    res["pressure2"] = float(np.trace(res["virial"])) / (3.0 * abs(float(np.linalg.det(h))))
    return res
