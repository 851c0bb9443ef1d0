"""Frequency sampler of the random batch Ewald method (FP64 reference).

TEST INFRASTRUCTURE ONLY (FP64 CPU oracle; imported by tests, the smoke check
and the benchmark's CPU-baseline leg, never by the product path).

What it follows:
* Section 4.2, eq. (S) and (psf): the normaliser S is the sum of
  exp(-|k|^2/(4 alpha)) over all nonzero k of the reciprocal lattice.  For an
  orthorhombic cell diag(l1, l2, l3) with k = 2 pi (m1/l1, m2/l2, m3/l3) the
  weight factorises over axes, w_j(m) = exp(-pi^2 m^2 / (alpha l_j^2)), so
  S = H1*H2*H3 - 1 with H_j the one-axis sum (cubic case: S = H^3 - 1).
* Section 4.2, eq. (probexpression): the law of one sample is
  S^-1 exp(-|k|^2/(4 alpha)) over k != 0, a product of one-axis discrete
  Gaussians restricted to m != 0.
* Appendix C, first remark on sampling: for a rectangular cell the three
  components are independent discrete Gaussians, each with its own side length.
* Section 4.3, the parallel sampling strategy (sample reuse, `ReusedDraws`):
  the batches of M consecutive steps are drawn at the first of them, from the
  law of the cell at that step; the paper notes the small error this adds
  while the cell changes slowly.

The paper draws the sample with a Metropolis chain (section 4.3).  This code
draws exact independent samples of the same law (reading: exact i.i.d.
sampling replaces the chain; the chain's burn-in and proposal details are not
fixed by the paper).  Stream specification shared with the device sampler:

  key      = (seed, system_id)
  counter  = (step, l, TAG_KSAMPLE, 0)  for sample l of a step
  u0..u3   = top 53 bits of the four Philox4x64-10 outputs, times 2^-53
  The nonzero event is split by its first nonzero axis:
     case x (m1 != 0)          with weight  T1 * H2 * H3
     case y (m1 == 0, m2 != 0) with weight  T2 * H3
     case z (m1 == m2 == 0)    with weight  T3
  where T_j = H_j - 1 is the one-axis sum over m != 0; so S = Tx*Hy*Hz + Ty*Hz + Tz.
  u0*S picks the case; the pivot axis is drawn from its m != 0 table with its
  own uniform, later axes from their full tables, earlier axes are 0.
  Axis j uses uniform u_{j+1}.  A table draw is the inverse CDF:
  the first index i with C[i] > u * C[last], C the running sum of weights
  in increasing m.
"""

import math
import numpy as np

from .philox import philox4x64, u01

TAG_KSAMPLE = 0x6B73616D   # 'ksam': stream tag of the frequency draws

# tail cut: weights below 2^-53 of the m = 0 weight are dropped
TAIL_LN = 53.0 * math.log(2.0)


def axis_mcut(alpha, ell):
    """Largest |m| kept on an axis: exp(-pi^2 m^2/(alpha l^2)) >= 2^-53."""
    return int(math.ceil(math.sqrt(TAIL_LN * alpha * ell * ell) / math.pi))


def axis_weights(alpha, ell):
    """(m values, weights) for one axis, m = -mcut..mcut in increasing order."""
    mc = axis_mcut(alpha, ell)
    m = np.arange(-mc, mc + 1, dtype=np.int64)
    w = np.exp(-(math.pi ** 2) * (m.astype(np.float64) ** 2) / (alpha * ell * ell))
    return m, w


def axis_tables(alpha, ell):
    """Full and m != 0 cumulative tables of one axis.

    Returns dict with m_full, c_full, m_nz, c_nz, H (= c_full[-1]),
    T (= c_nz[-1], the m != 0 mass).
    """
    m, w = axis_weights(alpha, ell)
    c_full = np.cumsum(w)
    nz = m != 0
    m_nz = m[nz]
    c_nz = np.cumsum(w[nz])
    return dict(m_full=m, c_full=c_full, m_nz=m_nz, c_nz=c_nz,
                H=float(c_full[-1]), T=float(c_nz[-1]))


def box_tables(alpha, box):
    """Per-axis tables plus the case weights and S for an orthorhombic box."""
    tabs = [axis_tables(alpha, float(l)) for l in box]
    Tx, Ty, Tz = (t["T"] for t in tabs)
    Hx, Hy, Hz = (1.0 + t["T"] for t in tabs)
    wx = Tx * Hy * Hz
    wy = Ty * Hz
    wz = Tz
    S = wx + wy + wz
    return dict(axes=tabs, case_w=(wx, wy, wz), S=S, H=(Hx, Hy, Hz))


def normaliser_poisson(alpha, box, nterms=8):
    """S from the Poisson-summed form of H (eq. psf): independent of the tables.

    H_j = sqrt(alpha l_j^2/pi) * sum_n exp(-alpha n^2 l_j^2).
    """
    Hs = []
    for l in box:
        pref = math.sqrt(alpha * l * l / math.pi)
        s = sum(math.exp(-alpha * n * n * l * l) for n in range(-nterms, nterms + 1))
        Hs.append(pref * s)
    return Hs[0] * Hs[1] * Hs[2] - 1.0


def _inverse_cdf(m_vals, cum, u):
    target = u * cum[-1]
    i = int(np.searchsorted(cum, target, side="right"))   # first C[i] > target
    if i >= len(cum):
        i = len(cum) - 1
    return int(m_vals[i])


def sample_k(alpha, box, P, seed, system_id, step, tables=None):
    """Draw P nonzero integer vectors m (P x 3 int64) for one step."""
    tb = box_tables(alpha, box) if tables is None else tables
    wx, wy, wz = tb["case_w"]
    S = tb["S"]
    ax = tb["axes"]
    out = np.zeros((P, 3), dtype=np.int64)
    key = (seed, system_id)
    for l in range(P):
        r = philox4x64((step, l, TAG_KSAMPLE, 0), key)
        u = [u01(x) for x in r]
        t = u[0] * S
        if t < wx:
            pivot = 0
        elif t < wx + wy:
            pivot = 1
        else:
            pivot = 2
        for j in range(3):
            if j < pivot:
                out[l, j] = 0
            elif j == pivot:
                out[l, j] = _inverse_cdf(ax[j]["m_nz"], ax[j]["c_nz"], u[j + 1])
            else:
                out[l, j] = _inverse_cdf(ax[j]["m_full"], ax[j]["c_full"], u[j + 1])
    return out


def marginal_pmf(alpha, box, axis, m):
    """Exact marginal pmf of component `axis` under the sampling law."""
    Hs = []
    for l in box:
        mm, w = axis_weights(alpha, float(l))
        Hs.append(float(np.sum(w)))
    S = Hs[0] * Hs[1] * Hs[2] - 1.0
    l = float(box[axis])
    m = np.asarray(m, dtype=np.float64)
    w = np.exp(-(math.pi ** 2) * m * m / (alpha * l * l))
    other = 1.0
    for j in range(3):
        if j != axis:
            other *= Hs[j]
    return w * (other - (m == 0)) / S


class ReusedDraws:
    """Sample reuse (section 4.3, parallel strategy).  The steps are grouped
    in blocks [kM, (k+1)M) of the step counter; the cell given at a block's
    first sampled step is frozen, and the batch of every step s of the block
    is the exact draw of step s (counter (s, l, 'ksam', 0)) from the frozen
    cell's law.  The draws of a block are independent, as the M independent
    sampling processes of the paper are; step j of a block takes the j-th.
    period = 1 is the exact sampler of the current cell."""

    def __init__(self, alpha, P, seed, system_id, period):
        self.alpha, self.P = alpha, P
        self.seed, self.system_id = seed, system_id
        self.period = int(period)
        self.block = None
        self.frozen = None

    def sample(self, box, step):
        block = int(step) // self.period
        if self.block is None or block != self.block:
            self.block = block
            self.frozen = tuple(float(b) for b in box)
        return sample_k(self.alpha, self.frozen, self.P, self.seed, self.system_id, step)
