"""Online Metropolis-Hastings frequency sampler (FP64 reference).

TEST INFRASTRUCTURE ONLY (FP64 CPU oracle; imported by tests, the smoke check
and the benchmark's CPU-baseline leg, never by the product path).

What it follows: section 4.3 (sampling the frequencies), the online approach.
Every step, each sample starts from its value at the previous step and takes
Metropolis-Hastings moves towards the law of eq. (probexpression), a product
over axes of exp(-pi^2 m_j^2/(alpha l_j^2)) on m != 0, with the current cell.
The proposal is the continuous Gaussian, rounded: the probability that it
falls into [m - 1/2, m + 1/2) is a difference of normal distribution
functions, so the acceptance ratio is cheap.

Readings (the paper fixes neither):
* per axis the discrete law is exp(-m^2/(2 sigma_j^2)) with
  sigma_j^2 = alpha l_j^2/(2 pi^2); the proposal draws z_j ~ N(0, sigma_j^2)
  and takes the integer m_j = floor(z_j + 1/2) whose interval holds it, so
  q_j(m) = Phi((m + 1/2)/sigma_j) - Phi((m - 1/2)/sigma_j);
* the proposal does not depend on the current state (an independence
  chain), so a move m -> m' is accepted with probability
  min(1, pi(m') q(m) / (pi(m) q(m'))), pi(0) = 0: a proposal m' = 0 is
  rejected;
* one chain per batch slot l (P independent chains), `iters` moves per step;
* a chain starts from an exact draw of the law (sampler.sample_k) at the
  first step it is used; its state then carries over from step to step,
  whatever the cell did in between.

Stream (key (seed, system_id)): move it of chain l at step s takes
  counter (s, l, TAG_MH, 2 it):      u0..u3 -> z_x = sqrt(-2 ln(1 - u0)) cos(2 pi u1),
                                     z_y = sqrt(-2 ln(1 - u0)) sin(2 pi u1),
                                     z_z = sqrt(-2 ln(1 - u2)) cos(2 pi u3);
  counter (s, l, TAG_MH, 2 it + 1):  u0 -> accept if u0 < the ratio.
The ratio is formed as exp(-sum_j (m'_j^2 - m_j^2)/(2 sigma_j^2)) times
prod_j q_j(m_j)/q_j(m'_j), axes in order x, y, z.
"""

import math

import numpy as np

from .philox import philox4x64, u01
from . import sampler as exact

TAG_MH = 0x6D686368   # 'mhch': stream tag of the chain moves

SQRT2 = math.sqrt(2.0)


def sigmas(alpha, box):
    """Per-axis sigma_j = sqrt(alpha) l_j/(pi sqrt 2) of the discrete law."""
    return [math.sqrt(alpha) * float(l) / (math.pi * SQRT2) for l in box]


def proposal_pmf(m, sigma):
    """q(m) = Phi((m + 1/2)/sigma) - Phi((m - 1/2)/sigma) for one axis, formed
    from the complementary error function on the side away from the mode
    (no cancellation in the tails)."""
    s = sigma * SQRT2
    if m == 0:
        return math.erf(0.5 / s)
    a = abs(m)
    return 0.5 * (math.erfc((a - 0.5) / s) - math.erfc((a + 0.5) / s))


def proposal(sig, z):
    """Rounded continuous Gaussian: the integer whose [m - 1/2, m + 1/2) holds sigma z."""
    return [int(math.floor(sig[j] * z[j] + 0.5)) for j in range(3)]


def acceptance(m, mp, sig):
    """min(1, pi(m') q(m) / (pi(m) q(m'))) for the independence proposal."""
    if mp[0] == 0 and mp[1] == 0 and mp[2] == 0:
        return 0.0
    e = 0.0
    for j in range(3):
        e += (mp[j] * mp[j] - m[j] * m[j]) / (2.0 * sig[j] * sig[j])
    r = math.exp(-e)
    for j in range(3):
        r *= proposal_pmf(m[j], sig[j]) / proposal_pmf(mp[j], sig[j])
    return min(1.0, r)


def _move_randoms(seed, system_id, step, l, it):
    r = philox4x64((step, l, TAG_MH, 2 * it), (seed, system_id))
    u = [u01(x) for x in r]
    a = math.sqrt(-2.0 * math.log(1.0 - u[0]))
    b = math.sqrt(-2.0 * math.log(1.0 - u[2]))
    z = (a * math.cos(2.0 * math.pi * u[1]), a * math.sin(2.0 * math.pi * u[1]),
         b * math.cos(2.0 * math.pi * u[3]))
    ua = u01(philox4x64((step, l, TAG_MH, 2 * it + 1), (seed, system_id))[0])
    return z, ua


def chain_moves(m_prev, alpha, box, seed, system_id, step, iters=1):
    """The batch of `step`: every chain l moved `iters` times from m_prev[l].
    Returns (m [P][3] int64, accepted moves)."""
    sig = sigmas(alpha, box)
    out = np.array(m_prev, dtype=np.int64).copy()
    acc = 0
    for l in range(out.shape[0]):
        m = [int(v) for v in out[l]]
        for it in range(iters):
            z, ua = _move_randoms(seed, system_id, step, l, it)
            mp = proposal(sig, z)
            if ua < acceptance(m, mp, sig):
                m = mp
                acc += 1
        out[l] = m
    return out, acc


class MHChains:
    """P chains carried from step to step (the first step draws them exactly)."""

    def __init__(self, alpha, P, seed, system_id, iters=1):
        self.alpha, self.P, self.iters = alpha, P, iters
        self.seed, self.sysid = seed, system_id
        self.m = None
        self.accepted = 0

    def sample(self, box, step):
        if self.m is None:
            self.m = exact.sample_k(self.alpha, box, self.P, seed=self.seed,
                                    system_id=self.sysid, step=step)
        else:
            self.m, a = chain_moves(self.m, self.alpha, box, self.seed, self.sysid, step,
                                    self.iters)
            self.accepted += a
        return self.m.copy()
