"""Pins of the online Metropolis-Hastings sampler oracle: the proposal pmf is
the rounded normal (library normal CDF, and the frequencies of the proposal
draw itself), the move kernel leaves the law of eq. (probexpression)
invariant (exact, on a truncated lattice), and chains started far from it
reach its marginals (chi^2)."""
import math

import numpy as np
import pytest

from oracle import mh_sampler as mh
from oracle import sampler as osamp


@pytest.mark.parametrize("sigma", [0.3, 1.35, 4.5, 14.5])
def test_proposal_pmf_is_the_rounded_normal(sigma):
    from scipy import stats
    M = int(math.ceil(12 * sigma)) + 2
    q = np.array([mh.proposal_pmf(m, sigma) for m in range(-M, M + 1)])
    assert abs(q.sum() - 1.0) < 1e-14
    for m in range(-int(3 * sigma) - 1, int(3 * sigma) + 2):
        ref = stats.norm.cdf((m + 0.5) / sigma) - stats.norm.cdf((m - 0.5) / sigma)
        assert abs(mh.proposal_pmf(m, sigma) - ref) < 1e-12 * max(ref, 1e-300) + 1e-16
    # the proposal draw (rounding sigma z) has exactly this pmf
    z = np.random.default_rng(3).standard_normal((60000, 3))
    sig = [sigma] * 3
    draws = np.array([mh.proposal(sig, zi)[0] for zi in z])
    vals, cnt = np.unique(draws, return_counts=True)
    exp = np.array([mh.proposal_pmf(int(v), sigma) for v in vals]) * len(draws)
    keep = exp > 20
    chi2 = ((cnt[keep] - exp[keep]) ** 2 / exp[keep]).sum()
    dof = max(int(keep.sum()) - 1, 1)
    assert stats.chi2.sf(chi2, dof) > 1e-4


def test_move_kernel_leaves_the_law_invariant():
    # every state m != 0 with |m_j| <= 4 (tails beyond are below 1e-30 at
    # these widths): the transition matrix of one move,
    # T(m -> m') = q(m') a(m, m') and T(m -> m) = 1 - sum of the rest, must
    # satisfy pi T = pi for the discrete Gaussian pi on m != 0
    alpha = 1.0
    box = [math.pi * math.sqrt(2.0) * s for s in (0.35, 0.42, 0.3)]   # sigma_j as given
    sig = mh.sigmas(alpha, box)
    assert np.allclose(sig, (0.35, 0.42, 0.3), rtol=1e-14)
    R = range(-4, 5)
    states = [(a, b, c) for a in R for b in R for c in R if (a, b, c) != (0, 0, 0)]
    n = len(states)
    pi = np.array([math.exp(-sum(m[j] ** 2 / (2 * sig[j] ** 2) for j in range(3)))
                   for m in states])
    pi /= pi.sum()
    q = np.array([np.prod([mh.proposal_pmf(m[j], sig[j]) for j in range(3)]) for m in states])
    T = np.zeros((n, n))
    for i, m in enumerate(states):
        for k, mp in enumerate(states):
            if k != i:
                T[i, k] = q[k] * mh.acceptance(list(m), list(mp), sig)
        T[i, i] = 1.0 - T[i].sum()
    assert (T >= -1e-15).all()
    assert np.abs(pi @ T - pi).max() < 1e-14
    # and the zero vector is never proposed into
    assert mh.acceptance([1, 0, 0], [0, 0, 0], sig) == 0.0


def test_chains_from_a_bad_start_reach_the_marginals():
    from scipy import stats
    alpha, box = 0.09, (14.0, 9.0, 20.0)          # sigma = 0.95, 0.61, 1.35
    P, iters = 3000, 25
    m0 = np.tile([3, 0, 0], (P, 1))                # far out in x, nothing elsewhere
    m, acc = mh.chain_moves(m0, alpha, box, seed=21, system_id=4, step=7, iters=iters)
    assert not (m == 0).all(axis=1).any()
    assert 0.3 < acc / (P * iters) < 1.0
    for axis in range(3):
        vals = np.arange(-8, 9)
        pmf = np.array([osamp.marginal_pmf(alpha, box, axis, int(v)) for v in vals])
        cnt = np.array([(m[:, axis] == v).sum() for v in vals])
        exp = pmf * P
        keep = exp > 10
        chi2 = ((cnt[keep] - exp[keep]) ** 2 / exp[keep]).sum()
        assert stats.chi2.sf(chi2, int(keep.sum()) - 1) > 1e-4, (axis, cnt, exp)


def test_first_step_is_an_exact_draw_then_moves():
    alpha, box, P = 0.09, (20.0, 20.0, 20.0), 50
    ch = mh.MHChains(alpha, P, seed=3, system_id=1, iters=2)
    m0 = ch.sample(box, 10)
    np.testing.assert_array_equal(m0, osamp.sample_k(alpha, box, P, seed=3, system_id=1, step=10))
    m1 = ch.sample((20.1, 20.1, 20.1), 11)
    m1b, _ = mh.chain_moves(m0, alpha, (20.1, 20.1, 20.1), 3, 1, 11, iters=2)
    np.testing.assert_array_equal(m1, m1b)
    assert (m1 != m0).any(axis=1).sum() > 0
