"""Pins of the sample-reuse oracle (section 4.3, parallel sampling strategy):
draws inside a block follow the law of the cell frozen at the block's first
step and not the current cell's (chi^2 against both marginals), period 1 is
the exact sampler of the current cell, and the expected estimator under a
stale law approaches the Ewald sum with a bias linear in the cell change."""
import numpy as np
import pytest

from oracle import ewald
from oracle import rbe as orbe
from oracle import sampler as osamp
from paper_2110_14362_amd import workloads


def _chi2_p(draws, alpha, box, axis):
    from scipy import stats
    vals = np.arange(-12, 13)
    pmf = np.array([osamp.marginal_pmf(alpha, box, axis, int(v)) for v in vals])
    cnt = np.array([(draws[:, axis] == v).sum() for v in vals])
    exp = pmf * len(draws)
    keep = exp > 10
    chi2 = ((cnt[keep] - exp[keep]) ** 2 / exp[keep]).sum()
    return stats.chi2.sf(chi2, int(keep.sum()) - 1)


def test_block_draws_follow_the_frozen_cell():
    alpha, P, M = 0.09, 400, 8
    small, large = (12.0, 12.0, 12.0), (17.0, 17.0, 17.0)
    rd = osamp.ReusedDraws(alpha, P, seed=5, system_id=2, period=M)
    # block 0: frozen at the small cell, the cell then jumps to the large one
    rd.sample(small, 0)
    inside = np.concatenate([rd.sample(large, s) for s in range(1, M)])
    # block 1: its first step freezes the large cell
    nxt = np.concatenate([rd.sample(large, s) for s in range(M, 2 * M - 1)])
    for axis in range(3):
        assert _chi2_p(inside, alpha, small, axis) > 1e-4
        assert _chi2_p(inside, alpha, large, axis) < 1e-8
        assert _chi2_p(nxt, alpha, large, axis) > 1e-4
        assert _chi2_p(nxt, alpha, small, axis) < 1e-8


def test_period_one_is_the_exact_sampler():
    alpha, P = 0.3, 40
    rd = osamp.ReusedDraws(alpha, P, seed=9, system_id=0, period=1)
    for s in range(5):
        box = (10.0 + 0.3 * s, 10.0, 10.5 - 0.2 * s)
        np.testing.assert_array_equal(rd.sample(box, s),
                                      osamp.sample_k(alpha, box, P, 9, 0, s))


def test_first_sampled_step_of_a_block_freezes_it():
    # a run that starts inside a block freezes the cell of its first call;
    # a call at a later block re-freezes even when steps were skipped
    alpha, P, M = 0.3, 16, 4
    rd = osamp.ReusedDraws(alpha, P, seed=1, system_id=3, period=M)
    b1, b2, b3 = (10.0, 10.0, 10.0), (10.4, 10.4, 10.4), (11.0, 11.0, 11.0)
    g = rd.sample(b1, 2)
    np.testing.assert_array_equal(g, osamp.sample_k(alpha, b1, P, 1, 3, 2))
    g = rd.sample(b2, 3)
    np.testing.assert_array_equal(g, osamp.sample_k(alpha, b1, P, 1, 3, 3))
    g = rd.sample(b3, 9)                 # block 2 (steps 8..11), block 1 skipped
    np.testing.assert_array_equal(g, osamp.sample_k(alpha, b3, P, 1, 3, 9))


def test_reuse_bias_is_first_order_in_the_cell_change():
    s = workloads.random_neutral(24, (9.0, 9.0, 9.0), seed=11)
    alpha = 0.3
    box = np.array([9.0, 9.0, 9.0])
    r, q = s["pos"], s["q"]
    exact = ewald.kspace_weighted(r, q, np.diag(box), alpha, *ewald.ewald_modes(np.diag(box), alpha))
    same = orbe.reuse_expected(r, q, box, box, alpha)
    scale = np.abs(exact["forces"]).max()
    # unbiased without reuse: the weights reduce to the Ewald ones
    assert np.abs(same["forces"] - exact["forces"]).max() < 1e-11 * scale
    assert abs(same["energy"] - exact["energy"]) < 1e-11 * abs(exact["energy"])
    biases = []
    for d in (1e-4, 2e-4, 4e-4):
        e = orbe.reuse_expected(r, q, box, box * (1.0 - d), alpha)
        biases.append(np.abs(e["forces"] - exact["forces"]).max() / scale)
    # linear in the cell change, and small: the expected force moves by a
    # fraction of order the relative cell change
    assert biases[1] / biases[0] == pytest.approx(2.0, rel=0.02)
    assert biases[2] / biases[1] == pytest.approx(2.0, rel=0.02)
    assert 1e-6 < biases[0] < 1e-2


def test_reuse_expected_is_the_mean_of_stale_batches():
    # Monte Carlo pin of reuse_expected at a stale cell: batches drawn by
    # ReusedDraws from the law of a frozen cell 4 % smaller than the current
    # one, each evaluated by the RBE estimator at the CURRENT cell (weight
    # S_now/p, eq. (appforce), (apppress)), average to reuse_expected within
    # a few standard errors, component by component.  A version without the
    # S_now/S_frozen factor (weights w_frozen(m) alone) lies many standard
    # errors away, and so does the unbiased Ewald sum.
    s = workloads.random_neutral(24, (9.0, 9.0, 9.0), seed=11)
    alpha, P, nb = 0.3, 400, 250
    box = np.array([9.0, 9.0, 9.0])
    frozen = box * 0.96
    r, q = s["pos"], s["q"]
    rd = osamp.ReusedDraws(alpha, P, seed=17, system_id=4, period=10 ** 6)
    rd.sample(tuple(frozen), 0)                     # the block's first step freezes this cell
    S_now = osamp.box_tables(alpha, tuple(box))["S"]
    self_e = ewald.self_energy(q, alpha, 1.0)
    est = []
    for step in range(1, nb + 1):
        m = rd.sample(tuple(box), step)
        e = orbe.rbe_kspace(r, q, box, alpha, m, S_now)
        est.append(np.concatenate([e["forces"].ravel(), e["virial"][np.triu_indices(3)],
                                   [e["energy"] - self_e]]))
    est = np.array(est)
    mean, se = est.mean(axis=0), est.std(axis=0, ddof=1) / np.sqrt(nb)

    def flat(d):
        return np.concatenate([d["forces"].ravel(), d["virial"][np.triu_indices(3)],
                               [d["energy"]]])

    z = (mean - flat(orbe.reuse_expected(r, q, box, frozen, alpha))) / se
    print("stale-law expectation: max |z| %.2f, mean z^2 %.2f over %d components"
          % (np.abs(z).max(), (z * z).mean(), len(z)))
    assert np.abs(z).max() < 4.5
    assert 0.6 < (z * z).mean() < 1.5
    # planted mistakes: the S_now/S_frozen factor dropped; no reuse bias at all
    m_all, _ = ewald.ewald_modes(np.diag(np.maximum(box, frozen)), alpha, 1e-16)
    k2f = (((2.0 * np.pi) * m_all / frozen[None, :]) ** 2).sum(axis=1)
    wrong = ewald.kspace_weighted(r, q, np.diag(box), alpha, m_all, np.exp(-k2f / (4.0 * alpha)))
    unbiased = ewald.kspace_weighted(r, q, np.diag(box), alpha,
                                     *ewald.ewald_modes(np.diag(box), alpha))
    for other in (wrong, unbiased):
        zo = (mean - flat(other)) / se
        assert np.abs(zo).max() > 8.0
        assert (zo * zo).mean() > 4.0
