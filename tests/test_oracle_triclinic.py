"""Pins of the triclinic-cell oracle (appendix C): the normaliser against its
Poisson-summed form, the envelope's validity, the rejection sampler's joint
law (chi-square over every mode of a skewed cell, with planted mistakes that
must fail), the estimator's forces against finite differences of its energy,
and its mean over many batches against the Ewald Fourier-space forces and
full virial tensor."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import ewald
from oracle import sampler as osamp
from oracle import triclinic as tri
from oracle.philox import philox4x64, u01
from paper_2110_14362_amd import workloads

SKEW = tri.cell_matrix(6.0, 5.0, 7.0, 1.5, -1.0, 2.0)
ALPHA = 0.3


@pytest.mark.parametrize("h", [SKEW, tri.cell_matrix(6.0, 5.0, 7.0),
                               tri.cell_matrix(9.0, 9.0, 9.0, 2.0, 0.0, -1.5)])
def test_normaliser_equals_poisson_form(h):
    S = tri.normaliser(ALPHA, h)
    assert abs(S - tri.normaliser_poisson(ALPHA, h)) < 1e-12 * S


def test_rectangular_cell_reduces_to_the_separable_sampler():
    h = tri.cell_matrix(6.0, 5.0, 7.0)
    S = osamp.box_tables(ALPHA, (6.0, 5.0, 7.0))["S"]
    assert abs(tri.normaliser(ALPHA, h) - S) < 1e-13 * S
    m, tries = tri.sample_k_cell(ALPHA, h, 3000, 5, 1, 4)
    ref = osamp.sample_k(ALPHA, (6.0, 5.0, 7.0), 3000, 5, 1, 4)
    assert np.all(tries == 1)                    # A is diagonal: every proposal accepted
    assert np.mean(np.all(m == ref, axis=1)) > 0.999


def test_envelope_lies_below_the_law():
    A = tri.quad_matrix(ALPHA, SKEW)
    d = tri.envelope(ALPHA, SKEW)
    assert np.linalg.eigvalsh(A - np.diag(d)).min() >= 0.0
    m, Q = tri.ellipsoid_modes(A, 60.0)
    assert np.all(Q - (m * m) @ d >= -1e-12 * np.maximum(Q, 1.0))


def _chi2_p(draws, modes, prob):
    index = {tuple(int(v) for v in mm): i for i, mm in enumerate(modes)}
    cnt = np.zeros(len(modes) + 1)
    for row in draws:
        cnt[index.get(tuple(int(v) for v in row), len(modes))] += 1
    exp = np.append(prob, 0.0) * len(draws)
    big = exp >= 5.0
    obs = np.append(cnt[big], cnt[~big].sum())
    ex = np.append(exp[big], exp[~big].sum())
    keep = ex > 0
    chi2 = ((obs[keep] - ex[keep]) ** 2 / ex[keep]).sum()
    return stats.chi2.sf(chi2, int(keep.sum()) - 1)


def test_rejection_sampler_draws_the_joint_law():
    modes, prob = tri.law(ALPHA, SKEW)
    draws = np.concatenate([tri.sample_k_cell(ALPHA, SKEW, 5000, 11, 0, s)[0] for s in range(4)])
    assert not np.any(np.all(draws == 0, axis=1))
    p_ok = _chi2_p(draws, modes, prob)
    # planted mistakes: every proposal accepted (the envelope's law); the
    # tilt ignored (a rectangular cell with the same diagonal of A)
    d = tri.envelope(ALPHA, SKEW)
    tab = tri.proposal_tables(d)
    no_reject = np.array([tri.propose(tab, [u01(x) for x in philox4x64((0, l, osamp.TAG_KSAMPLE, 0),
                                                                          (11, 0))])
                          for l in range(20000)])
    tab_diag = tri.proposal_tables(np.diag(tri.quad_matrix(ALPHA, SKEW)))
    no_tilt = np.array([tri.propose(tab_diag, [u01(x) for x in philox4x64((1, l, osamp.TAG_KSAMPLE, 0),
                                                                            (11, 0))])
                        for l in range(20000)])
    p_bad1 = _chi2_p(no_reject, modes, prob)
    p_bad2 = _chi2_p(no_tilt, modes, prob)
    print("joint law chi-square p: rejection sampler %.3g, no rejection %.3g, tilt ignored %.3g"
          % (p_ok, p_bad1, p_bad2))
    assert p_ok > 1e-3
    assert p_bad1 < 1e-8 and p_bad2 < 1e-8


def test_triclinic_estimator_force_is_minus_energy_gradient():
    s = workloads.random_neutral(20, (6.0, 5.0, 7.0), seed=4)
    r = s["pos"] @ np.linalg.inv(np.diag([6.0, 5.0, 7.0])).T @ SKEW.T     # into the skew cell
    S = tri.normaliser(ALPHA, SKEW)
    m, _ = tri.sample_k_cell(ALPHA, SKEW, 30, 3, 1, 0)
    res = tri.rbe_kspace_cell(r, s["q"], SKEW, ALPHA, m, S)
    F = res["forces"]
    eps = 1e-6
    for i, c in ((0, 0), (7, 1), (13, 2)):
        rp = r.copy(); rp[i, c] += eps
        rm = r.copy(); rm[i, c] -= eps
        fd = -(tri.rbe_kspace_cell(rp, s["q"], SKEW, ALPHA, m, S)["energy"]
               - tri.rbe_kspace_cell(rm, s["q"], SKEW, ALPHA, m, S)["energy"]) / (2 * eps)
        assert abs(fd - F[i, c]) < 1e-7 * max(1.0, np.abs(F).max())
    assert np.abs(F.sum(axis=0)).max() < 1e-11 * np.abs(F).max()


def test_triclinic_estimator_is_unbiased():
    # mean of the batch estimator over 2.5e4 draws against the Ewald
    # Fourier-space forces and full virial tensor of the skew cell, component
    # by component within a few standard errors; the same estimator on draws
    # of the envelope's law (every proposal accepted) is excluded.  (S itself
    # hardly depends on the tilt: it is (alpha/pi)^(3/2) V - 1 up to terms of
    # exp(-alpha |h n|^2).)
    s = workloads.random_neutral(16, (6.0, 5.0, 7.0), seed=9)
    r = s["pos"] @ np.linalg.inv(np.diag([6.0, 5.0, 7.0])).T @ SKEW.T
    q = s["q"]
    S = tri.normaliser(ALPHA, SKEW)
    modes, w = ewald.ewald_modes(SKEW, ALPHA)
    ref = ewald.kspace_weighted(r, q, SKEW, ALPHA, modes, w)
    est = []
    for b in range(100):
        m, _ = tri.sample_k_cell(ALPHA, SKEW, 250, 21, 0, b)
        e = tri.rbe_kspace_cell(r, q, SKEW, ALPHA, m, S)
        est.append(np.concatenate([e["forces"].ravel(), e["virial"].ravel()]))
    est = np.array(est)
    mean, se = est.mean(axis=0), est.std(axis=0, ddof=1) / math.sqrt(len(est))
    want = np.concatenate([ref["forces"].ravel(), ref["virial"].ravel()])
    z = (mean - want) / se
    print("triclinic estimator mean: max |z| %.2f, mean z^2 %.2f over %d components"
          % (np.abs(z).max(), (z * z).mean(), len(z)))
    assert np.abs(z).max() < 4.5 and (z * z).mean() < 1.6
    tab = tri.proposal_tables(tri.envelope(ALPHA, SKEW))
    bad = []
    for b in range(100):
        m = np.array([tri.propose(tab, [u01(x) for x in philox4x64((b, l, osamp.TAG_KSAMPLE, 0),
                                                                      (21, 0))])
                      for l in range(250)])
        e = tri.rbe_kspace_cell(r, q, SKEW, ALPHA, m, S)
        bad.append(np.concatenate([e["forces"].ravel(), e["virial"].ravel()]))
    zb = (np.mean(bad, axis=0) - want) / se
    assert (zb * zb).mean() > 4.0
