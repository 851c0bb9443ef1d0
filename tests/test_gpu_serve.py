"""Served batching (rbe_batch_*): a system's trajectory is the same alone and
in a mix of other systems admitted at different times, fused or with
per-system launches, and equal to the one-system API's; the served path
matches the oracle's trajectory; admission respects the memory budget."""
import numpy as np
import pytest

from paper_2110_14362_amd import serve, workloads
from paper_2110_14362_amd.rbe import Batch
from tests.md_cases import oracle_trajectory

pytestmark = pytest.mark.gpu

BUDGET = 4 << 30


def request(i, n, **kw):
    r = serve.make_requests(1, seed=7000 + i, nmin=n, nmax=n, steps=kw.pop("steps", 4),
                            kinds=kw.pop("kinds", ("ions",)), **kw)[0]
    r.rid = i
    r.desc.system_id = i
    return r


def run_alone(r, steps, fused=True, precision="fp32"):
    b = Batch(BUDGET, max_systems=2, precision=precision)
    slot = serve._admit(b, r)
    for _ in range(steps):
        b.step(fused=fused)
    b.sync()
    b.check(slot)
    out = b.read(slot)
    b.close()
    return out


def test_alone_equals_mix_bitwise(gpu):
    # the water system keeps real-space neighbour lists, the ions do not
    reqs = [request(0, 1500), request(1, 4000, kinds=("water",), skin=2.0), request(2, 9000)]
    assert reqs[1].md["skin"] > 0.0 and "skin" not in reqs[0].md
    print("sizes", [r.n for r in reqs], "boxes", [r.sysd["box"].round(2).tolist() for r in reqs],
          flush=True)
    b = Batch(BUDGET, max_systems=8, precision="fp32")
    s0 = serve._admit(b, reqs[0])
    s1 = serve._admit(b, reqs[1])
    b.step()
    b.step()
    s2 = serve._admit(b, reqs[2])         # joins while the others run
    for _ in range(3):
        b.step()
    b.sync()
    mix = {}
    for r, s in ((reqs[0], s0), (reqs[1], s1), (reqs[2], s2)):
        b.check(s)
        mix[r.rid] = (b.read(s), b.slot_step(s))
    b.close()
    assert mix[0][1] == 5 and mix[2][1] == 3
    assert mix[1][0]["rigid_count"] == reqs[1].n // 3
    for r in reqs:
        got, steps = mix[r.rid]
        for fused in (True, False):
            ref = run_alone(r, steps, fused=fused)
            np.testing.assert_array_equal(got["pos"], ref["pos"])
            np.testing.assert_array_equal(got["mom"], ref["mom"])
            np.testing.assert_array_equal(got["box"], ref["box"])
        print("request %d (N=%d, %d steps): box %s, identical alone and in the mix"
              % (r.rid, r.n, steps, got["box"]), flush=True)


def wide_splitting(r, g_rc=4.5):
    """The request with alpha raised so that sqrt(alpha) rc = g_rc."""
    sysd = dict(r.sysd)
    sysd["alpha"] = (g_rc / sysd["rc"]) ** 2
    w = serve.Request(r.rid, 0.0, sysd, r.md, r.steps)
    w.desc.system_id = r.rid
    return w


def test_mixed_erfcx_series_alone_equals_mix_bitwise(gpu):
    # systems with sqrt(alpha) rc > 4 take the full-range erfcx series, the
    # others the bounded-range one; in a fused launch each instance evaluates
    # only its own systems, so every system's trajectory stays bitwise its own
    reqs = [request(0, 1500), request(1, 3000, kinds=("water",), skin=2.0),
            wide_splitting(request(2, 2000)),
            wide_splitting(request(3, 3000, kinds=("water",), skin=2.0))]
    g_rc = [float(np.sqrt(r.sysd["alpha"]) * r.sysd["rc"]) for r in reqs]
    assert g_rc[0] <= 4.0 and g_rc[1] <= 4.0 and g_rc[2] > 4.0 and g_rc[3] > 4.0
    print("sizes", [r.n for r in reqs], "g rc", np.round(g_rc, 3).tolist(), flush=True)
    b = Batch(BUDGET, max_systems=8, precision="fp32")
    slots = [serve._admit(b, r) for r in reqs]
    for _ in range(3):
        b.step()
    b.sync()
    mix = {}
    for r, sl in zip(reqs, slots):
        b.check(sl)
        mix[r.rid] = b.read(sl)
    b.close()
    for r in reqs:
        got = mix[r.rid]
        for fused in (True, False):
            ref = run_alone(r, 3, fused=fused)
            np.testing.assert_array_equal(got["pos"], ref["pos"])
            np.testing.assert_array_equal(got["mom"], ref["mom"])
            np.testing.assert_array_equal(got["box"], ref["box"])
        print("request %d (N=%d, g rc %.2f): identical alone and in the mix"
              % (r.rid, r.n, g_rc[r.rid]), flush=True)


def test_served_equals_one_system_api(gpu):
    # the served runtime launches the Fourier step as two kernels; the
    # one-system API in that form gives the same bits, and in its default
    # single launch (another chunking, so another rounding) the same
    # trajectory to FP32 rounding
    from paper_2110_14362_amd.md import NPTSystem
    r = request(3, 2500)
    steps = 4
    ref = run_alone(r, steps)
    out = {}
    for fused in (False, True):
        md = dict(r.md, types=r.sysd["types"], lj=r.sysd["lj"], fused=fused)
        sysg = NPTSystem(r.sysd, md, precision="fp32", seed=r.desc.seed,
                         system_id=r.desc.system_id)
        sysg.step(steps)
        out[fused] = sysg.state()
    np.testing.assert_array_equal(out[False]["pos"], ref["pos"])
    np.testing.assert_array_equal(out[False]["mom"], ref["mom"])
    dr = np.abs(out[True]["pos"] - ref["pos"]).max()
    dp = np.abs(out[True]["mom"] - ref["mom"]).max() / np.abs(ref["mom"]).max()
    print("single launch vs two launches over %d NPT steps: max |dr| %.2e, rel |dp| %.2e"
          % (steps, dr, dp), flush=True)
    assert dr < 1e-6 and dp < 1e-4


@pytest.mark.parametrize("kind,skin", [("ions", 0.0), ("water", 0.0), ("water", 1.0)])
def test_served_trajectory_matches_oracle(gpu, kind, skin):
    r = request(4, 1000, kinds=(kind,), skin=skin)
    assert r.md.get("skin", 0.0) == skin
    steps = 3
    got = run_alone(r, steps, precision="fp64")
    md = dict(r.md, types=r.sysd["types"], lj=r.sysd["lj"], rigid=r.sysd.get("rigid"))
    o = oracle_trajectory(r.sysd, md, np.zeros((r.n, 3)), steps, seed=r.desc.seed,
                          system_id=r.desc.system_id)
    dpos = np.abs(got["pos"] - o["pos"]).max()
    dmom = np.abs(got["mom"] - o["mom"]).max() / np.abs(o["mom"]).max()
    dbox = np.abs(got["box"] - o["box"]).max() / o["box"].max()
    print("served %s N=%d skin %g: max |dr| %.2e, rel |dp| %.2e, rel |dl| %.2e"
          % (kind, r.n, skin, dpos, dmom, dbox), flush=True)
    assert dpos < 1e-9 and dmom < 1e-9 and dbox < 1e-11


def test_admission_respects_budget(gpu):
    a, c = request(5, 3000), request(6, 3000)
    budget = a.bytes + c.bytes // 2
    b = Batch(budget, max_systems=4, precision="fp32")
    sa = serve._admit(b, a)
    assert sa is not None
    assert serve._admit(b, c) is None            # over budget: refused, nothing held
    assert b.info()["bytes"] == a.bytes
    b.step()
    b.release(sa)
    assert b.info()["bytes"] == 0
    sc = serve._admit(b, c)
    assert sc is not None
    b.step()
    b.sync()
    b.check(sc)
    b.close()


def test_served_stream_runs(gpu):
    reqs = serve.make_requests(12, seed=9100, nmin=1000, nmax=20000, steps=5,
                               kinds=("ions", "water"), skin=2.0)
    for r, t in zip(reqs, serve.poisson_arrivals(len(reqs), rate=400.0)):
        r.arrival = float(t)
    b = Batch(BUDGET, max_systems=16, precision="fp32")
    st = serve.serve(b, reqs, fused=True)
    b.close()
    print(st, flush=True)
    assert st["steps"] == 60 and all(len(r.lat) == 5 for r in reqs)
    assert st["p99_ms"] >= st["p50_ms"] > 0


# ---------------------------------------------------------------------------
# the Fourier-space step alone, served (rbe_batch_step_fourier)

def fourier_alone(r, steps, fused=True, precision="fp32"):
    b = Batch(BUDGET, max_systems=2, precision=precision)
    slot = serve._admit(b, r)
    for _ in range(steps):
        b.step(fused=fused, fourier_only=True)
    b.sync()
    b.check(slot)
    out = b.read(slot)
    b.close()
    return out


def test_fourier_steps_alone_equal_mix_bitwise(gpu):
    reqs = [request(10, 1500), request(11, 4000, kinds=("water",)), request(12, 9000)]
    b = Batch(BUDGET, max_systems=8, precision="fp32")
    s0 = serve._admit(b, reqs[0])
    s1 = serve._admit(b, reqs[1])
    b.step(fourier_only=True)
    b.step(fourier_only=True)
    s2 = serve._admit(b, reqs[2])
    for _ in range(3):
        b.step(fourier_only=True)
    b.sync()
    mix = {}
    for r, s in ((reqs[0], s0), (reqs[1], s1), (reqs[2], s2)):
        b.check(s)
        mix[r.rid] = (b.read(s), b.slot_step(s))
    b.close()
    assert mix[10][1] == 5 and mix[12][1] == 3
    for r in reqs:
        got, steps = mix[r.rid]
        # positions untouched by Fourier-only steps
        np.testing.assert_array_equal(got["pos"], np.asarray(r.sysd["pos"], dtype=np.float64))
        for fused in (True, False):
            ref = fourier_alone(r, steps, fused=fused)
            np.testing.assert_array_equal(got["forces"], ref["forces"])
        print("request %d (N=%d, %d Fourier steps): forces identical alone and in the mix"
              % (r.rid, r.n, steps), flush=True)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_fourier_step_matches_oracle(gpu, precision, tol):
    from oracle import rbe as orbe
    from oracle import sampler as osamp
    r = request(13, 1200)
    steps = 2                        # the last step's batch is that of step 1
    got = fourier_alone(r, steps, precision=precision)
    s = r.sysd
    m = osamp.sample_k(s["alpha"], s["box"], s["p"], seed=r.desc.seed,
                       system_id=r.desc.system_id, step=steps - 1)
    S = osamp.box_tables(s["alpha"], s["box"])["S"]
    o = orbe.rbe_kspace(np.asarray(s["pos"]), s["q"], s["box"], s["alpha"], m, S,
                        coulomb=s["coulomb"])
    err = np.linalg.norm(got["forces"] - o["forces"]) / np.linalg.norm(o["forces"])
    print("served Fourier step %s: force RMS rel. %.2e" % (precision, err), flush=True)
    assert err < tol


# ---------------------------------------------------------------------------
# served systems on the online Metropolis-Hastings sampler

def test_mh_system_alone_equals_mix_bitwise(gpu):
    reqs = [request(20, 2000), request(21, 3000, sampler="mh"), request(22, 2500, kinds=("water",))]
    assert reqs[1].desc.sampler == 1 and reqs[0].desc.sampler == 0
    b = Batch(BUDGET, max_systems=8, precision="fp32")
    slots = [serve._admit(b, r) for r in reqs]
    for _ in range(4):
        b.step()
    b.sync()
    mix = {r.rid: b.read(s) for r, s in zip(reqs, slots)}
    b.close()
    for r in reqs:
        for fused in (True, False):
            ref = run_alone(r, 4, fused=fused)
            np.testing.assert_array_equal(mix[r.rid]["pos"], ref["pos"])
            np.testing.assert_array_equal(mix[r.rid]["mom"], ref["mom"])


def test_served_mh_fourier_steps_follow_the_oracle_chain(gpu):
    from oracle import mh_sampler as omh
    from oracle import rbe as orbe
    from oracle import sampler as osamp
    from tests.md_cases import INIT_STEP
    r = request(23, 900, sampler="mh")
    steps = 3
    got = fourier_alone(r, steps, precision="fp64")
    s = r.sysd
    chains = omh.MHChains(s["alpha"], s["p"], seed=r.desc.seed, system_id=r.desc.system_id)
    chains.sample(s["box"], INIT_STEP)              # the admission's evaluation
    for k in range(steps):
        m = chains.sample(s["box"], k)
    S = osamp.box_tables(s["alpha"], s["box"])["S"]
    o = orbe.rbe_kspace(np.asarray(s["pos"]), s["q"], s["box"], s["alpha"], m, S,
                        coulomb=s["coulomb"])
    err = np.linalg.norm(got["forces"] - o["forces"]) / np.linalg.norm(o["forces"])
    print("served MH Fourier step: force RMS rel. %.2e, oracle acceptance %.2f"
          % (err, chains.accepted / (steps * s["p"])), flush=True)
    assert err < 1e-10


def test_served_mh_npt_trajectory_matches_oracle(gpu):
    # NPT steps of a served system on the Metropolis-Hastings sampler: the
    # chains must move towards the law of the cell the integrator's first
    # half has just produced (the cell changes every step), so the trajectory
    # equals the oracle integrator driven by the oracle chains
    from oracle import mh_sampler as omh
    r = request(24, 1000, sampler="mh")
    steps = 4
    got = run_alone(r, steps, precision="fp64")
    s = r.sysd
    chains = omh.MHChains(s["alpha"], s["p"], seed=r.desc.seed, system_id=r.desc.system_id)
    md = dict(r.md, types=s["types"], lj=s["lj"], rigid=s.get("rigid"))
    o = oracle_trajectory(s, md, np.zeros((r.n, 3)), steps, seed=r.desc.seed,
                          system_id=r.desc.system_id, draw=chains.sample)
    dpos = np.abs(got["pos"] - o["pos"]).max()
    dmom = np.abs(got["mom"] - o["mom"]).max() / np.abs(o["mom"]).max()
    dbox = np.abs(got["box"] - o["box"]).max() / o["box"].max()
    moved = np.abs(o["box"] - np.asarray(s["box"])).max() / o["box"].max()
    print("served MH NPT N=%d: max |dr| %.2e, rel |dp| %.2e, rel |dl| %.2e (cell moved %.1e), "
          "oracle acceptance %.2f" % (r.n, dpos, dmom, dbox, moved,
                                      chains.accepted / ((steps + 1) * s["p"])), flush=True)
    assert moved > 1e-9
    assert dpos < 1e-9 and dmom < 1e-9 and dbox < 1e-11
