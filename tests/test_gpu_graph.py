"""HIP-graph replay of lbm_step (lbm_set_graph_steps) against plain launches.

Same arithmetic, so the states must be bitwise equal.  Every check follows several
replays with eager work in between (moments, population reads, host syncs), and
lbm_set_gamma / lbm_set_solid in the middle of a run drop the captured graphs, so
the replayed run must follow the new values exactly as the plain run does.
"""
import numpy as np
import pytest

from cases import case, mrt_rates

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _lbm():
    from paper_1909_12390_amd import lbm
    return lbm


def pair(lattice, shape, storage, graph_steps, solid=None, psi_wall=0.0, schedule="two_pass"):
    c = case(lattice, 3, shape, seed=5, u_amp=0.01)
    rates = mrt_rates(lattice, 0.8)
    kw = dict(collision="mrt", forcing="edm", storage=storage, mrt_s=rates, solid=solid, psi_wall=psi_wall,
              schedule=schedule)
    lbm = _lbm()
    a = lbm.LbmContext(c["mix"], lattice, c["shape"], c["T"], 0.8, 1.16, c["gamma"], c["rho0"], c["u0"], **kw)
    b = lbm.LbmContext(c["mix"], lattice, c["shape"], c["T"], 0.8, 1.16, c["gamma"], c["rho0"], c["u0"],
                       graph_steps=graph_steps, **kw)
    return c, a, b


def same(a, b):
    fa = a.get_populations().cpu().numpy()
    fb = b.get_populations().cpu().numpy()
    a.check()
    b.check()
    return np.array_equal(fa, fb)


@pytest.mark.parametrize("lattice,shape", [("D2Q9", (45, 70)), ("D3Q19", (13, 14, 15))])
@pytest.mark.parametrize("storage", ["f64", "f16"])
@pytest.mark.parametrize("schedule", ["two_pass", "blocked"])
def test_graph_replay_equals_plain_steps(lattice, shape, storage, schedule):
    print(f"case graph replay {lattice} {storage} {schedule}", flush=True)
    c, a, b = pair(lattice, shape, storage, graph_steps=9, schedule=schedule)   # rounded up to 10
    for n in (20, 7, 33, 10):          # several replays, a remainder, eager work between them
        a.step(n)
        b.step(n)
        ma = a.moments()
        mb = b.moments()
        assert np.array_equal(ma["mass"], mb["mass"])
        assert same(a, b)
    # new gamma: the captured graphs are dropped and recaptured with it
    g = np.asarray(c["gamma"]) * np.array([0.97, 0.98, 1.0])   # gamma stays in (0, 1]
    a.set_gamma(g)
    b.set_gamma(g)
    a.step(30)
    b.step(30)
    assert same(a, b)
    a.close()
    b.close()


@pytest.mark.parametrize("storage", ["f64", "f16"])
def test_graph_replay_with_walls_and_mask_change(storage):
    print(f"case graph replay walls {storage}", flush=True)
    from oracle import lbm as olbm
    from oracle_backend import to_mixture
    shape = (45, 70)
    solid = np.random.default_rng([9, 1]).uniform(size=shape) < 0.12
    c0 = case("D2Q9", 3, shape, seed=5, u_amp=0.01)
    pw = 1.3 * float(olbm.pseudo_potential(c0["rho0"][:, 0, 0][:, None], c0["T"], to_mixture(c0["mix"]), -1.0)[0])
    c, a, b = pair("D2Q9", shape, storage, graph_steps=8, solid=solid, psi_wall=pw)
    a.step(24)
    b.step(24)
    assert same(a, b)
    solid2 = solid.copy()
    solid2[5:9, 10:20] = True
    a.set_solid(solid2, 1.05 * pw)
    b.set_solid(solid2, 1.05 * pw)
    a.step(17)
    b.step(17)
    assert same(a, b)
    a.close()
    b.close()


def test_graph_steps_rejected_on_the_default_stream():
    lbm = _lbm()
    c = case("D2Q9", 2, (16, 16), seed=1)
    ctx = lbm.LbmContext(c["mix"], "D2Q9", c["shape"], c["T"], 0.8, 1.16, c["gamma"], c["rho0"], forcing="edm")
    if ctx.stream.cuda_stream == 0:
        with pytest.raises(lbm.LbmError):
            lbm._check(lbm.lib().lbm_set_graph_steps(ctx._ctx, 4))
    ctx.close()
