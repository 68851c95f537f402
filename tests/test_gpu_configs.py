"""Parity on the seeded benchmark configurations themselves, in the launch
configurations bench.py times.

* C1 (binary D2Q9 64^2 drop, float64, BGK + exact-difference forcing) and C2
  (ternary D2Q9 256^2 slab, MRT) are small enough for the oracle to step the whole
  field: element by element, float64 to 1e-12 after 1 and 10 steps, float32 offset
  storage to the reduced-precision budget; C1 also over its full 1000 steps.
* C3 (four-component D3Q19 128^3 drop, MRT + exact-difference forcing): every cell
  after one step from the GPU's own state, against the oracle stepping the whole
  field; float64 to 1e-12, float32 offsets to 1e-6, the benchmarked float16
  two-pass configuration to 1e-4 of max |f| (one re-encoding).
* C3 inside the synthetic porous medium the benchmark's walls section uses (random
  overlapping spheres of radius 6, solid fraction 0.30, psi_w midway between the
  phases): the same whole-field check with the oracle's wall model; solid cells
  hold zeros on both sides.
* C4 (512 independent boxes, tile 64, persistent grid): every box against the
  oracle stepping it alone.
"""
import numpy as np
import pytest

from cases import LAT
from oracle import lbm as olbm
from oracle_backend import BACKEND, to_mixture
from paper_1909_12390_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _lbm():
    from paper_1909_12390_amd import lbm
    return lbm


def rel_err(g, f):
    return max(float(np.max(np.abs(g[s] - f[s])) / np.max(np.abs(f[s]))) for s in range(f.shape[0]))


def oracle_prm(cfg, gamma=None):
    return olbm.StepParams(T=cfg.T, tau=cfg.tau, gamma=cfg.gamma if gamma is None else gamma, beta=cfg.beta,
                           collision=cfg.collision, forcing=cfg.forcing, mrt_s=cfg.mrt_s)


def context(cfg, storage, schedule="two_pass"):
    return _lbm().LbmContext(cfg.mix, cfg.lattice, cfg.shape, cfg.T, cfg.tau, cfg.beta, cfg.gamma, cfg.rho0,
                             collision=cfg.collision, forcing=cfg.forcing, storage=storage, schedule=schedule,
                             mrt_s=cfg.mrt_s)


@pytest.mark.parametrize("which,storage,tol1,tol10", [("C1", "f64", 1e-12, 1e-12), ("C2", "f64", 1e-12, 1e-12),
                                                      ("C2", "f32", 1e-6, 5e-6)])
def test_small_configs_whole_field(which, storage, tol1, tol10):
    cfg = inputs.config_c1(BACKEND) if which == "C1" else inputs.config_c2(BACKEND)
    print(f"case {which} {cfg.shape} nc={cfg.nc} {cfg.collision}+{cfg.forcing} {storage}", flush=True)
    ctx = context(cfg, storage)
    m = to_mixture(cfg.mix)
    f = olbm.init_populations(cfg.rho0, LAT[cfg.lattice])
    prm = oracle_prm(cfg)
    assert rel_err(ctx.get_populations().cpu().numpy(), f) < (1e-15 if storage == "f64" else 1e-6)
    ref = [f]
    for _ in range(10):
        f = olbm.step(f, m, prm, LAT[cfg.lattice])
        ref.append(f)
    ctx.step(1)
    e1 = rel_err(ctx.get_populations().cpu().numpy(), ref[1])
    ctx.step(9)
    e10 = rel_err(ctx.get_populations().cpu().numpy(), ref[10])
    ctx.check()
    print(f"  1 step {e1:.2e}  10 steps {e10:.2e}", flush=True)
    assert e1 < tol1 and e10 < tol10, (e1, e10)


def test_c1_full_length_whole_field():
    """C1 over its whole length (1000 steps) against the oracle stepping the same
    field (about 2 s on the host): float64, every population of every cell."""
    cfg = inputs.config_c1(BACKEND)
    print(f"case C1 {cfg.shape} nc={cfg.nc} {cfg.collision}+{cfg.forcing} f64, {cfg.steps} steps", flush=True)
    ctx = context(cfg, "f64")
    m = to_mixture(cfg.mix)
    f = olbm.init_populations(cfg.rho0, LAT[cfg.lattice])
    prm = oracle_prm(cfg)
    for _ in range(cfg.steps):
        f = olbm.step(f, m, prm, LAT[cfg.lattice])
    ctx.step(cfg.steps)
    ctx.check()
    e = rel_err(ctx.get_populations().cpu().numpy(), f)
    print(f"  {cfg.steps} steps {e:.2e}", flush=True)
    assert e < 1e-12, e


def c3_state_pair(cfg, storage, solid=None):
    """The GPU's state after 2 steps (a state with flow and forces) and after a
    third step, as canonical float64 populations; with walls, psi_w midway between
    the phases' psi."""
    ctx = context(cfg, storage)
    psi_w = 0.0
    if solid is not None:
        psi = ctx.moments(fields=True, totals=False)["psi"]
        h = cfg.shape[0] // 2
        psi_w = 0.5 * float(psi[0, 0, 0].item() + psi[h, h, h].item())
        del psi
        ctx.set_solid(solid, psi_w)
    ctx.step(2)
    ctx.check()
    f0 = ctx.get_populations().cpu().numpy()
    ctx.step(1)
    ctx.check()
    f1 = ctx.get_populations().cpu().numpy()
    del ctx
    torch.cuda.empty_cache()
    return f0, f1, psi_w


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-6), ("f16", 1e-4)])
def test_c3_full_size_whole_field(storage, tol):
    """Every cell of the 128^3 four-component drop after one step from the GPU's own
    state, against the oracle stepping the whole field (about 3 s on the host)."""
    cfg = inputs.config_c3(BACKEND)
    print(f"case C3 {cfg.shape} nc={cfg.nc} {storage} two_pass, whole field", flush=True)
    f0, f1, _ = c3_state_pair(cfg, storage)
    ref = olbm.step(f0, to_mixture(cfg.mix), oracle_prm(cfg), LAT["D3Q19"])
    del f0
    scale = np.max(np.abs(ref), axis=(1, 2, 3, 4))      # max |f| per component
    err = max(float(np.max(np.abs(f1[s] - ref[s]))) / scale[s] for s in range(cfg.nc))
    print(f"  max error / max |f| = {err:.2e} over {f1[0, 0].size} cells", flush=True)
    assert err < tol


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-6), ("f16", 1e-4)])
def test_c3_walls_full_size_whole_field(storage, tol):
    """The same drop inside the porous medium of the benchmark's walls section
    (random overlapping spheres of radius 6, solid fraction 0.30, psi_w midway
    between the phases), every cell against the oracle's wall model."""
    cfg = inputs.config_c3(BACKEND)
    solid = inputs.porous_spheres(cfg.shape, 0.30, 6.0, seed=0)
    print(f"case C3 walls {cfg.shape} {storage} solid fraction {solid.mean():.3f}, whole field", flush=True)
    f0, f1, psi_w = c3_state_pair(cfg, storage, solid)
    prm = oracle_prm(cfg)
    prm.solid = solid
    prm.psi_wall = psi_w
    ref = olbm.step(f0, to_mixture(cfg.mix), prm, LAT["D3Q19"])
    del f0
    assert np.all(f1[:, :, solid] == 0.0) and np.all(ref[:, :, solid] == 0.0)
    scale = np.max(np.abs(ref), axis=(1, 2, 3, 4))
    err = max(float(np.max(np.abs(f1[s] - ref[s]))) / scale[s] for s in range(cfg.nc))
    print(f"  max error / max |f| = {err:.2e} over {f1[0, 0].size} cells", flush=True)
    assert err < tol


def test_c4_full_batch_every_box():
    lbm = _lbm()
    cfgs = inputs.config_c4_boxes(BACKEND, nboxes=512)
    boxes = [{"mix": c.mix, "shape": c.shape, "T": c.T, "tau": c.tau, "beta": c.beta, "gamma": c.gamma,
              "rho0": c.rho0} for c in cfgs]
    print("case C4 512 boxes f64 tile 64, every box", flush=True)
    b = lbm.LbmBatch(boxes, "D2Q9", collision="bgk", forcing="edm", storage="f64", tile=64)
    b.step(2)
    f2 = b.fields(populations=True)[1]
    b.check()
    pick = list(range(len(cfgs)))
    got = {i: f2[i].cpu().numpy() for i in pick}
    del f2
    b.close()
    for i in pick:
        c = cfgs[i]
        f = olbm.init_populations(c.rho0, LAT["D2Q9"])
        prm = oracle_prm(c)
        for _ in range(2):
            f = olbm.step(f, to_mixture(c.mix), prm, LAT["D2Q9"])
        e = rel_err(got[i], f)
        assert e < 1e-12, (i, c.shape, e)


@pytest.mark.parametrize("lattice,shape", [("D2Q9", (5, 1)), ("D2Q9", (1, 7)), ("D2Q9", (1, 1)),
                                           ("D2Q9", (3, 64)), ("D2Q9", (2, 65)), ("D3Q19", (3, 1, 5)),
                                           ("D3Q19", (1, 1, 1)), ("D3Q19", (2, 3, 128))])
@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-6), ("f16", 1e-4)])
def test_degenerate_and_edge_boxes(lattice, shape, storage, tol):
    """One-cell-wide rows and columns, a single cell (every neighbour is the cell
    itself), rows of exactly 64 / 128 cells (the right neighbour of a wavefront's
    last lane wraps to x = 0) and of 65 (a one-cell second segment)."""
    from cases import case
    print(f"case edge box {lattice} {shape} {storage}", flush=True)
    c = case(lattice, 2, shape, seed=4, u_amp=0.01)
    ctx = _lbm().LbmContext(c["mix"], lattice, c["shape"], c["T"], 0.8, 1.16, c["gamma"], c["rho0"], c["u0"],
                            collision="bgk", forcing="edm", storage=storage)
    prm = olbm.StepParams(T=c["T"], tau=0.8, gamma=c["gamma"], beta=1.16, collision="bgk", forcing="edm")
    m = to_mixture(c["mix"])
    f = ctx.get_populations().cpu().numpy()          # the GPU's own (decoded) state
    for _ in range(3):
        ref = olbm.step(f, m, prm, LAT[lattice])
        ctx.step(1)
        f = ctx.get_populations().cpu().numpy()
        e = rel_err(f, ref)
        assert e < tol, (shape, storage, e)
    ctx.check()
