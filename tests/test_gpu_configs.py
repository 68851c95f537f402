"""Parity on the seeded benchmark configurations themselves, in the launch
configurations bench.py times.

* C1 (binary D2Q9 64^2 drop, float64, BGK + exact-difference forcing) and C2
  (ternary D2Q9 256^2 slab, MRT) are small enough for the oracle to step the whole
  field: element by element, float64 to 1e-12 after 1 and 10 steps, float32 offset
  storage to the reduced-precision budget.
* C3 (four-component D3Q19 128^3 drop, MRT + exact-difference forcing) is checked on
  sampled cells: one step at a cell depends only on cells within distance 2 (local
  densities, psi at the neighbours for the force at the source cell, one streaming
  hop), so the oracle steps a periodic 5^3 patch cut around the cell from the GPU's
  own input state and its centre is exact.  Samples include the row-segment edges
  (x = 0, 63, 64, 127) and the periodic faces.  float64 to 1e-12; the benchmarked
  float16 two-pass configuration to 1e-4 of max |f| (one re-encoding).
* C3 inside the synthetic porous medium the benchmark's walls section uses (random
  overlapping spheres of radius 6, solid fraction 0.30, psi_w midway between the
  phases): the same patch check with the patch of the solid mask, on cells next to
  walls, solid cells and row-segment edges; float64 to 1e-12, float16 to 1e-4.
* C4 (512 independent boxes, tile 64, persistent grid) is checked box by box on a
  sample of boxes of every side, against the oracle stepping each box alone.
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


def patch(f, center, r=2):
    """Periodic (2r+1)^3 patch of f [nc, Q, nz, ny, nx] around center (z, y, x)."""
    idx = [np.arange(c - r, c + r + 1) % n for c, n in zip(center, f.shape[2:])]
    return f[:, :, idx[0]][:, :, :, idx[1]][:, :, :, :, idx[2]]


def c3_samples(n, seed=3):
    rng = np.random.default_rng([12390, seed])
    pts = [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(24)]
    for x in (0, 63, 64, n - 1):
        for yz in ((0, 0), (n - 1, n // 2), (n // 2, n - 1), (n // 2, n // 2)):
            pts.append((yz[1], yz[0], x))
    # the drop's interface, where the force is largest
    for x in (n // 2 + n // 4 - 1, n // 2 + n // 4, n // 2 + n // 4 + 1):
        pts.append((n // 2, n // 2, x))
    return pts


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f16", 1e-4)])
def test_c3_full_size_sampled_cells(storage, tol):
    cfg = inputs.config_c3(BACKEND)
    n = cfg.shape[0]
    print(f"case C3 {cfg.shape} nc={cfg.nc} {storage} two_pass, sampled cells", flush=True)
    ctx = context(cfg, storage)
    ctx.step(2)                                   # a state with flow and forces
    ctx.check()
    f0 = ctx.get_populations().cpu().numpy()
    ctx.step(1)
    ctx.check()
    f1 = ctx.get_populations().cpu().numpy()
    del ctx
    torch.cuda.empty_cache()
    m = to_mixture(cfg.mix)
    prm = oracle_prm(cfg)
    scale = np.max(np.abs(f1), axis=(1, 2, 3, 4))      # max |f| per component
    worst = 0.0
    for c in c3_samples(n):
        ref = olbm.step(patch(f0, c), m, prm, LAT["D3Q19"])[:, :, 2, 2, 2]
        got = f1[:, :, c[0], c[1], c[2]]
        err = float(np.max(np.abs(got - ref) / scale[:, None]))
        worst = max(worst, err)
        assert err < tol, (c, err)
    print(f"  worst sampled error {worst:.2e} over {len(c3_samples(n))} cells", flush=True)


def wall_samples(solid, seed=5):
    """Fluid cells with a solid neighbour (D3Q19), solid cells, fluid cells at the
    row-segment edges x = 0, 63, 64, 127 and random fluid cells, as (z, y, x)."""
    rng = np.random.default_rng([12390, seed])
    near = np.zeros_like(solid)
    for e in LAT["D3Q19"].e[1:]:
        near |= np.roll(solid, shift=tuple(int(v) for v in e[::-1]), axis=(0, 1, 2))
    near &= ~solid
    pts = []
    for mask, k in ((near, 16), (solid, 4), (~solid, 6)):
        idx = np.argwhere(mask)
        pts += [tuple(int(v) for v in idx[i]) for i in rng.choice(len(idx), size=k, replace=False)]
    n = solid.shape[2]
    for x in (0, 63, 64, n - 1):
        col = np.argwhere(~solid[:, :, x])
        z, y = col[rng.integers(len(col))]
        pts.append((int(z), int(y), x))
    return pts


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f16", 1e-4)])
def test_c3_walls_full_size_sampled_cells(storage, tol):
    cfg = inputs.config_c3(BACKEND)
    solid = inputs.porous_spheres(cfg.shape, 0.30, 6.0, seed=0)
    print(f"case C3 walls {cfg.shape} {storage} solid fraction {solid.mean():.3f}, sampled cells", flush=True)
    ctx = context(cfg, storage)
    psi = ctx.moments(fields=True, totals=False)["psi"]
    h = cfg.shape[0] // 2
    psi_w = 0.5 * float(psi[0, 0, 0].item() + psi[h, h, h].item())   # midway between the phases
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
    m = to_mixture(cfg.mix)
    prm = oracle_prm(cfg)
    prm.psi_wall = psi_w
    scale = np.max(np.abs(f1), axis=(1, 2, 3, 4))
    worst = 0.0
    pts = wall_samples(solid)
    for c in pts:
        idx = [np.arange(v - 2, v + 3) % n for v, n in zip(c, solid.shape)]
        prm.solid = solid[idx[0]][:, idx[1]][:, :, idx[2]]
        ref = olbm.step(patch(f0, c), m, prm, LAT["D3Q19"])[:, :, 2, 2, 2]
        got = f1[:, :, c[0], c[1], c[2]]
        if solid[c]:
            assert np.all(got == 0.0) and np.all(ref == 0.0), c
            continue
        err = float(np.max(np.abs(got - ref) / scale[:, None]))
        worst = max(worst, err)
        assert err < tol, (c, err)
    print(f"  worst sampled error {worst:.2e} over {len(pts)} cells", flush=True)


def test_c4_full_batch_sampled_boxes():
    lbm = _lbm()
    cfgs = inputs.config_c4_boxes(BACKEND, nboxes=512)
    boxes = [{"mix": c.mix, "shape": c.shape, "T": c.T, "tau": c.tau, "beta": c.beta, "gamma": c.gamma,
              "rho0": c.rho0} for c in cfgs]
    print("case C4 512 boxes f64 tile 64, sampled boxes", flush=True)
    b = lbm.LbmBatch(boxes, "D2Q9", collision="bgk", forcing="edm", storage="f64", tile=64)
    b.step(2)
    f2 = b.fields(populations=True)[1]
    b.check()
    # one box of every side pair seen, up to 12 boxes
    seen, pick = set(), []
    for i, c in enumerate(cfgs):
        if c.shape not in seen and len(pick) < 12:
            seen.add(c.shape)
            pick.append(i)
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
@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f16", 1e-4)])
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
