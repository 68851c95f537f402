"""GPU parity of the HIP step (through the C ABI) against the CPU oracle.

Bar: float64 storage must match the oracle to 1e-12 relative per component
(max |f_gpu - f_oracle| / max |f_oracle|) after 1 and 10 steps from identical
states.  Boxes are ragged (cells not a multiple of the 256-thread block, sides
not multiples of the tile) and span several blocks.
"""
import numpy as np
import pytest

from cases import LAT, case, mrt_rates, oracle_params, oracle_run
from oracle import lbm as olbm
from oracle_backend import to_mixture

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHAPES = {"D2Q9": (45, 70), "D3Q19": (13, 14, 15)}
COMBOS = [("bgk", "guo"), ("bgk", "edm"), ("mrt", "guo"), ("mrt", "edm")]


def _lbm():
    from paper_1909_12390_amd import lbm
    return lbm


def rel_err(g, f):
    """max over components of max|g - f| / max|f|"""
    return max(float(np.max(np.abs(g[s] - f[s])) / np.max(np.abs(f[s]))) for s in range(f.shape[0]))


def gpu_context(c, lattice, collision, forcing, storage="f64", schedule="two_pass", tau=0.8, beta=1.7,
                mrt_s=None, accel=None):
    lbm = _lbm()
    return lbm.LbmContext(c["mix"], lattice, c["shape"], c["T"], tau, beta, c["gamma"], c["rho0"], c["u0"],
                          collision=collision, forcing=forcing, storage=storage, schedule=schedule,
                          mrt_s=mrt_s, accel=accel)


@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q19"])
@pytest.mark.parametrize("nc", [1, 2, 3, 4])
@pytest.mark.parametrize("collision,forcing", COMBOS)
def test_f64_step_matches_oracle(lattice, nc, collision, forcing):
    print(f"case f64 {lattice} nc={nc} {collision}+{forcing}", flush=True)
    c = case(lattice, nc, SHAPES[lattice], seed=nc, u_amp=0.01)
    rates = mrt_rates(lattice, 0.8) if collision == "mrt" else None
    prm = oracle_params(c, collision, forcing, mrt_s=rates)
    ref = oracle_run(c, lattice, prm, 10)
    ctx = gpu_context(c, lattice, collision, forcing, mrt_s=rates)
    f0 = ctx.get_populations().cpu().numpy()
    assert rel_err(f0, ref[0]) < 1e-15
    ctx.step(1)
    e1 = rel_err(ctx.get_populations().cpu().numpy(), ref[1])
    ctx.step(9)
    e10 = rel_err(ctx.get_populations().cpu().numpy(), ref[10])
    ctx.check()
    assert e1 < 1e-12 and e10 < 1e-12, (e1, e10)


@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q19"])
def test_moments_and_totals_match_oracle(lattice):
    print(f"case moments {lattice}", flush=True)
    c = case(lattice, 3, SHAPES[lattice], seed=7, u_amp=0.01)
    accel = [1e-5, -2e-5, 3e-5][: 2 if lattice == "D2Q9" else 3]
    prm = oracle_params(c, "bgk", "guo", accel=accel)
    ref = oracle_run(c, lattice, prm, 3)
    ctx = gpu_context(c, lattice, "bgk", "guo", accel=accel)
    ctx.step(3)
    m = ctx.moments()
    lat = LAT[lattice]
    om = olbm.macroscopic(ref[3], to_mixture(c["mix"]), prm, lat)
    ot = olbm.totals(ref[3], to_mixture(c["mix"]), prm, lat)
    for k in ("rho_s", "u", "p", "psi"):
        g = m[k].cpu().numpy()
        assert np.max(np.abs(g - om[k])) <= 1e-12 * np.max(np.abs(om[k])), k
    assert np.allclose(m["mass"], ot["mass"], rtol=1e-13)
    assert np.allclose(m["momentum"], ot["momentum"], rtol=1e-10, atol=1e-12)
    assert np.allclose(m["force"], ot["force"], atol=1e-12)


@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q19"])
@pytest.mark.parametrize("forcing", ["guo", "edm"])
def test_conservation_on_gpu(lattice, forcing):
    print(f"case conservation {lattice} {forcing}", flush=True)
    c = case(lattice, 2, SHAPES[lattice], seed=3)
    g = [2e-6, -1e-6, 1e-6][: 2 if lattice == "D2Q9" else 3]
    ctx = gpu_context(c, lattice, "bgk", forcing, accel=g)
    t0 = ctx.moments(fields=False)
    n = 200
    ctx.step(n)
    t1 = ctx.moments(fields=False)
    assert np.all(np.abs(t1["mass"] / t0["mass"] - 1) < 1e-13 * np.sqrt(n))
    assert np.all(np.abs(t1["force"]) < 1e-11)
    M = float(np.sum(t0["mass"]))
    assert np.allclose(t1["momentum"] - t0["momentum"], n * M * np.asarray(g), rtol=1e-9, atol=1e-11)


@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q19"])
@pytest.mark.parametrize("forcing,gamma", [("guo", (0.4, 1.0)), ("edm", (1.0, 1.0))])
def test_identical_components_equal_single_component_on_gpu(lattice, forcing, gamma):
    # Sec. 4.1 limiting case on the device: two identical components (segregated
    # initial fields, Eq. (initialMC)) evolve as the pure fluid.
    print(f"case limiting {lattice} {forcing}", flush=True)
    c1 = case(lattice, 1, SHAPES[lattice], seed=0, noise=0.0)
    mix2 = {k: (np.concatenate([v, v]) if k in ("a", "b", "omega", "M") else v) for k, v in c1["mix"].items()}
    mix2["k"] = np.zeros((2, 2))
    rho = c1["rho0"][0]
    rl, rv = rho.max(), rho.min()
    # split: component 1 carries the liquid excess, component 2 the vapor part
    r1 = rho - rv
    r2 = np.full_like(rho, rv)
    r1 = np.maximum(r1, 1e-3 * rl)
    r2 = rho - r1
    c2 = dict(c1, mix=mix2, rho0=np.stack([r1, r2]), gamma=np.array(gamma))
    a = gpu_context(c1, lattice, "bgk", forcing, tau=1.0, beta=1.3)
    b = gpu_context(c2, lattice, "bgk", forcing, tau=1.0, beta=1.3)
    a.step(20)
    b.step(20)
    fa = a.get_populations().cpu().numpy()[0]
    fb = b.get_populations().cpu().numpy().sum(0)
    a.check()
    b.check()
    assert np.max(np.abs(fa - fb)) < 1e-12 * np.max(np.abs(fa))


def test_domain_error_reported():
    lbm = _lbm()
    c = case("D2Q9", 2, (16, 20), seed=1)
    rho0 = c["rho0"].copy()
    rho0[0, 3, 4] = 50.0 / c["mix"]["b"][0] * c["mix"]["M"][0]      # b_m rho~ >> 1 in one cell
    c = dict(c, rho0=rho0)
    ctx = gpu_context(c, "D2Q9", "bgk", "edm")
    ctx.step(1)
    with pytest.raises(lbm.LbmError) as e:
        ctx.check()
    assert e.value.code == lbm.LBM_ERR_DOMAIN
    ctx.clear_error()


def test_set_get_populations_roundtrip():
    c = case("D3Q19", 2, (9, 10, 11), seed=5, u_amp=0.02)
    ctx = gpu_context(c, "D3Q19", "mrt", "edm", mrt_s=mrt_rates("D3Q19", 0.8))
    f = ctx.get_populations().cpu().numpy()
    rng = np.random.default_rng(0)
    g = f * (1 + 1e-3 * rng.uniform(-1, 1, f.shape))
    ctx.set_populations(g)
    assert np.array_equal(ctx.get_populations().cpu().numpy(), g)


# Reduced-precision storage.  Error budget relative to max|f| of a component:
#   f32 offsets: encode rounds f / b and the offset to float32 (~2 eps32 = 1.2e-7 of
#     f) and the float32 collision adds a few eps32 per step: <= 1e-6 after 1 step,
#     <= 5e-6 after 10 (errors also propagate through the psi stencil; measured
#     2.4e-7 / 4.6e-7);
#   f16 offsets: the stored offset r = f/b - w (|r| <~ 0.05 in these states) is
#     rounded to 11 bits (2^-11 |r| <~ 2.4e-5 b); relative to max|f| (>= w_0 b_max)
#     below 1e-4 per step, and the rounding does not accumulate over 10 steps
#     because every step re-encodes from float32 (measured 4e-5 / 3e-5).
@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q19"])
@pytest.mark.parametrize("storage,tol1,tol10", [("f32", 1e-6, 5e-6), ("f16", 1e-4, 2e-4)])
@pytest.mark.parametrize("collision,forcing", [("bgk", "guo"), ("mrt", "edm")])
@pytest.mark.parametrize("nc", [1, 2, 3, 4])
def test_reduced_precision_step_close_to_oracle(lattice, storage, tol1, tol10, collision, forcing, nc):
    # nc sets the width of the interleaved accesses (float16: 2, 4, 4 + 2, 8 bytes;
    # float32: 4, 8, 12, 16 bytes per direction and cell)
    print(f"case {storage} {lattice} nc={nc} {collision}+{forcing}", flush=True)
    c = case(lattice, nc, SHAPES[lattice], seed=11, u_amp=0.01)
    rates = mrt_rates(lattice, 0.8) if collision == "mrt" else None
    prm = oracle_params(c, collision, forcing, mrt_s=rates, beta=1.16 if forcing == "edm" else 1.945)
    ref = oracle_run(c, lattice, prm, 10)
    ctx = gpu_context(c, lattice, collision, forcing, storage=storage, mrt_s=rates,
                      beta=1.16 if forcing == "edm" else 1.945)
    e0 = rel_err(ctx.get_populations().cpu().numpy(), ref[0])
    ctx.step(1)
    e1 = rel_err(ctx.get_populations().cpu().numpy(), ref[1])
    ctx.step(9)
    e10 = rel_err(ctx.get_populations().cpu().numpy(), ref[10])
    ctx.check()
    print(f"  {storage}: init {e0:.2e}  1 step {e1:.2e}  10 steps {e10:.2e}", flush=True)
    assert e1 < tol1 and e10 < tol10, (e0, e1, e10)


@pytest.mark.parametrize("lattice,shape,slab", [("D2Q9", (45, 70), 7), ("D3Q19", (13, 14, 15), 4),
                                                ("D3Q19", (13, 14, 15), 1)])
@pytest.mark.parametrize("storage", ["f64", "f16"])
@pytest.mark.parametrize("schedule", ["blocked", "overlap"])
def test_blocked_schedule_equals_two_pass(lattice, shape, slab, storage, schedule):
    # same arithmetic, different launch order (and streams): bitwise identical states
    print(f"case {schedule} {lattice} slab={slab} {storage}", flush=True)
    c = case(lattice, 3, shape, seed=9, u_amp=0.01)
    rates = mrt_rates(lattice, 0.8)
    a = gpu_context(c, lattice, "mrt", "edm", storage=storage, mrt_s=rates, beta=1.16)
    lbm = _lbm()
    b = lbm.LbmContext(c["mix"], lattice, c["shape"], c["T"], 0.8, 1.16, c["gamma"], c["rho0"], c["u0"],
                       collision="mrt", forcing="edm", storage=storage, schedule=schedule, mrt_s=rates,
                       slab_planes=slab)
    a.step(7)
    b.step(7)
    fa = a.get_populations().cpu().numpy()
    fb = b.get_populations().cpu().numpy()
    a.check()
    b.check()
    assert np.array_equal(fa, fb)


def test_gamma_from_the_flash_at_init():
    # gamma left to lbm_init: the library's flash at (T, p*, z) (Eq. gamma) gives the
    # same run as passing that flash's gamma explicitly, bitwise; it agrees with the
    # oracle's flash
    print("case gamma from the flash at init", flush=True)
    from cases import BACKEND
    from paper_1909_12390_amd import inputs
    lbm = _lbm()
    mix, T, z, p, fl = inputs.pick_state(inputs.rng_for(777, 0), BACKEND, 3, 0.7, 0.95, 0.05, {})
    lib_fl = lbm.lbm_flash(mix, T, p, z)
    assert np.allclose(lib_fl.gamma[:3], fl.gamma, rtol=1e-9)
    shape = (40, 52)
    rho0 = inputs.drop_profile(shape, 10.0, 4.0, fl.rbar_l, fl.rbar_v)
    runs = []
    for gamma, kw in ((list(lib_fl.gamma[:3]), {}), (None, {"p_flash": p, "z_flash": z})):
        ctx = lbm.LbmContext(mix, "D2Q9", shape, T, 0.8, 1.3, gamma, rho0, collision="bgk", forcing="edm",
                             storage="f64", **kw)
        ctx.step(20)
        runs.append(ctx.get_populations().cpu().numpy())
        ctx.check()
    assert np.array_equal(runs[0], runs[1])
