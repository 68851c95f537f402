"""Hand-written adjoint on the GPU (lbm_step_adjoint, lbm_adjoint) against the
oracle's discrete adjoint and against central differences of the GPU forward.

* one reverse step at a float64 state equals the oracle's reverse product of the
  step (population adjoint and EOS-table adjoint) to 1e-11;
* a checkpointed gradient run equals the oracle gradient of the same loss
  (float64 1e-9; float32 offset storage 1e-5, float16 2e-4 of the largest entry);
  the checkpoint interval only changes the recomputation, so gradients for
  K = 1, 4 and nsteps are bitwise equal;
* at the full adjoint case (ternary D2Q9 128x128 drop, 2000 steps, checkpoints
  every 100) the float64 gradient agrees with central differences (h = 1e-6) of
  the GPU forward's loss to 1e-5 relative, and the float32-storage gradient is
  reported against it;
* the torch.autograd.Function returns the library gradient.
"""
import numpy as np
import pytest

from cases import LAT, case, mrt_rates, oracle_params
from oracle import adjoint as oadj
from oracle import lbm as olbm
from oracle_backend import BACKEND, to_mixture
from paper_1909_12390_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _lbm():
    from paper_1909_12390_amd import lbm
    return lbm


def context(c, lattice, storage="f64", beta=1.16, tau=0.8, forcing="edm", accel=None, collision="bgk",
            mrt_s=None):
    return _lbm().LbmContext(c["mix"], lattice, c["shape"], c["T"], tau, beta, c["gamma"], c["rho0"],
                             collision=collision, forcing=forcing, storage=storage, accel=accel, mrt_s=mrt_s)


@pytest.mark.parametrize("collision,forcing,accel", [("bgk", "edm", None), ("bgk", "guo", None),
                                                     ("bgk", "guo", (2e-5, -1e-5, 3e-6)), ("mrt", "edm", None),
                                                     ("mrt", "guo", (1e-5, 2e-5, -1e-5))])
@pytest.mark.parametrize("lattice,nc,shape", [("D2Q9", 3, (12, 14)), ("D2Q9", 1, (10, 9)), ("D2Q9", 4, (9, 11)),
                                              ("D3Q19", 2, (5, 6, 7))])
def test_step_adjoint_matches_oracle(lattice, nc, shape, collision, forcing, accel):
    print(f"case step adjoint {lattice} nc={nc} {shape} {collision} {forcing} accel={accel}", flush=True)
    c = case(lattice, nc, shape, seed=1, u_amp=0.01)
    c["u0"] = None
    D = 2 if lattice == "D2Q9" else 3
    acc = None if accel is None else np.asarray(accel[:D])
    beta = 1.16 if forcing == "edm" else 1.7
    rates = mrt_rates(lattice, 0.8) if collision == "mrt" else None
    ctx = context(c, lattice, forcing=forcing, beta=beta, accel=acc, collision=collision, mrt_s=rates)
    ctx.step(3)
    f = ctx.get_populations().cpu().numpy()
    h = np.random.default_rng(5).standard_normal(f.shape)
    hout, daa, db = ctx.step_adjoint(h)
    ctx.check()
    assert np.array_equal(ctx.get_populations().cpu().numpy(), f)   # state untouched
    base = to_mixture(c["mix"])
    prm = oracle_params(c, collision, forcing, tau=0.8, beta=beta, accel=acc, mrt_s=rates)
    aa, b = oadj.eos_tables(torch.as_tensor(oadj.theta_of(base), dtype=oadj.DT), base, c["T"])
    gf, gaa, gb = oadj.step_vjp_tables(f, h, aa.numpy(), b.numpy(), base, prm, LAT[lattice])
    assert np.max(np.abs(hout.cpu().numpy() - gf)) <= 1e-11 * np.max(np.abs(gf))
    assert np.max(np.abs(daa - gaa)) <= 1e-10 * np.max(np.abs(gaa))
    assert np.max(np.abs(db - gb)) <= 1e-10 * np.max(np.abs(gb))


def small_problem(seed=2, shape=(12, 14), nsteps=12):
    c = case("D2Q9", 3, shape, seed=seed)
    mask = inputs.drop_mask(shape, min(shape) / 4.0)
    base = to_mixture(c["mix"])
    f0 = olbm.init_populations(c["rho0"], LAT["D2Q9"])
    x0 = oadj.mole_fractions(torch.as_tensor(f0, dtype=oadj.DT), base.M, mask).numpy()
    x_tgt = x0 + np.array([0.01, -0.015, 0.005])
    return c, mask, base, f0, x_tgt, nsteps


def gpu_gradient(c, mask, x_tgt, nsteps, K, storage="f64", forcing="edm", collision="bgk"):
    from paper_1909_12390_amd import adjoint as padj
    rates = mrt_rates("D2Q9", 0.8) if collision == "mrt" else None
    ctx = context(c, "D2Q9", storage, forcing=forcing, beta=1.16 if forcing == "edm" else 1.7, collision=collision,
                  mrt_s=rates)
    r = ctx.adjoint(nsteps, K, mask, x_tgt)
    ctx.close()
    return r, padj.pack_gradient(r["d_k"], r["d_a"], r["d_b"])


@pytest.mark.parametrize("collision,forcing", [("bgk", "edm"), ("bgk", "guo"), ("mrt", "edm")])
def test_gradient_run_matches_oracle_gradient(collision, forcing):
    print(f"case adjoint run vs oracle {collision} {forcing}", flush=True)
    c, mask, base, f0, x_tgt, nsteps = small_problem()
    rates = mrt_rates("D2Q9", 0.8) if collision == "mrt" else None
    prm = oracle_params(c, collision, forcing, tau=0.8, beta=1.16 if forcing == "edm" else 1.7, mrt_s=rates)
    L, g = oadj.gradient(oadj.theta_of(base), f0, base, prm, LAT["D2Q9"], nsteps, mask, x_tgt)
    r, gg = gpu_gradient(c, mask, x_tgt, nsteps, K=5, forcing=forcing, collision=collision)
    assert abs(r["loss"] - L) <= 1e-11 * L
    assert np.max(np.abs(gg - g)) <= 1e-9 * np.max(np.abs(g))
    # float32 storage: same gradient to the precision of the stored states
    r32, g32 = gpu_gradient(c, mask, x_tgt, nsteps, K=5, storage="f32", forcing=forcing, collision=collision)
    rel32 = float(np.max(np.abs(g32 - g)) / np.max(np.abs(g)))
    print(f"  float32-storage gradient vs oracle: max rel {rel32:.2e}", flush=True)
    assert rel32 <= 1e-5
    # float16 offsets: the recomputed states carry the offsets' rounding, 2^-11 of
    # the offset (<= ~2.4e-5 of a population, see test_gpu_step), which the
    # gradient inherits over the 12 steps within a small factor (measured 1.7e-5 to
    # 6.9e-5 over the three schemes); bar at about 3x the largest
    r16, g16 = gpu_gradient(c, mask, x_tgt, nsteps, K=5, storage="f16", forcing=forcing, collision=collision)
    rel16 = float(np.max(np.abs(g16 - g)) / np.max(np.abs(g)))
    print(f"  float16-storage gradient vs oracle: max rel {rel16:.2e}", flush=True)
    assert rel16 <= 2e-4


def test_checkpoint_interval_does_not_change_gradient():
    print("case adjoint checkpoint intervals", flush=True)
    c, mask, base, f0, x_tgt, nsteps = small_problem(seed=3, shape=(10, 16), nsteps=9)
    outs = [gpu_gradient(c, mask, x_tgt, nsteps, K)[1] for K in (1, 4, 9, 20)]
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_autograd_function_returns_library_gradient():
    print("case adjoint autograd.Function", flush=True)
    from paper_1909_12390_amd import adjoint as padj
    c, mask, base, f0, x_tgt, nsteps = small_problem(seed=4, shape=(12, 12), nsteps=6)
    spec = padj.AdjointSpec(mix=c["mix"], lattice="D2Q9", shape=c["shape"], T=c["T"], tau=0.8, beta=1.16,
                            gamma=c["gamma"], rho0=c["rho0"], mask=mask, x_target=x_tgt, nsteps=nsteps,
                            checkpoint_every=4, storage="f64")
    theta = torch.tensor(padj.theta_of(c["mix"]), dtype=torch.float64, requires_grad=True)
    L = padj.liquid_composition_loss(theta, spec)
    (g,) = torch.autograd.grad(3.0 * L, theta)
    _, gg = gpu_gradient(c, mask, x_tgt, nsteps, K=4)
    assert np.allclose(g.numpy(), 3.0 * gg, rtol=0, atol=0)
    # without a gradient request only the forward steps run; same loss
    L0 = padj.liquid_composition_loss(theta.detach(), spec)
    assert abs(float(L0) - float(L)) <= 1e-12 * abs(float(L))
    # a float32 theta receives the float64 gradient cast once
    th32 = torch.tensor(padj.theta_of(c["mix"]), dtype=torch.float32, requires_grad=True)
    (g32,) = torch.autograd.grad(padj.liquid_composition_loss(th32, spec), th32)
    assert g32.dtype == torch.float32 and torch.isfinite(g32).all()


def host_loss(ctx, mask, M, x_tgt):
    rho = ctx.moments(totals=False)["rho_s"].cpu().numpy()
    n = rho / np.asarray(M).reshape(-1, 1, 1)
    Ni = np.array([n[i][mask].sum() for i in range(n.shape[0])])
    x = Ni / Ni.sum()
    return float(np.sum((x - x_tgt) ** 2))


def test_full_case_gradient_matches_central_differences():
    """Ternary D2Q9 128x128 drop, 2000 steps, checkpoints every 100 (the adjoint
    configuration); FD on the float64 GPU forward with a loss computed on the host."""
    from paper_1909_12390_amd import adjoint as padj
    cfg = inputs.config_c5(BACKEND)
    mask = inputs.drop_mask(cfg.shape, cfg.geometry["R0"])
    x_tgt = inputs.adjoint_target(cfg)
    print(f"case adjoint full {cfg.shape} nc={cfg.nc} steps={cfg.steps}", flush=True)
    spec = padj.AdjointSpec(mix=cfg.mix, lattice="D2Q9", shape=cfg.shape, T=cfg.T, tau=cfg.tau, beta=cfg.beta,
                            gamma=cfg.gamma, rho0=cfg.rho0, mask=mask, x_target=x_tgt, nsteps=cfg.steps,
                            checkpoint_every=100, storage="f64")
    theta = padj.theta_of(cfg.mix)
    L, x, g = padj.run(theta, spec)
    h = 1e-6
    for i in range(theta.size):
        vals = []
        for sgn in (1.0, -1.0):
            t = theta.copy()
            t[i] += sgn * h
            ctx = _lbm().LbmContext(padj.mixture_with(t, cfg.mix), "D2Q9", cfg.shape, cfg.T, cfg.tau, cfg.beta,
                                    cfg.gamma, cfg.rho0, collision="bgk", forcing="edm", storage="f64")
            ctx.step(cfg.steps)
            ctx.check()
            vals.append(host_loss(ctx, mask, cfg.mix["M"], x_tgt))
            ctx.close()
        fd = (vals[0] - vals[1]) / (2 * h)
        print(f"  theta[{i}] adjoint {g[i]:.10e} fd {fd:.10e}", flush=True)
        assert abs(g[i] - fd) <= 1e-5 * abs(fd) + 1e-7 * np.max(np.abs(g)), (i, g[i], fd)
    spec32 = padj.AdjointSpec(**{**spec.__dict__, "storage": "f32"})
    L32, _, g32 = padj.run(theta, spec32)
    rel = float(np.max(np.abs(g32 - g)) / np.max(np.abs(g)))
    print(f"  float32-storage gradient vs float64: max rel {rel:.3e}; loss {L32:.6e} vs {L:.6e}", flush=True)
    assert rel < 1e-5


def porous(shape, seed, frac=0.15):
    return np.random.default_rng([7, seed]).uniform(size=shape) < frac


def wall_psi(c):
    corner = c["rho0"][(slice(None),) + (0,) * len(c["shape"])]
    return 1.3 * float(olbm.pseudo_potential(corner[:, None], c["T"], to_mixture(c["mix"]), -1.0)[0])


@pytest.mark.parametrize("collision,forcing", [("bgk", "edm"), ("bgk", "guo"), ("mrt", "edm"), ("mrt", "guo")])
@pytest.mark.parametrize("lattice,nc,shape", [("D2Q9", 3, (12, 14)), ("D3Q19", 2, (5, 6, 7))])
def test_step_adjoint_with_walls_matches_oracle(lattice, nc, shape, collision, forcing):
    print(f"case step adjoint walls {lattice} nc={nc} {shape} {collision} {forcing}", flush=True)
    c = case(lattice, nc, shape, seed=1, u_amp=0.01)
    c["u0"] = None
    beta = 1.16 if forcing == "edm" else 1.7
    rates = mrt_rates(lattice, 0.8) if collision == "mrt" else None
    solid, pw = porous(shape, 11), wall_psi(c)
    ctx = _lbm().LbmContext(c["mix"], lattice, c["shape"], c["T"], 0.8, beta, c["gamma"], c["rho0"],
                            collision=collision, forcing=forcing, storage="f64", mrt_s=rates, solid=solid,
                            psi_wall=pw)
    ctx.step(3)
    f = ctx.get_populations().cpu().numpy()
    h = np.random.default_rng(5).standard_normal(f.shape)
    hout, daa, db = ctx.step_adjoint(h)
    ctx.check()
    base = to_mixture(c["mix"])
    prm = oracle_params(c, collision, forcing, tau=0.8, beta=beta, mrt_s=rates)
    prm.solid, prm.psi_wall = solid, pw
    aa, b = oadj.eos_tables(torch.as_tensor(oadj.theta_of(base), dtype=oadj.DT), base, c["T"])
    gf, gaa, gb = oadj.step_vjp_tables(f, h, aa.numpy(), b.numpy(), base, prm, LAT[lattice])
    ho = hout.cpu().numpy()
    assert np.all(ho[:, :, solid] == 0.0)
    assert np.max(np.abs(ho - gf)) <= 1e-11 * np.max(np.abs(gf))
    assert np.max(np.abs(daa - gaa)) <= 1e-10 * np.max(np.abs(gaa))
    assert np.max(np.abs(db - gb)) <= 1e-10 * np.max(np.abs(gb))


@pytest.mark.parametrize("collision,forcing", [("bgk", "edm"), ("mrt", "guo")])
def test_gradient_run_with_walls_matches_oracle_gradient(collision, forcing):
    print(f"case adjoint run with walls {collision} {forcing}", flush=True)
    shape = (12, 14)
    c = case("D2Q9", 3, shape, seed=2)
    base = to_mixture(c["mix"])
    solid, pw = porous(shape, 12), wall_psi(c)
    mask = inputs.drop_mask(shape, min(shape) / 2.0) & ~solid
    f0 = olbm.init_populations(c["rho0"], LAT["D2Q9"])
    f0[:, :, solid] = 0.0
    x0 = oadj.mole_fractions(torch.as_tensor(f0, dtype=oadj.DT), base.M, mask).numpy()
    x_tgt = x0 + np.array([0.01, -0.015, 0.005])
    beta = 1.16 if forcing == "edm" else 1.7
    rates = mrt_rates("D2Q9", 0.8) if collision == "mrt" else None
    prm = oracle_params(c, collision, forcing, tau=0.8, beta=beta, mrt_s=rates)
    prm.solid, prm.psi_wall = solid, pw
    nsteps = 10
    L, g = oadj.gradient(oadj.theta_of(base), f0, base, prm, LAT["D2Q9"], nsteps, mask, x_tgt)
    from paper_1909_12390_amd import adjoint as padj
    ctx = _lbm().LbmContext(c["mix"], "D2Q9", shape, c["T"], 0.8, beta, c["gamma"], c["rho0"], collision=collision,
                            forcing=forcing, storage="f64", mrt_s=rates, solid=solid, psi_wall=pw)
    r = ctx.adjoint(nsteps, 4, mask, x_tgt)
    ctx.close()
    gg = padj.pack_gradient(r["d_k"], r["d_a"], r["d_b"])
    assert abs(r["loss"] - L) <= 1e-11 * L
    assert np.max(np.abs(gg - g)) <= 1e-9 * np.max(np.abs(g))
