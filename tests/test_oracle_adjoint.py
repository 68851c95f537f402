"""Pins of the oracle's discrete adjoint (oracle/adjoint.py).

* the torch forward step is the NumPy oracle step (so the map being
  differentiated is the pinned one);
* dL/dtheta equals central differences of the NumPy oracle's loss, which shares
  no code with the torch forward or its differentiation;
* forward and reverse products obey <J v, w> = <v, J^T w>;
* at a target equal to the reached composition, L and dL/dtheta vanish.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from cases import LAT, case, mrt_rates, oracle_params  # noqa: E402
from oracle import adjoint as oadj  # noqa: E402
from oracle import lbm as olbm  # noqa: E402
from oracle_backend import to_mixture  # noqa: E402


def drop_mask(shape, R0):
    g = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    r = np.sqrt(sum((x - n / 2.0) ** 2 for x, n in zip(g, shape)))
    return r <= R0 / 2.0


def numpy_loss(theta, base, f0, prm, lat, nsteps, mask, x_tgt):
    """The loss from the NumPy oracle alone (independent of oracle/adjoint.py's
    forward and of any differentiation)."""
    mix = oadj.mixture_of(theta, base)
    f = f0
    for _ in range(nsteps):
        f = olbm.step(f, mix, prm, lat)
    n = f.sum(axis=1) / base.M.reshape((-1,) + (1,) * (f.ndim - 2))
    Ni = np.array([n[i][mask].sum() for i in range(n.shape[0])])
    x = Ni / Ni.sum()
    return float(np.sum((x - x_tgt) ** 2))


def setup(lattice, nc, shape, collision, forcing, seed=0):
    c = case(lattice, nc, shape, seed=seed)
    lat = LAT[lattice]
    rates = mrt_rates(lattice, 0.8) if collision == "mrt" else None
    prm = oracle_params(c, collision, forcing, beta=1.16 if forcing == "edm" else 1.7, mrt_s=rates)
    base = to_mixture(c["mix"])
    f0 = olbm.init_populations(c["rho0"], lat)
    return c, lat, prm, base, f0


@pytest.mark.parametrize("lattice,nc,shape", [("D2Q9", 3, (9, 11)), ("D2Q9", 2, (8, 10)), ("D3Q19", 2, (5, 6, 7))])
@pytest.mark.parametrize("collision,forcing", [("bgk", "edm"), ("bgk", "guo"), ("mrt", "edm"), ("mrt", "guo")])
def test_torch_step_is_the_numpy_step(lattice, nc, shape, collision, forcing):
    c, lat, prm, base, f0 = setup(lattice, nc, shape, collision, forcing)
    aa, b = oadj.eos_tables(torch.as_tensor(oadj.theta_of(base), dtype=oadj.DT), base, prm.T)
    f_np, f_t = f0, torch.as_tensor(f0, dtype=oadj.DT)
    for _ in range(3):
        f_np = olbm.step(f_np, base, prm, lat)
        f_t = oadj.step(f_t, aa, b, base, prm, lat)
        err = np.max(np.abs(f_t.numpy() - f_np)) / np.max(np.abs(f_np))
        assert err < 1e-13


@pytest.mark.parametrize("collision,forcing", [("bgk", "edm"), ("bgk", "guo"), ("mrt", "edm")])
def test_gradient_matches_central_differences_of_numpy_oracle(collision, forcing):
    shape = (10, 12)
    c, lat, prm, base, f0 = setup("D2Q9", 3, shape, collision, forcing, seed=2)
    mask = drop_mask(shape, min(shape) / 4.0)
    nsteps = 12
    theta = oadj.theta_of(base)
    x0 = oadj.mole_fractions(torch.as_tensor(f0, dtype=oadj.DT), base.M, mask).numpy()
    x_tgt = x0 + np.array([0.01, -0.015, 0.005])
    L, g = oadj.gradient(theta, f0, base, prm, lat, nsteps, mask, x_tgt)
    assert abs(L - numpy_loss(theta, base, f0, prm, lat, nsteps, mask, x_tgt)) <= 1e-14 * L
    h = 1e-6
    for i in range(theta.size):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (numpy_loss(tp, base, f0, prm, lat, nsteps, mask, x_tgt)
              - numpy_loss(tm, base, f0, prm, lat, nsteps, mask, x_tgt)) / (2 * h)
        assert abs(g[i] - fd) <= 1e-6 * np.max(np.abs(g)) + 1e-7 * abs(g[i]), (i, g[i], fd)


def test_dot_product_identity():
    shape = (9, 10)
    c, lat, prm, base, f0 = setup("D2Q9", 3, shape, "bgk", "edm", seed=3)
    f = olbm.step(f0, base, prm, lat)
    theta = oadj.theta_of(base)
    rng = np.random.default_rng(7)
    df = rng.standard_normal(f.shape) * 1e-3
    dth = rng.standard_normal(theta.shape) * 1e-3
    w = rng.standard_normal(f.shape)
    jv = oadj.step_jvp(f, df, dth, theta, base, prm, lat)
    gf, gth = oadj.step_vjp(f, w, theta, base, prm, lat)
    lhs = float(np.sum(jv * w))
    rhs = float(np.sum(df * gf) + np.sum(dth * gth))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + abs(rhs))


def test_zero_loss_and_gradient_at_reached_composition():
    shape = (8, 10)
    c, lat, prm, base, f0 = setup("D2Q9", 3, shape, "bgk", "edm", seed=4)
    mask = drop_mask(shape, min(shape) / 4.0)
    theta = oadj.theta_of(base)
    nsteps = 5
    f = f0
    for _ in range(nsteps):
        f = olbm.step(f, base, prm, lat)
    n = f.sum(axis=1) / base.M.reshape((-1, 1, 1))
    Ni = np.array([n[i][mask].sum() for i in range(3)])
    L, g = oadj.gradient(theta, f0, base, prm, lat, nsteps, mask, Ni / Ni.sum())
    assert L < 1e-28
    assert np.max(np.abs(g)) < 1e-12


def test_vjp_over_eos_tables_chains_to_theta():
    """The adjoint with respect to the EOS tables ((a alpha)_ij (1 - k_ij), b_i),
    pushed through the tables' own derivative in theta, is the theta adjoint."""
    shape = (8, 9)
    c, lat, prm, base, f0 = setup("D2Q9", 3, shape, "bgk", "edm", seed=5)
    f = olbm.step(f0, base, prm, lat)
    theta = oadj.theta_of(base)
    w = np.random.default_rng(8).standard_normal(f.shape)
    th = torch.as_tensor(theta, dtype=oadj.DT)
    aa, b = oadj.eos_tables(th, base, prm.T)
    gf1, gaa, gb = oadj.step_vjp_tables(f, w, aa.numpy(), b.numpy(), base, prm, lat)
    gf2, gth = oadj.step_vjp(f, w, theta, base, prm, lat)
    assert np.max(np.abs(gf1 - gf2)) <= 1e-14 * np.max(np.abs(gf2))
    thr = th.clone().requires_grad_(True)
    aa2, b2 = oadj.eos_tables(thr, base, prm.T)
    (chain,) = torch.autograd.grad((aa2 * torch.as_tensor(gaa)).sum() + (b2 * torch.as_tensor(gb)).sum(), thr)
    assert np.max(np.abs(chain.numpy() - gth)) <= 1e-13 * np.max(np.abs(gth))


def porous_mask(shape, seed, frac=0.15):
    return np.random.default_rng([7, seed]).uniform(size=shape) < frac


def wall_psi(c, base):
    corner = c["rho0"][(slice(None),) + (0,) * len(c["shape"])]
    return 1.3 * float(olbm.pseudo_potential(corner[:, None], c["T"], base, -1.0)[0])


@pytest.mark.parametrize("lattice,nc,shape", [("D2Q9", 3, (12, 14)), ("D3Q19", 2, (6, 7, 8))])
@pytest.mark.parametrize("collision,forcing", [("bgk", "edm"), ("bgk", "guo"), ("mrt", "edm"), ("mrt", "guo")])
def test_torch_step_is_the_numpy_step_with_walls(lattice, nc, shape, collision, forcing):
    c, lat, prm, base, f0 = setup(lattice, nc, shape, collision, forcing, seed=4)
    prm.solid, prm.psi_wall = porous_mask(shape, 4), wall_psi(c, base)
    f0 = f0.copy()
    f0[:, :, prm.solid] = 0.0
    aa, b = oadj.eos_tables(torch.as_tensor(oadj.theta_of(base), dtype=oadj.DT), base, prm.T)
    f_np, f_t = f0, torch.as_tensor(f0, dtype=oadj.DT)
    for _ in range(3):
        f_np = olbm.step(f_np, base, prm, lat)
        f_t = oadj.step(f_t, aa, b, base, prm, lat)
        err = np.max(np.abs(f_t.numpy() - f_np)) / np.max(np.abs(f_np))
        assert err < 1e-13


@pytest.mark.parametrize("collision,forcing", [("bgk", "edm"), ("mrt", "guo")])
def test_gradient_with_walls_matches_central_differences(collision, forcing):
    shape = (12, 14)
    c, lat, prm, base, f0 = setup("D2Q9", 3, shape, collision, forcing, seed=5)
    prm.solid, prm.psi_wall = porous_mask(shape, 5), wall_psi(c, base)
    f0 = f0.copy()
    f0[:, :, prm.solid] = 0.0
    mask = drop_mask(shape, min(shape) / 2.0) & ~prm.solid
    nsteps = 10
    theta = oadj.theta_of(base)
    x0 = oadj.mole_fractions(torch.as_tensor(f0, dtype=oadj.DT), base.M, mask).numpy()
    x_tgt = x0 + np.array([0.01, -0.015, 0.005])
    L, g = oadj.gradient(theta, f0, base, prm, lat, nsteps, mask, x_tgt)
    assert np.all(np.isfinite(g))
    assert abs(L - numpy_loss(theta, base, f0, prm, lat, nsteps, mask, x_tgt)) <= 1e-14 * L
    h = 1e-6
    for i in range(theta.size):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (numpy_loss(tp, base, f0, prm, lat, nsteps, mask, x_tgt)
              - numpy_loss(tm, base, f0, prm, lat, nsteps, mask, x_tgt)) / (2 * h)
        assert abs(g[i] - fd) <= 1e-6 * np.max(np.abs(g)) + 1e-7 * abs(g[i]), (i, g[i], fd)
