"""Pins of the oracle LB step (oracle/lbm.py, oracle/lattice.py).

Each test checks the oracle against something fixed by the paper or by
mathematics rather than against itself:
  * lattice isotropy moments and MRT row orthogonality;
  * equilibrium moments of Eq. (equilibrium a) and Guo-term moments of Eq. (equilibrium b);
  * exact per-component mass conservation and the momentum balance with forcing
    (sum_x F = 0 in a periodic box, Eq. (coupledMCforce));
  * MRT with every rate 1/tau is BGK;
  * Sec. 4.1 limiting case: N identical components reproduce a single-component
    Shan-Chen LBE, implemented independently below from Eq. (SCpengrobinson);
  * the stencil of Eq. (coupledMCforce) on a linear psi gives -G c_s^2 psi grad(psi)
    for every beta; F does not depend on |G|;
  * a uniform resting state is a fixed point; streaming moves a population by e_a.
"""
import numpy as np
import pytest

from oracle import lattice as L
from oracle import lbm, thermo

LATS = [L.d2q9(), L.d3q19()]


def _binary_mix(k12=0.02):
    return thermo.Mixture(a=[2 / 49, 0.08], b=[2 / 21, 0.15], omega=[0.15, 0.25],
                          M=[1.0, 1.6], k=[[0, k12], [k12, 0]], R=1.0)


def _drop_state(lat, shape, mix, seed=0):
    """Two-phase-like smooth densities (drop of liquid-ish values in vapor-ish values)."""
    rng = np.random.default_rng(seed)
    grids = np.meshgrid(*[np.arange(n, dtype=float) for n in shape], indexing="ij")
    r = np.sqrt(sum((g - n / 2) ** 2 for g, n in zip(grids, shape)))
    t = np.tanh(2 * (r - min(shape) / 4) / 4.0)
    inner = np.array([1.8, 4.2])[: mix.nc]
    outer = np.array([0.25, 0.15])[: mix.nc]
    rho = 0.5 * (inner + outer)[:, None] - 0.5 * (inner - outer)[:, None] * t.reshape(1, -1)
    rho = rho.reshape((mix.nc,) + tuple(shape)) * (1 + 1e-3 * rng.uniform(-1, 1, (mix.nc,) + tuple(shape)))
    u = 0.02 * rng.uniform(-1, 1, (lat.D,) + tuple(shape))
    return lbm.init_populations(rho, lat, u)


def _params(lat, collision="bgk", forcing="guo", beta=1.5, tau=0.8, gamma=(0.6, 1.0), accel=None, rates=None):
    T = 0.8 * min(_binary_mix().Tc)
    s = None
    if collision == "mrt":
        s = rates if rates is not None else np.linspace(0.9, 1.6, lat.Q)
    return lbm.StepParams(T=T, tau=tau, gamma=np.array(gamma), beta=beta, collision=collision,
                          forcing=forcing, mrt_s=s, accel=accel)


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_lattice_isotropy(lat):
    e = lat.e.astype(float)
    w = lat.w
    cs2 = L.CS2
    I = np.eye(lat.D)
    assert abs(w.sum() - 1) < 1e-15
    assert np.allclose(np.einsum("a,ai->i", w, e), 0, atol=1e-16)
    assert np.allclose(np.einsum("a,ai,aj->ij", w, e, e), cs2 * I, atol=1e-16)
    assert np.allclose(np.einsum("a,ai,aj,ak->ijk", w, e, e, e), 0, atol=1e-16)
    m4 = np.einsum("a,ai,aj,ak,al->ijkl", w, e, e, e, e)
    iso = cs2 * cs2 * (np.einsum("ij,kl->ijkl", I, I) + np.einsum("ik,jl->ijkl", I, I)
                       + np.einsum("il,jk->ijkl", I, I))
    assert np.allclose(m4, iso, atol=1e-16)
    # every velocity has its opposite
    for a in range(lat.Q):
        assert any(np.all(lat.e[b] == -lat.e[a]) for b in range(lat.Q))


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_mrt_rows_orthogonal(lat):
    M = L.mrt_basis(lat)
    G = M @ M.T
    assert np.allclose(G - np.diag(np.diag(G)), 0, atol=1e-12)
    assert np.linalg.matrix_rank(M) == lat.Q
    assert np.allclose(M[0], 1.0)
    for d in range(lat.D):   # momentum rows are the velocity components
        assert any(np.allclose(M[k], lat.e[:, d]) for k in range(lat.Q))


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_equilibrium_moments(lat):
    rng = np.random.default_rng(1)
    rho = rng.uniform(0.1, 5, size=(7,))
    u = rng.uniform(-0.1, 0.1, size=(lat.D, 7))
    feq = lbm.equilibrium(rho, u, lat)
    e = lat.e.astype(float)
    assert np.allclose(feq.sum(0), rho, rtol=1e-14)
    assert np.allclose(np.einsum("ac,ai->ic", feq, e), rho * u, atol=1e-14)
    P = np.einsum("ac,ai,aj->ijc", feq, e, e)
    want = rho * (L.CS2 * np.eye(lat.D)[:, :, None] + u[:, None] * u[None, :])
    assert np.allclose(P, want, atol=1e-14)


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_guo_source_moments(lat):
    rng = np.random.default_rng(2)
    u = rng.uniform(-0.1, 0.1, size=(lat.D, 5))
    F = rng.uniform(-0.01, 0.01, size=(lat.D, 5))
    tau = 0.8
    S = (1 - 0.5 / tau) * lbm.guo_shape(F, u, lat)
    e = lat.e.astype(float)
    assert np.allclose(S.sum(0), 0, atol=1e-17)
    assert np.allclose(np.einsum("ac,ai->ic", S, e), (1 - 0.5 / tau) * F, atol=1e-17)
    second = np.einsum("ac,ai,aj->ijc", S, e, e)
    want = (1 - 0.5 / tau) * (u[:, None] * F[None, :] + F[:, None] * u[None, :])
    assert np.allclose(second, want, atol=1e-17)


def _shape(lat):
    return (12, 14) if lat.D == 2 else (6, 7, 8)


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
@pytest.mark.parametrize("collision,forcing", [("bgk", "guo"), ("bgk", "edm"), ("mrt", "guo"), ("mrt", "edm")])
def test_mass_and_momentum_conservation(lat, collision, forcing):
    mix = _binary_mix()
    f = _drop_state(lat, _shape(lat), mix)
    prm = _params(lat, collision, forcing)
    t0 = lbm.totals(f, mix, prm, lat)
    for _ in range(10):
        f = lbm.step(f, mix, prm, lat)
    t1 = lbm.totals(f, mix, prm, lat)
    assert np.all(np.abs(t1["mass"] / t0["mass"] - 1) < 1e-13)
    assert np.all(np.abs(t1["force"]) < 1e-13)
    assert np.all(np.abs(t1["momentum"] - t0["momentum"]) < 1e-12)


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
@pytest.mark.parametrize("forcing", ["guo", "edm"])
def test_momentum_balance_with_body_acceleration(lat, forcing):
    mix = _binary_mix()
    f = _drop_state(lat, _shape(lat), mix)
    g = np.array([1e-5, -2e-5, 3e-5][: lat.D])
    prm = _params(lat, "bgk", forcing, accel=g)
    t0 = lbm.totals(f, mix, prm, lat)
    M = t0["mass"].sum()
    n = 6
    for _ in range(n):
        f = lbm.step(f, mix, prm, lat)
    t1 = lbm.totals(f, mix, prm, lat)
    assert np.allclose(t1["momentum"] - t0["momentum"], n * M * g, rtol=1e-10, atol=1e-13)


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
@pytest.mark.parametrize("forcing", ["guo", "edm"])
def test_mrt_equal_rates_is_bgk(lat, forcing):
    mix = _binary_mix()
    f = _drop_state(lat, _shape(lat), mix)
    tau = 0.8
    a = lbm.step(f, mix, _params(lat, "bgk", forcing, tau=tau), lat)
    b = lbm.step(f, mix, _params(lat, "mrt", forcing, tau=tau, rates=np.full(lat.Q, 1 / tau)), lat)
    assert np.max(np.abs(a - b)) < 1e-14 * np.max(np.abs(a))


def single_component_step(f, a, b, omega, T, tau, beta, lat, forcing):
    """Independent single-component Shan-Chen LBE (the model the limiting case of
    Sec. 4.1 must reproduce): pure PR pressure in mass density, psi, the beta force,
    BGK with Guo or exact-difference forcing, periodic streaming."""
    cs2 = 1.0 / 3.0
    G = -1.0
    rho = f.sum(0)
    e = lat.e
    j = np.tensordot(e.T.astype(float), f, axes=([1], [0]))
    p = thermo.pure_pressure_mass(rho, T, a, b, omega, 1.0)
    psi = np.sqrt(2 * (p - cs2 * rho) / (G * cs2))
    nd = lat.D
    axes = {d: f.ndim - 2 - d for d in range(nd)}   # axes of a spatial array

    def nb(arr, ea):  # arr(x + e)
        out = arr
        for d in range(nd):
            if ea[d]:
                out = np.roll(out, -ea[d], axis=axes[d])
        return out

    F = np.zeros((nd,) + rho.shape)
    for al in range(1, lat.Q):
        pn = nb(psi, e[al])
        for d in range(nd):
            F[d] += lat.w[al] * e[al, d] * (-beta * G * psi * pn - 0.5 * (1 - beta) * G * pn * pn)

    def feq(r, u):
        uu = (u * u).sum(0)
        out = np.empty_like(f)
        for al in range(lat.Q):
            eu = sum(e[al, d] * u[d] for d in range(nd))
            out[al] = r * lat.w[al] * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * uu)
        return out

    if forcing == "guo":
        u = (j + 0.5 * F) / rho
        src = np.empty_like(f)
        for al in range(lat.Q):
            eu = sum(e[al, d] * u[d] for d in range(nd))
            src[al] = (1 - 0.5 / tau) * lat.w[al] * sum(
                (3 * (e[al, d] - u[d]) + 9 * eu * e[al, d]) * F[d] for d in range(nd))
        post = f - (f - feq(rho, u)) / tau + src
    else:
        u = j / rho
        post = f - (f - feq(rho, u)) / tau + feq(rho, u + F / rho) - feq(rho, u)
    out = np.empty_like(f)
    for al in range(lat.Q):
        moved = post[al]
        for d in range(nd):
            if e[al, d]:
                moved = np.roll(moved, e[al, d], axis=axes[d] - 0)
        out[al] = moved
    return out


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
@pytest.mark.parametrize("forcing,gamma", [("guo", (1.0, 1.0)), ("guo", (0.4, 1.0)), ("edm", (1.0, 1.0))])
def test_identical_components_reproduce_single_component(lat, forcing, gamma):
    # Sec. 4.1: water + water behaves as pure water.  With Guo forcing the total
    # population is the single-component one for ANY gamma (the split is linear).
    a, b, om = 2 / 49, 2 / 21, 0.344
    mix = thermo.Mixture(a=[a, a], b=[b, b], omega=[om, om], M=[1.0, 1.0], k=np.zeros((2, 2)), R=1.0)
    T = 0.9 * mix.Tc[0]
    shape = _shape(lat)
    grids = np.meshgrid(*[np.arange(n, dtype=float) for n in shape], indexing="ij")
    r = np.sqrt(sum((g - n / 2) ** 2 for g, n in zip(grids, shape)))
    W = 3.0
    r0 = min(shape) / 3
    rho_l, rho_v = 5.90796, 0.58007
    th_ = np.tanh(2 * (r - r0) / W)
    r1 = rho_l / 2 - rho_l / 2 * th_        # Eq. (initialMC), component 1
    r2 = rho_v / 2 + rho_v / 2 * th_        # Eq. (initialMC), component 2
    f = lbm.init_populations(np.stack([r1, r2]), lat)
    fsc = f.sum(0)
    prm = lbm.StepParams(T=T, tau=1.0, gamma=np.array(gamma), beta=1.3, forcing=forcing)
    for _ in range(5):
        f = lbm.step(f, mix, prm, lat)
        fsc = single_component_step(fsc, a, b, om, T, 1.0, 1.3, lat, forcing)
    assert np.max(np.abs(f.sum(0) - fsc)) < 1e-13 * np.max(fsc)


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
@pytest.mark.parametrize("beta", [1.0, 1.945, 0.5])
def test_force_stencil_on_linear_psi(lat, beta):
    shape = (20, 22) if lat.D == 2 else (9, 10, 11)
    xs = np.meshgrid(*[np.arange(n, dtype=float) for n in shape], indexing="ij")[::-1]
    g = np.array([0.013, -0.021, 0.017][: lat.D])
    psi = 1.7 + sum(g[d] * xs[d] for d in range(lat.D))
    G = -1.0
    F = lbm.total_force(psi, beta, G, lat)
    want = np.stack([-G * L.CS2 * psi * g[d] for d in range(lat.D)])
    interior = tuple([slice(None)] + [slice(1, n - 1) for n in shape])
    assert np.max(np.abs(F[interior] - want[interior])) < 1e-15
    # uniform psi gives no force anywhere
    F0 = lbm.total_force(np.full(shape, 2.3), beta, G, lat)
    assert np.max(np.abs(F0)) < 1e-15


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_force_independent_of_G_magnitude(lat):
    mix = _binary_mix()
    f = _drop_state(lat, _shape(lat), mix)
    rho_s = lbm.densities(f)
    T = 0.8 * min(mix.Tc)
    F1 = lbm.total_force(lbm.pseudo_potential(rho_s, T, mix, -1.0), 1.7, -1.0, lat)
    F2 = lbm.total_force(lbm.pseudo_potential(rho_s, T, mix, -2.5), 1.7, -2.5, lat)
    assert np.max(np.abs(F1 - F2)) < 1e-15 * max(1.0, np.max(np.abs(F1))) * 10


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
@pytest.mark.parametrize("collision,forcing", [("bgk", "guo"), ("mrt", "edm")])
def test_uniform_state_is_fixed_point(lat, collision, forcing):
    mix = _binary_mix()
    shape = _shape(lat)
    rho = np.stack([np.full(shape, 1.2), np.full(shape, 0.7)])
    f = lbm.init_populations(rho, lat)
    f1 = lbm.step(f, mix, _params(lat, collision, forcing), lat)
    assert np.max(np.abs(f1 - f)) < 1e-15


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_shift_moves_by_velocity(lat):
    shape = _shape(lat)
    for a in range(lat.Q):
        arr = np.zeros(shape)
        src = tuple(n // 2 for n in shape)
        arr[src] = 1.0
        out = lbm.shift(arr, lat.e[a], lead=0)
        # destination index: x + e (x is the last axis)
        dst = list(src)
        for d in range(lat.D):
            ax = len(shape) - 1 - d
            dst[ax] = (dst[ax] + lat.e[a, d]) % shape[ax]
        assert out[tuple(dst)] == 1.0 and out.sum() == 1.0


def test_split_sums_to_total():
    rng = np.random.default_rng(4)
    rho_s = rng.uniform(0.1, 3, (3, 5, 6))
    F = rng.uniform(-1, 1, (2, 5, 6))
    Fs = lbm.split_force(F, rho_s, [0.3, 0.7, 1.0])
    assert np.allclose(Fs.sum(0), F, atol=1e-15)
    # chi_i proportional to gamma_i rbar_i (Eq. (distributionforce))
    ratio = Fs[0, 0] / Fs[2, 0]
    assert np.allclose(ratio, 0.3 * rho_s[0] / rho_s[2])


def test_domain_errors():
    lat = L.d2q9()
    mix = _binary_mix()
    T = 0.8 * min(mix.Tc)
    # b_m rho~ >= 1
    rho_s = np.stack([np.full((4, 4), 11.0), np.full((4, 4), 0.1)])
    with pytest.raises(lbm.DomainError):
        lbm.pseudo_potential(rho_s, T, mix, -1.0)
    # positive G makes the square-root argument negative
    rho_s = np.stack([np.full((4, 4), 1.0), np.full((4, 4), 0.5)])
    with pytest.raises(lbm.DomainError):
        lbm.pseudo_potential(rho_s, T, mix, +1.0)
    del lat


def _default_rates(lat, tau):
    from paper_1909_12390_amd.inputs import default_mrt_rates
    return default_mrt_rates(lat.name, tau)


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
@pytest.mark.parametrize("collision", ["bgk", "mrt"])
@pytest.mark.parametrize("forcing", ["guo", "edm"])
def test_per_component_momentum_change_follows_split(lat, collision, forcing):
    # Sec. 3.1: component s receives chi_s F, chi_s = gamma_s rbar_s / Gamma
    # (Eq. (distributionforce)).  Both forcings change the component momentum by
    #   j_s* - j_s = -(j_s - rbar_s U)/tau + (1 - 1/(2 tau)) chi_s F,
    # U = (j + F/2)/rho the barycentric velocity (Guo's first moment; for EDM the
    # relaxation towards U - du_s/2 plus the jump du_s give the same).  With MRT the
    # benchmark rates relax the component momentum rows at 1/tau, so the same holds.
    mix = _binary_mix()
    f = _drop_state(lat, _shape(lat), mix)
    tau = 0.8
    gamma = np.array([0.45, 1.0])
    rates = _default_rates(lat, tau) if collision == "mrt" else None
    prm = _params(lat, collision, forcing, tau=tau, gamma=gamma, rates=rates)
    _, fld = lbm.step(f, mix, prm, lat, return_fields=True)
    e = lat.e.astype(float)
    Gam = gamma[0] * fld["rho_s"][0] + gamma[1] * fld["rho_s"][1]
    rho = fld["rho_s"].sum(axis=0)
    U = (np.einsum("sa...,ai->i...", f, e) + 0.5 * fld["F"]) / rho
    for s in range(2):
        j_s = np.einsum("a...,ai->i...", f[s], e)
        j_post = np.einsum("a...,ai->i...", fld["fstar"][s], e)
        Fs = gamma[s] * fld["rho_s"][s] / Gam * fld["F"]
        want = j_s - (j_s - fld["rho_s"][s] * U) / tau + (1.0 - 0.5 / tau) * Fs
        assert np.max(np.abs(j_post - want)) < 1e-14


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
@pytest.mark.parametrize("collision", ["bgk", "mrt"])
@pytest.mark.parametrize("forcing", ["guo", "edm"])
def test_resting_components_receive_their_force_share(lat, collision, forcing):
    # Eq. (hydrostatic1) of Sec. 3.1: at rest every component balances its partial
    # pressure gradient with its own share chi_s F of the force, which requires the
    # step to deliver exactly chi_s F to component s.  A resting component
    # (velocity (j_s + F_s/2)/rbar_s = 0, i.e. j_s = -F_s/2) must leave the
    # collision with j_s* = +F_s/2, whatever tau, the collision rates or the
    # composition.
    mix = _binary_mix()
    f0 = _drop_state(lat, _shape(lat), mix)
    tau = 0.7
    gamma = np.array([0.3, 1.0])
    rates = _default_rates(lat, tau) if collision == "mrt" else None
    prm = _params(lat, collision, forcing, tau=tau, gamma=gamma, rates=rates)
    rho_s = lbm.densities(f0)
    _, fld = lbm.step(f0, mix, prm, lat, return_fields=True)      # F depends on the densities only
    Fs = fld["F_s"]
    f = np.stack([lbm.equilibrium(rho_s[s], -0.5 * Fs[s] / rho_s[s], lat) for s in range(2)])
    _, fld = lbm.step(f, mix, prm, lat, return_fields=True)
    scale = np.max(np.abs(Fs))
    assert np.max(np.abs(fld["F_s"] - Fs)) < 1e-13 * scale
    e = lat.e.astype(float)
    for s in range(2):
        j_post = np.einsum("a...,ai->i...", fld["fstar"][s], e)
        assert np.max(np.abs(j_post - 0.5 * Fs[s])) < 1e-12 * scale
