"""Physics pins of the oracle step: long CPU runs of small versions of the paper's
validation cases (marked slow; about two minutes together).

* Sec. 4.1 limiting case: two identical water-like components (a = 2/49, b = 2/21,
  omega = 0.344, T = 0.9 Tc, tau = 1, Guo forcing) at a flat interface.  With the
  blended force of Eq. (coupledMCforce) at the paper's beta = 1.945 the bulk
  densities land within 0.5 % (liquid) and 5 % (vapour) of the Maxwell values
  5.90796 / 0.58007; with the original force (beta = 1, Eq. (correctMCforce)) the
  vapour misses by more than 20 % -- the inconsistency Sec. 3.3 sets out to remove.
  The paper's own setting, a drop, is run too: its bulk densities are reported
  against Maxwell (the Laplace pressure of a drop of radius 16 raises the vapour
  density by about 10 %, so only the liquid is gated, within 2 %) and its two bulk
  phases must satisfy the iso-fugacity rule of Sec. 3.2 (f_l = f_v for one
  component) within 5 % (2.5 % measured; the flat interface's vapour sits 3 %
  above Maxwell at this beta).
* Sec. 4.2 flat interface of 40 % propane / 60 % n-pentane at T = Tc(C3) (Table 1
  data in the lattice units of Sec. 4.2, Eq. (initialdensity) with the slab position
  of Eq. (initialdensity2)) in an 80 x 1 box: the bulk phases must match the
  flash (iso-fugacity solution) within 5 % in composition and 3 % in phase density
  (the paper: 4.0 % and 2.1 % at 1600 x 2) -- Guo forcing with beta = 1.945 at
  200 psia, and the exact-difference forcing with its own beta = 1.3 at 240 psia.
  The exact-difference forcing must deliver chi_s F to each component (the reading
  of the oracle's step); relaxing every component towards feq(j/rho) instead misses
  the flash by tens of per cent.
* Sec. 4.3 Laplace's law: three small drops (n = 40, 48, 56, R0 = n/5, beta = 1.915,
  200 psia): dp against 1/R is a straight line (R^2 > 0.999); the surface tension of
  each drop, dp R, lies within 10 % of the paper's 0.1289 and grows towards it
  with the drop size (the GPU validation of sizes 50...800 converges to it).
"""
import numpy as np
import pytest

from golden_io import maxwell, table1
from oracle import lattice as L
from oracle import lbm, thermo

pytestmark = pytest.mark.slow
LAT = L.d2q9()
R_FIELD = 10.7316          # psia ft^3 / (lbmol degR): Table 1's R_s = R / M to its printed digits


def lattice_mixture(names=("C3", "nC5")):
    """Table 1 components in the lattice units of Sec. 4.2 (a_1 = 2/49, b_1 = 2/21,
    M_1 = 1, R = 1); returns the mixture and the factors that turn a field
    temperature [degR] and pressure [psia] into lattice units."""
    t = table1()
    phys = thermo.mixture_from_critical([t[n]["pc"] for n in names], [t[n]["Tc"] for n in names],
                                        [t[n]["omega"] for n in names], [t[n]["M"] for n in names], R=R_FIELD)
    sn = (2.0 / 21.0) / phys.b[0]                 # molar density scale: b_lb = b sn
    sp = phys.a[0] * sn * sn / (2.0 / 49.0)       # pressure scale: a_lb = a sn^2 / sp
    sT = sp / (R_FIELD * sn)                      # temperature scale: R_lb = 1
    mix = thermo.Mixture(a=phys.a * sn * sn / sp, b=phys.b * sn, omega=phys.omega, M=phys.M / phys.M[0],
                         k=np.zeros((len(names), len(names))), R=1.0)
    return mix, 1.0 / sT, 1.0 / sp


def run(f, mix, prm, steps, probe=None, every=2000):
    """Advance `steps` steps; returns the final populations and the largest
    relative change of probe(f) over the last `every` steps."""
    last = None
    change = np.inf
    for i in range(1, steps + 1):
        f = lbm.step(f, mix, prm, LAT)
        if probe is not None and i % every == 0:
            v = probe(f)
            if last is not None:
                change = float(np.max(np.abs(v - last) / np.abs(last)))
            last = v
    return f, change


# ---------------------------------------------------------------------------
# Sec. 4.1: limiting case against the Maxwell construction
# ---------------------------------------------------------------------------

def _water_pair():
    g = maxwell()
    mix = thermo.Mixture(a=[g["a"]] * 2, b=[g["b"]] * 2, omega=[g["omega"]] * 2, M=[1.0, 1.0],
                         k=np.zeros((2, 2)), R=1.0)
    return mix, g["T_over_Tc"] * mix.Tc[0], g["rho_l"], g["rho_v"]


def _identical_split(rho_l, rho_v, t):
    """Eq. (initialMC): component 1 carries the liquid, component 2 the vapour."""
    return np.stack([0.5 * rho_l - 0.5 * rho_l * t, 0.5 * rho_v + 0.5 * rho_v * t])


@pytest.mark.parametrize("beta", [1.945, 1.0])
def test_limiting_case_flat_coexistence_against_maxwell(beta):
    mix, T, rl, rv = _water_pair()
    n = 64
    x = np.arange(n, dtype=float)
    t = np.tanh(2.0 * (np.abs(x - n / 2) - n / 4) / 8.0)
    f = lbm.init_populations(_identical_split(rl, rv, t)[:, None, :], LAT)
    prm = lbm.StepParams(T=T, tau=1.0, gamma=np.array([1.0, 1.0]), beta=beta, collision="bgk", forcing="guo")
    bulk = lambda g: lbm.densities(g).sum(axis=0)[0, [n // 2, 0]]
    f, change = run(f, mix, prm, 8000, bulk)
    dl, dv = bulk(f) / np.array([rl, rv]) - 1.0
    print(f"beta {beta}: rho_l {bulk(f)[0]:.5f} ({dl:+.2%}), rho_v {bulk(f)[1]:.5f} ({dv:+.2%}), change {change:.1e}")
    assert change < 1e-6
    if beta == 1.0:
        assert dv < -0.2                       # the original force: vapour far below Maxwell
    else:
        assert abs(dl) < 5e-3 and abs(dv) < 5e-2


def test_limiting_case_drop_of_sec_4_1():
    mix, T, rl, rv = _water_pair()
    n = 64
    g = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float), indexing="ij")
    r = np.sqrt((g[0] - n / 2) ** 2 + (g[1] - n / 2) ** 2)
    t = np.tanh(2.0 * (r - n / 4) / 8.0)         # Eq. (initialden), W = 8, r0 = n/4
    f = lbm.init_populations(_identical_split(rl, rv, t), LAT)
    prm = lbm.StepParams(T=T, tau=1.0, gamma=np.array([1.0, 1.0]), beta=1.945, collision="bgk", forcing="guo")
    bulk = lambda h: lbm.densities(h).sum(axis=0)[[n // 2, 0], [n // 2, 0]]
    f, change = run(f, mix, prm, 5000, bulk)
    d_l, d_v = bulk(f)
    # one component: molar density = mass density (M = 1); f_i = phi_i p
    pure = thermo.Mixture(a=mix.a[:1], b=mix.b[:1], omega=mix.omega[:1], M=mix.M[:1], k=np.zeros((1, 1)), R=1.0)
    fl = thermo.state_from_molar(pure, T, [d_l])["fug"][0]
    fv = thermo.state_from_molar(pure, T, [d_v])["fug"][0]
    print(f"drop: rho_l {d_l:.5f} ({d_l / rl - 1:+.2%} vs Maxwell), rho_v {d_v:.5f} ({d_v / rv - 1:+.2%}), "
          f"f_l/f_v - 1 = {fl / fv - 1:.2e}, change {change:.1e}")
    assert change < 1e-4
    assert abs(d_l / rl - 1.0) < 2e-2
    assert abs(fl / fv - 1.0) < 5e-2


# ---------------------------------------------------------------------------
# Sec. 4.2: flat interface against the flash
# ---------------------------------------------------------------------------

def slab_vapour_width(rbar_l, rbar_v, M, z1, L):
    """Eq. (initialdensity2): the vapour width L0 at each end of the box for which a
    sharp liquid slab between two vapour regions holds the overall mole fraction z1
    (mole numbers per unit area: (L - 2 L0) n_l + 2 L0 n_v per component)."""
    nl = np.asarray(rbar_l) / M
    nv = np.asarray(rbar_v) / M
    return L * (nl[0] - z1 * nl.sum()) / (2.0 * (z1 * (nv.sum() - nl.sum()) - nv[0] + nl[0]))


def flat_interface(p_psia, forcing, beta, nx=80, steps=20000, z1=0.4, D=8.0):
    mix, perT, perp = lattice_mixture()
    T = table1()["C3"]["Tc"] * perT
    p = p_psia * perp
    z = np.array([z1, 1.0 - z1])
    fl = thermo.flash(mix, T, p, z)
    L0 = slab_vapour_width(fl.rbar_l, fl.rbar_v, mix.M, z1, float(nx))
    x = np.arange(nx, dtype=float)
    lv = 0.5 * (fl.rbar_l + fl.rbar_v)[:, None]
    hw = 0.5 * (fl.rbar_l - fl.rbar_v)[:, None]
    left = lv + hw * np.tanh(2.0 * (x - L0) / D)                 # Eq. (initialdensity)
    right = lv - hw * np.tanh(2.0 * (x - nx + L0) / D)
    rho0 = np.where(x <= nx / 2, left, right)[:, None, :]
    f = lbm.init_populations(rho0, LAT)
    prm = lbm.StepParams(T=T, tau=0.8, gamma=fl.gamma, beta=beta, collision="bgk", forcing=forcing)
    bulk = lambda g: lbm.densities(g)[:, 0, [nx // 2, 0]].T.ravel()     # (liquid comps, vapour comps)
    f, change = run(f, mix, prm, steps, bulk)
    rl, rv = bulk(f).reshape(2, 2)
    nl, nv = rl / mix.M, rv / mix.M
    x_lb, y_lb = nl / nl.sum(), nv / nv.sum()
    err_c = max(np.max(np.abs(x_lb - fl.x) / fl.x), np.max(np.abs(y_lb - fl.y) / fl.y))
    err_d = max(abs(rl.sum() / fl.rbar_l.sum() - 1.0), abs(rv.sum() / fl.rbar_v.sum() - 1.0))
    sl, sv = thermo.state_from_molar(mix, T, nl), thermo.state_from_molar(mix, T, nv)
    res = thermo.iso_fugacity_residual(sl["fug"], sv["fug"])     # Eq. (error) at the LB bulk states
    print(f"{forcing} beta {beta} {p_psia} psia: x1 {x_lb[0]:.4f} (flash {fl.x[0]:.4f}), y1 {y_lb[0]:.4f} "
          f"(flash {fl.y[0]:.4f}); composition err {err_c:.2%}, density err {err_d:.2%}, "
          f"Eq. (error) residual {res:.2e}, LB pressure {0.5 * (sl['p'] + sv['p']) / perp:.1f} psia, change {change:.1e}")
    return err_c, err_d, res, change


@pytest.mark.parametrize("forcing,beta,p_psia", [("guo", 1.945, 200.0), ("edm", 1.3, 240.0)])
def test_flat_interface_matches_flash(forcing, beta, p_psia):
    err_c, err_d, res, change = flat_interface(p_psia, forcing, beta)
    assert change < 1e-4
    assert err_c < 0.05 and err_d < 0.03
    assert res < 1e-2


# ---------------------------------------------------------------------------
# Sec. 4.3: Laplace's law on small drops
# ---------------------------------------------------------------------------

def drop_radius_and_dp(rho_s, mix, T):
    """Radius where the total density crosses (rho_centre + rho_corner)/2 on the
    four axis rays from the centre (linear interpolation, averaged) and the
    pressure jump p_EOS(centre) - p_EOS(corner)."""
    rho = rho_s.sum(axis=0)
    n = rho.shape[0]
    c = n // 2
    level = 0.5 * (rho[c, c] + rho[0, 0])
    radii = []
    for prof in (rho[c, c:], rho[c, c::-1], rho[c:, c], rho[c::-1, c]):
        k = int(np.argmax(prof < level))
        radii.append(k - 1 + (prof[k - 1] - level) / (prof[k - 1] - prof[k]))
    p = thermo.pressure_molar((rho_s[:, [c, 0], [c, 0]] / mix.M[:, None]), T, mix)
    return float(np.mean(radii)), float(p[0] - p[1])


def test_laplace_law_small_drops():
    mix, perT, perp = lattice_mixture()
    T = table1()["C3"]["Tc"] * perT
    fl = thermo.flash(mix, T, 200.0 * perp, np.array([0.4, 0.6]))
    inv_r, dps = [], []
    for n in (40, 48, 56):
        g = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float), indexing="ij")
        r = np.sqrt((g[0] - n / 2) ** 2 + (g[1] - n / 2) ** 2)
        t = np.tanh(2.0 * (r - n / 5.0) / 4.0)
        rho0 = 0.5 * (fl.rbar_l + fl.rbar_v)[:, None, None] - 0.5 * (fl.rbar_l - fl.rbar_v)[:, None, None] * t
        f = lbm.init_populations(rho0, LAT)
        prm = lbm.StepParams(T=T, tau=0.8, gamma=fl.gamma, beta=1.915, collision="bgk", forcing="guo")
        f, change = run(f, mix, prm, 6000, lambda h: np.array(drop_radius_and_dp(lbm.densities(h), mix, T)))
        R, dp = drop_radius_and_dp(lbm.densities(f), mix, T)
        print(f"n {n}: R {R:.3f}, dp {dp:.6f}, sigma_n = dp R = {dp * R:.4f}, change {change:.1e}")
        assert change < 1e-3
        inv_r.append(1.0 / R)
        dps.append(dp)
    inv_r, dps = np.array(inv_r), np.array(dps)
    slope, icpt = np.polyfit(inv_r, dps, 1)
    fit = slope * inv_r + icpt
    r2 = 1.0 - np.sum((dps - fit) ** 2) / np.sum((dps - dps.mean()) ** 2)
    # lattice units of pressure x length: the paper quotes sigma in the same units
    print(f"sigma (slope) {slope:.4f} (paper 0.1289), intercept {icpt:.2e}, R^2 {r2:.6f}")
    assert r2 > 0.999
    sig = dps / inv_r
    assert np.all(np.abs(sig / 0.1289 - 1.0) < 0.10)     # Laplace's law drop by drop
    assert np.all(np.diff(sig) > 0.0)                     # and approaching the paper's value with size
