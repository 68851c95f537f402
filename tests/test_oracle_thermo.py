"""Pins of the oracle thermodynamics (oracle/thermo.py) against the paper and mathematics.

Pins used here:
  * Sec. 4.1: Maxwell densities of the pure PR fluid (golden/maxwell_pure_pr.txt),
    reached twice: through the Gibbs/fugacity route and by an equal-area quadrature
    of the EOS that uses none of the fugacity formulas.
  * Table 2 (Sec. 4.2) with Table 1 data (golden/table2_c3_nc5.txt).
  * Identities: the EOS-derived Z solves the (corrected) cubic; dG of
    Eq. (solutionselection) equals sum_i c_i [ln phi_i(Zmax) - ln phi_i(Zmin)];
    ln phi_i equals the composition derivative of the residual Helmholtz energy
    obtained by quadrature of the EOS pressure; the binary Rachford-Rice root has a
    closed form; a two-identical-component mixture reproduces the pure EOS.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from golden_io import maxwell, table1, table2
from oracle import thermo as th

R_FIELD = 10.7316    # psia ft^3 / (lbmol degR); Table 1 lists R_i = R / M_i


def c3_nc5():
    t1 = table1()
    c3, c5 = t1["C3"], t1["nC5"]
    return th.mixture_from_critical([c3["pc"], c5["pc"]], [c3["Tc"], c5["Tc"]],
                                    [c3["omega"], c5["omega"]], [c3["M"], c5["M"]], R=R_FIELD)


def test_table1_gas_constant_consistent():
    # Table 1's specific gas constants are R / M_i to the printed three digits
    for name, row in table1().items():
        assert abs(R_FIELD / row["M"] - row["Rs"]) <= 0.0015, name


def test_m_of_omega_branches_continuous_enough():
    # the two branches of m(omega) agree to 5e-3 at the switch omega = 0.49 (Sec. 3.2)
    lo = 0.374640 + 1.54226 * 0.49 - 0.26992 * 0.49 ** 2
    hi = 0.379642 + 1.48503 * 0.49 - 0.164423 * 0.49 ** 2 + 0.016666 * 0.49 ** 3
    assert abs(th.m_of_omega(0.49) - lo) < 1e-15
    assert abs(th.m_of_omega(0.4901) - (0.379642 + 1.48503 * 0.4901 - 0.164423 * 0.4901 ** 2
                                        + 0.016666 * 0.4901 ** 3)) < 1e-15
    assert abs(lo - hi) < 5e-3


def test_maxwell_pure_by_fugacity_matches_paper():
    g = maxwell()
    mix1 = th.Mixture(a=[g["a"]], b=[g["b"]], omega=[g["omega"]], M=[1.0], k=[[0.0]], R=1.0)
    T = g["T_over_Tc"] * mix1.Tc[0]
    p, rl, rv = th.maxwell_by_fugacity(mix1, T)
    assert abs(rl / g["rho_l"] - 1) < 1e-4
    assert abs(rv / g["rho_v"] - 1) < 1e-4
    # equal pressure and equal ln(phi) at the two densities (state_from_molar uses Z=p/(rho R T))
    sl = th.state_from_molar(mix1, T, [rl])
    sv = th.state_from_molar(mix1, T, [rv])
    assert abs(sl["p"] - sv["p"]) < 1e-14
    assert abs(sl["lnphi"][0] - sv["lnphi"][0]) < 1e-11


def test_maxwell_equal_area_independent_route():
    g = maxwell()
    Tc = (th.OMEGA_B / th.OMEGA_A) * g["a"] / g["b"]
    p, rl, rv = th.maxwell_equal_area(g["a"], g["b"], g["omega"], g["T_over_Tc"] * Tc)
    assert abs(rl / g["rho_l"] - 1) < 1e-4
    assert abs(rv / g["rho_v"] - 1) < 1e-4
    mix1 = th.Mixture(a=[g["a"]], b=[g["b"]], omega=[g["omega"]], M=[1.0], k=[[0.0]], R=1.0)
    p2, rl2, rv2 = th.maxwell_by_fugacity(mix1, g["T_over_Tc"] * Tc)
    assert abs(p / p2 - 1) < 1e-11 and abs(rl / rl2 - 1) < 1e-11 and abs(rv / rv2 - 1) < 1e-10


def test_pure_limit_of_mixture_eos():
    # two identical components (M = 1) behave as the pure substance, Eq. (SCpengrobinson)
    a, b, om = 2 / 49, 2 / 21, 0.344
    mix = th.Mixture(a=[a, a], b=[b, b], omega=[om, om], M=[1.0, 1.0], k=np.zeros((2, 2)), R=1.0)
    T = 0.9 * mix.Tc[0]
    rng = np.random.default_rng(0)
    n = rng.uniform(0.05, 4.0, size=(2, 50))
    p_mix = th.pressure_molar(n, T, mix)
    p_pure = th.pure_pressure_mass(n.sum(0), T, a, b, om, 1.0)
    assert np.max(np.abs(p_mix - p_pure) / np.abs(p_pure).max()) < 1e-14


@pytest.mark.parametrize("row", [r for r in table2() if not math.isnan(r["Zv"]) and not math.isnan(r["Zl"])],
                         ids=lambda r: f"p{r['p']:.0f}")
def test_table2_two_phase_rows(row):
    mix = c3_nc5()
    fr = th.flash(mix, 666.06, row["p"], [0.4, 0.6])
    assert abs(fr.Zl / row["Zl"] - 1) < 2e-4
    assert abs(fr.Zv / row["Zv"] - 1) < 2e-4
    # mole fractions: printed to 5 decimals, systematically 4e-5..9e-5 above a 1e-13
    # converged flash (likely a slightly different R in the paper): 1.2e-4 absolute
    # (the literal A_i of Eq. (cubiccoeff) would move x1 by ~0.3)
    assert abs(fr.x[0] - row["x1"]) < 1.2e-4
    assert abs(fr.y[0] - row["y1"]) < 1.2e-4
    # cell-volume densities (lb/ft^3), printed to 3 decimals.  The printed densities
    # differ by up to ~4e-4 relative from p/(Z R T) x_i M_i evaluated with the table's
    # own Z and x (a slightly different R or M_i in the paper), hence half a unit of
    # the last digit + 5e-4 relative.
    got = [fr.rbar_l[0], fr.rbar_l[1], fr.rbar_v[0], fr.rbar_v[1]]
    want = [row["r1l"], row["r2l"], row["r1v"], row["r2v"]]
    for g_, w_ in zip(got, want):
        assert abs(g_ - w_) <= 5e-4 + 5e-4 * abs(w_)
    assert abs(fr.gamma[0] - row["gamma1"]) < 5e-5
    assert fr.gamma[1] == 1.0
    # iso-fugacity, Eq. (error), and material balance z = V y + (1 - V) x
    assert fr.residual < 1e-20
    assert np.allclose(fr.V * fr.y + (1 - fr.V) * fr.x, [0.4, 0.6], atol=1e-13)
    # gamma by the second form of Eq. (gamma): ln(rho~l/rho~v) and K
    L = math.log(fr.rho_l / fr.rho_v)
    g2 = (L - math.log(fr.K[0])) / (L - math.log(fr.K[1]))
    assert abs(g2 - fr.gamma[0]) < 1e-13


def test_table2_bubble_and_dew_rows():
    mix = c3_nc5()
    rows = {r["p"]: r for r in table2()}
    pb = th.bubble_pressure(mix, 666.06, [0.4, 0.6])
    pd = th.dew_pressure(mix, 666.06, [0.4, 0.6])
    assert abs(pb - 246.0) < 0.5          # printed rounded to 246.0
    assert abs(pd - 127.9) < 0.1
    Zl, _ = th.phase_state(mix, 666.06, 246.0, [0.4, 0.6])
    Zv, _ = th.phase_state(mix, 666.06, 127.9, [0.4, 0.6])
    assert abs(Zl / rows[246.0]["Zl"] - 1) < 2e-4
    assert abs(Zv / rows[127.9]["Zv"] - 1) < 2e-4
    rho_l = 246.0 / (Zl * R_FIELD * 666.06)
    assert abs(rho_l * 0.4 * 44.097 - rows[246.0]["r1l"]) < 5e-4 + 5e-4 * rows[246.0]["r1l"]
    rho_v = 127.9 / (Zv * R_FIELD * 666.06)
    assert abs(rho_v * 0.6 * 72.15 - rows[127.9]["r2v"]) < 5e-4 + 5e-4 * rows[127.9]["r2v"]


def random_states(mix, T, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        c = rng.dirichlet(np.ones(mix.nc))
        rho_t = rng.uniform(0.02, 0.9) / float(c @ mix.b)
        n = c * rho_t
        out.append(n)
    return out


def test_eos_z_solves_corrected_cubic_and_not_printed_one():
    mix = c3_nc5()
    T = 666.06
    worst_fixed, best_printed = 0.0, np.inf
    for n in random_states(mix, T, 40, 1):
        p = float(th.pressure_molar(n, T, mix))
        if p <= 0:
            continue
        c = n / n.sum()
        Z = p / (n.sum() * mix.R * T)
        A, B, _, _ = th.cubic_AB(mix, T, p, c)
        co = th.cubic_coefficients(A, B)
        res = ((Z + co[1]) * Z + co[2]) * Z + co[3]
        scale = abs(Z) ** 3 + abs(co[1] * Z * Z) + abs(co[2] * Z) + abs(co[3])
        worst_fixed = max(worst_fixed, abs(res) / scale)
        printed = Z ** 3 + (B - 1) * Z ** 2 + (A - 2 * B * B - 2 * B) * Z - (A * B - B * B - B)
        best_printed = min(best_printed, abs(printed) / scale)
    assert worst_fixed < 1e-14
    assert best_printed > 1e-6     # the coefficients as printed are not the EOS


def test_gibbs_difference_identity():
    mix = c3_nc5()
    T = 666.06
    hits = 0
    for p in [100.0, 150.0, 200.0, 250.0]:
        for c1 in [0.2, 0.4, 0.6]:
            c = np.array([c1, 1 - c1])
            A, B, Aij, Bi = th.cubic_AB(mix, T, p, c)
            r = th.cubic_roots(A, B)
            if len(r) < 3:
                continue
            hits += 1
            dG = th.gibbs_difference(r[-1], r[0], A, B)
            lmax = th.ln_phi(r[-1], A, B, Aij, Bi, c)
            lmin = th.ln_phi(r[0], A, B, Aij, Bi, c)
            assert abs(dG - float(c @ (lmax - lmin))) < 1e-13
    assert hits >= 3


def residual_helmholtz(n, T, mix):
    """A_res / RT at unit volume by quadrature of the EOS pressure:
    A_res = int_V^inf (p - n R T / V') dV' = int_0^1 (p(n s) - R T s sum n) / s^2 ds."""
    ntot = float(np.sum(n))

    def integrand(s):
        if s == 0.0:
            return 0.0
        return (float(th.pressure_molar(np.asarray(n) * s, T, mix)) - mix.R * T * s * ntot) / (s * s)

    val, _ = quad(integrand, 0.0, 1.0, epsabs=1e-15, epsrel=1e-14, limit=200)
    return val / (mix.R * T)


def test_ln_phi_is_derivative_of_residual_helmholtz():
    mix = c3_nc5()
    mix.k = np.array([[0.0, 0.03], [0.03, 0.0]])   # exercise the interaction term
    T = 666.06
    for n in random_states(mix, T, 4, 2):
        s = th.state_from_molar(mix, T, n)
        for i in range(mix.nc):
            h = 1e-4 * n[i]
            up = n.copy(); up[i] += h
            dn = n.copy(); dn[i] -= h
            d = (residual_helmholtz(up, T, mix) - residual_helmholtz(dn, T, mix)) / (2 * h)
            lnphi_fd = d - math.log(s["Z"])
            assert abs(lnphi_fd - s["lnphi"][i]) < 2e-7, (i, lnphi_fd, s["lnphi"][i])


def test_rachford_rice_binary_closed_form():
    rng = np.random.default_rng(3)
    for _ in range(20):
        z1 = rng.uniform(0.1, 0.9)
        K1 = rng.uniform(1.2, 5.0)
        K2 = rng.uniform(0.05, 0.9)
        z = np.array([z1, 1 - z1])
        V = th.rachford_rice(z, [K1, K2])
        closed = -(z1 * (K1 - 1) + (1 - z1) * (K2 - 1)) / ((K1 - 1) * (K2 - 1))
        assert abs(V - closed) < 1e-13
        assert 1 / (1 - K1) < V < 1 / (1 - K2)


def test_three_component_flash_iso_fugacity():
    t1 = table1()
    names = ["C1", "C3", "nC5"]
    mix = th.mixture_from_critical([t1[n]["pc"] for n in names], [t1[n]["Tc"] for n in names],
                                   [t1[n]["omega"] for n in names], [t1[n]["M"] for n in names], R=R_FIELD)
    fr = th.flash(mix, 600.0, 500.0, [0.3, 0.3, 0.4])
    assert fr.residual < 1e-20
    assert 0 < fr.V < 1
    assert np.allclose(fr.V * fr.y + (1 - fr.V) * fr.x, [0.3, 0.3, 0.4], atol=1e-13)
    # least volatile component (heaviest) has gamma 1, the others less
    assert fr.gamma[2] == 1.0 and np.all(fr.gamma[:2] < 1.0) and np.all(fr.gamma > 0)
    # independent fugacity evaluation of both phases through the density route
    sl = th.state_from_molar(mix, 600.0, fr.rho_l * fr.x)
    sv = th.state_from_molar(mix, 600.0, fr.rho_v * fr.y)
    assert abs(sl["p"] / 500.0 - 1) < 1e-12 and abs(sv["p"] / 500.0 - 1) < 1e-12
    assert np.allclose(sl["fug"], sv["fug"], rtol=1e-11)


def test_single_phase_flash_rejected():
    mix = c3_nc5()
    with pytest.raises(th.SinglePhase):
        th.flash(mix, 666.06, 400.0, [0.4, 0.6])
