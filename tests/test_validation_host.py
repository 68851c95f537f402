"""Host side of the flat-interface validation (Sec. 4.2): lattice-unit scaling,
slab position and initial profile (no device call)."""
import numpy as np
import pytest

from golden_io import table1, table2
from paper_1909_12390_amd import lbm, validation


def test_table1_copy_matches_fixture():
    t = table1()
    for name, (pc, Tc, om, M) in validation.TABLE1.items():
        assert (pc, Tc, om, M) == (t[name]["pc"], t[name]["Tc"], t[name]["omega"], t[name]["M"])


def test_lattice_units_fix_component_one():
    u = validation.LatticeUnits(validation.field_mixture())
    m = u.mixture()
    assert m["a"][0] == pytest.approx(2.0 / 49.0, rel=1e-15)
    assert m["b"][0] == pytest.approx(2.0 / 21.0, rel=1e-15)
    assert m["M"][0] == 1.0 and m["R"] == 1.0
    # ratios to component 1 are unit-free
    f = validation.field_mixture()
    assert m["a"][1] / m["a"][0] == pytest.approx(f["a"][1] / f["a"][0], rel=1e-14)
    assert m["b"][1] / m["b"][0] == pytest.approx(f["b"][1] / f["b"][0], rel=1e-14)


def test_lattice_flash_reproduces_table2():
    """The rescaled mixture flashed in lattice units at the rescaled pressures gives
    Table 2's compositions, gamma_1 and (rescaled) densities."""
    case = validation.flat_case(240.0, nx=64)
    u, mix, T = case["units"], case["mix"], case["T"]
    for r in table2():
        if not np.isfinite(r["gamma1"]):
            continue
        fl = lbm.lbm_flash(mix, T, u.p(r["p"]), np.array([0.4, 0.6]))
        assert fl.x[0] == pytest.approx(r["x1"], abs=2e-4)
        assert fl.y[0] == pytest.approx(r["y1"], abs=2e-4)
        assert fl.gamma[0] == pytest.approx(r["gamma1"], abs=5e-5)
        printed = np.array([r["r1l"], r["r2l"], r["r1v"], r["r2v"]])
        ours = np.array([fl.rbar_l[0], fl.rbar_l[1], fl.rbar_v[0], fl.rbar_v[1]])
        assert np.allclose(ours, u.mass_density(printed), rtol=1.5e-3)


def test_slab_start_gives_overall_composition_for_sharp_profile():
    l, v = np.array([1.398, 5.3997]), np.array([0.2159, 0.1948])
    M = np.array([1.0, 1.636])
    z1, L = 0.4, 1600.0
    L0 = validation.slab_start(l, v, z1, M[0] / M[1], L)
    N = ((L - 2 * L0) * l + 2 * L0 * v) / M
    assert N[0] / N.sum() == pytest.approx(z1, abs=1e-12)
    assert 0.0 < L0 < L / 2


def test_flat_profile_limits_and_symmetry():
    l, v = np.array([2.0, 5.0]), np.array([0.3, 0.2])
    prof = validation.flat_profile(400, 2, 120.0, 8.0, l, v)
    assert prof.shape == (2, 2, 400)
    assert np.allclose(prof[:, :, 200], l[:, None], atol=1e-12)
    assert np.allclose(prof[:, :, 0], v[:, None], atol=1e-12)
    assert np.allclose(prof[:, 0, 1:], prof[:, 0, 1:][:, ::-1], atol=1e-12)


def test_convergence_recovers_a_known_order():
    """v_n = 1 + 0.3 n^-p against a reference size far enough out that its own
    error is below rounding: errors 0.3 n^-p, observed order p between sizes."""
    for p in (1.0, 2.0):
        vals = {n: 1.0 + 0.3 * n ** -p for n in (50, 100, 200, 400)}
        vals[10 ** 9] = 1.0 + 0.3 * (10.0 ** 9) ** -p
        rows = validation.convergence(vals)
        for r in rows[:3]:
            assert r["error"] == pytest.approx(0.3 * r["n"] ** -p / (1.0 + 0.3e-9 ** p), rel=1e-6)
            assert r["order"] == pytest.approx(p, rel=1e-6)
        assert rows[-1]["order"] is None


def test_flat_and_sigma_convergence_group_by_pressure():
    reps = [{"p_psia": p, "nx": n, "rho_l": 5.0 + 1.0 / n + p, "rho_v": 0.5 + 2.0 / n} for p in (200.0, 240.0)
            for n in (100, 200, 400)]
    out = validation.flat_convergence(reps)
    assert set(out) == {"200.0", "240.0"} and out["200.0"]["reference_nx"] == 400
    e = out["240.0"]["rho_v"][0]["error"]
    assert e == pytest.approx((2.0 / 100 - 2.0 / 400) / (0.5 + 2.0 / 400), rel=1e-12)
    lap = {"pressures": {"200.0": {"drops": [{"n": n, "dp": 0.13 / (n / 5) * (1 + 1 / n), "R": n / 5}
                                             for n in (50, 100, 200)]}}}
    s = validation.sigma_convergence(lap)["200.0"]
    assert s["sigma"]["100"] == pytest.approx(0.13 * 1.01, rel=1e-12)
    assert s["convergence"][0]["error"] == pytest.approx((0.13 * 1.02 - 0.13 * 1.005) / (0.13 * 1.005), rel=1e-12)


def test_stretch_flat_keeps_interfaces_bulk_and_masses():
    """A tanh slab of a 400-cell box stretched to 800 cells is the tanh slab of the
    800-cell box with the same width (interfaces at the scaled positions), and the
    optional rescale hits the requested component totals."""
    l, v = np.array([4.0, 2.5]), np.array([0.6, 0.2])
    small = validation.flat_profile(400, 2, 120.0, 8.0, l, v)
    big = validation.flat_profile(800, 2, 240.0, 8.0, l, v)
    st = validation.stretch_flat(small, 800)
    assert st.shape == big.shape
    # the kept band (24 cells) ends where the tanh tail is 1 - tanh(6) ~ 1e-5 from the bulk
    assert np.max(np.abs(st - big)) < 1e-5 * l.max()
    mass = big.reshape(2, -1).sum(axis=1) * np.array([1.001, 0.999])
    st2 = validation.stretch_flat(small, 800, mass=mass)
    assert np.allclose(st2.reshape(2, -1).sum(axis=1), mass, rtol=1e-13, atol=0)


@pytest.mark.parametrize("theta", [45.0, 90.0, 120.0, 150.0])
def test_contact_angle_of_a_circular_cap(theta):
    """A tanh-profiled circular cap meeting the wall y = 2.5 at a known angle: the
    measured angle (circle through the top and the crossings 3 cells above the
    wall) recovers it within 1.5 degrees."""
    ny, nx, yw, R = 90, 200, 2.5, 30.0
    yc = yw - R * np.cos(np.radians(theta))
    y, x = np.meshgrid(np.arange(ny, dtype=float), np.arange(nx, dtype=float), indexing="ij")
    r = np.sqrt((x - nx // 2) ** 2 + (y - yc) ** 2)
    rho = 3.2 - 2.6 * np.tanh(2.0 * (r - R) / 4.0)
    rho[:3] = 0.6
    m = validation.contact_angle(rho, yw)
    assert abs(m["theta_deg"] - theta) < 1.5, m
    assert abs(m["R"] - R) < 1.0


def test_sphere_measurement_recovers_radius_and_dissolution():
    """A tanh sphere of radius 17.3 in a 64^3 box: the six-ray level crossing gives
    the radius; centre and corner hold the flash's coexisting phases, so their
    pressures agree (the Laplace jump appears only once the drop equilibrates); a
    uniform vapour box reads as dissolved."""
    n, R = 64, 17.3
    g = np.meshgrid(*[np.arange(n, dtype=float)] * 3, indexing="ij")
    r = np.sqrt(sum((x - n // 2) ** 2 for x in g))
    prof = 0.5 * (1 - np.tanh(2.0 * (r - R) / 4.0))
    c = validation.drop3d_case(200.0, 8)
    l, v = np.asarray(c["flash"].rbar_l), np.asarray(c["flash"].rbar_v)
    rho = v[:, None, None, None] + (l - v)[:, None, None, None] * prof[None]
    m = validation.drop3d_measure(rho, c["mix"], c["T"])
    assert abs(m["R"] - R) < 0.05
    assert abs(m["dp"]) < 1e-5 * m["p_l"]
    assert validation.drop3d_measure(np.broadcast_to(v[:, None, None, None], rho.shape), c["mix"], c["T"]) is None
