"""Flat-interface validation of Sec. 4.2 on the GPU: 40 % propane / 60 % n-pentane
at T = Tc(C3), 400 x 2 periodic box, BGK + Guo forcing, beta = 1.945, tau = 0.8,
nominal pressures 200 and 240 psia.  The bulk compositions and phase densities at
steady state must agree with the flash (Table 2) within the errors the paper
reports for this model (4.0 % in composition, 2.1 % in phase density), the two
bulk phases must sit at one pressure, and the light component must be enriched in
the vapour."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_flat_interface_matches_flash():
    from paper_1909_12390_amd import validation as V
    print("case flat interface 400x2, 200 and 240 psia, Guo, beta 1.945", flush=True)
    cases = [V.flat_case(p, nx=400) for p in (200.0, 240.0)]
    reps = V.run_flat(cases, collision="bgk", forcing="guo", max_steps=1_600_000, check_every=100_000, tol=1e-10)
    for r in reps:
        print(f"  p={r['p_psia']}: composition err {r['err_composition']:.4f}, density err {r['err_density']:.4f}, "
              f"steps {r['steps']}", flush=True)
        assert r["err_composition"] < 0.040
        assert r["err_density"] < 0.021
        assert abs(r["p_l"] - r["p_v"]) < 1e-6 * r["p_l"]
        assert r["y"][0] > r["x"][0]
        assert r["p_lb_psia"] == pytest.approx(r["p_psia"], rel=0.02)


def test_flat_interface_with_exact_difference_forcing():
    """The same flat interface with the exact-difference forcing (reading R8 of the
    velocities) at its calibrated beta = 1.3 (the paper calibrates beta for Guo only
    and notes that it depends on the forcing, Sec. 4.2): 160 and 240 psia, the ends
    of the calibrated range, within the same bars as Guo, and the iso-fugacity
    residual of Eq. (error) at the LB bulk states below 1e-3."""
    from paper_1909_12390_amd import validation as V
    print("case flat interface 400x2, 160 and 240 psia, EDM, beta 1.3", flush=True)
    cases = [V.flat_case(p, nx=400, beta=1.3) for p in (160.0, 240.0)]
    reps = V.run_flat(cases, collision="bgk", forcing="edm", max_steps=3_000_000, check_every=100_000, tol=1e-9)
    for r in reps:
        print(f"  p={r['p_psia']}: composition err {r['err_composition']:.4f}, density err {r['err_density']:.4f}, "
              f"residual {r['residual_eq_error']:.1e}, steps {r['steps']}", flush=True)
        assert r["err_composition"] < 0.040
        assert r["err_density"] < 0.021
        assert r["residual_eq_error"] < 1e-3
        assert r["y"][0] > r["x"][0]


def test_laplace_law_on_drops():
    """Sec. 4.3: drops of initial radius n/5 in n x n boxes (n = 50, 100, 200),
    200 psia, Guo forcing, beta = 1.915: dp = p_l - p_v is linear in 1/R and its
    slope is the paper's surface tension 0.1289 (lattice units) within 10 %."""
    from paper_1909_12390_amd import validation as V
    print("case Laplace drops 50/100/200, 200 psia", flush=True)
    out = V.run_laplace(p_list=(200.0,), sizes=(50, 100, 200), beta=1.915, max_steps=400_000,
                        check_every=50_000, tol=1e-6)
    r = out["pressures"]["200.0"]
    print(f"  sigma {r['sigma']:.4f} (paper 0.1289), r2 {r['r2']:.5f}, steps {out['steps']}", flush=True)
    assert r["r2"] > 0.999
    assert r["sigma"] == pytest.approx(0.1289, rel=0.10)
    for d in r["drops"]:
        assert d["dp"] > 0.0 and d["y"][0] > d["x"][0]


def test_oscillating_drop_period():
    """Sec. 4.3 / Table 3: elliptical drop (h = 0.9, R0 = 0.15 n) at 580 degR and
    70 psia (density ratio ~58), Guo forcing, beta = 1.815, n = 200.  The period
    of the axis oscillation must agree with the model period of Table 3 (2407)
    within 6 % and with Lamb's period (2129) within 10 %."""
    import os
    from paper_1909_12390_amd import validation as V
    rows = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "table3_periods.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                n, th, mo = line.split()
                rows[int(n)] = (float(th), float(mo))
    print("case oscillating drop n=200", flush=True)
    out = V.run_oscillation(sizes=(200,), steps=7500, sample_every=25)
    period = out["drops"][0]["period"]
    theory, model = rows[200]
    print(f"  period {period:.0f} (paper model {model:.0f}, theory {theory:.0f})", flush=True)
    assert period == pytest.approx(model, rel=0.06)
    assert period == pytest.approx(theory, rel=0.10)


def test_laplace_3d_spheres():
    """D3Q19 spheres (initial radius n/5 in n^3, n = 60 and 80, 200 psia, BGK + Guo,
    beta = 1.915): both survive, Laplace's law per sphere (sigma_n = dp R / 2) rises
    with the radius as in two dimensions, and at R ~ 14 lies within 5 % of the
    paper's two-dimensional 0.1289 (Sec. 4.3; flat-interface tension does not depend
    on the lattice dimension)."""
    from paper_1909_12390_amd import validation
    print("case laplace 3d n = 60, 80, 60000 steps", flush=True)
    out = validation.run_laplace3d((200.0,), sizes=(60, 80), max_steps=60000, check_every=20000, tol=0.0)
    d = out["pressures"]["200.0"]
    assert d["dissolved"] == []
    s = [m["sigma_n"] for m in d["drops"]]
    print("  sigma_n", s, "R", [m["R"] for m in d["drops"]], flush=True)
    assert s[1] > s[0]
    assert abs(s[1] - 0.1289) < 0.05 * 0.1289
