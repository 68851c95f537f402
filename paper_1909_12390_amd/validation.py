"""Flat-interface validation of the model on the GPU (Sec. 4.2) and calibration of
the force-blending parameter beta of Eq. (coupledMCforce).

Case of Sec. 4.2: propane (component 1) and n-pentane (component 2) with the
Table 1 properties, overall composition z1 = 0.4, T = Tc of propane, a periodic
nx x 2 box holding a liquid slab between two vapour regions, initialised with
Eq. (initialdensity) and the slab position L0 of Eq. (initialdensity2) from the
flashed phase densities (Table 2), tau = 0.8.  Lattice units follow Sec. 4.2:
the physical EOS parameters are rescaled so that a_1 = 2/49, b_1 = 2/21, M_1 = 1
and R = 1, the others keeping their ratios to component 1.

Several pressures (or several beta values) are advanced together as the boxes of
one batch (lbm_batch_*), each box with its own phase densities, gamma and beta.
At steady state the bulk values are read at the centre of the liquid slab and at
the box edge (the centre of the vapour region); they are compared with the flash
at the nominal pressure (what the paper's comparison reports: 4.0 % in
composition and 2.1 % in phase density over 240-140 psia with Guo forcing and
beta = 1.945), and their own iso-fugacity residual at the LB pressure is given.

Everything here is orchestration: the steps run in the HIP library; the flash,
pressures and fugacities come from the library's host thermodynamics.
"""
from __future__ import annotations

import math

import numpy as np

from . import lbm

# Table 1 (Sec. 4.2; from Danesh): critical pressure [psia], critical temperature
# [degR], acentric factor, molar mass [lbm/lbmol]
TABLE1 = {
    "C3": (616.00, 666.06, 0.1522, 44.097),
    "nC5": (488.60, 845.80, 0.2514, 72.150),
}
R_FIELD = 10.7316          # psia ft^3 / (lbmol degR)
OMEGA_A, OMEGA_B = 0.45724, 0.0778


def field_mixture(names=("C3", "nC5")) -> dict:
    """Peng-Robinson parameters per mole in field units (Sec. 3.2 definitions)."""
    pc = np.array([TABLE1[n][0] for n in names])
    Tc = np.array([TABLE1[n][1] for n in names])
    om = np.array([TABLE1[n][2] for n in names])
    M = np.array([TABLE1[n][3] for n in names])
    a = OMEGA_A * R_FIELD ** 2 * Tc ** 2 / pc
    b = OMEGA_B * R_FIELD * Tc / pc
    nc = len(names)
    return {"a": a, "b": b, "omega": om, "M": M, "k": np.zeros((nc, nc)), "R": R_FIELD}


class LatticeUnits:
    """Scales between field units and the lattice units of Sec. 4.2 (a_1 = 2/49,
    b_1 = 2/21, M_1 = 1, R = 1): molar density n_lb = n / sn, pressure
    p_lb = p / sp, temperature T_lb = T / sT, molar mass M_lb = M / M_1."""

    def __init__(self, fmix: dict):
        a1, b1 = float(fmix["a"][0]), float(fmix["b"][0])
        self.sn = (2.0 / 21.0) / b1                 # b_lb = b sn
        self.sp = a1 * self.sn ** 2 / (2.0 / 49.0)  # a_lb = a sn^2 / sp
        self.sT = self.sp / (fmix["R"] * self.sn)   # R_lb = R sT sn / sp = 1
        self.M1 = float(fmix["M"][0])
        self.fmix = fmix

    def mixture(self) -> dict:
        f = self.fmix
        return {"a": f["a"] * self.sn ** 2 / self.sp, "b": f["b"] * self.sn, "omega": f["omega"].copy(),
                "M": f["M"] / self.M1, "k": f["k"].copy(), "R": 1.0}

    def T(self, T_field):
        return T_field / self.sT

    def p(self, p_field):
        return p_field / self.sp

    def mass_density(self, rho_field):
        """lbm/ft^3 -> lattice mass density (n M with the scaled n and M)."""
        return rho_field / (self.sn * self.M1)


def slab_start(rbar_l, rbar_v, z1, theta, L):
    """L0 of Eq. (initialdensity2): the vapour width at each end of the box that
    gives the overall mole fraction z1 for a sharp profile (theta = M1 / M2)."""
    l1, l2 = rbar_l
    v1, v2 = rbar_v
    num = (l1 * z1 + theta * l2 * z1 - l1) * L
    den = 2.0 * (v1 - l1 - v1 * z1 - theta * v2 * z1 + l1 * z1 + theta * l2 * z1)
    return num / den


def flat_profile(nx, ny, L0, D, rbar_l, rbar_v):
    """Eq. (initialdensity): vapour at both ends, liquid in the middle, along x;
    array (nc, ny, nx)."""
    x = np.arange(nx, dtype=np.float64)
    L = float(nx)
    l = np.asarray(rbar_l, dtype=np.float64)[:, None]
    v = np.asarray(rbar_v, dtype=np.float64)[:, None]
    left = 0.5 * (l + v) + 0.5 * (l - v) * np.tanh(2.0 * (x - L0) / D)
    right = 0.5 * (l + v) - 0.5 * (l - v) * np.tanh(2.0 * (x - L + L0) / D)
    prof = np.where(x[None, :] <= L / 2.0, left, right)
    return np.repeat(prof[:, None, :], ny, axis=1)


def flat_case(p_psia, nx=1600, ny=2, D=8.0, z1=0.4, beta=1.945, tau=0.8, T_over_Tc1=1.0, names=("C3", "nC5")):
    """One box of the flat-interface case at nominal pressure p_psia."""
    fmix = field_mixture(names)
    u = LatticeUnits(fmix)
    mix = u.mixture()
    T = u.T(T_over_Tc1 * TABLE1[names[0]][1])
    z = np.array([z1, 1.0 - z1])
    fl = lbm.lbm_flash(mix, T, u.p(p_psia), z)
    theta = mix["M"][0] / mix["M"][1]
    L0 = slab_start(fl.rbar_l, fl.rbar_v, z1, theta, float(nx))
    rho0 = flat_profile(nx, ny, L0, D, fl.rbar_l, fl.rbar_v)
    return {"mix": mix, "shape": (ny, nx), "T": T, "tau": tau, "beta": beta, "gamma": np.asarray(fl.gamma),
            "rho0": rho0, "p_lb": u.p(p_psia), "p_psia": p_psia, "z": z, "flash": fl, "units": u, "L0": L0}


def bulk_state(rho_s, mix):
    """Bulk rbar at the centre of the liquid slab and of the vapour, each averaged
    over y; returns (rbar_l, rbar_v).  The slab starts centred (liquid at x = nx/2,
    vapour at x = 0) but may drift along the periodic x axis, so the liquid centre is
    taken as the middle of the cells whose total density lies above the mean of its
    extremes (x = nx/2 while the slab stays put) and the vapour centre half a box
    away."""
    r = np.asarray(rho_s)
    nx = r.shape[-1]
    tot = r.sum(axis=0).mean(axis=0)
    dense = tot > 0.5 * (tot.max() + tot.min())
    # circular mean of the dense cells' positions
    ang = 2.0 * np.pi * np.arange(nx) / nx
    c = np.arctan2(np.sin(ang[dense]).sum(), np.cos(ang[dense]).sum())
    xl = int(round(c / (2.0 * np.pi) * nx)) % nx
    xv = (xl + nx // 2) % nx
    return r[:, :, xl].mean(axis=1), r[:, :, xv].mean(axis=1)


def phase_report(mix, T, rbar_l, rbar_v, flash):
    """Compositions, densities, pressures and iso-fugacity residual of the LB bulk
    phases, and their relative errors against the flash."""
    M = np.asarray(mix["M"], dtype=np.float64)
    nl, nv = rbar_l / M, rbar_v / M
    x, y = nl / nl.sum(), nv / nv.sum()
    fug = lbm.lbm_fugacity(mix, T, np.stack([nl, nv]))
    p_l, p_v = float(fug["p"][0]), float(fug["p"][1])
    fl, fv = fug["fug"][0], fug["fug"][1]
    res = float(np.max(np.abs(fl - fv) / np.abs(fv)))
    res_sq = float(np.sum((fl / fv - 1.0) ** 2))          # Eq. (error)
    rho_l, rho_v = float(rbar_l.sum()), float(rbar_v.sum())
    frho_l, frho_v = float(flash.rbar_l.sum()), float(flash.rbar_v.sum())
    out = {"x": x.tolist(), "y": y.tolist(), "rho_l": rho_l, "rho_v": rho_v, "p_l": p_l, "p_v": p_v,
           "fugacity_residual": res, "residual_eq_error": res_sq,
           "err_x": float(np.max(np.abs(x - flash.x) / flash.x)),
           "err_y": float(np.max(np.abs(y - flash.y) / flash.y)),
           "err_rho_l": abs(rho_l - frho_l) / frho_l, "err_rho_v": abs(rho_v - frho_v) / frho_v}
    out["err_composition"] = max(out["err_x"], out["err_y"])
    out["err_density"] = max(out["err_rho_l"], out["err_rho_v"])
    return out


def overall_composition(rho_s, M):
    """Mole fractions of the whole box (conserved by the step)."""
    n = np.asarray(rho_s).reshape(len(M), -1).sum(axis=1) / np.asarray(M, dtype=np.float64)
    return n / n.sum()


def reflash_gamma(case, rho_s):
    """State-dependent gamma: flash at the box's LB bulk pressure (p_EOS of the bulk
    liquid and vapour, averaged) and its overall composition; returns the new
    gamma and the pressure, or (None, p) if the flash finds one phase or a gamma
    outside (0, 1]."""
    mix, T = case["mix"], case["T"]
    rl, rv = bulk_state(rho_s, mix)
    M = np.asarray(mix["M"], dtype=np.float64)
    p = lbm.lbm_pressure(mix, T, np.stack([rl / M, rv / M]))
    p_lb = 0.5 * float(p[0] + p[1])
    try:
        fl = lbm.lbm_flash(mix, T, p_lb, overall_composition(rho_s, M))
    except lbm.LbmError:
        return None, p_lb
    g = np.asarray(fl.gamma)
    if not np.all((g > 0.0) & (g <= 1.0)):     # outside the model's range: keep the old gamma
        return None, p_lb
    return g, p_lb


def run_flat(cases, collision="bgk", forcing="guo", storage="f64", max_steps=2_000_000, check_every=20_000,
             tol=1e-9, graph_steps=1000, progress=None, gamma_update=False, fields_out=None):
    """Advance the boxes together until the bulk densities of every box change by
    less than tol (relative) over check_every steps.  Returns the reports;
    progress(steps, change) is called after every check.  With gamma_update, every
    check re-flashes each box at its current bulk pressure and overall composition
    and replaces its gamma (state-dependent gamma, Sec. 3.1).  A list passed as
    fields_out receives the final per-component density fields of the boxes."""
    boxes = [{"mix": c["mix"], "shape": c["shape"], "T": c["T"], "tau": c["tau"], "beta": c["beta"],
              "gamma": c["gamma"], "rho0": c["rho0"]} for c in cases]
    rates = None
    if collision == "mrt":
        from .inputs import default_mrt_rates
        rates = default_mrt_rates("D2Q9", cases[0]["tau"])
    b = lbm.LbmBatch(boxes, "D2Q9", collision=collision, forcing=forcing, storage=storage,
                     graph_steps=min(graph_steps, check_every), mrt_s=rates)
    prev = None
    steps = 0
    change = float("inf")
    try:
        while steps < max_steps:
            b.step(check_every)
            steps += check_every
            bad = b.box_errors()
            if bad.any():
                raise lbm.LbmError(lbm.LBM_ERR_DOMAIN, f"boxes {np.nonzero(bad)[0].tolist()} left the EOS domain")
            rho = [r.cpu().numpy() for r in b.fields()]
            bulk = [np.concatenate(bulk_state(r, c["mix"])) for r, c in zip(rho, cases)]
            if gamma_update:
                for k, (r, c) in enumerate(zip(rho, cases)):
                    g, _ = reflash_gamma(c, r)
                    if g is not None:
                        b.set_gamma(k, g)
                        c["gamma"] = g
            if prev is not None:
                change = max(float(np.max(np.abs(u - v) / np.abs(v))) for u, v in zip(bulk, prev))
            if progress is not None:
                progress(steps, change)
            if change < tol:
                break
            prev = bulk
        b.check()
    finally:
        b.close()
    reports = []
    for r, c in zip(rho, cases):
        rl, rv = bulk_state(r, c["mix"])
        try:
            rep = phase_report(c["mix"], c["T"], rl, rv, c["flash"])
        except lbm.LbmError as e:      # no two bulk phases left in this box (e.g. the slab evaporated)
            reports.append({"p_psia": c["p_psia"], "nx": int(c["shape"][1]), "beta": c["beta"], "steps": steps,
                            "error": str(e), "err_composition": float("inf"), "err_density": float("inf"),
                            "rbar_l": rl.tolist(), "rbar_v": rv.tolist()})
            continue
        rep.update({"p_psia": c["p_psia"], "nx": int(c["shape"][1]), "beta": c["beta"], "steps": steps,
                    "last_change": change,
                    "p_lb_psia": 0.5 * (rep["p_l"] + rep["p_v"]) * c["units"].sp,
                    "gamma": np.asarray(c["gamma"]).tolist()})
        # the same bulk states against the flash at the LB pressure and overall composition
        try:
            fl_lb = lbm.lbm_flash(c["mix"], c["T"], 0.5 * (rep["p_l"] + rep["p_v"]),
                                  overall_composition(r, c["mix"]["M"]))
            lb = phase_report(c["mix"], c["T"], rl, rv, fl_lb)
            rep["err_composition_at_lb_pressure"] = lb["err_composition"]
            rep["err_density_at_lb_pressure"] = lb["err_density"]
        except lbm.LbmError:          # the LB pressure lies outside the two-phase range of z
            rep["err_composition_at_lb_pressure"] = float("inf")
            rep["err_density_at_lb_pressure"] = float("inf")
        reports.append(rep)
    if fields_out is not None:
        fields_out.extend(rho)
    return reports


def calibrate_beta(p_list=(200.0, 240.0), forcing="edm", collision="bgk", betas=None, nx=400, **run_kw):
    """Sweep beta on the flat case (one box per (beta, pressure)); returns the
    sweep and the beta with the smallest worst-case composition error.  A finer
    search repeats the sweep on a narrower grid around the best value."""
    if betas is None:
        betas = np.linspace(1.0, 2.0, 11)
    cases = [flat_case(p, nx=nx, beta=float(bt)) for bt in betas for p in p_list]
    reps = run_flat(cases, collision=collision, forcing=forcing, **run_kw)
    table = {}
    for rep in reps:
        table.setdefault(rep["beta"], []).append(rep)
    score = {bt: max(r["err_composition"] for r in rs) for bt, rs in table.items()}
    best = min(score, key=score.get)
    return {"sweep": [{"beta": bt, "worst_composition_err": score[bt],
                       "worst_density_err": max(r["err_density"] for r in table[bt])} for bt in sorted(table)],
            "best_beta": best, "best_err": score[best], "reports": reps}


# ---------------------------------------------------------------------------
# Grid convergence (Sec. 4.2: phase densities of the flat interface against the
# finest box; Sec. 4.3: surface tension against the largest drop)
# ---------------------------------------------------------------------------

def convergence(values: dict) -> list:
    """values: {n: v}.  Relative error of each v against the value at the largest n,
    |v_n - v_max| / |v_max|, and the observed order between consecutive sizes,
    log(e_a / e_b) / log(n_b / n_a) (None where the next error is the last one or zero)."""
    ns = sorted(values)
    ref = values[ns[-1]]
    errs = [abs(values[n] - ref) / abs(ref) for n in ns[:-1]]
    rows = []
    for i, n in enumerate(ns[:-1]):
        order = None
        if i + 1 < len(errs) and errs[i] > 0.0 and errs[i + 1] > 0.0:
            order = math.log(errs[i] / errs[i + 1]) / math.log(ns[i + 1] / n)
        rows.append({"n": n, "error": errs[i], "order": order})
    return rows


def flat_convergence(reports) -> dict:
    """Per pressure, the liquid and vapour mass densities of the flat-interface
    reports (any number of runs; one report per (pressure, nx)) against the
    largest nx."""
    out = {}
    for p in sorted({r["p_psia"] for r in reports}):
        rs = {r["nx"]: r for r in reports if r["p_psia"] == p}
        out[str(p)] = {"reference_nx": max(rs),
                       "rho_l": convergence({n: r["rho_l"] for n, r in rs.items()}),
                       "rho_v": convergence({n: r["rho_v"] for n, r in rs.items()})}
    return out


def sigma_convergence(laplace: dict) -> dict:
    """Per pressure of a run_laplace result, the surface tension of each drop by
    Laplace's law alone, sigma_n = dp_n R_n, against the largest box."""
    out = {}
    for p, d in laplace["pressures"].items():
        sig = {m["n"]: m["dp"] * m["R"] for m in d["drops"]}
        out[p] = {"sigma": {str(n): v for n, v in sorted(sig.items())}, "convergence": convergence(sig)}
    return out


def _level_crossing(prof, level, i0, i1, rising):
    """Fractional index of the first crossing of level in prof[i0:i1]."""
    for i in range(max(i0, 1), i1):
        a, b = prof[i - 1], prof[i]
        if (a < level <= b) if rising else (a >= level > b):
            return i - 1 + (level - a) / (b - a)
    raise ValueError("no interface found")


def stretch_flat(rho_s, nx_new, mass=None, keep=24):
    """A starting state for a larger flat-interface box from a converged smaller
    one (nc, ny, nx): the slab stays centred and its length scales with the box,
    the profiles within `keep` cells of each interface are carried over (linear
    interpolation at the shifted positions), the rest is filled with the bulk
    values of the small box.  With mass (per-component totals) each component is
    rescaled to its total, so the run conserves the same amounts as a box
    initialised directly at nx_new."""
    r = np.asarray(rho_s, dtype=np.float64)
    nc, ny, nx = r.shape
    prof = r.mean(axis=1)
    tot = prof.sum(axis=0)
    c_old = nx // 2
    level = 0.5 * (tot[c_old] + tot[0])
    xl = _level_crossing(tot, level, 1, c_old + 1, rising=True)
    xr = _level_crossing(tot, level, c_old, nx, rising=False)
    s = nx_new / nx
    c_new = nx_new // 2
    xl_new = c_new - (c_old - xl) * s
    xr_new = c_new + (xr - c_old) * s
    liq, vap = prof[:, c_old], prof[:, 0]
    xs = np.arange(nx, dtype=np.float64)
    new = np.empty((nc, nx_new))
    for X in range(nx_new):
        if X < c_new:
            d, x_old, inside = X - xl_new, xl + (X - xl_new), X > xl_new
        else:
            d, x_old, inside = X - xr_new, xr + (X - xr_new), X < xr_new
        if abs(d) <= keep:
            new[:, X] = [np.interp(x_old, xs, prof[i]) for i in range(nc)]
        else:
            new[:, X] = liq if inside else vap
    out = np.repeat(new[:, None, :], ny, axis=1)
    if mass is not None:
        out *= (np.asarray(mass, dtype=np.float64) / out.reshape(nc, -1).sum(axis=1))[:, None, None]
    return out


# ---------------------------------------------------------------------------
# Laplace's law for a drop (Sec. 4.3)
# ---------------------------------------------------------------------------

def drop_case(p_psia, n, beta=1.915, tau=0.8, W=4.0, z1=0.4, names=("C3", "nC5")):
    """A drop of initial radius R0 = n/5 at the centre of an n x n periodic box,
    Eq. (initialdensity_droplet) with the liquid inside (the sign of
    Eq. (initialden)), phase densities from the flash at p_psia."""
    fmix = field_mixture(names)
    u = LatticeUnits(fmix)
    mix = u.mixture()
    T = u.T(TABLE1[names[0]][1])
    fl = lbm.lbm_flash(mix, T, u.p(p_psia), np.array([z1, 1.0 - z1]))
    y, x = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64), indexing="ij")
    r = np.sqrt((x - n / 2.0) ** 2 + (y - n / 2.0) ** 2)
    t = np.tanh(2.0 * (r - n / 5.0) / W)
    l = np.asarray(fl.rbar_l)[:, None, None]
    v = np.asarray(fl.rbar_v)[:, None, None]
    rho0 = 0.5 * (l + v) - 0.5 * (l - v) * t[None]
    return {"mix": mix, "shape": (n, n), "T": T, "tau": tau, "beta": beta, "gamma": np.asarray(fl.gamma),
            "rho0": rho0, "p_psia": p_psia, "flash": fl, "units": u, "n": n}


def drop_measure(rho_s, mix, T):
    """Radius at the level 0.5 (rho_l + rho_v) of the total density along the four
    axis rays from the centre (linear interpolation, averaged), and the pressures
    p_EOS at the centre and at the box corner."""
    r = np.asarray(rho_s)
    rho = r.sum(axis=0)
    n = rho.shape[0]
    c = n // 2
    rl, rv = rho[c, c], rho[0, 0]
    level = 0.5 * (rl + rv)
    radii = []
    for prof in (rho[c, c:], rho[c, c::-1], rho[c:, c], rho[c::-1, c]):
        k = int(np.argmax(prof < level))
        a, b = prof[k - 1], prof[k]
        radii.append(k - 1 + (a - level) / (a - b))
    M = np.asarray(mix["M"], dtype=np.float64)
    n_l, n_v = r[:, c, c] / M, r[:, 0, 0] / M
    p = lbm.lbm_pressure(mix, T, np.stack([n_l, n_v]))
    return {"R": float(np.mean(radii)), "p_l": float(p[0]), "p_v": float(p[1]), "dp": float(p[0] - p[1]),
            "x": (n_l / n_l.sum()).tolist(), "y": (n_v / n_v.sum()).tolist()}


def run_laplace(p_list=(200.0, 240.0), sizes=(50, 100, 200, 400, 800), beta=1.915, forcing="guo",
                collision="bgk", max_steps=400_000, check_every=20_000, tol=1e-8, progress=None):
    """All (pressure, size) drops as one batch to steady state; per pressure the
    surface tension is the least-squares slope of dp against 1/R (with intercept)."""
    cases = [drop_case(p, n, beta=beta) for p in p_list for n in sizes]
    boxes = [{"mix": c["mix"], "shape": c["shape"], "T": c["T"], "tau": c["tau"], "beta": c["beta"],
              "gamma": c["gamma"], "rho0": c["rho0"]} for c in cases]
    b = lbm.LbmBatch(boxes, "D2Q9", collision=collision, forcing=forcing, storage="f64",
                     graph_steps=min(1000, check_every))
    steps, prev, change = 0, None, float("inf")
    try:
        while steps < max_steps:
            b.step(check_every)
            steps += check_every
            bad = b.box_errors()
            if bad.any():
                raise lbm.LbmError(lbm.LBM_ERR_DOMAIN, f"boxes {np.nonzero(bad)[0].tolist()} left the EOS domain")
            meas = [drop_measure(r.cpu().numpy(), c["mix"], c["T"]) for r, c in zip(b.fields(), cases)]
            cur = np.array([[m["R"], m["dp"]] for m in meas])
            if prev is not None:
                change = float(np.max(np.abs(cur - prev) / np.abs(prev)))
            if progress is not None:
                progress(steps, change)
            if change < tol:
                break
            prev = cur
        b.check()
    finally:
        b.close()
    out = {"steps": steps, "last_change": change, "beta": beta, "forcing": forcing, "pressures": {}}
    for p in p_list:
        rows = [(c["n"], m) for c, m in zip(cases, meas) if c["p_psia"] == p]
        invR = np.array([1.0 / m["R"] for _, m in rows])
        dp = np.array([m["dp"] for _, m in rows])
        A = np.stack([invR, np.ones_like(invR)], axis=1)
        (sigma, icpt), *_ = np.linalg.lstsq(A, dp, rcond=None)
        fit = A @ np.array([sigma, icpt])
        r2 = 1.0 - float(np.sum((dp - fit) ** 2) / np.sum((dp - dp.mean()) ** 2)) if len(dp) > 2 else 1.0
        out["pressures"][str(p)] = {"sigma": float(sigma), "intercept": float(icpt), "r2": r2,
                                    "drops": [{"n": n, **m} for n, m in rows]}
    return out


# ---------------------------------------------------------------------------
# Laplace's law in three dimensions (D3Q19): a sphere has dp = 2 sigma / R, and the
# tension of the flat interface does not depend on the lattice dimension, so the
# slope should reproduce the two-dimensional sigma (a cross-check of the 3-D path)
# ---------------------------------------------------------------------------

def drop3d_case(p_psia, n, beta=1.915, tau=0.8, W=4.0, z1=0.4, names=("C3", "nC5")):
    """A sphere of initial radius n/5 at the centre of an n^3 periodic box, the
    radial profile of drop_case, phase densities from the flash at p_psia."""
    c2 = drop_case(p_psia, 8, beta=beta, tau=tau, W=W, z1=z1, names=names)
    fl = c2["flash"]
    g = np.meshgrid(*[np.arange(n, dtype=np.float64)] * 3, indexing="ij")
    r = np.sqrt(sum((x - n / 2.0) ** 2 for x in g))
    t = np.tanh(2.0 * (r - n / 5.0) / W)
    l = np.asarray(fl.rbar_l)[:, None, None, None]
    v = np.asarray(fl.rbar_v)[:, None, None, None]
    rho0 = 0.5 * (l + v) - 0.5 * (l - v) * t[None]
    return {**c2, "shape": (n, n, n), "rho0": rho0, "n": n}


def drop3d_measure(rho_s, mix, T):
    """Radius at the level 0.5 (rho_l + rho_v) along the six axis rays from the
    centre (averaged) and p_EOS at the centre and at the box corner; None once the
    sphere has dissolved (below a critical size a small drop evaporates into the
    vapour of a closed box)."""
    r = np.asarray(rho_s)
    rho = r.sum(axis=0)
    n = rho.shape[0]
    c = n // 2
    rl, rv = rho[c, c, c], rho[0, 0, 0]
    if not rl > 1.5 * rv:
        return None
    level = 0.5 * (rl + rv)
    radii = []
    for prof in (rho[c, c, c:], rho[c, c, c::-1], rho[c, c:, c], rho[c, c::-1, c], rho[c:, c, c], rho[c::-1, c, c]):
        k = int(np.argmax(prof < level))
        a, b = prof[k - 1], prof[k]
        radii.append(k - 1 + (a - level) / (a - b))
    M = np.asarray(mix["M"], dtype=np.float64)
    n_l, n_v = r[:, c, c, c] / M, r[:, 0, 0, 0] / M
    p = lbm.lbm_pressure(mix, T, np.stack([n_l, n_v]))
    return {"R": float(np.mean(radii)), "p_l": float(p[0]), "p_v": float(p[1]), "dp": float(p[0] - p[1])}


def run_laplace3d(p_list=(200.0,), sizes=(40, 60, 80, 100), beta=1.915, forcing="guo", max_steps=200_000,
                  check_every=10_000, tol=1e-6, progress=None):
    """All (pressure, size) spheres as one D3Q19 batch to steady state; per pressure
    sigma is the least-squares slope of dp against 2/R (with intercept), and
    sigma_n = dp_n R_n / 2 per sphere."""
    cases = [drop3d_case(p, n, beta=beta) for p in p_list for n in sizes]
    boxes = [{"mix": c["mix"], "shape": c["shape"], "T": c["T"], "tau": c["tau"], "beta": c["beta"],
              "gamma": c["gamma"], "rho0": c["rho0"]} for c in cases]
    b = lbm.LbmBatch(boxes, "D3Q19", collision="bgk", forcing=forcing, storage="f64",
                     graph_steps=min(1000, check_every))
    steps, prev, change = 0, None, float("inf")
    try:
        while steps < max_steps:
            b.step(check_every)
            steps += check_every
            bad = b.box_errors()
            if bad.any():
                raise lbm.LbmError(lbm.LBM_ERR_DOMAIN, f"boxes {np.nonzero(bad)[0].tolist()} left the EOS domain")
            meas = [drop3d_measure(r.cpu().numpy(), c["mix"], c["T"]) for r, c in zip(b.fields(), cases)]
            cur = np.array([[m["R"], m["dp"]] if m is not None else [np.nan, np.nan] for m in meas])
            if prev is not None:
                ok = ~np.isnan(cur[:, 0]) & ~np.isnan(prev[:, 0])
                change = float(np.max(np.abs(cur[ok] - prev[ok]) / np.abs(prev[ok]))) if ok.any() else 0.0
            if progress is not None:
                progress(steps, change)
            if change < tol:
                break
            prev = cur
        b.check()
    finally:
        b.close()
    out = {"steps": steps, "last_change": change, "beta": beta, "forcing": forcing, "pressures": {}}
    for p in p_list:
        rows = [(c["n"], m) for c, m in zip(cases, meas) if c["p_psia"] == p and m is not None]
        gone = [c["n"] for c, m in zip(cases, meas) if c["p_psia"] == p and m is None]
        x = np.array([2.0 / m["R"] for _, m in rows])
        dp = np.array([m["dp"] for _, m in rows])
        sigma = icpt = float("nan")
        if len(rows) >= 2:
            A = np.stack([x, np.ones_like(x)], axis=1)
            (sigma, icpt), *_ = np.linalg.lstsq(A, dp, rcond=None)
        out["pressures"][str(p)] = {"sigma": float(sigma), "intercept": float(icpt), "dissolved": gone,
                                    "drops": [{"n": n, "sigma_n": 0.5 * m["dp"] * m["R"], **m} for n, m in rows]}
    return out


# ---------------------------------------------------------------------------
# Oscillating elliptical drop (Sec. 4.3, Table 3)
# ---------------------------------------------------------------------------

def ellipse_case(n, p_psia=70.0, T_degR=580.0, beta=1.815, tau=0.8, W=4.0, h=0.9, z1=0.4, names=("C3", "nC5")):
    """Elliptical drop, Eq. (ellipsedroplet) with the liquid inside: semi-axes R0
    along x and R0 h along y, R0 = 0.15 n, in an n x n periodic box; phase
    densities from the flash at (T_degR, p_psia)."""
    fmix = field_mixture(names)
    u = LatticeUnits(fmix)
    mix = u.mixture()
    T = u.T(T_degR)
    fl = lbm.lbm_flash(mix, T, u.p(p_psia), np.array([z1, 1.0 - z1]))
    R0 = 0.15 * n
    y, x = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64), indexing="ij")
    r = np.sqrt((x - n / 2.0) ** 2 + ((y - n / 2.0) / h) ** 2)
    t = np.tanh(2.0 * (r - R0) / W)
    l = np.asarray(fl.rbar_l)[:, None, None]
    v = np.asarray(fl.rbar_v)[:, None, None]
    rho0 = 0.5 * (l + v) - 0.5 * (l - v) * t[None]
    return {"mix": mix, "shape": (n, n), "T": T, "tau": tau, "beta": beta, "gamma": np.asarray(fl.gamma),
            "rho0": rho0, "n": n, "R0": R0, "h": h, "flash": fl, "units": u}


def _axis_radius(line, level):
    """Distance from the centre (index 0 of `line`) to where `line` drops below level."""
    k = int(np.argmax(line < level))
    a, b = line[k - 1], line[k]
    return k - 1 + (a - level) / (a - b)


def axes_of(rho_s):
    """Semi-axes along x and y of a centred drop: where the total density crosses
    the mean of its centre and corner values on the axis rays (averaged over the
    two rays of each axis)."""
    import torch
    rho = rho_s.sum(dim=0)
    n = rho.shape[0]
    c = n // 2
    m = n - c
    rows = torch.stack([rho[c, c:], torch.flip(rho[c, c - m + 1:c + 1], [0]), rho[c:, c],
                        torch.flip(rho[c - m + 1:c + 1, c], [0])]).cpu().numpy()
    level = 0.5 * (float(rows[0, 0]) + float(rho[0, 0]))
    rx = 0.5 * (_axis_radius(rows[0], level) + _axis_radius(rows[1], level))
    ry = 0.5 * (_axis_radius(rows[2], level) + _axis_radius(rows[3], level))
    return rx, ry


def oscillation_period(t, d):
    """Period from the zero crossings of d(t) = Rx - Ry (linear interpolation);
    consecutive crossings are half a period apart."""
    t = np.asarray(t, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    z = []
    for k in range(1, len(d)):
        if d[k - 1] == 0.0 or d[k - 1] * d[k] < 0.0:
            z.append(t[k - 1] + (t[k] - t[k - 1]) * d[k - 1] / (d[k - 1] - d[k]))
    if len(z) < 3:
        return float("nan"), z
    return float(2.0 * np.mean(np.diff(z))), z


def run_oscillation(sizes=(200, 300, 400, 600, 800), steps=None, sample_every=50, periods=3.0, beta=1.815,
                    forcing="guo", progress=None):
    """All sizes as one batch; the semi-axes are sampled every sample_every steps
    (computed on the device from the density field); returns the periods."""
    cases = [ellipse_case(n, beta=beta) for n in sizes]
    if steps is None:
        # enough for `periods` periods of the largest drop, from the paper's Table 3 scale (T ~ n^1.5)
        steps = int(periods * 18112.0 * (max(sizes) / 800.0) ** 1.5) + 2000
    boxes = [{"mix": c["mix"], "shape": c["shape"], "T": c["T"], "tau": c["tau"], "beta": c["beta"],
              "gamma": c["gamma"], "rho0": c["rho0"]} for c in cases]
    b = lbm.LbmBatch(boxes, "D2Q9", collision="bgk", forcing=forcing, storage="f64", graph_steps=sample_every)
    series = [[] for _ in cases]
    t = []
    try:
        done = 0
        while done < steps:
            b.step(sample_every)
            done += sample_every
            t.append(done)
            for k, r in enumerate(b.fields()):
                series[k].append(axes_of(r))
            if progress is not None and len(t) % 200 == 0:
                progress(done, float("nan"))
        bad = b.box_errors()
        if bad.any():
            raise lbm.LbmError(lbm.LBM_ERR_DOMAIN, f"boxes {np.nonzero(bad)[0].tolist()} left the EOS domain")
        b.check()
    finally:
        b.close()
    out = []
    for c, ser in zip(cases, series):
        ser = np.asarray(ser)
        period, crossings = oscillation_period(t, ser[:, 0] - ser[:, 1])
        out.append({"n": c["n"], "period": period, "crossings": crossings[:12],
                    "rx_final": float(ser[-1, 0]), "ry_final": float(ser[-1, 1])})
    return {"steps": steps, "sample_every": sample_every, "beta": beta, "drops": out}


# ---------------------------------------------------------------------------
# Wetting: contact angle of a drop on a wall against psi_w (solid walls are a
# design of this library; the paper's porous-media motivation, Sec. 1)
# ---------------------------------------------------------------------------

# the single-component fluid of Sec. 4.1 and its Maxwell densities at T = 0.9 Tc
PURE = {"a": np.array([2.0 / 49.0]), "b": np.array([2.0 / 21.0]), "omega": np.array([0.344]),
        "M": np.array([1.0]), "k": np.zeros((1, 1)), "R": 1.0}
MAXWELL_09 = (5.90796, 0.58007)


def sessile_case(nx=160, ny=80, R0=25.0, W=4.0, floor=3):
    """A drop resting on a solid floor (rows 0 .. floor-1, periodic in x and y, so
    the floor is a slab with vapour below it as well): a half disk of radius R0
    centred on the wall surface y = floor - 1/2, tanh profile of width W."""
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    yw = floor - 0.5
    r = np.sqrt((x - nx / 2.0) ** 2 + (y - yw) ** 2)
    rl, rv = MAXWELL_09
    rho = 0.5 * (rl + rv) - 0.5 * (rl - rv) * np.tanh(2.0 * (r - R0) / W)
    solid = np.zeros((ny, nx), dtype=bool)
    solid[:floor] = True
    rho[solid] = rv
    return {"rho0": rho[None], "solid": solid, "wall_y": yw, "shape": (ny, nx)}


def _crossing(prof, level, start):
    """First fractional index >= start where prof falls below level."""
    for i in range(start + 1, len(prof)):
        if prof[i - 1] >= level > prof[i]:
            return i - 1 + (prof[i - 1] - level) / (prof[i - 1] - prof[i])
    raise ValueError("no crossing")


def contact_angle(rho, wall_y, base_offset=3.0):
    """Angle (degrees, measured through the liquid) of the circle through the
    drop's top and its two level crossings base_offset above the wall surface,
    where it meets the wall: cos(theta) = (wall_y - y_c) / R.  The level is the
    mean of the drop's interior density (the largest on the centre column; next
    to a repellent wall the liquid is depleted) and the far-vapour density."""
    ny, nx = rho.shape
    cx = nx // 2
    y0 = int(np.ceil(wall_y))
    col = rho[:, cx]
    liquid = float(np.max(col[y0:]))
    vapour = rho[y0 + (ny - y0) // 2, 0]        # mid-height of the fluid, far from the drop
    level = 0.5 * (liquid + vapour)
    top = _crossing(col, level, y0)
    yb = wall_y + base_offset
    j = int(np.floor(yb))
    row = rho[j] + (yb - j) * (rho[j + 1] - rho[j])
    right = _crossing(row, level, cx)
    left = _crossing(row[::-1], level, nx - 1 - cx)
    half = 0.5 * (right - (nx - 1 - left))
    hgt = top - yb
    R = (half * half + hgt * hgt) / (2.0 * hgt)
    yc = top - R
    c = np.clip((wall_y - yc) / R, -1.0, 1.0)
    return {"theta_deg": float(np.degrees(np.arccos(c))), "R": float(R), "top": float(top), "half_width": float(half),
            "liquid": float(liquid), "vapour": float(vapour)}


def run_contact_angles(psi_fracs=(0.1, 0.3, 0.5, 0.7, 0.9), steps=60000, nx=160, ny=80, R0=25.0, tau=1.0,
                       beta=1.945, progress=None, fields_out=None):
    """One box per psi_w = psi_v + t (psi_l - psi_v) (psi of the Maxwell vapour and
    liquid), BGK + Guo, float64, run for `steps`; returns the angles (None where
    no cap sits on the wall).  A dict passed as fields_out receives the final
    density fields."""
    T = 0.9 * float(lbm.LibThermo().critical_temperature(PURE)[0])
    case = sessile_case(nx, ny, R0)
    probe = lbm.LbmContext(PURE, "D2Q9", case["shape"], T, tau, beta, [1.0], case["rho0"], forcing="guo")
    psi = probe.moments(totals=False)["psi"].cpu().numpy()
    probe.close()
    y0 = int(np.ceil(case["wall_y"]))
    psi_l, psi_v = float(psi[y0 + 2, nx // 2]), float(psi[y0 + (ny - y0) // 2, 0])
    out = {"T": T, "steps": steps, "psi_l": psi_l, "psi_v": psi_v, "tau": tau, "beta": beta, "drops": []}
    for t in psi_fracs:
        pw = psi_v + t * (psi_l - psi_v)
        ctx = lbm.LbmContext(PURE, "D2Q9", case["shape"], T, tau, beta, [1.0], case["rho0"], forcing="guo",
                             solid=case["solid"], psi_wall=pw)
        try:
            ctx.step(steps)
            ctx.check()
            rho = ctx.moments(totals=False)["rho_s"].cpu().numpy()[0]
            ctx.step(steps // 10)
            ctx.check()
            rho2 = ctx.moments(totals=False)["rho_s"].cpu().numpy()[0]
        except lbm.LbmError as e:   # a strongly wetting wall condenses liquid past the EOS domain
            out["drops"].append({"psi_frac": t, "psi_wall": pw, "theta_deg": None, "error": str(e)})
            continue
        finally:
            ctx.close()
        if fields_out is not None:
            fields_out[f"psi_frac_{t:g}"] = rho2
        try:
            a, b = contact_angle(rho, case["wall_y"]), contact_angle(rho2, case["wall_y"])
        except ValueError:          # no cap on the wall (the drop left it, or spread into a film)
            out["drops"].append({"psi_frac": t, "psi_wall": pw, "theta_deg": None})
            continue
        out["drops"].append({"psi_frac": t, "psi_wall": pw, **b, "theta_change_last_tenth": b["theta_deg"] - a["theta_deg"]})
        if progress is not None:
            progress(t, b["theta_deg"])
    return out


def main():
    import argparse
    import json

    ap = argparse.ArgumentParser(description="flat-interface validation (Sec. 4.2) and beta calibration")
    ap.add_argument("--pressures", default="240,220,200,180,160,140")
    ap.add_argument("--nx", type=int, default=1600)
    ap.add_argument("--beta", type=float, default=1.945)
    ap.add_argument("--forcing", default="guo")
    ap.add_argument("--collision", default="bgk")
    ap.add_argument("--max-steps", type=int, default=2_000_000)
    ap.add_argument("--check-every", type=int, default=50_000)
    ap.add_argument("--tol", type=float, default=1e-9)
    ap.add_argument("--gamma-update", action="store_true", help="re-flash gamma at every check")
    ap.add_argument("--calibrate", action="store_true", help="sweep beta instead")
    ap.add_argument("--laplace", action="store_true", help="Laplace's law on drops instead (Sec. 4.3)")
    ap.add_argument("--sizes", default="50,100,200,400,800")
    ap.add_argument("--oscillation", action="store_true", help="oscillating elliptical drop instead (Table 3)")
    ap.add_argument("--betas", default="", help="comma list for --calibrate (default 1.0..2.0 step 0.1)")
    ap.add_argument("--convergence", action="store_true",
                    help="flat interface at every nx of --sizes (grid convergence, Sec. 4.2)")
    ap.add_argument("--save-state", default="", help="flat runs: write the final fields to this .npz")
    ap.add_argument("--init-from", default="",
                    help="flat runs: start each box from the largest smaller box of this .npz (stretch_flat)")
    ap.add_argument("--combine", nargs="+", default=None,
                    help="merge the reports of flat-run JSON files into convergence tables and exit")
    ap.add_argument("--sigma-convergence", default="",
                    help="surface-tension convergence of a --laplace JSON file and exit")
    ap.add_argument("--contact-angle", action="store_true", help="sessile drop on a wall against psi_w instead")
    ap.add_argument("--laplace3d", action="store_true", help="Laplace's law on D3Q19 spheres instead")
    ap.add_argument("--psi-fracs", default="0.1,0.3,0.5,0.7,0.9")
    args = ap.parse_args()
    ps = [float(p) for p in args.pressures.split(",")]
    import sys

    def progress(steps, change):
        print(f"steps {steps} max relative change of the bulk densities {change:.3e}", file=sys.stderr, flush=True)

    kw = dict(max_steps=args.max_steps, check_every=args.check_every, tol=args.tol, progress=progress)
    if args.combine:
        reps = []
        for path in args.combine:
            with open(path) as fh:
                reps += json.loads(fh.read().strip().splitlines()[-1])["reports"]
        print(json.dumps(flat_convergence(reps), default=float))
        return
    if args.sigma_convergence:
        with open(args.sigma_convergence) as fh:
            print(json.dumps(sigma_convergence(json.loads(fh.read().strip().splitlines()[-1])), default=float))
        return
    if args.laplace3d:
        out = run_laplace3d(ps, sizes=[int(n) for n in args.sizes.split(",")], beta=args.beta, forcing=args.forcing,
                            **kw)
        print(json.dumps(out, default=float))
        return
    if args.contact_angle:
        fields = {}
        out = run_contact_angles([float(t) for t in args.psi_fracs.split(",")], steps=args.max_steps,
                                 beta=args.beta, fields_out=fields,
                                 progress=lambda t, th: print(f"psi fraction {t}: theta {th:.2f}",
                                                              file=sys.stderr, flush=True))
        if args.save_state:
            np.savez(args.save_state, **fields)
        print(json.dumps(out, default=float))
        return
    if args.oscillation:
        out = run_oscillation(sizes=[int(n) for n in args.sizes.split(",")], beta=args.beta, forcing=args.forcing,
                              progress=progress)
    elif args.laplace:
        out = run_laplace(ps, sizes=[int(n) for n in args.sizes.split(",")], beta=args.beta, forcing=args.forcing,
                          collision=args.collision, **kw)
    elif args.calibrate:
        betas = [float(b) for b in args.betas.split(",")] if args.betas else None
        out = calibrate_beta(ps, forcing=args.forcing, collision=args.collision, nx=args.nx, betas=betas, **kw)
    else:
        sizes = [int(n) for n in args.sizes.split(",")] if args.convergence else [args.nx]
        cases = [flat_case(p, nx=n, beta=args.beta) for p in ps for n in sizes]
        if args.init_from:
            saved = np.load(args.init_from)
            for c in cases:
                nx = c["shape"][1]
                keys = [k for k in saved.files if k.startswith(f"p{c['p_psia']:g}_nx")]
                smaller = [int(k.split("_nx")[1]) for k in keys if int(k.split("_nx")[1]) < nx]
                if smaller:
                    src = saved[f"p{c['p_psia']:g}_nx{max(smaller)}"]
                    mass = c["rho0"].reshape(c["rho0"].shape[0], -1).sum(axis=1)
                    c["rho0"] = stretch_flat(src, nx, mass=mass)
        fields = []
        reps = run_flat(cases, collision=args.collision, forcing=args.forcing, gamma_update=args.gamma_update,
                        fields_out=fields, **kw)
        if args.save_state:
            np.savez(args.save_state, **{f"p{c['p_psia']:g}_nx{c['shape'][1]}": f for c, f in zip(cases, fields)})
        out = {"reports": reps, "worst_composition_err": max(r["err_composition"] for r in reps),
               "worst_density_err": max(r["err_density"] for r in reps)}
        if len(sizes) > 1:
            out["convergence"] = flat_convergence(reps)
    print(json.dumps(out, default=float))


if __name__ == "__main__":
    main()
