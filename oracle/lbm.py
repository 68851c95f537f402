"""One time step of the multi-component pseudo-potential LB model, plain float64.

Oracle; test infrastructure only.  Array layout: populations f[sigma, alpha, *space]
with space = (ny, nx) in 2-D and (nz, ny, nx) in 3-D; velocity component d (0 = x,
1 = y, 2 = z) runs along the array axis counted from the right.  All boundaries are
periodic (Sec. 4 uses periodic domains throughout).

Step order (Sec. 3.4, the list of implementation steps, and Eq. (LBE) of Sec. 2.1):
  1. cell-volume densities rbar_sigma = sum_alpha f (Sec. 2.1) and momentum j;
  2. p_EOS from the mixture EOS with molar densities rbar_sigma / M_sigma,
     Eq. (MCPengRobinson) with Eq. (randommixingrule);
  3. psi from Eq. (psicorrected) with the phase mass density rho = sum rbar;
  4. total force, Eq. (coupledMCforce) (beta = 1 gives Eq. (correctMCforce));
  5. split F_sigma = chi_sigma F, chi from Eq. (distributionforce);
  6. velocity, equilibrium Eq. (equilibrium a), collision with forcing
     (Guo's term Eq. (equilibrium b), or the exact-difference method);
  7. streaming, the left-hand side of Eq. (LBE).

Readings (the paper is silent on these):
  * u with Guo forcing is the shared barycentric velocity U = (sum_sigma j_sigma + F/2)/rho.
  * The exact-difference method (EDM) is not in the paper; for several components it
    is read so that the per-component balance of Sec. 3.1, Eq. (hydrostatic1), holds
    as it does with Guo's term: component sigma receives the velocity jump
    du_sigma = F_sigma / rbar_sigma = gamma_sigma F / Gamma and relaxes towards
    feq(rbar_sigma, U - du_sigma / 2), followed by the jump
    feq(rbar_sigma, U + du_sigma / 2) - feq(rbar_sigma, U - du_sigma / 2).  Its
    component momentum then changes by -(j_sigma - rbar_sigma U)/tau + (1 - 1/(2 tau)) F_sigma
    (the same first moment as Guo's scheme), so that a resting component whose
    momentum is -F_sigma/2 gains exactly F_sigma per step; with one component it is
    the standard EDM (relaxation towards feq(j/rho)).  Relaxing every component
    towards the shared feq(j/rho) instead would add a drift between the components
    that depends on their mass fractions and on tau, i.e. a different split than
    Eq. (distributionforce).
  * psi uses the densities of the populations being collided (no time lag).
  * A negative argument of the square root in Eq. (psicorrected), or b_m rho~ >= 1,
    is an error (DomainError); nothing is clamped.
  * G = -1; the force does not depend on |G| (Sec. 4.1 remarks G only fixes the sign).
  * MRT (not in the paper): m^eq = M f^eq, so equal rates reduce exactly to BGK; with
    Guo forcing the source is M^-1 (I - S/2) M Fbar.
  * Optional uniform body acceleration g adds rbar_sigma g to F_sigma (a test hook
    for momentum balance with forcing).

Solid walls (beyond the paper: porous media are its motivation in Sec. 1, but it
defines no boundary; this is the design used here).  An optional boolean mask
marks solid cells.  Solid cells hold no fluid (their populations are zero); in the
force stencil their psi is a wetting constant psi_w (a larger psi_w attracts the
fluid, G < 0).  Streaming uses halfway bounce-back: a population that would arrive
at a fluid cell x from a solid cell x - e_a is instead the post-collision
population of the opposite direction at x itself (it left x towards the wall and
returned reversed within the step).  Collision, force split and velocity are
evaluated on fluid cells only.

Pins (tests/test_oracle_lbm.py, tests/test_oracle_walls.py): per-component mass,
momentum balance, equilibrium and forcing moment identities, MRT==BGK at equal
rates, identical components == single-component model (Sec. 4.1), force stencil
on linear psi, invariance to |G|, uniform-state fixed point; with walls: the
streaming is a permutation of the fluid cells' values, mass is conserved, a
uniform resting fluid with psi_w = psi(rho) is a fixed point, the wetting sign,
and the BGK Poiseuille profile that halfway bounce-back reproduces exactly at
(tau - 1/2)^2 = 3/16.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import thermo
from .lattice import CS2, VelocitySet, mrt_basis


class DomainError(ValueError):
    """Raised when the EOS or the pseudo-potential leaves its domain."""


@dataclass
class StepParams:
    T: float
    tau: float
    gamma: np.ndarray
    G: float = -1.0
    beta: float = 1.0
    collision: str = "bgk"      # "bgk" | "mrt"
    forcing: str = "guo"        # "guo" | "edm"
    mrt_s: np.ndarray = None    # relaxation rate per moment row (MRT only)
    accel: np.ndarray = field(default=None)
    solid: np.ndarray = None    # boolean mask of solid cells (space shape); None = no walls
    psi_wall: float = 0.0       # psi of the solid cells in the force stencil


def _axis(d: int, nspace: int, lead: int) -> int:
    """Array axis of velocity component d for an array with `lead` leading axes."""
    return lead + (nspace - 1 - d)


def shift(a: np.ndarray, e, lead: int) -> np.ndarray:
    """b(x) = a(x - e), periodic, over the trailing spatial axes."""
    nspace = a.ndim - lead
    out = a
    for d, ed in enumerate(e):
        if ed != 0:
            out = np.roll(out, int(ed), axis=_axis(d, nspace, lead))
    return out


def densities(f: np.ndarray) -> np.ndarray:
    return f.sum(axis=1)


def momentum(f: np.ndarray, lat: VelocitySet) -> np.ndarray:
    j = np.zeros((lat.D,) + f.shape[2:])
    for s in range(f.shape[0]):
        for a in range(lat.Q):
            for d in range(lat.D):
                if lat.e[a, d] != 0:
                    j[d] += f[s, a] * lat.e[a, d]
    return j


def eos_pressure(rho_s: np.ndarray, T: float, mix: thermo.Mixture) -> np.ndarray:
    """p_EOS from cell-volume densities: molar densities rbar_i / M_i into
    Eq. (MCPengRobinson)."""
    n = rho_s / mix.M.reshape((-1,) + (1,) * (rho_s.ndim - 1))
    Bn = np.einsum("i...,i->...", n, mix.b)
    if np.any(Bn >= 1.0):
        raise DomainError("b_m * rho~ >= 1")
    return thermo.pressure_molar(n, T, mix)


def pseudo_potential(rho_s: np.ndarray, T: float, mix: thermo.Mixture, G: float) -> np.ndarray:
    """psi = sqrt(2 (p_EOS - c_s^2 rho) / (G c_s^2)), Eq. (psicorrected), delta t = 1,
    rho = sum of cell-volume densities."""
    p = eos_pressure(rho_s, T, mix)
    rho = rho_s.sum(axis=0)
    X = 2.0 * (p - CS2 * rho) / (G * CS2)
    if np.any(X < 0.0) or not np.all(np.isfinite(X)):
        raise DomainError("negative argument under the square root of Eq. (psicorrected)")
    return np.sqrt(X)


def total_force(psi: np.ndarray, beta: float, G: float, lat: VelocitySet) -> np.ndarray:
    """Eq. (coupledMCforce):
    F = -beta G psi(x) sum_a w_a psi(x+e_a) e_a - (1-beta)/2 G sum_a w_a psi(x+e_a)^2 e_a."""
    F = np.zeros((lat.D,) + psi.shape)
    for a in range(1, lat.Q):
        e = lat.e[a]
        psi_n = shift(psi, -e, lead=0)          # psi(x + e_a)
        for d in range(lat.D):
            if e[d] != 0:
                F[d] += (-beta * G * psi * lat.w[a] * psi_n * e[d]
                         - 0.5 * (1.0 - beta) * G * lat.w[a] * psi_n * psi_n * e[d])
    return F


def split_force(F: np.ndarray, rho_s: np.ndarray, gamma, fluid=None) -> np.ndarray:
    """F_sigma = chi_sigma F with chi_sigma = gamma_sigma rbar_sigma / sum_i gamma_i rbar_i,
    Eq. (forcedistribution) and Eq. (distributionforce).  With a fluid mask, solid
    cells get F_sigma = 0 and are not checked."""
    gamma = np.asarray(gamma, dtype=np.float64)
    gshape = (-1,) + (1,) * (rho_s.ndim - 1)
    Gam = np.sum(gamma.reshape(gshape) * rho_s, axis=0)
    if fluid is None:
        fluid = np.ones(Gam.shape, dtype=bool)
    if np.any(Gam[fluid] <= 0.0):
        raise DomainError("sum_i gamma_i rbar_i <= 0")
    chi = np.where(fluid, gamma.reshape(gshape) * rho_s / np.where(fluid, Gam, 1.0), 0.0)
    return chi[:, None] * F[None]          # (N, D, *space)


def equilibrium(rho_sig: np.ndarray, u: np.ndarray, lat: VelocitySet) -> np.ndarray:
    """Eq. (equilibrium a): rbar w_a [1 + e.u/cs2 + (e.u)^2/(2 cs4) - u.u/(2 cs2)]."""
    uu = np.sum(u * u, axis=0)
    feq = np.empty((lat.Q,) + rho_sig.shape)
    for a in range(lat.Q):
        eu = sum(lat.e[a, d] * u[d] for d in range(lat.D))
        feq[a] = rho_sig * lat.w[a] * (1.0 + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2))
    return feq


def guo_shape(F_sig: np.ndarray, u: np.ndarray, lat: VelocitySet) -> np.ndarray:
    """w_a [(e_a - u)/cs2 + (e_a.u) e_a / cs4] . F_sigma (Eq. (equilibrium b) without
    its (1 - 1/(2 tau)) prefactor)."""
    out = np.empty((lat.Q,) + F_sig.shape[1:])
    for a in range(lat.Q):
        eu = sum(lat.e[a, d] * u[d] for d in range(lat.D))
        acc = 0.0
        for d in range(lat.D):
            acc = acc + ((lat.e[a, d] - u[d]) / CS2 + eu * lat.e[a, d] / (CS2 * CS2)) * F_sig[d]
        out[a] = lat.w[a] * acc
    return out


def _rates(prm: StepParams, lat: VelocitySet) -> np.ndarray:
    if prm.mrt_s is None:
        raise ValueError("MRT needs a relaxation rate for every moment row")
    s = np.asarray(prm.mrt_s, dtype=np.float64)
    assert s.shape == (lat.Q,)
    return s


def _apply_matrix(Mx: np.ndarray, g: np.ndarray) -> np.ndarray:
    """(Q x Q) matrix times populations g[alpha, *space]."""
    return np.tensordot(Mx, g, axes=([1], [0]))


def opposite(lat: VelocitySet) -> np.ndarray:
    """Index of -e_a for every direction a."""
    return np.array([next(b for b in range(lat.Q) if np.array_equal(lat.e[b], -lat.e[a])) for a in range(lat.Q)])


def stream(fstar: np.ndarray, lat: VelocitySet, solid=None) -> np.ndarray:
    """f(x, t + 1) = f*(x - e_a, t), periodic; with a solid mask, halfway
    bounce-back: at a fluid cell x whose source x - e_a is solid the arriving
    population is f*_{opp(a)}(x), and solid cells receive nothing (zero)."""
    fnew = np.empty_like(fstar)
    for s in range(fstar.shape[0]):
        for a in range(lat.Q):
            fnew[s, a] = shift(fstar[s, a], lat.e[a], lead=0)
    if solid is None:
        return fnew
    opp = opposite(lat)
    for a in range(lat.Q):
        from_wall = shift(solid, lat.e[a], lead=0) & ~solid      # x fluid, x - e_a solid
        for s in range(fstar.shape[0]):
            fnew[s, a][from_wall] = fstar[s, opp[a]][from_wall]
    fnew[:, :, solid] = 0.0
    return fnew


def step(f: np.ndarray, mix: thermo.Mixture, prm: StepParams, lat: VelocitySet, return_fields=False):
    """Advance the populations by one time step; see the module docstring."""
    N = f.shape[0]
    D = lat.D
    gshape = (-1,) + (1,) * (f.ndim - 2)
    solid = prm.solid
    fluid = None if solid is None else ~solid
    if solid is not None:
        f = np.where(solid[None, None], 0.0, f)        # solid cells hold no fluid
    # 1. densities and momentum
    rho_s = densities(f)
    rho = rho_s.sum(axis=0)
    j = momentum(f, lat)
    # 2-3. EOS and pseudo-potential (psi_w on solid cells)
    if solid is None:
        psi = pseudo_potential(rho_s, prm.T, mix, prm.G)
    else:
        psi = np.full(rho.shape, float(prm.psi_wall))
        psi[fluid] = pseudo_potential(rho_s[:, fluid], prm.T, mix, prm.G)
    # 4. total interaction force
    F = total_force(psi, prm.beta, prm.G, lat)
    # 5. split into components (+ optional body acceleration)
    F_s = split_force(F, rho_s, prm.gamma, fluid)
    g = np.zeros(D) if prm.accel is None else np.asarray(prm.accel, dtype=np.float64)
    for d in range(D):
        F_s[:, d] += rho_s * g[d]
    F_tot = F_s.sum(axis=0)
    rho_div = rho if solid is None else np.where(solid, 1.0, rho)   # solid cells: u = 0
    # 6. velocity, equilibrium, collision with forcing
    if prm.forcing not in ("guo", "edm"):
        raise ValueError(prm.forcing)
    u = (j + 0.5 * F_tot) / rho_div        # barycentric velocity U (both forcings)
    if prm.forcing == "edm":
        gamma = np.asarray(prm.gamma, dtype=np.float64)
        Gam = np.sum(gamma.reshape(gshape) * rho_s, axis=0)
        if solid is not None:
            Gam = np.where(solid, 1.0, Gam)
    if prm.collision == "mrt":
        Mx = mrt_basis(lat)
        Minv = np.linalg.inv(Mx)
        S = np.diag(_rates(prm, lat))
        relax = Minv @ S @ Mx
        guo_mat = Minv @ (np.eye(lat.Q) - 0.5 * S) @ Mx
    fstar = np.empty_like(f)
    for s in range(N):
        if prm.forcing == "edm":
            du = np.empty_like(u)           # velocity jump of component s
            for d in range(D):
                du[d] = prm.gamma[s] * F[d] / Gam + g[d]
            ueq = u - 0.5 * du              # its equilibrium velocity
        else:
            ueq = u
        feq = equilibrium(rho_s[s], ueq, lat)
        if prm.collision == "bgk":
            post = f[s] - (f[s] - feq) / prm.tau
        elif prm.collision == "mrt":
            post = f[s] - _apply_matrix(relax, f[s] - feq)
        else:
            raise ValueError(prm.collision)
        if prm.forcing == "guo":
            shape = guo_shape(F_s[s], u, lat)
            if prm.collision == "bgk":
                post = post + (1.0 - 0.5 / prm.tau) * shape
            else:
                post = post + _apply_matrix(guo_mat, shape)
        else:
            post = post + equilibrium(rho_s[s], ueq + du, lat) - feq
        fstar[s] = post
    if solid is not None:
        fstar[:, :, solid] = 0.0
    # 7. streaming: f(x + e_a, t + 1) = f*(x, t) (bounce-back at solid sources)
    fnew = stream(fstar, lat, solid)
    if return_fields:
        return fnew, {"rho_s": rho_s, "rho": rho, "j": j, "psi": psi, "F": F,
                      "F_s": F_s, "u": u, "fstar": fstar}
    return fnew


def macroscopic(f: np.ndarray, mix: thermo.Mixture, prm: StepParams, lat: VelocitySet):
    """Fields reported for a population state: rbar_sigma, the physical velocity
    u = (j + F_total/2)/rho, p (= p_EOS, equal to the hydrodynamic pressure of
    Eq. (hydropressure) by construction of psi) and psi."""
    solid = prm.solid
    if solid is not None:
        f = np.where(solid[None, None], 0.0, f)
    rho_s = densities(f)
    rho = rho_s.sum(axis=0)
    j = momentum(f, lat)
    if solid is None:
        p = eos_pressure(rho_s, prm.T, mix)
        psi = pseudo_potential(rho_s, prm.T, mix, prm.G)
    else:                                   # solid cells: p = 0, psi = psi_w
        p = np.zeros(rho.shape)
        p[~solid] = eos_pressure(rho_s[:, ~solid], prm.T, mix)
        psi = np.full(rho.shape, float(prm.psi_wall))
        psi[~solid] = pseudo_potential(rho_s[:, ~solid], prm.T, mix, prm.G)
    F = total_force(psi, prm.beta, prm.G, lat)
    g = np.zeros(lat.D) if prm.accel is None else np.asarray(prm.accel, dtype=np.float64)
    F_tot = F + rho[None] * g.reshape((-1,) + (1,) * rho.ndim)
    if solid is None:
        u = (j + 0.5 * F_tot) / rho
    else:                                   # solid cells: no fluid, u = 0, F = 0
        F = np.where(solid[None], 0.0, F)
        F_tot = np.where(solid[None], 0.0, F_tot)
        u = (j + 0.5 * F_tot) / np.where(solid, 1.0, rho)
    return {"rho_s": rho_s, "u": u, "p": p, "psi": psi, "F": F, "j": j}


def totals(f: np.ndarray, mix: thermo.Mixture, prm: StepParams, lat: VelocitySet):
    """Conservation sums: mass of each component, total momentum sum(j + F_total/2)
    and the net interaction force sum F."""
    m = macroscopic(f, mix, prm, lat)
    rho = m["rho_s"].sum(axis=0)
    g = np.zeros(lat.D) if prm.accel is None else np.asarray(prm.accel, dtype=np.float64)
    F_tot = m["F"] + rho[None] * g.reshape((-1,) + (1,) * rho.ndim)
    axes = tuple(range(1, f.ndim - 1))
    return {"mass": m["rho_s"].sum(axis=axes),
            "momentum": (m["j"] + 0.5 * F_tot).sum(axis=axes),
            "force": m["F"].sum(axis=axes)}


def init_populations(rho_s: np.ndarray, lat: VelocitySet, u: np.ndarray = None) -> np.ndarray:
    """Initial populations f = f^eq(rbar_sigma, u) (u = 0 unless given): the paper
    initialises densities only; the populations start at equilibrium."""
    N = rho_s.shape[0]
    if u is None:
        u = np.zeros((lat.D,) + rho_s.shape[1:])
    f = np.empty((N, lat.Q) + rho_s.shape[1:])
    for s in range(N):
        f[s] = equilibrium(rho_s[s], u, lat)
    return f
