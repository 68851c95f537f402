"""Peng-Robinson mixture thermodynamics, plain float64 (oracle; test infrastructure only).

Follows Sec. 3.2 of the paper ("Peng-Robinson EOS for multi-component hydrocarbon
mixtures") and the volatility coefficient of Sec. 3.1, Eq. (gamma).

Readings taken where the printed text is garbled (each one pinned by a test):
  * Eq. (PRcubic): the Z coefficient is A - 3B^2 - 2B and the constant term is
    -(AB - B^2 - B^3).  This is the cubic that Eq. (MCPengRobinson) gives on
    substituting Z = p/(rho~ R T); the printed coefficients are not satisfied by
    the EOS.
  * Eq. (cubiccoeff): A_i carries p_ri / T_ri^2 (not p_ri / T_ri), which is what
    a_i alpha_i p / (R T)^2 evaluates to with a_i from the definitions below it.
  * The flash algorithm is not given (end of Sec. 3.2): Wilson start, successive
    substitution on K, Rachford-Rice by bisection on its bracket.
  * gamma for more than two components: Eq. (gamma) applied per component against
    the least volatile component (smallest K), whose gamma is 1 (Sec. 3.1).

Pins (tests/test_oracle_thermo.py): the Maxwell densities quoted in Sec. 4.1,
Table 2 (Sec. 4.2) with Table 1 data, the Gibbs-difference identity, the
Gibbs-Duhem/finite-difference check of ln(phi), the EOS-vs-cubic identity.

Parity unpinned (no value the paper prints and no identity separates them from a
plausible mistake): the omega > 0.49 branch of m(omega) (Table 1's components and
every synthetic workload lie below 0.49; its test only retypes the formula), and
the sign of the interaction factor (1 - zeta_ij) for zeta_ij != 0 (Table 2 has
zeta = 0; the ln(phi) identity holds for either sign, since the pressure and
ln(phi) share the mixing rule).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Sec. 3.2: constants Omega_a^o and Omega_b^o of the Peng-Robinson EOS.
OMEGA_A = 0.45724
OMEGA_B = 0.0778
SQRT2 = math.sqrt(2.0)


@dataclass
class Mixture:
    """Component data in one consistent unit system.

    a, b   : attraction and co-volume parameters per mole (Sec. 3.2 definitions)
    omega  : Pitzer acentric factor
    M      : molar mass (converts cell-volume mass density to molar density)
    k      : binary interaction coefficients zeta_ij (symmetric, zero diagonal)
    R      : universal gas constant in the same units
    """
    a: np.ndarray
    b: np.ndarray
    omega: np.ndarray
    M: np.ndarray
    k: np.ndarray
    R: float = 1.0

    def __post_init__(self):
        self.a = np.asarray(self.a, dtype=np.float64)
        self.b = np.asarray(self.b, dtype=np.float64)
        self.omega = np.asarray(self.omega, dtype=np.float64)
        self.M = np.asarray(self.M, dtype=np.float64)
        self.k = np.asarray(self.k, dtype=np.float64)
        self.R = float(self.R)

    @property
    def nc(self) -> int:
        return int(self.a.shape[0])

    @property
    def Tc(self) -> np.ndarray:
        # invert a_i = Omega_a R^2 Tc^2 / pc and b_i = Omega_b R Tc / pc (Sec. 3.2)
        return (OMEGA_B / OMEGA_A) * self.a / (self.b * self.R)

    @property
    def pc(self) -> np.ndarray:
        return OMEGA_B * self.R * self.Tc / self.b


def mixture_from_critical(pc, Tc, omega, M, k=None, R=1.0) -> Mixture:
    """Build a Mixture from critical constants: a_i, b_i of Sec. 3.2."""
    pc = np.asarray(pc, dtype=np.float64)
    Tc = np.asarray(Tc, dtype=np.float64)
    a = OMEGA_A * R * R * Tc * Tc / pc
    b = OMEGA_B * R * Tc / pc
    nc = pc.shape[0]
    if k is None:
        k = np.zeros((nc, nc))
    return Mixture(a=a, b=b, omega=omega, M=M, k=k, R=R)


def m_of_omega(omega):
    """m_i as a function of the acentric factor, two branches split at 0.49 (Sec. 3.2)."""
    omega = np.asarray(omega, dtype=np.float64)
    low = 0.374640 + 1.54226 * omega - 0.26992 * omega ** 2
    high = 0.379642 + 1.48503 * omega - 0.164423 * omega ** 2 + 0.016666 * omega ** 3
    return np.where(omega <= 0.49, low, high)


def alpha(mix: Mixture, T: float) -> np.ndarray:
    """alpha_i(T) = [1 + m_i (1 - sqrt(T/Tc_i))]^2 (Sec. 3.2)."""
    return (1.0 + m_of_omega(mix.omega) * (1.0 - np.sqrt(T / mix.Tc))) ** 2


def aalpha_pair(mix: Mixture, T: float) -> np.ndarray:
    """sqrt(a_i alpha_i a_j alpha_j) (1 - zeta_ij): the summand of the random mixing
    rule, Eq. (randommixingrule)."""
    aa = mix.a * alpha(mix, T)
    return np.sqrt(np.outer(aa, aa)) * (1.0 - mix.k)


# ---------------------------------------------------------------------------
# Equation of state in terms of molar densities
# ---------------------------------------------------------------------------

def pressure_molar(n, T: float, mix: Mixture):
    """Mixture Peng-Robinson pressure, Eq. (MCPengRobinson) with Eq. (randommixingrule).

    n : molar densities of each component, shape (nc, ...).  The molar density of
        the phase is rho~ = sum_i n_i and the local composition is c_i = n_i / rho~
        (the reading of Sec. 3.2 that c_i is the local phase composition).
    """
    n = np.asarray(n, dtype=np.float64)
    rho_t = n.sum(axis=0)
    c = n / rho_t
    pair = aalpha_pair(mix, T)
    aalpha_m = np.einsum("i...,j...,ij->...", c, c, pair)
    b_m = np.einsum("i...,i->...", c, mix.b)
    return (rho_t * mix.R * T / (1.0 - b_m * rho_t)
            - aalpha_m * rho_t ** 2 / (1.0 + 2.0 * b_m * rho_t - (b_m * rho_t) ** 2))


def pure_pressure_mass(rho, T, a, b, omega, Rs=1.0):
    """Single-substance Peng-Robinson pressure in mass density, Eq. (SCpengrobinson)."""
    Tc = (OMEGA_B / OMEGA_A) * a / (b * Rs)
    al = (1.0 + m_of_omega(omega) * (1.0 - math.sqrt(T / Tc))) ** 2
    return rho * Rs * T / (1.0 - b * rho) - a * al * rho ** 2 / (1.0 + 2.0 * b * rho - b * b * rho * rho)


# ---------------------------------------------------------------------------
# Cubic in Z, fugacity coefficients, Gibbs root selection
# ---------------------------------------------------------------------------

def cubic_AB(mix: Mixture, T: float, p: float, c):
    """Mixture A, B and the component A_ij, B_i of Eq. (cubiccoeff), written with the
    reduced quantities p_ri = p/pc_i, T_ri = T/Tc_i (A_i with T_ri^2, see header)."""
    c = np.asarray(c, dtype=np.float64)
    Tr = T / mix.Tc
    pr = p / mix.pc
    m = m_of_omega(mix.omega)
    Ai = OMEGA_A * pr / Tr ** 2 * (1.0 + m * (1.0 - np.sqrt(Tr))) ** 2
    Bi = OMEGA_B * pr / Tr
    Aij = np.sqrt(np.outer(Ai, Ai)) * (1.0 - mix.k)
    A = float(c @ Aij @ c)
    B = float(c @ Bi)
    return A, B, Aij, Bi


def cubic_coefficients(A: float, B: float):
    """Coefficients of Z^3 + (B-1) Z^2 + (A - 3B^2 - 2B) Z - (AB - B^2 - B^3) = 0,
    Eq. (PRcubic) in the corrected form (see header)."""
    return np.array([1.0, B - 1.0, A - 3.0 * B * B - 2.0 * B, -(A * B - B * B - B ** 3)])


def cubic_roots(A: float, B: float):
    """Real roots of Eq. (PRcubic) greater than B, ascending.

    numpy.roots (companion-matrix eigenvalues) gives the roots; each real one is
    refined by Newton on the same cubic to remove eigen-solver rounding.
    """
    coef = cubic_coefficients(A, B)
    r = np.roots(coef)
    out = []
    for z in r:
        if abs(z.imag) > 1e-7 * max(1.0, abs(z.real)):
            continue
        x = float(z.real)
        for _ in range(4):
            f = ((x + coef[1]) * x + coef[2]) * x + coef[3]
            d = (3.0 * x + 2.0 * coef[1]) * x + coef[2]
            if d == 0.0:
                break
            x -= f / d
        if x > B:
            out.append(x)
    out.sort()
    return out


def ln_phi(Z: float, A: float, B: float, Aij, Bi, c):
    """Fugacity coefficients ln(phi_i) of Eq. (fugacitycoeff2)."""
    c = np.asarray(c, dtype=np.float64)
    sum_Aij_c = Aij @ c
    return (-np.log(Z - B) + Bi / B * (Z - 1.0)
            + A / (2.0 * SQRT2 * B) * (2.0 * sum_Aij_c / A - Bi / B)
            * np.log((Z + (1.0 - SQRT2) * B) / (Z + (1.0 + SQRT2) * B)))


def gibbs_difference(Zmax: float, Zmin: float, A: float, B: float) -> float:
    """dG/RT = G(Zmax) - G(Zmin), Eq. (solutionselection)."""
    return ((Zmax - Zmin) + math.log((Zmin - B) / (Zmax - B))
            + A / (2.0 * SQRT2 * B) * math.log(
                ((Zmin + (1.0 + SQRT2) * B) * (Zmax + (1.0 - SQRT2) * B))
                / ((Zmin + (1.0 - SQRT2) * B) * (Zmax + (1.0 + SQRT2) * B))))


def select_root(roots, A: float, B: float) -> float:
    """One root: use it.  Three roots: drop the middle one and keep Zmin if dG > 0,
    else Zmax (Sec. 3.2).  A tie (dG == 0) keeps Zmin."""
    if len(roots) == 0:
        raise ValueError("cubic has no root above B")
    if len(roots) == 1:
        return roots[0]
    zmin, zmax = roots[0], roots[-1]
    return zmin if gibbs_difference(zmax, zmin, A, B) >= 0.0 else zmax


def phase_state(mix: Mixture, T: float, p: float, c, root: str = "gibbs"):
    """Z and ln(phi) of a phase of composition c at (T, p).

    root = "gibbs" (Sec. 3.2 criterion), "min" or "max" (the typical approach the
    paper mentions, used only to probe metastable branches).
    """
    A, B, Aij, Bi = cubic_AB(mix, T, p, c)
    roots = cubic_roots(A, B)
    if root == "gibbs":
        Z = select_root(roots, A, B)
    elif root == "min":
        Z = roots[0]
    else:
        Z = roots[-1]
    return Z, ln_phi(Z, A, B, Aij, Bi, c)


def state_from_molar(mix: Mixture, T: float, n):
    """Thermodynamic state of one homogeneous cell from molar densities n_i:
    p from Eq. (MCPengRobinson), Z = p/(rho~ R T) (no root choice), c_i, ln(phi_i)
    from Eq. (fugacitycoeff2) and fugacities f_i = phi_i c_i p (Eq. (fugacity))."""
    n = np.asarray(n, dtype=np.float64)
    rho_t = float(n.sum())
    c = n / rho_t
    p = float(pressure_molar(n, T, mix))
    Z = p / (rho_t * mix.R * T)
    A, B, Aij, Bi = cubic_AB(mix, T, p, c)
    lphi = ln_phi(Z, A, B, Aij, Bi, c)
    fug = np.exp(lphi) * c * p
    return {"p": p, "Z": Z, "c": c, "lnphi": lphi, "fug": fug}


def fugacity(mix: Mixture, T: float, p: float, c, root="gibbs"):
    """f_i = phi_i c_i p, Eq. (fugacity)."""
    Z, lphi = phase_state(mix, T, p, c, root)
    return np.exp(lphi) * np.asarray(c) * p


def iso_fugacity_residual(f_l, f_v) -> float:
    """sum_i (f_li / f_vi - 1)^2, Eq. (error)."""
    f_l = np.asarray(f_l)
    f_v = np.asarray(f_v)
    return float(np.sum((f_l / f_v - 1.0) ** 2))


# ---------------------------------------------------------------------------
# Two-phase flash and derived quantities
# ---------------------------------------------------------------------------

def wilson_K(mix: Mixture, T: float, p: float):
    """Wilson's correlation, the usual starting K for a flash."""
    return mix.pc / p * np.exp(5.373 * (1.0 + mix.omega) * (1.0 - mix.Tc / T))


def rachford_rice(z, K):
    """Vapor mole fraction V solving sum_i z_i (K_i - 1) / (1 + V (K_i - 1)) = 0.

    Plain bisection on the open bracket (1/(1-Kmax), 1/(1-Kmin)) where the function
    is monotone decreasing; run until the bracket stops shrinking.
    """
    z = np.asarray(z, dtype=np.float64)
    K = np.asarray(K, dtype=np.float64)
    kmax, kmin = K.max(), K.min()
    if not (kmax > 1.0 and kmin < 1.0):
        raise ValueError("Rachford-Rice has no two-phase bracket")
    lo = 1.0 / (1.0 - kmax)
    hi = 1.0 / (1.0 - kmin)

    def g(V):
        return float(np.sum(z * (K - 1.0) / (1.0 + V * (K - 1.0))))

    for _ in range(2000):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if g(mid) > 0.0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


@dataclass
class FlashResult:
    T: float
    p: float
    z: np.ndarray
    V: float
    x: np.ndarray
    y: np.ndarray
    K: np.ndarray
    Zl: float
    Zv: float
    rho_l: float          # molar density of the liquid phase
    rho_v: float          # molar density of the vapor phase
    rbar_l: np.ndarray    # cell-volume (mass) densities of each component in the liquid
    rbar_v: np.ndarray    # ... in the vapor
    gamma: np.ndarray
    residual: float
    iterations: int
    fug_l: np.ndarray = field(default=None)
    fug_v: np.ndarray = field(default=None)


class SinglePhase(Exception):
    pass


def flash(mix: Mixture, T: float, p: float, z, tol: float = 1e-13, max_iter: int = 20000) -> FlashResult:
    """Two-phase flash at (T, p, z) by successive substitution (the paper gives no
    algorithm, end of Sec. 3.2): K <- phi_l / phi_v with Z chosen per phase by the
    Gibbs criterion; the phase split V by Rachford-Rice."""
    z = np.asarray(z, dtype=np.float64)
    K = wilson_K(mix, T, p)
    it = 0
    for it in range(1, max_iter + 1):
        V = rachford_rice(z, K)
        x = z / (1.0 + V * (K - 1.0))
        y = K * x
        x = x / x.sum()
        y = y / y.sum()
        _, lphi_l = phase_state(mix, T, p, x)
        _, lphi_v = phase_state(mix, T, p, y)
        lnK_new = lphi_l - lphi_v
        dlnK = np.max(np.abs(lnK_new - np.log(K)))
        K = np.exp(lnK_new)
        if np.max(np.abs(lnK_new)) < 1e-6:
            raise SinglePhase("flash converged to the trivial solution")
        if dlnK < tol:
            break
    V = rachford_rice(z, K)
    if not (0.0 < V < 1.0):
        raise SinglePhase(f"vapor fraction {V} outside (0, 1)")
    x = z / (1.0 + V * (K - 1.0))
    y = K * x
    x = x / x.sum()
    y = y / y.sum()
    Zl, lphi_l = phase_state(mix, T, p, x)
    Zv, lphi_v = phase_state(mix, T, p, y)
    rho_l = p / (Zl * mix.R * T)
    rho_v = p / (Zv * mix.R * T)
    # Sec. 2.2: rbar_{i,l} = rho_l x_i M_i / sum_j x_j M_j with rho_l the mass density,
    # i.e. (molar density) * x_i * M_i.
    rbar_l = rho_l * x * mix.M
    rbar_v = rho_v * y * mix.M
    fug_l = np.exp(lphi_l) * x * p
    fug_v = np.exp(lphi_v) * y * p
    res = FlashResult(T=T, p=p, z=z, V=V, x=x, y=y, K=y / x, Zl=Zl, Zv=Zv,
                      rho_l=rho_l, rho_v=rho_v, rbar_l=rbar_l, rbar_v=rbar_v,
                      gamma=gamma_from_phases(rbar_l, rbar_v, y / x),
                      residual=iso_fugacity_residual(fug_l, fug_v), iterations=it,
                      fug_l=fug_l, fug_v=fug_v)
    return res


def gamma_from_phases(rbar_l, rbar_v, K):
    """Volatility coefficients, Eq. (gamma): gamma_i = ln(rbar_il/rbar_iv) /
    ln(rbar_ref,l / rbar_ref,v) with ref the least volatile component (smallest K),
    for which gamma = 1 (Sec. 3.1)."""
    rbar_l = np.asarray(rbar_l)
    rbar_v = np.asarray(rbar_v)
    ref = int(np.argmin(K))
    return np.log(rbar_l / rbar_v) / math.log(rbar_l[ref] / rbar_v[ref])


def bubble_pressure(mix: Mixture, T: float, z, p0=None, tol=1e-13, max_iter=20000):
    """Bubble-point pressure: liquid of composition z in equilibrium with an incipient
    vapor.  Successive substitution on K and on p (p <- p * sum_i K_i z_i)."""
    z = np.asarray(z, dtype=np.float64)
    p = float(np.sum(z * mix.pc * np.exp(5.373 * (1 + mix.omega) * (1 - mix.Tc / T)))) if p0 is None else p0
    K = wilson_K(mix, T, p)
    for _ in range(max_iter):
        y = K * z / np.sum(K * z)
        _, lphi_l = phase_state(mix, T, p, z)
        _, lphi_v = phase_state(mix, T, p, y)
        K = np.exp(lphi_l - lphi_v)
        S = float(np.sum(K * z))
        p_new = p * S
        if abs(S - 1.0) < tol:
            return p_new
        p = p_new
    raise RuntimeError("bubble-point iteration did not converge")


def dew_pressure(mix: Mixture, T: float, z, p0=None, tol=1e-13, max_iter=20000):
    """Dew-point pressure: vapor of composition z with an incipient liquid.
    Successive substitution on K and on p (p <- p / sum_i z_i / K_i)."""
    z = np.asarray(z, dtype=np.float64)
    if p0 is None:
        Kw = wilson_K(mix, T, 1.0)
        p = 1.0 / float(np.sum(z / Kw))
    else:
        p = p0
    K = wilson_K(mix, T, p)
    for _ in range(max_iter):
        x = z / K / np.sum(z / K)
        _, lphi_l = phase_state(mix, T, p, x)
        _, lphi_v = phase_state(mix, T, p, z)
        K = np.exp(lphi_l - lphi_v)
        S = float(np.sum(z / K))
        p_new = p / S
        if abs(S - 1.0) < tol:
            return p_new
        p = p_new
    raise RuntimeError("dew-point iteration did not converge")


# ---------------------------------------------------------------------------
# Pure-substance coexistence (Sec. 3.2: Maxwell rule as the pure case of iso-fugacity)
# ---------------------------------------------------------------------------

def _three_root_interval(mix1: Mixture, T: float):
    """Pressure interval in which the pure cubic has three roots above B (scan)."""
    pc = float(mix1.pc[0])
    ps = np.linspace(1e-6 * pc, pc, 4001)
    three = [p for p in ps if len(cubic_roots(*cubic_AB(mix1, T, p, [1.0])[:2])) == 3]
    return min(three), max(three)


def maxwell_by_fugacity(mix1: Mixture, T: float):
    """Saturation pressure of a pure component where the liquid and vapor roots have
    equal ln(phi) (dG = 0 of Eq. (solutionselection)); returns (p, rho_l, rho_v) with
    molar densities."""
    from scipy.optimize import brentq

    def dG(p):
        A, B, _, _ = cubic_AB(mix1, T, p, [1.0])
        r = cubic_roots(A, B)
        return gibbs_difference(r[-1], r[0], A, B)

    lo, hi = _three_root_interval(mix1, T)
    p = brentq(dG, lo, hi, xtol=1e-16, rtol=1e-15, maxiter=500)
    A, B, _, _ = cubic_AB(mix1, T, p, [1.0])
    r = cubic_roots(A, B)
    R = mix1.R
    return p, p / (r[0] * R * T), p / (r[-1] * R * T)


def maxwell_equal_area(a: float, b: float, omega: float, T: float, Rs: float = 1.0):
    """Maxwell equal-area construction on the pure EOS in mass density,
    Eq. (SCpengrobinson): find p with integral_{v_l}^{v_v} (p_EOS(v) - p) dv = 0.
    Independent of the fugacity formulas (quadrature of the EOS itself)."""
    from scipy.integrate import quad
    from scipy.optimize import brentq

    def p_of_v(v):
        return pure_pressure_mass(1.0 / v, T, a, b, omega, Rs)

    Tc = (OMEGA_B / OMEGA_A) * a / (b * Rs)
    # locate the spinodals on a fine density grid
    rho = np.linspace(1e-4, 0.999 / b, 200001)
    pr = pure_pressure_mass(rho, T, a, b, omega, Rs)
    dp = np.diff(pr)
    i_max = int(np.argmax(dp < 0))                  # first local max (vapor spinodal)
    i_min = i_max + int(np.argmax(dp[i_max:] > 0))  # following local min
    p_hi = pr[i_max]
    p_lo = max(pr[i_min], 2.0 * pr[0])   # keep the vapor root inside the grid

    def roots_at(p):
        sign = np.sign(pr - p)
        idx = np.nonzero(np.diff(sign))[0]
        rts = []
        for i in idx:
            rts.append(brentq(lambda r: pure_pressure_mass(r, T, a, b, omega, Rs) - p,
                              rho[i], rho[i + 1], xtol=1e-15, rtol=1e-15))
        return rts

    def area(p):
        rts = roots_at(p)
        rv, rl = rts[0], rts[-1]
        val, _ = quad(lambda v: p_of_v(v) - p, 1.0 / rl, 1.0 / rv, limit=400,
                      epsabs=1e-14, epsrel=1e-13)
        return val

    eps = 1e-9 * (p_hi - p_lo)
    p = brentq(area, p_lo + eps, p_hi - eps, xtol=1e-15, rtol=1e-15)
    rts = roots_at(p)
    del Tc
    return p, rts[-1], rts[0]
