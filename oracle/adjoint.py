"""Discrete adjoint of the LB step and gradient of a phase-composition loss,
plain float64 on the CPU (oracle; test infrastructure only).

The forward map is the step of ``oracle.lbm`` (Sec. 3.4 order of operations,
Eq. (LBE) of Sec. 2.1) written once more over torch tensors, so that torch's
reverse-mode differentiation yields the exact derivative of the discrete map (the
discrete adjoint).  A tensor library's automatic differentiation is used here as
a primitive, the way a matmul would be; the forward it differentiates is pinned
to the NumPy step, and the gradient to central differences of the NumPy oracle.

Parameters (reading; the paper does not differentiate the model):
  theta = (k_ij for i < j in row-major order, a_1..a_nc, b_1..b_nc).
  alpha_i = alpha(T / Tc_i) follows a_i and b_i through Tc_i = (Omega_b/Omega_a)
  a_i / (b_i R) (Sec. 3.2), so a derivative in a or b includes the one through
  alpha.  M_i, omega_i, T, gamma_i and the initial fields are held fixed.

Loss (reading): L = sum_i (x_i - x_i^tgt)^2 with x_i = N_i / sum_j N_j,
N_i = sum over a fixed cell mask of rbar_i / M_i, from the post-streaming
populations after the last step (the liquid mask of a drop is r <= R0/2).

Solid walls (prm.solid, prm.psi_wall) follow oracle.lbm: solid cells hold no fluid,
carry psi_w, and streaming bounces back; their EOS, force split and velocity are
evaluated on harmless stand-in values and masked, so that no NaN reaches the
reverse pass.

Pins (tests/test_oracle_adjoint.py): the torch step equals the NumPy step (with and
without walls); the gradient equals central differences of the NumPy oracle's
loss; forward- and reverse-mode products satisfy the dot-product identity; L and
its gradient vanish when the target is the reached composition.
"""
from __future__ import annotations

import numpy as np
import torch

from . import thermo
from .lattice import CS2, VelocitySet, mrt_basis
from .lbm import opposite

DT = torch.float64


# ---------------------------------------------------------------------------
# parameters
# ---------------------------------------------------------------------------

def pair_index(nc: int):
    """(i, j) pairs with i < j in row-major order: the k entries of theta."""
    return [(i, j) for i in range(nc) for j in range(i + 1, nc)]


def theta_of(mix: thermo.Mixture) -> np.ndarray:
    nc = mix.nc
    k = [mix.k[i, j] for i, j in pair_index(nc)]
    return np.concatenate([np.asarray(k, dtype=np.float64), mix.a, mix.b])


def mixture_of(theta, base: thermo.Mixture) -> thermo.Mixture:
    """NumPy mixture with theta's k, a, b and base's omega, M, R."""
    theta = np.asarray(theta, dtype=np.float64)
    nc = base.nc
    npair = nc * (nc - 1) // 2
    k = np.zeros((nc, nc))
    for v, (i, j) in zip(theta[:npair], pair_index(nc)):
        k[i, j] = k[j, i] = v
    return thermo.Mixture(a=theta[npair:npair + nc].copy(), b=theta[npair + nc:].copy(),
                          omega=base.omega, M=base.M, k=k, R=base.R)


def eos_tables(theta: torch.Tensor, base: thermo.Mixture, T: float):
    """(aalpha)_ij (1 - k_ij) and b_i as torch functions of theta (Sec. 3.2,
    Eq. (randommixingrule))."""
    nc = base.nc
    npair = nc * (nc - 1) // 2
    a = theta[npair:npair + nc]
    b = theta[npair + nc:]
    Tc = (thermo.OMEGA_B / thermo.OMEGA_A) * a / (b * base.R)
    m = torch.as_tensor(thermo.m_of_omega(base.omega), dtype=DT)
    alpha = (1.0 + m * (1.0 - torch.sqrt(T / Tc))) ** 2
    aal = a * alpha
    one_minus_k = [[None] * nc for _ in range(nc)]
    for i in range(nc):
        one_minus_k[i][i] = torch.ones((), dtype=DT)
    for v, (i, j) in zip(theta[:npair], pair_index(nc)):
        one_minus_k[i][j] = 1.0 - v
        one_minus_k[j][i] = 1.0 - v
    rows = [torch.stack([torch.sqrt(aal[i] * aal[j]) * one_minus_k[i][j] for j in range(nc)])
            for i in range(nc)]
    return torch.stack(rows), b


# ---------------------------------------------------------------------------
# forward step over torch tensors (same operations as oracle.lbm.step)
# ---------------------------------------------------------------------------

def _axis(d: int, nspace: int, lead: int) -> int:
    return lead + (nspace - 1 - d)


def shift(a: torch.Tensor, e, lead: int) -> torch.Tensor:
    """b(x) = a(x - e), periodic."""
    nspace = a.dim() - lead
    out = a
    for d, ed in enumerate(e):
        if ed != 0:
            out = torch.roll(out, int(ed), dims=_axis(d, nspace, lead))
    return out


def pressure(rho_s, T, aa, b, M, R):
    """Eq. (MCPengRobinson) with the random mixing rule, molar densities rbar/M."""
    n = rho_s / torch.as_tensor(M, dtype=DT).reshape((-1,) + (1,) * (rho_s.dim() - 1))
    rho_t = n.sum(dim=0)
    c = n / rho_t
    am = torch.einsum("i...,j...,ij->...", c, c, aa)
    bm = torch.einsum("i...,i->...", c, b)
    return rho_t * R * T / (1.0 - bm * rho_t) - am * rho_t ** 2 / (1.0 + 2.0 * bm * rho_t - (bm * rho_t) ** 2)


def equilibrium(rho_sig, u, lat: VelocitySet):
    uu = (u * u).sum(dim=0)
    out = []
    for a in range(lat.Q):
        eu = sum(float(lat.e[a, d]) * u[d] for d in range(lat.D))
        out.append(rho_sig * lat.w[a] * (1.0 + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2)))
    return torch.stack(out)


def guo_shape(F_sig, u, lat: VelocitySet):
    out = []
    for a in range(lat.Q):
        eu = sum(float(lat.e[a, d]) * u[d] for d in range(lat.D))
        acc = 0.0
        for d in range(lat.D):
            acc = acc + ((float(lat.e[a, d]) - u[d]) / CS2 + eu * float(lat.e[a, d]) / (CS2 * CS2)) * F_sig[d]
        out.append(lat.w[a] * acc)
    return torch.stack(out)


def step(f, aa, b, base: thermo.Mixture, prm, lat: VelocitySet):
    """One step (prm: oracle.lbm.StepParams); f[sigma, alpha, *space] post-streaming."""
    N = f.shape[0]
    D = lat.D
    gshape = (-1,) + (1,) * (f.dim() - 2)
    solid = None if getattr(prm, "solid", None) is None else torch.as_tensor(np.asarray(prm.solid, dtype=bool))
    if solid is not None:
        f = torch.where(solid, torch.zeros((), dtype=DT), f)       # solid cells hold no fluid
    rho_s = f.sum(dim=1)
    rho = rho_s.sum(dim=0)
    j = torch.stack([sum(float(lat.e[a, d]) * f[s, a] for s in range(N) for a in range(lat.Q)
                         if lat.e[a, d] != 0) for d in range(D)])
    rho_eos = rho_s if solid is None else torch.where(solid, torch.full((), 1e-3, dtype=DT), rho_s)
    p = pressure(rho_eos, prm.T, aa, b, base.M, base.R)
    X = 2.0 * (p - CS2 * rho_eos.sum(dim=0)) / (prm.G * CS2)
    psi = torch.sqrt(X)
    if solid is not None:
        psi = torch.where(solid, torch.full((), float(prm.psi_wall), dtype=DT), psi)
        rho = torch.where(solid, torch.ones((), dtype=DT), rho)    # u = j / rho = 0 there
    F = [torch.zeros_like(psi) for _ in range(D)]
    for a in range(1, lat.Q):
        e = lat.e[a]
        psi_n = shift(psi, -e, lead=0)
        for d in range(D):
            if e[d] != 0:
                F[d] = F[d] + (-prm.beta * prm.G * psi * lat.w[a] * psi_n * float(e[d])
                               - 0.5 * (1.0 - prm.beta) * prm.G * lat.w[a] * psi_n * psi_n * float(e[d]))
    F = torch.stack(F)
    gamma = torch.as_tensor(np.asarray(prm.gamma, dtype=np.float64), dtype=DT)
    Gam = (gamma.reshape(gshape) * rho_s).sum(dim=0)
    if solid is not None:
        Gam = torch.where(solid, torch.ones((), dtype=DT), Gam)
    g = np.zeros(D) if prm.accel is None else np.asarray(prm.accel, dtype=np.float64)
    F_s = torch.stack([torch.stack([gamma[s] * rho_s[s] / Gam * F[d] + rho_s[s] * float(g[d])
                                    for d in range(D)]) for s in range(N)])
    u = (j + 0.5 * F_s.sum(dim=0)) / rho        # barycentric velocity (both forcings)
    if prm.collision == "mrt":
        Mx = mrt_basis(lat)
        Minv = np.linalg.inv(Mx)
        S = np.diag(np.asarray(prm.mrt_s, dtype=np.float64))
        relax = torch.as_tensor(Minv @ S @ Mx, dtype=DT)
        guo_mat = torch.as_tensor(Minv @ (np.eye(lat.Q) - 0.5 * S) @ Mx, dtype=DT)
    posts = []
    for s in range(N):
        if prm.forcing == "edm":       # jump du_s, equilibrium velocity U - du_s / 2 (oracle.lbm)
            du = torch.stack([gamma[s] * F[d] / Gam + float(g[d]) for d in range(D)])
            ueq = u - 0.5 * du
        else:
            ueq = u
        feq = equilibrium(rho_s[s], ueq, lat)
        if prm.collision == "bgk":
            post = f[s] - (f[s] - feq) / prm.tau
        else:
            post = f[s] - torch.tensordot(relax, f[s] - feq, dims=([1], [0]))
        if prm.forcing == "guo":
            shape = guo_shape(F_s[s], u, lat)
            if prm.collision == "bgk":
                post = post + (1.0 - 0.5 / prm.tau) * shape
            else:
                post = post + torch.tensordot(guo_mat, shape, dims=([1], [0]))
        else:
            post = post + equilibrium(rho_s[s], ueq + du, lat) - feq
        posts.append(post)
    fstar = torch.stack(posts)
    if solid is None:
        return torch.stack([torch.stack([shift(fstar[s, a], lat.e[a], lead=0) for a in range(lat.Q)])
                            for s in range(N)])
    # halfway bounce-back: a fluid cell whose source x - e_a is solid receives its
    # own opposite post-collision population; solid cells receive nothing
    opp = opposite(lat)
    zero = torch.zeros((), dtype=DT)
    out = []
    for s in range(N):
        row = []
        for a in range(lat.Q):
            from_wall = shift(solid, lat.e[a], lead=0) & ~solid
            v = torch.where(from_wall, fstar[s, opp[a]], shift(fstar[s, a], lat.e[a], lead=0))
            row.append(torch.where(solid, zero, v))
        out.append(torch.stack(row))
    return torch.stack(out)


# ---------------------------------------------------------------------------
# loss and gradients
# ---------------------------------------------------------------------------

def mole_fractions(f, M, mask):
    """x_i over the mask from post-streaming populations."""
    rho_s = f.sum(dim=1)
    n = rho_s / torch.as_tensor(M, dtype=DT).reshape((-1,) + (1,) * (rho_s.dim() - 1))
    m = torch.as_tensor(mask, dtype=torch.bool)
    Ni = torch.stack([n[i][m].sum() for i in range(n.shape[0])])
    return Ni / Ni.sum()


def loss_of_state(f, M, mask, x_tgt):
    x = mole_fractions(f, M, mask)
    return ((x - torch.as_tensor(x_tgt, dtype=DT)) ** 2).sum()


def run_loss(theta, f0, base, prm, lat, nsteps, mask, x_tgt):
    """L(theta) after nsteps from the populations f0 (torch scalar)."""
    aa, b = eos_tables(theta, base, prm.T)
    f = torch.as_tensor(f0, dtype=DT)
    for _ in range(nsteps):
        f = step(f, aa, b, base, prm, lat)
    return loss_of_state(f, base.M, mask, x_tgt)


def gradient(theta, f0, base, prm, lat, nsteps, mask, x_tgt):
    """(L, dL/dtheta) as float and NumPy array."""
    th = torch.tensor(np.asarray(theta, dtype=np.float64), dtype=DT, requires_grad=True)
    L = run_loss(th, f0, base, prm, lat, nsteps, mask, x_tgt)
    (g,) = torch.autograd.grad(L, th)
    return float(L.detach()), g.numpy()


def step_vjp(f, fbar_next, theta, base, prm, lat):
    """Reverse product of one step at state f: given the adjoint of the
    post-streaming populations after the step, return the adjoint of f and the
    step's contribution to dL/dtheta (NumPy arrays)."""
    ft = torch.tensor(np.asarray(f, dtype=np.float64), dtype=DT, requires_grad=True)
    th = torch.tensor(np.asarray(theta, dtype=np.float64), dtype=DT, requires_grad=True)
    aa, b = eos_tables(th, base, prm.T)
    out = step(ft, aa, b, base, prm, lat)
    gf, gt = torch.autograd.grad(out, (ft, th), grad_outputs=torch.as_tensor(fbar_next, dtype=DT))
    return gf.numpy(), gt.numpy()


def step_vjp_tables(f, fbar_next, aa, b, base, prm, lat):
    """As step_vjp, but the parameter adjoint is returned for the EOS tables
    themselves: (fbar, d/d aa_ij as an nc x nc array over ordered pairs, d/d b_i)."""
    ft = torch.tensor(np.asarray(f, dtype=np.float64), dtype=DT, requires_grad=True)
    aat = torch.tensor(np.asarray(aa, dtype=np.float64), dtype=DT, requires_grad=True)
    bt = torch.tensor(np.asarray(b, dtype=np.float64), dtype=DT, requires_grad=True)
    out = step(ft, aat, bt, base, prm, lat)
    gf, ga, gb = torch.autograd.grad(out, (ft, aat, bt), grad_outputs=torch.as_tensor(fbar_next, dtype=DT))
    return gf.numpy(), ga.numpy(), gb.numpy()


def step_jvp(f, df, dtheta, theta, base, prm, lat):
    """Forward product of one step: directional derivative of the post-streaming
    populations along (df, dtheta)."""
    def fn(ft, th):
        aa, b = eos_tables(th, base, prm.T)
        return step(ft, aa, b, base, prm, lat)
    _, out = torch.func.jvp(fn, (torch.as_tensor(f, dtype=DT), torch.as_tensor(theta, dtype=DT)),
                            (torch.as_tensor(df, dtype=DT), torch.as_tensor(dtheta, dtype=DT)))
    return out.numpy()
