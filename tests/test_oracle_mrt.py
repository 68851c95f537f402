"""Pins of the oracle's MRT collision at the rates the benchmark configurations use
(``inputs.default_mrt_rates``: shear and component-momentum rows at 1/tau, energy
rows at 0.5, the others at 1).

MRT is not in the paper; what its rates must deliver is fixed by hydrodynamics:
  * a shear wave decays as exp(-nu k^2 t) with nu = c_s^2 (1/s_nu - 1/2), the BGK
    viscosity at s_nu = 1/tau -- one wave per independent shear row (D2Q9: p_xy
    and, on the diagonal, p_xx; D3Q19: p_xy, p_yz, p_xz and the two normal-stress
    rows through the xy and yz diagonals);
  * a composition wave between two identical components (uniform total density,
    hence uniform psi and zero force) decays as exp(-D k^2 t) with the
    inter-diffusion coefficient D = c_s^2 (1/s_j - 1/2) of the component momentum
    rows, one wave per axis.
The measured coefficients must equal (tau - 1/2)/3 to 1e-3 relative (lattice
corrections at these wavelengths are ~1e-4).  A rate attached to the wrong moment
row, or two basis rows swapped, changes one of them by tens of per cent.
"""
import numpy as np
import pytest

from oracle import lattice as L
from oracle import lbm, thermo
from paper_1909_12390_amd.inputs import default_mrt_rates

TAU = 0.8
NU = (TAU - 0.5) / 3.0


def _positions(lat, shape):
    grids = np.meshgrid(*[np.arange(n, dtype=float) for n in shape], indexing="ij")
    return [grids[lat.D - 1 - d] for d in range(lat.D)]      # velocity component d lives on axis D-1-d


def _decay_rate(lat, mix, rho, u, phase, k2, measure, n1=60, n2=460, forcing="guo"):
    f = lbm.init_populations(rho, lat, u)
    prm = lbm.StepParams(T=0.8 * float(np.min(mix.Tc)), tau=TAU, gamma=np.ones(mix.nc), beta=1.5,
                         collision="mrt", forcing=forcing, mrt_s=default_mrt_rates(lat.name, TAU))
    amp = {}
    for t in range(n2 + 1):
        if t in (n1, n2):
            amp[t] = measure(f, prm)
        if t < n2:
            f = lbm.step(f, mix, prm, lat)
    return -np.log(amp[n2] / amp[n1]) / (k2 * (n2 - n1))


SHEAR = [  # (lattice, shape (array axes), velocity direction, wave vector in units of 2 pi / n)
    ("D2Q9", (96, 1), (1, 0), (0, 1)),              # p_xy
    ("D2Q9", (48, 48), (1, -1), (1, 1)),             # p_xx (normal-stress difference)
    ("D3Q19", (1, 96, 1), (1, 0, 0), (0, 1, 0)),     # p_xy
    ("D3Q19", (96, 1, 1), (0, 1, 0), (0, 0, 1)),     # p_yz
    ("D3Q19", (1, 1, 96), (0, 0, 1), (1, 0, 0)),     # p_xz
    ("D3Q19", (1, 48, 48), (1, -1, 0), (1, 1, 0)),   # xx - yy: 3 p_xx and p_ww rows
    ("D3Q19", (48, 48, 1), (0, 1, -1), (0, 1, 1)),   # yy - zz: p_ww row
]


@pytest.mark.parametrize("latname,shape,uvec,kvec", SHEAR)
def test_shear_wave_viscosity(latname, shape, uvec, kvec):
    lat = L.d2q9() if latname == "D2Q9" else L.d3q19()
    mix = thermo.Mixture(a=[2 / 49], b=[2 / 21], omega=[0.2], M=[1.0], k=[[0.0]], R=1.0)
    n = max(shape)
    kv = 2 * np.pi / n * np.asarray(kvec, dtype=float)
    pos = _positions(lat, shape)
    phase = sum(kv[d] * pos[d] for d in range(lat.D))
    uhat = np.asarray(uvec, dtype=float) / np.linalg.norm(uvec)
    u = np.stack([1e-3 * uhat[d] * np.sin(phase) for d in range(lat.D)])
    rho = np.full((1,) + tuple(shape), 0.3)            # uniform vapour: uniform psi, F = 0

    def measure(f, prm):
        m = lbm.macroscopic(f, mix, prm, lat)
        ul = sum(uhat[d] * m["u"][d] for d in range(lat.D))
        return 2.0 * np.mean(ul * np.sin(phase))

    nu = _decay_rate(lat, mix, rho, u, phase, float(kv @ kv), measure)
    assert abs(nu / NU - 1.0) < 1e-3, (nu, NU)


DIFFUSION = [("D2Q9", (96, 1), (0, 1)), ("D2Q9", (1, 96), (1, 0)),
             ("D3Q19", (1, 1, 96), (1, 0, 0)), ("D3Q19", (1, 96, 1), (0, 1, 0)), ("D3Q19", (96, 1, 1), (0, 0, 1))]


@pytest.mark.parametrize("latname,shape,kvec", DIFFUSION)
@pytest.mark.parametrize("forcing", ["guo", "edm"])
def test_interdiffusion_coefficient(latname, shape, kvec, forcing):
    lat = L.d2q9() if latname == "D2Q9" else L.d3q19()
    mix = thermo.Mixture(a=[2 / 49] * 2, b=[2 / 21] * 2, omega=[0.2] * 2, M=[1.0] * 2,
                         k=[[0.0, 0.0], [0.0, 0.0]], R=1.0)
    n = max(shape)
    kv = 2 * np.pi / n * np.asarray(kvec, dtype=float)
    pos = _positions(lat, shape)
    phase = sum(kv[d] * pos[d] for d in range(lat.D))
    rho = np.stack([0.15 * (1 + 0.01 * np.sin(phase)), 0.15 * (1 - 0.01 * np.sin(phase))])

    def measure(f, prm):
        r = lbm.densities(f)
        return 2.0 * np.mean((r[0] - r[1]) * np.sin(phase))

    D = _decay_rate(lat, mix, rho, None, phase, float(kv @ kv), measure, forcing=forcing)
    assert abs(D / NU - 1.0) < 1e-3, (D, NU)
