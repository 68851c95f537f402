"""Seeded test cases: a mixture in a two-phase state (flashed by the oracle) laid
out as a noisy drop.  Shared by the GPU parity tests (test infrastructure)."""
import numpy as np

from oracle import lattice as olat
from oracle import lbm as olbm
from oracle import thermo as oth
from oracle_backend import BACKEND, to_mixture
from paper_1909_12390_amd import inputs

LAT = {"D2Q9": olat.d2q9(), "D3Q19": olat.d3q19()}


def pure_water_mix():
    # Sec. 4.1 limiting-case fluid: a = 2/49, b = 2/21, R = 1, acentric factor 0.344
    return {"a": np.array([2 / 49]), "b": np.array([2 / 21]), "omega": np.array([0.344]),
            "M": np.array([1.0]), "k": np.zeros((1, 1)), "R": 1.0}


def case(lattice, nc, shape, seed=0, noise=1e-3, u_amp=0.0):
    rng = inputs.rng_for(100 + nc, seed)
    if nc == 1:
        mix = pure_water_mix()
        m = to_mixture(mix)
        T = 0.9 * m.Tc[0]
        _, rl, rv = oth.maxwell_by_fugacity(m, T)
        rbar_l, rbar_v, gamma = np.array([rl]), np.array([rv]), np.array([1.0])
    else:
        mix, T, z, p, fl = inputs.pick_state(rng, BACKEND, nc, 0.7, 0.95, 0.05, {})
        rbar_l, rbar_v, gamma = fl.rbar_l, fl.rbar_v, fl.gamma
    R0 = min(shape) / 4.0
    rho0 = inputs.drop_profile(shape, R0, 4.0, rbar_l, rbar_v)
    rho0 = rho0 * inputs.multiplicative_noise(inputs.rng_for(200 + nc, seed), rho0.shape, noise)
    D = 2 if lattice == "D2Q9" else 3
    u0 = None
    if u_amp > 0:
        u0 = u_amp * inputs.rng_for(300 + nc, seed).uniform(-1, 1, (D,) + tuple(shape))
    return {"mix": mix, "T": T, "gamma": np.asarray(gamma), "rho0": rho0, "u0": u0, "shape": tuple(shape)}


def mrt_rates(lattice, tau):
    return inputs.default_mrt_rates(lattice, tau) * np.linspace(0.97, 1.03, 9 if lattice == "D2Q9" else 19)


def oracle_params(c, collision, forcing, tau=0.8, beta=1.7, mrt_s=None, accel=None):
    return olbm.StepParams(T=c["T"], tau=tau, gamma=c["gamma"], beta=beta, collision=collision,
                           forcing=forcing, mrt_s=mrt_s, accel=accel)


def oracle_run(c, lattice, prm, steps):
    lat = LAT[lattice]
    mix = to_mixture(c["mix"])
    f = olbm.init_populations(c["rho0"], lat, c["u0"])
    out = [f]
    for _ in range(steps):
        f = olbm.step(f, mix, prm, lat)
        out.append(f)
    return out
