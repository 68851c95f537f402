"""Adapter exposing oracle.thermo through the backend interface of
paper_1909_12390_amd.inputs (test infrastructure)."""
import numpy as np

from oracle import thermo


def to_mixture(mix):
    return thermo.Mixture(a=mix["a"], b=mix["b"], omega=mix["omega"], M=mix["M"],
                          k=mix["k"], R=mix["R"])


class OracleThermo:
    def critical_temperature(self, mix):
        return to_mixture(mix).Tc

    def bubble_pressure(self, mix, T, z):
        return thermo.bubble_pressure(to_mixture(mix), T, z)

    def dew_pressure(self, mix, T, z):
        return thermo.dew_pressure(to_mixture(mix), T, z)

    def flash(self, mix, T, p, z):
        return thermo.flash(to_mixture(mix), T, p, z)

    def pressure(self, mix, T, n):
        m = to_mixture(mix)
        n = np.atleast_2d(np.asarray(n, dtype=np.float64))
        p = thermo.pressure_molar(n.T, T, m)
        inside = (n @ m.b) < 1.0
        return np.where(inside, p, np.nan)


BACKEND = OracleThermo()
