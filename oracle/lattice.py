"""Velocity sets and MRT moment bases (oracle; test infrastructure only).

The paper does not name its velocity set (Sec. 2.1 speaks only of "weighting
factors").  Reading: the standard D2Q9 and D3Q19 sets with c_s^2 = 1/3, and the
same weights w_alpha in the equilibrium and in the force stencil, which is what
makes the hydrodynamic pressure of Eq. (hydropressure) come out (the stencil's
second moment sum_alpha w_alpha e_alpha e_alpha equals c_s^2 I).

MRT is not in the paper.  Its bases are the orthogonal polynomial sets of
Lallemand & Luo (2000) for D2Q9 and d'Humieres et al. (2002) for D3Q19, built
here directly from their defining polynomials in the velocity components.

Pins: tests/test_oracle_lbm.py checks the isotropy moments of each set
(sum w = 1, sum w e = 0, sum w e e = c_s^2 I, sum w e e e = 0, fourth moment
c_s^4 (d_ij d_kl + d_ik d_jl + d_il d_jk)) and the mutual orthogonality of the
MRT rows; tests/test_oracle_mrt.py checks what the rates attached to the rows
deliver: the shear viscosity of every shear row and the inter-diffusion
coefficient of the component momentum rows.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

CS2 = 1.0 / 3.0


@dataclass(frozen=True)
class VelocitySet:
    name: str
    D: int
    e: np.ndarray      # (Q, D) integer velocities
    w: np.ndarray      # (Q,)

    @property
    def Q(self) -> int:
        return int(self.e.shape[0])


def d2q9() -> VelocitySet:
    e = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1],
                  [1, 1], [-1, 1], [-1, -1], [1, -1]], dtype=np.int64)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    return VelocitySet("D2Q9", 2, e, w)


def d3q19() -> VelocitySet:
    e = [[0, 0, 0],
         [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
         [1, 1, 0], [-1, 1, 0], [1, -1, 0], [-1, -1, 0],
         [1, 0, 1], [-1, 0, 1], [1, 0, -1], [-1, 0, -1],
         [0, 1, 1], [0, -1, 1], [0, 1, -1], [0, -1, -1]]
    e = np.array(e, dtype=np.int64)
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    return VelocitySet("D3Q19", 3, e, w)


def mrt_basis(lat: VelocitySet) -> np.ndarray:
    """Rows of the moment matrix M (Q x Q), orthogonal under the plain dot product."""
    e = lat.e.astype(np.float64)
    if lat.D == 2:
        ex, ey = e[:, 0], e[:, 1]
        e2 = ex * ex + ey * ey
        rows = [np.ones_like(ex),                    # rho
                -4.0 + 3.0 * e2,                     # e (energy)
                4.0 - 10.5 * e2 + 4.5 * e2 * e2,     # epsilon (energy squared)
                ex,                                  # j_x
                (-5.0 + 3.0 * e2) * ex,              # q_x
                ey,                                  # j_y
                (-5.0 + 3.0 * e2) * ey,              # q_y
                ex * ex - ey * ey,                   # p_xx
                ex * ey]                             # p_xy
    else:
        ex, ey, ez = e[:, 0], e[:, 1], e[:, 2]
        e2 = ex * ex + ey * ey + ez * ez
        rows = [np.ones_like(ex),                             # rho
                19.0 * e2 - 30.0,                             # e
                (21.0 * e2 * e2 - 53.0 * e2 + 24.0) / 2.0,    # epsilon
                ex, (5.0 * e2 - 9.0) * ex,                    # j_x, q_x
                ey, (5.0 * e2 - 9.0) * ey,                    # j_y, q_y
                ez, (5.0 * e2 - 9.0) * ez,                    # j_z, q_z
                3.0 * ex * ex - e2,                           # 3 p_xx
                (3.0 * e2 - 5.0) * (3.0 * ex * ex - e2),      # 3 pi_xx
                ey * ey - ez * ez,                            # p_ww
                (3.0 * e2 - 5.0) * (ey * ey - ez * ez),       # pi_ww
                ex * ey, ey * ez, ex * ez,                    # p_xy, p_yz, p_xz
                (ey * ey - ez * ez) * ex,                     # m_x
                (ez * ez - ex * ex) * ey,                     # m_y
                (ex * ex - ey * ey) * ez]                     # m_z
    return np.array(rows)

