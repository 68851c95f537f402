"""Host chain rule of the library's adjoint (lbm_eos_param_grad) against the
oracle's differentiation of the EOS tables (CPU only: no device call)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import adjoint as oadj  # noqa: E402
from oracle_backend import to_mixture  # noqa: E402
from paper_1909_12390_amd import inputs, lbm  # noqa: E402


@pytest.mark.parametrize("nc,seed", [(1, 0), (2, 1), (3, 2), (4, 3)])
def test_eos_param_grad_matches_oracle_chain(nc, seed):
    rng = inputs.rng_for(900, seed)
    mix = inputs.draw_components(rng, nc, k_max=0.08)
    base = to_mixture(mix)
    T = 0.8 * float(np.min(base.Tc))
    d_aa = rng.standard_normal((nc, nc))
    d_b = rng.standard_normal(nc)
    dk, da, db = lbm.eos_param_grad(mix, T, d_aa, d_b)
    th = torch.tensor(oadj.theta_of(base), dtype=oadj.DT, requires_grad=True)
    aa, b = oadj.eos_tables(th, base, T)
    (g,) = torch.autograd.grad((aa * torch.as_tensor(d_aa)).sum() + (b * torch.as_tensor(d_b)).sum(), th)
    g = g.numpy()
    npair = nc * (nc - 1) // 2
    lib_theta = np.concatenate([[dk[i, j] for i, j in oadj.pair_index(nc)], da, db])
    assert np.allclose(lib_theta, g, rtol=1e-12, atol=1e-14 * np.max(np.abs(g)))
    assert np.allclose(dk, dk.T) and np.all(np.diag(dk) == 0.0)
    assert lib_theta.shape == (npair + 2 * nc,)


def test_eos_param_grad_rejects_bad_input():
    mix = inputs.draw_components(inputs.rng_for(901), 2)
    with pytest.raises(lbm.LbmError):
        lbm.eos_param_grad(mix, -1.0, np.zeros((2, 2)), np.zeros(2))
