"""lbm_moments_noalloc (partial sums in the library's static device scratch) against
lbm_moments (partial sums in the context's workspace), through the C ABI: the same
kernels in the same order, so fields and totals must agree bitwise -- on two
calls in a row, the second on a smaller box, whose partial sums overwrite only a
prefix of what the first call left in the scratch; and a box whose partial sums do
not fit the scratch is rejected with an error while lbm_moments still serves it."""
import numpy as np
import pytest

from cases import case, pure_water_mix
from oracle_backend import to_mixture

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _ctx(lattice, nc, shape, storage, steps):
    from paper_1909_12390_amd import lbm
    c = case(lattice, nc, shape, seed=7, u_amp=0.01)
    ctx = lbm.LbmContext(c["mix"], lattice, c["shape"], c["T"], 0.8, 1.3, c["gamma"], c["rho0"], c["u0"],
                         collision="mrt" if lattice == "D3Q19" else "bgk", forcing="edm", storage=storage,
                         mrt_s=None if lattice == "D2Q9" else
                         __import__("paper_1909_12390_amd.inputs", fromlist=["x"]).default_mrt_rates("D3Q19", 0.8))
    ctx.step(steps)
    ctx.check()
    return ctx


def _compare(ctx):
    a = ctx.moments(noalloc=False)
    b = ctx.moments(noalloc=True)
    for k in ("rho_s", "u", "p", "psi"):
        assert torch.equal(a[k], b[k]), k
    for k in ("mass", "momentum", "force", "negative_cells"):
        assert np.array_equal(a[k], b[k]), (k, a[k], b[k])
    return b


def test_noalloc_moments_match_workspace_moments_on_two_calls():
    print("case moments_noalloc: D3Q19 nc=4 (24, 40, 64) f16, then D2Q9 nc=2 (20, 36) f64", flush=True)
    big = _ctx("D3Q19", 4, (24, 40, 64), "f16", 3)
    rb = _compare(big)
    assert rb["mass"].shape == (4,) and np.all(rb["mass"] > 0)
    big.close()
    small = _ctx("D2Q9", 2, (20, 36), "f64", 2)
    rs = _compare(small)
    assert rs["mass"].shape == (2,) and np.all(rs["mass"] > 0)
    small.close()


def test_noalloc_moments_reject_boxes_beyond_the_scratch():
    from paper_1909_12390_amd import lbm
    shape = (2400, 2400)          # partial sums: 22,504 blocks x 6 doubles > 1 MiB - 256 B
    print(f"case moments_noalloc: D2Q9 nc=1 {shape} f16 (beyond the scratch)", flush=True)
    mix = pure_water_mix()
    T = 0.9 * to_mixture(mix).Tc[0]
    rho0 = np.full((1,) + shape, 0.58)
    ctx = lbm.LbmContext(mix, "D2Q9", shape, T, 0.8, 1.3, np.array([1.0]), rho0, collision="bgk",
                         forcing="edm", storage="f16")
    with pytest.raises(lbm.LbmError) as err:
        ctx.moments(noalloc=True)
    assert err.value.code == lbm.LBM_ERR_ARG and "too large" in str(err.value)
    m = ctx.moments()             # the workspace form serves every size
    assert m["mass"][0] == pytest.approx(0.58 * shape[0] * shape[1], rel=1e-6)
    ctx.close()
