"""The copy kernel bench.py measures its bandwidth ceiling with (lbm_stream_copy):
it must copy every byte, for any size that is a multiple of 16 and any grid, and
refuse what it cannot do (on the host, before any launch)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes", [16, 16 * 61, 65536 + 48, (1 << 20) + 16 * 7])
@pytest.mark.parametrize("grid", [0, 1, 7, 4096])
def test_stream_copy_copies_every_byte(nbytes, grid):
    from paper_1909_12390_amd import lbm
    print(f"case stream copy {nbytes} B grid {grid}", flush=True)
    rng = np.random.default_rng(nbytes + grid)
    src = torch.from_numpy(rng.integers(0, 256, nbytes + 64, dtype=np.uint8)).cuda()
    dst = torch.zeros(nbytes + 64, dtype=torch.uint8, device="cuda")
    lbm.stream_copy(dst, src, nbytes, grid)
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src[:nbytes])
    assert int(dst[nbytes:].abs().sum()) == 0          # nothing past the end


def test_stream_copy_refuses_bad_arguments():
    from paper_1909_12390_amd import lbm
    print("case stream copy arguments", flush=True)
    a = torch.zeros(256, dtype=torch.uint8, device="cuda")
    b = torch.zeros(256, dtype=torch.uint8, device="cuda")
    with pytest.raises(lbm.LbmError):
        lbm.stream_copy(a, b, 24)                        # not a multiple of 16
    with pytest.raises(lbm.LbmError):
        lbm.stream_copy(a[8:], b[8:], 16)                # 8-byte aligned only
    with pytest.raises(ValueError):
        lbm.stream_copy(a, b, 512)                       # beyond the tensors
    lbm.stream_copy(a, b, 0)                             # nothing to do
