"""The bandwidth probes move exactly the data they claim to (so the
denominators bench.py reports are for real copies)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2607_05668_amd import lbm  # noqa: E402

CX = [0, 1, 0, -1, 0, 1, -1, -1, 1]
CY = [0, 0, 1, 0, -1, 1, 1, -1, -1]


@pytest.mark.parametrize("shape,fields", [((48, 70), 3), ((17, 256), 6)])
def test_streams_probe_is_the_d2q9_pull(shape, fields):
    ny, nx = shape
    src = torch.randn(9 * fields, ny, nx, device="cuda")
    dst = torch.full_like(src, float("nan"))
    lbm.bw_streams(dst, src, nx, ny, fields)
    torch.cuda.synchronize()
    s, d = src.cpu().numpy(), dst.cpu().numpy()
    for j in range(9 * fields):
        i = j % 9
        assert np.array_equal(d[j], np.roll(s[j], (CY[i], CX[i]), axis=(0, 1))), j


def test_copy_probe_copies_with_a_ragged_tail():
    n = (1 << 20) + 7
    src = torch.randint(0, 255, (n,), dtype=torch.uint8, device="cuda")
    dst = torch.zeros_like(src)
    lbm.bw_copy(dst, src, n)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)


def test_probes_reject_bad_arguments():
    a = torch.zeros(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        lbm.bw_streams(a, a, 64, 64, 3)
    lib = lbm.load_library()
    assert lib.lbm_bw_streams(a.data_ptr(), a.data_ptr(), 1, 1, 4, None) == lbm.LBM_EINVAL
