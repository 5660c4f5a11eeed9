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


def _to_tiles(planes):
    """[N, ny, nx] -> the tile-blocked layout [tiles][N][64] of the
    population buffers (cells y nx + x cut into tiles of 64, last one padded
    with NaN)."""
    N = planes.shape[0]
    P = planes.shape[1] * planes.shape[2]
    T = (P + 63) // 64
    flat = np.full((N, T * 64), np.nan, dtype=np.float32)
    flat[:, :P] = planes.reshape(N, P)
    return np.ascontiguousarray(flat.reshape(N, T, 64).transpose(1, 0, 2)).ravel()


def _from_tiles(buf, N, ny, nx):
    T = (ny * nx + 63) // 64
    return buf.reshape(T, N, 64).transpose(1, 0, 2).reshape(N, T * 64)[:, :ny * nx].reshape(N, ny, nx)


@pytest.mark.parametrize("shape,fields", [((48, 70), 3), ((17, 256), 6), ((5, 13), 3)])
def test_streams_probe_is_the_d2q9_pull(shape, fields):
    """The pattern probe pulls every plane at the D2Q9 offsets in the step's
    tile-blocked layout (ragged last tile included) and never reads padding."""
    ny, nx = shape
    N = 9 * fields
    planes = np.random.default_rng(3).normal(size=(N, ny, nx)).astype(np.float32)
    src = torch.tensor(_to_tiles(planes), device="cuda")
    dst = torch.full_like(src, float("nan"))
    lbm.bw_streams(dst, src, nx, ny, fields)
    torch.cuda.synchronize()
    d = _from_tiles(dst.cpu().numpy(), N, ny, nx)
    for j in range(N):
        i = j % 9
        assert np.array_equal(d[j], np.roll(planes[j], (CY[i], CX[i]), axis=(0, 1))), j


CX3 = [0, 1, -1, 0, 0, 0, 0]
CY3 = [0, 0, 0, 1, -1, 0, 0]
CZ3 = [0, 0, 0, 0, 0, 1, -1]


def _to_tiles3(planes):
    """[N, nz, ny, nx] -> the 3D step's layout [nz][tiles][N][64] (each
    z-slab's cells y nx + x cut into tiles of 64, the last one padded with
    NaN)."""
    return np.concatenate([_to_tiles(planes[:, z]) for z in range(planes.shape[1])])


def _from_tiles3(buf, N, nz, ny, nx):
    slab = buf.size // nz
    return np.stack([_from_tiles(buf[z * slab:(z + 1) * slab], N, ny, nx) for z in range(nz)], axis=1)


@pytest.mark.parametrize("shape,fields", [((3, 5, 13), 17), ((4, 16, 32), 14), ((2, 9, 70), 17)])
def test_streams3_probe_is_the_d3q7_pull(shape, fields):
    """The 3D pattern probe pulls every plane at the D3Q7 offsets in the
    step's tile-blocked z-slab layout (ragged last tile of each slab
    included) and never reads padding."""
    nz, ny, nx = shape
    N = 7 * fields
    planes = np.random.default_rng(5).normal(size=(N, nz, ny, nx)).astype(np.float32)
    src = torch.tensor(_to_tiles3(planes), device="cuda")
    dst = torch.full_like(src, float("nan"))
    lbm.bw_streams3(dst, src, nx, ny, nz, fields)
    torch.cuda.synchronize()
    d = _from_tiles3(dst.cpu().numpy(), N, nz, ny, nx)
    for j in range(N):
        i = j % 7
        assert np.array_equal(d[j], np.roll(planes[j], (CZ3[i], CY3[i], CX3[i]), axis=(0, 1, 2))), j


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
    assert lib.lbm_bw_streams3(a.data_ptr(), a.data_ptr(), 1, 1, 1, 4, None) == lbm.LBM_EINVAL
    assert lib.lbm_bw_streams3(a.data_ptr(), a.data_ptr(), 1, 1, 0, 17, None) == lbm.LBM_EINVAL
    with pytest.raises(ValueError):
        lbm.bw_streams3(a, a, 64, 64, 2, 17)
