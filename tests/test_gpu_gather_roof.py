"""The gather-roof measurement kernel (lsdf_gather_roof) reads what it says:
8 corners of in-range cells, summed in the stated order."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_12543_amd import lsdf
    lsdf.load_library()
    return lsdf


def mix32(x):
    x = np.uint64(x) & np.uint64(0xFFFFFFFF)
    x ^= x >> np.uint64(16)
    x = (x * np.uint64(0x7feb352d)) & np.uint64(0xFFFFFFFF)
    x ^= x >> np.uint64(15)
    x = (x * np.uint64(0x846ca68b)) & np.uint64(0xFFFFFFFF)
    x ^= x >> np.uint64(16)
    return int(x)


def test_gather_roof_constant_grid(B):
    n, iters, threads = 33, 7, 5000
    g = torch.full((n ** 3,), 0.5, dtype=torch.float32, device="cuda")
    out = B.gather_roof(g, n, iters, threads)
    assert torch.all(out == 8 * 0.5 * iters)


def test_gather_roof_cells_match_the_hash(B):
    n, threads = 64, 300
    vals = np.arange(n ** 3, dtype=np.float32)            # exact in FP32 (< 2^24)
    out = B.gather_roof(torch.as_tensor(vals, device="cuda"), n, 1, threads).cpu().numpy()
    m = n - 1
    for t in range(threads):
        h = mix32((t * 0x9e3779b9 + 0x165667b1) & 0xFFFFFFFF) % (m ** 3)
        ix, iy, iz = h % m, (h // m) % m, h // (m * m)
        c = iz * n * n + iy * n + ix
        f = np.float32
        v = (f(vals[c]) + f(vals[c + 1]) + (f(vals[c + n]) + f(vals[c + n + 1]))) + \
            ((f(vals[c + n * n]) + f(vals[c + n * n + 1])) + (f(vals[c + n * n + n]) + f(vals[c + n * n + n + 1])))
        assert out[t] == np.float32(0.0) + v, t
