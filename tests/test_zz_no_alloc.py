"""The allocation-free map2alm (csmap_map2alm_noalloc) against csmap_map2alm.

Both run the same kernels; the allocation-free entry point takes its scratch
from the library's fixed device array instead of allocating it.  Two calls
in a row, the second on a smaller map, must each equal the allocating entry
point's result bit for bit (the kernels sum in a fixed order), and a size
whose scratch exceeds the fixed array is refused."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    from paper_1204_5041_amd import binding
    assert torch.cuda.is_available()
    return binding


def _map(nside, seed):
    rng = np.random.default_rng(seed)
    return torch.from_numpy(rng.standard_normal(12 * nside * nside)).cuda()


def test_noalloc_map2alm_equals_map2alm_on_two_calls(B):
    # The larger case first, so the second call runs on scratch that still
    # holds the first call's values.
    for nside, lmax, seed in ((512, 1024, 1), (64, 100, 2)):
        say(f"map2alm_noalloc nside={nside} lmax={lmax}")
        m = _map(nside, seed)
        ref = torch.view_as_real(B.map2alm(m, lmax)).contiguous().view(-1)
        out = torch.full((2 * B.alm_size(lmax),), float("nan"), dtype=torch.float64,
                         device="cuda")
        B.map2alm_noalloc(m, lmax, out)
        torch.cuda.synchronize()
        got, want = out.cpu().numpy(), ref.cpu().numpy()
        assert np.all(np.isfinite(got))
        assert np.array_equal(got, want), np.max(np.abs(got - want))


def test_noalloc_map2alm_refuses_oversized_scratch(B):
    m = _map(1024, 3)
    out = torch.empty(2 * B.alm_size(1024), dtype=torch.float64, device="cuda")
    with pytest.raises(B.CsmapError):
        B.map2alm_noalloc(m, 1024, out)
