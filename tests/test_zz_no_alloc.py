"""rogs_elev_loss_static, the allocation-free variant of rogs_elev_loss (block
partial sums in the library's fixed device array), against rogs_elev_loss
with a caller-owned scratch buffer: same kernels, so the same bits.  Two
calls in a row, the second smaller, so that the array still holds the first
call's partials when the second runs."""
import numpy as np
import pytest
import torch

from paper_2405_14342_amd import binding as B
from paper_2405_14342_amd import synth

pytestmark = pytest.mark.gpu
MAX_N = 16777216            # ROGS_ELEV_STATIC_MAX_N


def _compare(rg, n_along, n_across, seed):
    n = n_along * n_across
    rng = np.random.default_rng(seed)
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device="cuda")
    z = f(rng.normal(0.0, 0.1, n))
    zbar = f(rng.normal(0.0, 0.1, n))
    nbr = torch.as_tensor(np.ascontiguousarray(synth.grid_neighbours(n_along, n_across), np.int32),
                          device="cuda")
    base = rng.normal(0.0, 1.0, n)           # both calls add into the same starting gradient
    dz_ref, dz = f(base), f(base)
    loss_ref, loss = f([0.25]), f([0.25])
    scratch = torch.empty(B.elev_scratch_bytes(n), dtype=torch.uint8, device="cuda")
    rg.elev_loss(n, z, nbr, 1.0, zbar, 0.02, dz_ref, loss_ref, scratch)
    rg.elev_loss_static(n, z, nbr, 1.0, zbar, 0.02, dz, loss)
    torch.cuda.synchronize()
    assert torch.equal(dz, dz_ref)
    assert torch.equal(loss, loss_ref)
    assert float(loss) != 0.25


def test_static_partials_match_caller_scratch_on_two_calls():
    rg = B.Rogs()
    print("[no-alloc] 1000 x 300 surfels, then 37 x 11", flush=True)
    _compare(rg, 1000, 300, 1)      # 300,000 surfels: 1172 partial sums
    _compare(rg, 37, 11, 2)         # 407 surfels: 2 partial sums


def test_static_rejects_counts_above_its_array():
    rg = B.Rogs()
    z = torch.zeros(4, dtype=torch.float32, device="cuda")
    r = rg.elev_loss_static(MAX_N + 1, z, None, 1.0, z, 0.02, z, z, check=False)
    assert r == B.EINVAL
    assert "ROGS_ELEV_STATIC_MAX_N" in rg.last_error()
    assert rg.elev_loss_static(0, z, None, 1.0, z, 0.02, z, z, check=False) == B.EINVAL
