"""The event-set comparison's zero-allocation entry point (its bitmaps in the
library's fixed device array) against the entry point with a caller scratch:
identical distances on two calls in a row, the second on a smaller grid and
fewer events (so a stale bitmap of the first would show), and the size limit."""
import numpy as np
import pytest
import torch

from paper_2303_02608_amd import binding as B
from parity_util import say

pytestmark = pytest.mark.gpu


def _events(rng, n, W, H, T):
    return dict(x=torch.from_numpy(rng.integers(0, W, n).astype(np.int32)).cuda(),
                y=torch.from_numpy(rng.integers(0, H, n).astype(np.int32)).cuda(),
                t=torch.from_numpy(rng.integers(0, T, n).astype(np.int32)).cuda(),
                p=torch.from_numpy(rng.choice(np.array([-1, 1], np.int8), n)).cuda())


def test_noalloc_matches_scratch_call_twice():
    rng = np.random.default_rng(23)
    for (W, H, T, ns, nq) in ((640, 480, 120, 400000, 300000), (96, 64, 12, 3000, 5000)):
        say(f"no-alloc nn distances {W}x{H}x{T}, {ns} sources, {nq} queries")
        assert B.load().esim_nn_scratch_bytes(W, H, T) <= B.NN_STATIC_BYTES
        src, qry = _events(rng, ns, W, H, T), _events(rng, nq, W, H, T)
        ref = B.nn_distances(src, qry, W, H, T, 0.05)
        d = torch.full((nq,), -1.0, dtype=torch.float64, device="cuda")
        B.nn_distances_noalloc(src, qry, W, H, T, 0.05, d)
        torch.cuda.synchronize()
        a, b = ref.cpu().numpy(), d.cpu().numpy()
        assert np.isfinite(a).sum() > nq // 10
        assert np.array_equal(a, b)


def test_noalloc_rejects_grids_beyond_the_fixed_array():
    W, H, T = 1920, 1080, 500
    assert B.load().esim_nn_scratch_bytes(W, H, T) > B.NN_STATIC_BYTES
    rng = np.random.default_rng(1)
    src = _events(rng, 10, W, H, T)
    d = torch.empty(10, dtype=torch.float64, device="cuda")
    with pytest.raises(B.EsimError) as e:
        B.nn_distances_noalloc(src, src, W, H, T, 0.05, d)
    assert e.value.status == B.E_CAPACITY
