"""GPU: expm_batched_noalloc (the library's own device scratch, no workspace) against
expm_batched on the same batches, through the C ABI: two calls in a row, the second with a
smaller batch of smaller orders, each compared with expm_batched element by element (the same
kernels run on the same matrices, so results, (m, s) and status must be identical), plus an
oracle sample at the relative 1-norm error bound of the FP64 method, 1e-12."""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

TOL = 1e-12


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _check_against_batched(P, orc, mats, selector):
    from paper_1710_10989_amd.expm import Batch
    B = Batch.from_host(mats)
    E0, m0, s0, st0 = P.batched(B, selector=selector)
    E1, m1, s1, st1 = P.batched_noalloc(B, selector=selector)
    torch.cuda.synchronize()
    assert torch.equal(st1, st0) and torch.equal(m1, m0) and torch.equal(s1, s0)
    assert bool((st1 == 0).all())
    assert torch.equal(E1, E0)
    outs = B.unpack(E1)
    sample = np.random.default_rng(len(mats)).choice(len(mats), 12, replace=False)
    refs, _ = orc.expm_taylor_batch([mats[i] for i in sample], prec="ld")
    for i, R in zip(sample, refs):
        assert orc.rel_err_1(outs[i], R) <= TOL, i


@pytest.mark.parametrize("selector", ["plain", "alpha"])
def test_noalloc_matches_batched_two_calls(orc, selector):
    import paper_1710_10989_amd as P
    from paper_1710_10989_amd import workloads as W
    assert torch.cuda.is_available()
    mats, _ = W.mixed_batch(count=900, seed_stream=41)  # orders 16..128, the headline mix
    say("case noalloc first call", selector, len(mats))
    _check_against_batched(P, orc, mats, selector)
    small, _ = W.mixed_batch(count=130, sizes=(16, 32, 48, 64), seed_stream=42)
    say("case noalloc second call (smaller)", selector, len(small))
    _check_against_batched(P, orc, small, selector)
