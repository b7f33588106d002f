"""GPU: the autotuner on the device, and every launch configuration it can choose giving the
results of the default one (the same kernels on the same matrices: identical bits; order 16
on the 4-wave kernel instead of one wave per matrix: the oracle's 1e-12)."""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_quick_tune_and_reload(tmp_path):
    from paper_1710_10989_amd import autotune as T
    try:
        say("case quick autotune")
        entry = T.tune(quick=True, log=say)
        path = str(tmp_path / "cache.json")
        T.save(entry, path)
        T.defaults()
        assert T.install(path) == entry["tune"]
        assert T.to_dict(T.get()) == entry["tune"]
        lim = T.limits()
        t = entry["tune"]
        assert all(0 <= a <= 3 for a in t["arrangement"]) and t["small_kernel"] in (1, 2)
        assert all(0 <= v <= max(1, lim.per_cu[k]) for k, v in enumerate(t["per_cu"]))
    finally:
        T.defaults()


def test_configurations_give_default_results(orc):
    import paper_1710_10989_amd as P
    from paper_1710_10989_amd import autotune as T
    from paper_1710_10989_amd import workloads as W
    from paper_1710_10989_amd.expm import Batch
    mats, _ = W.mixed_batch(count=700, sizes=(16, 32, 48, 64, 96, 128, 144, 200), seed_stream=77)
    B = Batch.from_host(mats)
    try:
        T.defaults()
        E0, m0, s0, st0 = P.batched(B)
        torch.cuda.synchronize()
        lim = T.limits()
        cfgs = [{"arrangement": [a, a, a]} for a in (1, 2, 3)]
        cfgs.append({"per_cu": [1] * 6})
        cfgs.append({"per_cu": [max(1, v - 1) for v in lim.per_cu], "arrangement": [2, 2, 2]})
        for c in cfgs:
            T.set_tune(T.from_dict(c))
            say("case configuration", c)
            ws = torch.empty(P.workspace_bytes(B.n_max, len(mats)), dtype=torch.uint8, device="cuda")
            E1, m1, s1, st1 = P.batched(B, workspace=ws)
            torch.cuda.synchronize()
            assert torch.equal(st1, st0) and torch.equal(m1, m0) and torch.equal(s1, s0), c
            assert torch.equal(E1, E0), c
        # order 16 on the 4-wave kernel: other kernel, same method
        T.set_tune(T.from_dict({"small_kernel": 2}))
        E2, m2, s2, st2 = P.batched(B)
        torch.cuda.synchronize()
        assert torch.equal(m2, m0) and torch.equal(s2, s0) and bool((st2 == 0).all())
        outs = B.unpack(E2)
        small = [i for i, A in enumerate(mats) if A.shape[0] == 16][:40]
        refs, _ = orc.expm_taylor_batch([mats[i] for i in small], prec="ld")
        for i, R in zip(small, refs):
            assert orc.rel_err_1(outs[i], R) <= 1e-12, i
        # tiled path with fewer and more tiles per launch: the same kernels per matrix
        A = torch.from_numpy(np.stack(W.large_dense(6, 384, seed_stream=3))).cuda()
        T.defaults()
        R0 = P.batched_uniform(A)[0]
        for tiles in (9, 18):  # one and two matrices of order 384 (9 tiles each) per group
            T.set_tune(T.from_dict({"tiles_per_launch": [tiles] * 4}))
            R1 = P.batched_uniform(A)[0]
            torch.cuda.synchronize()
            assert torch.equal(R1, R0), tiles
    finally:
        T.defaults()
