"""Autotuner of the library's launch configuration (expm_tune_t, include/expm.h).

Nothing here changes what the method computes: every candidate runs the same kernels on the
same matrices; only how the work is laid out on the GPU differs.  For each knob the tuner
times every candidate on a synthetic batch of the order range, precision and selector the knob
serves (HIP events on the current stream, after untimed warm-up calls), keeps the fastest, and
records all timings.  The winners are kept in a JSON cache keyed by the GPU architecture
(``tuning_cache.json`` beside this file); ``install()`` loads the entry of the current
device's architecture into the library (``expm_tune_set``), ``defaults()`` restores the
untuned configuration (every field 0: the library's built-in choices).

Knobs (one cache entry each, key ``<knob>/<order range>/<precision>/<selector>``):
  arrangement   how expm_batched spreads its sweeps over two streams, per selector, timed on
                the batched workload (4096 matrices, orders 16..128)
  small_kernel  order <= 16 on one wavefront per matrix or on the 4-wave on-chip kernel
  per_cu        persistent workgroups per CU of each sweep kernel, timed on a uniform batch
                of the order range that kernel serves
  tiles         output tiles per launch of the tiled path, per precision, timed on
                n = 1024 matrices

Command line:  python -m paper_1710_10989_amd.autotune [--quick] [--out PATH]
"""
import argparse
import ctypes
import datetime
import json
import os

import numpy as np
import torch

from . import _native as N
from . import expm as X

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning_cache.json")

KERNELS = ("fused4", "fused8", "res4", "splitrow", "res8", "onewave")
PRECS = ("fp64", "fp32", "bf16x3", "fp32all")
SELS = ("plain", "alpha", "learned")
# uniform batch that exercises each sweep kernel: (real order, matrices); fused4 serves only the
# learned selector's feature rows and is not timed
KERNEL_CASE = {"fused8": (256, 512), "res4": (48, 4096), "splitrow": (96, 2048), "res8": (128, 2048),
               "onewave": (16, 65536)}  # onewave: Gaussian entries, like the other cases


def arch():
    """GPU architecture name of the current device (e.g. gfx950)."""
    return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]


def to_dict(t):
    return {"arrangement": list(t.arrangement), "small_kernel": int(t.small_kernel), "per_cu": list(t.per_cu),
            "tiles_per_launch": list(t.tiles_per_launch)}


def from_dict(d):
    t = N.ExpmTune()
    for i, v in enumerate(d.get("arrangement", [0, 0, 0])):
        t.arrangement[i] = int(v)
    t.small_kernel = int(d.get("small_kernel", 0))
    for i, v in enumerate(d.get("per_cu", [0] * 6)):
        t.per_cu[i] = int(v)
    for i, v in enumerate(d.get("tiles_per_launch", [0] * 4)):
        t.tiles_per_launch[i] = int(v)
    return t


def get():
    t = N.ExpmTune()
    N.check(N.lib().expm_tune_get(ctypes.byref(t)), "expm_tune_get")
    return t


def set_tune(t):
    N.check(N.lib().expm_tune_set(ctypes.byref(t)), "expm_tune_set")


def limits():
    t = N.ExpmTune()
    N.check(N.lib().expm_tune_limits(ctypes.byref(t)), "expm_tune_limits")
    return t


def defaults():
    """Back to the untuned configuration."""
    set_tune(N.ExpmTune())


def load(path=CACHE):
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def install(path=CACHE, which=None):
    """Installs the cached configuration of architecture `which` (default: the current
    device's).  Returns the installed dict, or None (defaults kept) when the cache has no entry."""
    d = load(path).get(which or arch())
    if not d:
        return None
    set_tune(from_dict(d["tune"]))
    return d["tune"]


def _time(fn, warmup, reps):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def _pick(base, set_field, candidates, fn, warmup, reps):
    """Times fn() under each candidate value of one field (the others as in `base`); returns
    (best, {value: ms}) and leaves `base` with the best value set."""
    times = {}
    for v in candidates:
        set_field(base, v)
        set_tune(base)
        times[v] = _time(fn, warmup, reps)
    best = min(times, key=lambda v: (times[v], v))
    set_field(base, best)
    set_tune(base)
    return best, times


def tune(quick=False, log=print):
    """Runs every knob's candidates on the current device; returns the cache entry
    {"tune": ..., "entries": ..., ...} of this architecture (the winners stay installed)."""
    from . import workloads as W
    from .expm import Batch
    lim = limits()
    cur = N.ExpmTune()
    set_tune(cur)
    warm, reps = (2, 3) if quick else (10, 20)
    scale = 8 if quick else 1
    entries = {}

    # batched workload: arrangement per selector, then the order-16 kernel
    mats, _ = W.mixed_batch(count=4096 // scale)
    B = Batch.from_host(mats)
    nb = len(mats)
    ws = torch.empty(X.workspace_bytes(B.n_max, nb), dtype=torch.uint8, device="cuda")
    outs = (torch.empty_like(B.packed), torch.empty(nb, dtype=torch.int32, device="cuda"),
            torch.empty(nb, dtype=torch.int32, device="cuda"), torch.empty(nb, dtype=torch.int32, device="cuda"))
    for si, sel in enumerate(SELS[:2]):
        def run(sel=sel):
            X.batched(B, selector=sel, workspace=ws, outs=outs)

        def setf(t, v, si=si):
            t.arrangement[si] = v
        best, times = _pick(cur, setf, list(range(lim.arrangement[si] + 1)), run, warm, reps)
        entries["arrangement/16-128/fp64/%s" % sel] = {"choice": best, "ms": times}
        log("arrangement %s: %s -> %d" % (sel, times, best))

    del B, ws, outs

    # order 16: one wavefront per matrix or the 4-wave kernel, on a uniform order-16 batch
    # (the exponents of an exponential integrator: 65536 skew-symmetric matrices)
    A16 = torch.from_numpy(W.small_skew_batch(count=65536 // scale, n=16)).cuda()
    ws16 = torch.empty(X.workspace_bytes(16, A16.shape[0]), dtype=torch.uint8, device="cuda")
    E16 = torch.empty_like(A16)
    o16 = tuple(torch.empty(A16.shape[0], dtype=torch.int32, device="cuda") for _ in range(3))

    def run_16():
        X.batched_uniform(A16, workspace=ws16, out=E16, outs=o16)

    def set_small(t, v):
        t.small_kernel = v
    best, times = _pick(cur, set_small, [1, 2], run_16, warm, reps)
    entries["small_kernel/16/fp64/plain"] = {"choice": best, "ms": times, "matrices": int(A16.shape[0])}
    log("small_kernel: %s -> %d" % (times, best))
    del A16, ws16, E16, o16

    # persistent grid of each sweep kernel on a uniform batch of its order range
    g = np.random.default_rng(1710)
    for k, name in enumerate(KERNELS):
        if name == "onewave" and cur.small_kernel == 2:
            continue  # order 16 runs on the 4-wave kernel: the one-wave grid is never launched
        if name not in KERNEL_CASE or lim.per_cu[k] <= 1:
            if name in KERNEL_CASE:
                entries["per_cu/%s/fp64/plain" % name] = {"choice": 0, "ms": {}}
            continue
        n, count = KERNEL_CASE[name]
        count = max(count // scale, 64)
        A = torch.from_numpy(g.standard_normal((count, n, n)) * (2.0 / n)).cuda()
        wsk = torch.empty(X.workspace_bytes(n, count), dtype=torch.uint8, device="cuda")
        E = torch.empty_like(A)
        o3 = tuple(torch.empty(count, dtype=torch.int32, device="cuda") for _ in range(3))

        def run_u():
            X.batched_uniform(A, workspace=wsk, out=E, outs=o3)

        def set_pc(t, v, k=k):
            t.per_cu[k] = v
        best, times = _pick(cur, set_pc, list(range(1, lim.per_cu[k] + 1)), run_u, warm, reps)
        entries["per_cu/%s/fp64/plain" % name] = {"choice": best, "ms": times, "order": n, "matrices": count}
        log("per_cu %s (n=%d, %d matrices): %s -> %d" % (name, n, count, times, best))
        del A, wsk, E

    # tiled path: tiles per launch per precision (n = 1024)
    n = 1024
    count = 16 if quick else 64
    A = torch.from_numpy(np.stack(W.large_dense(count, n, seed_stream=9))).cuda()
    E = torch.empty_like(A)
    o3 = tuple(torch.empty(count, dtype=torch.int32, device="cuda") for _ in range(3))
    for pi, prec in enumerate(PRECS):
        times = {}
        for v in (1024, 2048, 4096, 8192):
            cur.tiles_per_launch[pi] = v
            set_tune(cur)
            wsk = torch.empty(X.workspace_bytes(n, count, prec=prec), dtype=torch.uint8, device="cuda")
            times[v] = _time(lambda: X.batched_uniform(A, prec=prec, workspace=wsk, out=E, outs=o3),
                             1, 1 if quick else 3)
            del wsk
        best = min(times, key=lambda v: (times[v], v))
        cur.tiles_per_launch[pi] = best
        set_tune(cur)
        entries["tiles/1024/%s/plain" % prec] = {"choice": best, "ms": times, "matrices": count}
        log("tiles %s: %s -> %d" % (prec, times, best))
    return {"tune": to_dict(cur), "entries": entries, "device": torch.cuda.get_device_name(),
            "quick": bool(quick), "when": datetime.datetime.now(datetime.timezone.utc).isoformat()}


def save(entry, path=CACHE, which=None):
    d = load(path)
    d[which or arch()] = entry
    with open(path, "w") as fh:
        json.dump(d, fh, indent=1, sort_keys=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="smaller batches, fewer repetitions")
    ap.add_argument("--out", default=CACHE)
    args = ap.parse_args()
    entry = tune(quick=args.quick, log=lambda s: print(s, flush=True))
    save(entry, args.out)
    print(json.dumps(entry["tune"]), flush=True)


if __name__ == "__main__":
    main()
