"""Throughput of the matrix-exponential hot path on one MI355X.

Default workload (batched): 4096 FP64 matrices of uneven order n in {16, 32, 48, 64, 96, 128},
||A||_1 log-uniform in [1e-3, 1e2], structure mix 40 % dense Gaussian / 20 % skew-symmetric /
20 % strictly upper triangular / 20 % diagonal + rank 4 (seeded, synthetic).  One step = one
expm_batched call on the whole batch (device work-queue ordering + the persistent resident
kernels: norm, (m, s) selection, product-reduced Taylor polynomial, squarings), inputs
already resident in HBM.  The dominant kernel (orders 112..128) is then timed alone, phase by
phase, for its roofline.

Other workloads (one JSON line each, selected with --workload):
  single     one 64 x 64 FP64 matrix, ||A||_1 = 2 (latency-bound; repeated expm_taylor calls)
  precision  256 matrices n = 1024 + 16 matrices n = 4096, N(0,1)/sqrt(n) entries scaled to
             ||A||_1 uniform in [0.5, 50]; --prec fp64 / fp32 / bf16x3
  learned    20000 held-out FP64 matrices, n in {32, 64, 128, 256}, ||A||_1 log-uniform in
             [1e-2, 1e3], the batched structure mix; plain vs alpha vs learned selector (the
             network is trained on 200k matrices of the same distribution by
             `python -m paper_1710_10989_amd.learned train`; its checkpoint is loaded if present)
  complex    512 complex matrices -i H dt (H Hermitian, spectral radius 1, n = 256,
             dt log-uniform in [1e-2, 1e2]) + one dense FP64 n = 8192 with ||A||_1 = 20
  small      65536 skew-symmetric FP64 matrices of order 16, ||A||_1 log-uniform in [0.05, 1]
             (the exponents of a Magnus integrator; one wave per matrix)
  magnus     one fourth-order Magnus step for 65536 linear systems Y' = (S0 + u(t) S1) Y of
             order 16 (expm_magnus4_step: exponent, e^Omega and its product with Y on chip)
  triangular 64 upper triangular FP64 matrices of order 512 with a widely spread diagonal, with
             and without the triangular refinement (EXPM_FLAG_TRI)
  copy       device-to-device copy of a 1 GiB buffer (the known-size calibration kernel
             for HBM byte counters; not a matrix-exponential figure)

The JSON line carries matrices/s, the roofline of the dominant kernel (executed flops =
sum over matrices of (products(m) + s) * 2 n^3 for the real order n the kernels run on,
divided by the kernel's duration measured with HIP events on the launch stream, against the
MI355X dense FP64 MFMA peak, 78.6 TFLOP/s) and the CPU oracle (direct Taylor) timed on a
bounded sample of the same workload on the host cores.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

PRODUCTS = {1: 0, 2: 1, 4: 2, 8: 3, 12: 4, 18: 5}
PS_PRODUCTS = {1: 0, 2: 1, 4: 2, 6: 3, 9: 4, 12: 5, 16: 6}  # Paterson-Stockmeyer (Table 3)
PEAK_FP64 = 78.6e12
PEAK_FP32 = 157.3e12
HERE = os.path.dirname(os.path.abspath(__file__))


KERNEL_SOURCES = ("coefs.h", "expm_api.cpp", "expm_fused.h", "expm_fused.hip", "expm_internal.h", "resident.h")


def sources_sha256(files=KERNEL_SOURCES):
    """Digest of the csrc files a kernel and its launch are built from."""
    import hashlib
    d = os.path.join(HERE, "paper_1710_10989_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(files):
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(tag):
    """HBM bytes per launch of a kernel from its committed PMC summary (FETCH_SIZE and
    WRITE_SIZE, each scaled by the same counter's reading on a copy of known size), or None
    when the summary was taken on other sources of that kernel than the current ones."""
    path = os.path.join(HERE, "profiles", tag + "_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    files = d.get("sources", [])
    if not files or d.get("sources_sha256") != sources_sha256(files):
        return None
    return d.get("bytes_per_launch")


def executed_flops(ms, ss, ns, prods=PRODUCTS):
    return float(sum((prods[int(m)] + int(s)) * 2.0 * float(n) ** 3 for m, s, n in zip(ms, ss, ns) if m > 0))


def host_cpu():
    """(threads the oracle may use, nproc, CPU model): the cores this process may run on,
    capped at 16 (the host share of one GPU)."""
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return min(nproc, 16), nproc, model


def cpu_oracle(mats, seconds, label, single_seconds=3.0):
    """Whole passes of the FP64 direct-Taylor oracle over `mats` until about `seconds`, on an
    explicitly set number of OpenMP threads; then the single-thread rate on a sub-sample."""
    import oracle
    want, nproc, model = host_cpu()
    threads = oracle.set_threads(want)
    oracle.expm_taylor_batch(mats[:1], prec="d")
    done, c0 = 0, time.perf_counter()
    while True:
        oracle.expm_taylor_batch(mats, prec="d")
        done += 1
        if time.perf_counter() - c0 >= seconds:
            break
    c1 = time.perf_counter()
    # one thread: passes over every 16th matrix (the same mix of orders) for about single_seconds
    sub = mats[::16] if len(mats) >= 64 else mats
    oracle.set_threads(1)
    d1, s0 = 0, time.perf_counter()
    while True:
        oracle.expm_taylor_batch(sub, prec="d")
        d1 += 1
        if time.perf_counter() - s0 >= single_seconds:
            break
    s1 = time.perf_counter()
    oracle.set_threads(want)
    return {"value": done * len(mats) / (c1 - c0), "unit": "matrices/s", "cores": threads, "kind": "oracle",
            "nproc": nproc, "cpu_model": model,
            "single_core": {"value": d1 * len(sub) / (s1 - s0), "unit": "matrices/s",
                            "sample": "%d pass(es) over %d matrices (every 16th), %.1f s" % (d1, len(sub), s1 - s0)},
            "sample": "%d pass(es) over %s, FP64 direct Taylor (own scaling ||X||_1 <= 1/2), OpenMP over "
                      "matrices on %d threads, %.1f s" % (done, label, threads, c1 - c0)}


def line(args, metric, value, ms_step, dtype, config, roofline, cpu, unit="matrices/s", vs_baseline=None):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": vs_baseline, "dtype": dtype, "data": "synthetic", "config": config, "roofline": roofline,
            "cpu_baseline": cpu}


def run_batched(args, torch, P, W):
    from paper_1710_10989_amd.expm import Batch
    mats, kinds = W.mixed_batch(count=args.count)
    B = Batch.from_host(mats)
    ws = torch.empty(P.workspace_bytes(B.n_max, len(mats)), dtype=torch.uint8, device="cuda")
    nb = len(mats)
    outs = (torch.empty_like(B.packed), torch.empty(nb, dtype=torch.int32, device="cuda"),
            torch.empty(nb, dtype=torch.int32, device="cuda"), torch.empty(nb, dtype=torch.int32, device="cuda"))
    stream = torch.cuda.current_stream()

    def step():
        # one step = one expm_batched call on the whole batch
        P.batched(B, selector=args.selector, workspace=ws, outs=outs)

    def staged(ev):
        # the same work in its three phases on one stream, events bracketing phase 1: the 8-wave
        # resident kernel (orders 112..128), the dominant kernel of this workload, run alone
        P.batched(B, selector=args.selector, workspace=ws, outs=outs, stage=0)
        ev[0].record(stream)
        P.batched(B, selector=args.selector, workspace=ws, outs=outs, stage=1)
        ev[1].record(stream)
        P.batched(B, selector=args.selector, workspace=ws, outs=outs, stage=2)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for i in range(args.steps):
        step()
    t1.record(stream)
    torch.cuda.synchronize()
    ms_step = t0.elapsed_time(t1) / args.steps
    kev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for i in range(args.steps):
        staged(kev[i])
    torch.cuda.synchronize()
    ms_k8 = sum(a.elapsed_time(b) for a, b in kev) / args.steps
    _, m, s, st = (x.cpu().numpy() for x in outs)
    assert np.all(st == 0), "non-ok status in the batch"
    plain = plain_per_matrix(torch, P, B, mats, outs[0], m, s, args.plain_passes) if args.plain_passes > 0 else None
    ns = np.array([a.shape[0] for a in mats], dtype=np.float64)
    big = ((ns + 15) // 16) >= 7  # real orders handled by the 8-wave resident kernel (112..128)
    flops = executed_flops(m, s, ns)
    flops_k8 = executed_flops(m[big], s[big], ns[big])
    achieved = flops_k8 / (ms_k8 * 1e-3)
    cpu = None if args.no_cpu else cpu_oracle(mats, args.cpu_seconds, "all %d matrices of the workload" % nb)
    config = {"workload": "4096 FP64 matrices, n uniform in {16,32,48,64,96,128}, ||A||_1 log-uniform [1e-3,1e2], "
                          "40/20/20/20 dense/skew/nilpotent/diag+rank4; one expm_batched call per step",
              "selector": args.selector,
              "mean_products_plus_squarings": float(np.mean([PRODUCTS[int(a)] + int(b) for a, b in zip(m, s)]))}
    roof = {"bound": "mfma", "kernel": "expm_resident_kernel<8> (orders 112..128 of the batch)",
            "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64,
            "traffic": measured_traffic("expm_resident_kernel8_batched_4096_mixed"), "kernel_ms": ms_k8,
            "kernel_timing": "HIP events around the kernel's phase, run alone (expm_batched_stage 1), "
                             "%d steps right after the timed region" % args.steps,
            "step_tflops": flops / (ms_step * 1e-3) / 1e12}
    config["plain_fp64_form"] = plain
    value = nb / (ms_step * 1e-3)
    return line(args, "expm matrices/s (rel err <= 1e-12, FP64)", value, ms_step, "f64", config,
                roof, cpu, vs_baseline=value / plain["value"] if plain else None)


def plain_per_matrix(torch, P, B, mats, E_batched, m_b, s_b, passes):
    """The method's plain FP64 form on the same workload: one expm_taylor call (one launch) per
    matrix, norm-based (m, s), matrices in the workload's order on one stream.  Checks that
    every (m, s) equals the batched call's and that the results agree to 1e-12."""
    from paper_1710_10989_amd import _native as N
    import ctypes
    L = N.lib()
    nb = len(mats)
    o = N.ExpmOpts(N.EXPM_F64, N.EXPM_PREC_FP64, N.EXPM_SEL_PLAIN, 0, 0.0)
    nmax = max(a.shape[0] for a in mats)
    ws = torch.empty(L.expm_workspace_bytes(nmax, 1, ctypes.byref(o)), dtype=torch.uint8, device="cuda")
    E = torch.empty_like(B.packed)
    ms = torch.empty((nb, 3), dtype=torch.int32, device="cuda")
    offs = B.offsets.cpu().numpy()
    a0, e0, m0 = B.packed.data_ptr(), E.data_ptr(), ms.data_ptr()
    calls = [(ctypes.c_void_p(a0 + 8 * int(offs[b])), ctypes.c_void_p(e0 + 8 * int(offs[b])), mats[b].shape[0],
              ctypes.c_void_p(m0 + 12 * b), ctypes.c_void_p(m0 + 12 * b + 4), ctypes.c_void_p(m0 + 12 * b + 8))
             for b in range(nb)]
    wsp, wsn, op = ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.byref(o)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    fn = L.expm_taylor

    def one_pass():
        for a, e, n, pm, ps, pst in calls:
            if fn(a, e, n, op, pm, ps, pst, wsp, wsn, stream) != 0:
                raise RuntimeError("expm_taylor failed")

    one_pass()
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    h0 = time.perf_counter()
    t0.record()
    for _ in range(passes):
        one_pass()
    t1.record()
    h1 = time.perf_counter()
    torch.cuda.synchronize()
    ms_pass = t0.elapsed_time(t1) / passes
    msh = ms.cpu().numpy()
    assert np.all(msh[:, 2] == 0)
    assert np.array_equal(msh[:, 0], m_b) and np.array_equal(msh[:, 1], s_b)
    diff = (E - E_batched).abs()
    dev = 0.0
    for b in range(0, nb, 97):  # sampled matrices: relative 1-norm difference of the two forms
        n, o_ = mats[b].shape[0], int(offs[b])
        Xb = E[o_:o_ + n * n].view(n, n)
        Db = diff[o_:o_ + n * n].view(n, n)
        dev = max(dev, float(Db.sum(0).max() / Xb.abs().sum(0).max()))
    assert dev <= 1e-12, dev
    return {"value": nb / (ms_pass * 1e-3), "unit": "matrices/s", "ms_per_pass": ms_pass,
            "host_ms_per_pass": (h1 - h0) * 1e3 / passes, "passes": passes,
            "form": "plain FP64: one expm_taylor call (one kernel launch) per matrix, norm-based (m, s), "
                    "one stream, after one untimed pass",
            "max_rel_diff_vs_batched_sampled": dev}


def run_single(args, torch, P, W):
    A = torch.from_numpy(W.single_dense(64, 2.0)).cuda()
    ws = torch.empty(P.workspace_bytes(64, 1), dtype=torch.uint8, device="cuda")
    out, outs = torch.empty_like(A), torch.empty(3, dtype=torch.int32, device="cuda")  # reused by every call
    for _ in range(args.warmup):
        E, m, s, st = P.taylor(A, selector=args.selector, workspace=ws, out=out, outs=outs)
    torch.cuda.synchronize()
    reps = args.steps * 50
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        E, m, s, st = P.taylor(A, selector=args.selector, workspace=ws, out=out, outs=outs)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    fl = executed_flops([int(m.item())], [int(s.item())], [64])
    cpu = None if args.no_cpu else cpu_oracle([A.cpu().numpy()] * 64, args.cpu_seconds, "64 copies of the matrix")
    one_cu = PEAK_FP64 / 256
    roof = {"bound": "mfma", "kernel": "expm_resident_kernel<4> (one workgroup of four waves, latency-bound)",
            "achieved": fl / (ms * 1e-3) / 1e12, "peak": one_cu / 1e12, "unit": "TFLOP/s",
            "frac": fl / (ms * 1e-3) / one_cu, "traffic": None, "note": "peak of the one CU a single matrix runs on"}
    config = {"workload": "one 64x64 FP64 matrix, N(0,1) scaled to ||A||_1 = 2, one expm_taylor call per step "
                          "(calls back to back with reused output buffers, %d per timed step)" % 50,
              "selector": args.selector,
              "m_s": [int(m.item()), int(s.item())], "us_per_matrix": ms * 1e3}
    return line(args, "expm matrices/s (single 64x64, rel err <= 1e-12)", 1e3 / ms, ms * 50, "f64", config, roof, cpu)


def run_precision(args, torch, P, W):
    mats1 = W.large_dense(256, 1024, seed_stream=0)
    mats4 = W.large_dense(16, 4096, seed_stream=1)
    A1 = torch.from_numpy(np.stack(mats1)).cuda()
    A4 = torch.from_numpy(np.stack(mats4)).cuda()
    del mats4
    mt = args.method
    ws1 = torch.empty(P.workspace_bytes(1024, 256, prec=args.prec, method=mt), dtype=torch.uint8, device="cuda")
    ws4 = torch.empty(P.workspace_bytes(4096, 16, prec=args.prec, method=mt), dtype=torch.uint8, device="cuda")
    E1, E4 = torch.empty_like(A1), torch.empty_like(A4)

    def step():
        r1 = P.batched_uniform(A1, prec=args.prec, selector=args.selector, workspace=ws1, out=E1, method=mt)
        r4 = P.batched_uniform(A4, prec=args.prec, selector=args.selector, workspace=ws4, out=E4, method=mt)
        return r1, r4

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(args.steps):
        (_, m1, s1, st1), (_, m4, s4, st4) = step()
    t1.record()
    torch.cuda.synchronize()
    ms_step = t0.elapsed_time(t1) / args.steps
    m1, s1, m4, s4 = (x.cpu().numpy() for x in (m1, s1, m4, s4))
    prods = PS_PRODUCTS if mt == "ps" else PRODUCTS
    flops = executed_flops(m1, s1, [1024] * 256, prods) + executed_flops(m4, s4, [4096] * 16, prods)
    err = None
    if args.prec != "fp64" or mt != "reduced":  # error against the FP64 path (pinned to the oracle)
        R1 = P.batched_uniform(A1, selector=args.selector)[0]
        R4 = P.batched_uniform(A4, selector=args.selector)[0]
        torch.cuda.synchronize()

        def rel(X, R):
            return float((X - R).abs().sum(dim=-2).amax(dim=-1).div(R.abs().sum(dim=-2).amax(dim=-1)).max())
        err = max(rel(E1, R1), rel(E4, R4))
    cpu = None if args.no_cpu else cpu_oracle(mats1[:1], args.cpu_seconds, "1 of the 256 n = 1024 matrices")
    peak, note = PEAK_FP64, "executed flops over the whole step against the FP64 peak (FP64-equivalent rate)"
    if args.prec == "fp32all":  # every product in FP32: the FP32 MFMA peak is the bound
        peak, note = PEAK_FP32, "executed flops over the whole step against the FP32 MFMA peak"
    roof = {"bound": "mfma", "kernel": "lg_gemm_kernel (tiled 128x128, all GEMM steps of the step)",
            "achieved": flops / (ms_step * 1e-3) / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
            "frac": flops / (ms_step * 1e-3) / peak, "traffic": None, "note": note}
    # accuracy against the bound each form states for this workload (FP64: 1e-12 against the
    # oracle, checked by the GPU tests at these sizes); the reduced forms are measured here
    # against the FP64 path, itself within 1e-12 of the oracle
    stated = {"fp64": 1e-12, "fp32": 1e-6, "bf16x3": 1e-9, "fp32all": 1e-6}[args.prec]
    smax = int(max(np.max(s1), np.max(s4)))
    accuracy = {"stated_bound": stated, "max_rel_err_vs_fp64_path": err,
                "meets_stated_bound": None if err is None else bool(err <= stated),
                "derived_bound_4sqrt(n)u32*2^s": None if args.prec == "fp64" else 4.0 * 64 * 2.0 ** -24 * 2.0 ** smax}
    config = {"workload": "256 FP64 n=1024 + 16 FP64 n=4096, N(0,1)/sqrt(n) scaled to ||A||_1 ~ U[0.5,50]; two "
                          "expm_batched_uniform calls per step", "selector": args.selector, "prec": args.prec,
              "method": mt, "max_rel_err_vs_fp64_path": err, "accuracy": accuracy,
              "mean_products_plus_squarings": float(np.mean([prods[int(a)] + int(b) for a, b in
                                                             zip(np.r_[m1, m4], np.r_[s1, s4])]))}
    name = args.prec if mt == "reduced" else "%s, Paterson-Stockmeyer" % args.prec
    return line(args, "expm matrices/s (precision workload, %s)" % name, 272 / (ms_step * 1e-3), ms_step,
                {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3+f32", "fp32all": "f32"}[args.prec], config, roof,
                cpu)


def run_complex(args, torch, P, W):
    mats, dts = W.hermitian_unitary_batch(count=512, n=256)
    Z = torch.from_numpy(np.stack(mats)).cuda()
    big = torch.from_numpy(W.single_dense(8192, 20.0, seed_stream=5)).cuda()
    wsz = torch.empty(P.workspace_bytes(256, 512, dtype=torch.complex128), dtype=torch.uint8, device="cuda")
    wsb = torch.empty(P.workspace_bytes(8192, 1), dtype=torch.uint8, device="cuda")
    Ez, Eb = torch.empty_like(Z), torch.empty_like(big)
    for _ in range(args.warmup):
        P.batched_uniform(Z, selector=args.selector, workspace=wsz, out=Ez)
        P.taylor(big, selector=args.selector, workspace=wsb)
    torch.cuda.synchronize()
    t0, t1, t2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    t0.record()
    for _ in range(args.steps):
        _, mz, sz, _ = P.batched_uniform(Z, selector=args.selector, workspace=wsz, out=Ez)
    t1.record()
    for _ in range(args.steps):
        _, mb, sb, _ = P.taylor(big, selector=args.selector, workspace=wsb)
    t2.record()
    torch.cuda.synchronize()
    ms_z = t0.elapsed_time(t1) / args.steps
    ms_b = t1.elapsed_time(t2) / args.steps
    mz, sz = mz.cpu().numpy(), sz.cpu().numpy()
    # algorithmic flops: a complex product is 8 n^3 real flops (4 real products)
    fl_z = 4 * executed_flops(mz, sz, [256] * 512)
    fl_b = executed_flops([int(mb.item())], [int(sb.item())], [8192])
    EzH = Ez.conj().transpose(-1, -2).contiguous()
    unit = float((torch.matmul(EzH, Ez) - torch.eye(256, dtype=torch.complex128, device="cuda")).abs().sum(-2).amax())
    cpu = None
    if not args.no_cpu:  # the oracle's complex direct Taylor on a few of the matrices, one thread
        import oracle
        oracle.set_threads(1)
        done, c0 = 0, time.perf_counter()
        while time.perf_counter() - c0 < args.cpu_seconds:
            oracle.expm_taylor(mats[done % 4])
            done += 1
        c1 = time.perf_counter()
        want, nproc, model = host_cpu()
        oracle.set_threads(want)
        cpu = {"value": done / (c1 - c0), "unit": "matrices/s", "cores": 1, "kind": "oracle", "nproc": nproc,
               "cpu_model": model, "sample": "%d of the 512 complex matrices (4 distinct), long-double complex direct "
                                             "Taylor, one thread, %.1f s" % (done, c1 - c0)}
    roof = {"bound": "mfma", "kernel": "lg_gemm_kernel (complex batch natively: four real products per complex "
                                         "product; n = 8192 matrix)",
            "achieved": (fl_z + fl_b) / ((ms_z + ms_b) * 1e-3) / 1e12, "peak": PEAK_FP64 / 1e12,
            "unit": "TFLOP/s", "frac": (fl_z + fl_b) / ((ms_z + ms_b) * 1e-3) / PEAK_FP64, "traffic": None,
            "note": "algorithmic flops: 8 n^3 per complex product, which is what the native complex path executes",
            "complex_batch_tflops": fl_z / (ms_z * 1e-3) / 1e12}
    config = {"workload": "512 complex128 -iH dt (n=256, Hermitian, spectral radius 1, dt log-U[1e-2,1e2]) + 1 FP64 "
                          "n=8192 ||A||_1=20", "selector": args.selector, "ms_complex_batch": ms_z,
              "ms_n8192": ms_b, "n8192_m_s": [int(mb.item()), int(sb.item())], "max_unitarity_err": unit}
    return line(args, "expm matrices/s (complex unitary + n=8192)", 513 / ((ms_z + ms_b) * 1e-3), ms_z + ms_b,
                "c128/f64", config, roof, cpu)


def run_learned(args, torch, P, W):
    from paper_1710_10989_amd import learned as LS
    from paper_1710_10989_amd.expm import Batch
    if os.path.exists(LS.DEFAULT_CKPT):
        net = LS.MLP()
        net.load(LS.DEFAULT_CKPT)
        trained = "checkpoint " + os.path.basename(LS.DEFAULT_CKPT)
    else:
        net = LS.train(LS.make_dataset(24576, seed=11), epochs=8)
        trained = "24576 matrices, 8 epochs (no checkpoint found)"
    LS.install(net)
    gen = torch.Generator().manual_seed(20000)
    stacks = [LS.device_batch(5000, n, gen) for n in LS.SIZES]
    packed = torch.cat([a.reshape(-1) for a in stacks])
    ns = torch.cat([torch.full((5000,), n, dtype=torch.int32) for n in LS.SIZES]).cuda()
    sizes = torch.cat([torch.full((5000,), n * n, dtype=torch.int64) for n in LS.SIZES])
    offs = torch.cat([torch.zeros(1, dtype=torch.int64), torch.cumsum(sizes, 0)[:-1]]).cuda()
    B = Batch(packed, offs, ns, 256)
    nb = 20000
    ws = torch.empty(P.workspace_bytes(256, nb), dtype=torch.uint8, device="cuda")
    outs = (torch.empty_like(packed), torch.empty(nb, dtype=torch.int32, device="cuda"),
            torch.empty(nb, dtype=torch.int32, device="cuda"), torch.empty(nb, dtype=torch.int32, device="cuda"))
    res = {}
    for sel in ("plain", "alpha", "learned"):
        for _ in range(args.warmup):
            P.batched(B, selector=sel, workspace=ws, outs=outs)
        torch.cuda.synchronize()
        if sel == "learned":
            LS.install(net)  # reset the counters
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(args.steps):
            P.batched(B, selector=sel, workspace=ws, outs=outs)
        t1.record()
        torch.cuda.synchronize()
        m, s, st = (x.cpu().numpy() for x in outs[1:])
        assert np.all(st == 0)
        nsh = ns.cpu().numpy()
        res[sel] = {"ms": t0.elapsed_time(t1) / args.steps, "m": m, "s": s,
                    "cost": float(np.mean([PRODUCTS[int(a)] + int(b) for a, b in zip(m, s)])),
                    "tflops": executed_flops(m, s, nsh) / (t0.elapsed_time(t1) / args.steps * 1e-3) / 1e12}
    acc, rej = LS.counts()
    acc //= max(1, args.steps)
    rej //= max(1, args.steps)
    nsh = ns.cpu().numpy()
    # dominant kernel of the learned run (order 256 on the 8-wave global-memory kernel): time
    # its phase alone with events
    kev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for i in range(args.steps):
        P.batched(B, selector="learned", workspace=ws, outs=outs, stage=0)
        kev[i][0].record()
        P.batched(B, selector="learned", workspace=ws, outs=outs, stage=3)
        kev[i][1].record()
        for stg in (1, 4, 5):
            P.batched(B, selector="learned", workspace=ws, outs=outs, stage=stg)
    torch.cuda.synchronize()
    ms_k8 = sum(a.elapsed_time(b) for a, b in kev) / args.steps
    big = ((nsh + 15) // 16) > 8
    ml, sl = res["learned"]["m"], res["learned"]["s"]
    achieved = executed_flops(ml[big], sl[big], nsh[big]) / (ms_k8 * 1e-3)
    cpu = None
    if not args.no_cpu:
        sample = [stacks[i % 4][i].cpu().numpy() for i in range(16)]
        cpu = cpu_oracle(sample, args.cpu_seconds, "16 of the held-out matrices (4 per order)")
    roof = {"bound": "mfma", "kernel": "expm_fused_kernel<8> (orders 144..256, learned selector)",
            "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64,
            "traffic": None, "kernel_ms": ms_k8}
    config = {"workload": "20000 held-out FP64 matrices, n in {32,64,128,256} (5000 each), ||A||_1 log-U[1e-2,1e3], "
                          "40/20/20/20 structure mix; one expm_batched call per step", "selector": "learned",
              "trained": trained,
              "matrices_per_s": {k: nb / (v["ms"] * 1e-3) for k, v in res.items()},
              "mean_products_plus_squarings": {k: v["cost"] for k, v in res.items()},
              "step_tflops": {k: v["tflops"] for k, v in res.items()},
              "learned_accepted": int(acc), "learned_rejected": int(rej)}
    return line(args, "expm matrices/s (learned selector, rel err <= 1e-12)", nb / (res["learned"]["ms"] * 1e-3),
                res["learned"]["ms"], "f64", config, roof, cpu)


PEAK_HBM = 8.0e12


def timed(torch, args, fn):
    """Average ms of fn() over args.steps calls after args.warmup, HIP events on the current
    stream (the launch stream of the calls)."""
    for _ in range(args.warmup):
        fn()
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(args.steps):
        fn()
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / args.steps


def run_small(args, torch, P, W):
    count, n = 65536, 16
    A = W.small_skew_batch(count=count, n=n)
    Ad = torch.from_numpy(A).cuda()
    ws = torch.empty(P.workspace_bytes(n, count, method=args.method), dtype=torch.uint8, device="cuda")
    out = torch.empty_like(Ad)
    outs = tuple(torch.empty(count, dtype=torch.int32, device="cuda") for _ in range(3))

    mt = args.method

    def step():
        P.batched_uniform(Ad, selector=args.selector, workspace=ws, out=out, outs=outs, method=mt)

    ms = timed(torch, args, step)
    m, s, st = (x.cpu().numpy() for x in outs)
    assert np.all(st == 0)
    prods = {"reduced": PRODUCTS, "ps": PS_PRODUCTS, "pade": {10: 3 + 4.0 / 3.0, 26: 6 + 4.0 / 3.0}}[mt]
    nbytes = count * (16 * n * n + 12)  # A in, e^A out, (m, s, status) out
    achieved = nbytes / (ms * 1e-3)
    roof = {"bound": "hbm", "kernel": "expm_tiny_kernel (one wave per matrix)", "achieved": achieved / 1e9,
            "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": achieved / PEAK_HBM,
            "traffic": measured_traffic("expm_tiny_kernel_65536_n16"), "kernel_ms": ms,
            "step_tflops": executed_flops(m, s, [n] * count, prods) / (ms * 1e-3) / 1e12}
    cpu = None
    if not args.no_cpu:
        cpu = cpu_oracle([A[i] for i in range(4096)], args.cpu_seconds, "4096 of the matrices")
    config = {"workload": "%d FP64 skew-symmetric matrices of order %d (Magnus-integrator exponents), "
                          "||A||_1 log-uniform [0.05, 1]; one expm_batched_uniform call per step" % (count, n),
              "selector": args.selector, "method": mt,
              "mean_products_plus_squarings": float(np.mean([prods[int(a)] + int(b) for a, b in zip(m, s)]))}
    return line(args, "expm matrices/s (rel err <= 1e-12, FP64)", count / (ms * 1e-3), ms, "f64", config, roof, cpu)


def run_magnus(args, torch, P, W):
    count, n, h = 65536, 16, 0.1
    S0, S1, Y0, a, w, phi = W.magnus_systems(count=count, n=n)
    u1, u2 = W.control_at_gauss_points(a, w, phi, 0.0, h)
    d = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (S0, S1, Y0, u1, u2)]
    Yo = torch.empty_like(d[2])
    outs = tuple(torch.empty(count, dtype=torch.int32, device="cuda") for _ in range(3))

    def step():
        P.magnus4_step(d[0], d[1], d[2], d[3], d[4], h, selector=args.selector, out=Yo, outs=outs)

    ms = timed(torch, args, step)
    m, s, st = (x.cpu().numpy() for x in outs)
    assert np.all(st == 0)
    nbytes = count * (4 * 8 * n * n + 16 + 12)  # S0, S1, Y in, Y out; u1, u2; (m, s, status)
    achieved = nbytes / (ms * 1e-3)
    gemms = [3 + PRODUCTS[int(a_)] + int(b_) for a_, b_ in zip(m, s)]  # commutator (2), e^Omega, e^Omega Y
    roof = {"bound": "hbm", "kernel": "expm_magnus4_kernel (one wave per system)", "achieved": achieved / 1e9,
            "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": achieved / PEAK_HBM,
            "traffic": measured_traffic("expm_magnus4_kernel_65536_n16"), "kernel_ms": ms,
            "step_tflops": sum(gemms) * 2.0 * n ** 3 / (ms * 1e-3) / 1e12}
    cpu = None
    if not args.no_cpu:
        import oracle
        done, c0 = 0, time.perf_counter()
        while time.perf_counter() - c0 < args.cpu_seconds:
            b = done % count
            oracle.magnus4_step(S0[b], S1[b], Y0[b], u1[b], u2[b], h, prec="d")
            done += 1
        c1 = time.perf_counter()
        cpu = {"value": done / (c1 - c0), "unit": "steps/s", "cores": 1, "kind": "oracle",
               "sample": "%d systems of the workload, one step each (FP64 Omega, FP64 direct-Taylor "
                         "exponential, one thread), %.1f s" % (done, c1 - c0)}
    config = {"workload": "%d linear systems Y' = (S0 + u(t) S1) Y of order %d, S0, S1 skew (||.||_1 = 2, 1), "
                          "u = a cos(w t + phi), one fourth-order Magnus step of h = %g per step "
                          "(expm_magnus4_step)" % (count, n, h),
              "selector": args.selector,
              "mean_products_plus_squarings": float(np.mean([PRODUCTS[int(a_)] + int(b_) for a_, b_ in zip(m, s)]))}
    return line(args, "Magnus-4 system steps/s (FP64)", count / (ms * 1e-3), ms, "f64", config, roof, cpu,
                unit="steps/s")


def run_triangular(args, torch, P, W):
    count, n = 64, 512
    A = W.triangular_batch(count=count, n=n)
    Ad = torch.from_numpy(A).cuda()
    ws = torch.empty(P.workspace_bytes(n, count, method="tri"), dtype=torch.uint8, device="cuda")
    out = torch.empty_like(Ad)
    outs = tuple(torch.empty(count, dtype=torch.int32, device="cuda") for _ in range(3))
    d = torch.from_numpy(np.exp(A[:, np.arange(n), np.arange(n)])).cuda()
    res = {}
    for mt in ("reduced", "tri"):  # both on the tiled path (n = 512)
        ms = timed(torch, args, lambda: P.batched_uniform(Ad, workspace=ws, out=out, outs=outs, method=mt))
        diag = torch.diagonal(out, dim1=1, dim2=2)
        res[mt] = {"ms": ms, "max_rel_err_diagonal": float(((diag - d).abs() / d).max())}
    m, s, st = (x.cpu().numpy() for x in outs)
    assert np.all(st == 0)
    ms = res["tri"]["ms"]
    flops = executed_flops(m, s, [n] * count)
    roof = {"bound": "mfma", "kernel": "lg_gemm_kernel (tiled 128x128, all GEMM steps) + lg_tri_fix_kernel",
            "achieved": flops / (ms * 1e-3) / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
            "frac": flops / (ms * 1e-3) / PEAK_FP64, "traffic": None, "kernel_ms": ms}
    cpu = None if args.no_cpu else cpu_oracle([A[0]], args.cpu_seconds, "1 of the 64 matrices")
    config = {"workload": "%d upper triangular FP64 matrices of order %d, diagonal uniform in [-40, 0], strictly "
                          "upper N(0,1)/sqrt(n); one expm_batched_uniform call per step with the triangular "
                          "refinement (EXPM_FLAG_TRI)" % (count, n),
              "unrefined_ms": res["reduced"]["ms"], "refined_ms": ms,
              "max_rel_err_diagonal": {k: v["max_rel_err_diagonal"] for k, v in res.items()},
              "mean_products_plus_squarings": float(np.mean([PRODUCTS[int(a)] + int(b) for a, b in zip(m, s)]))}
    return line(args, "expm matrices/s (triangular refinement, FP64)", count / (ms * 1e-3), ms, "f64", config, roof,
                cpu)


def run_comparison(args, torch, P, W):
    """The paper's cost comparison (Sec. 4, Table 3; abstract: 10-30 % cheaper than Pade) as
    MI355X wall time: the product-reduced Taylor method, the Paterson-Stockmeyer evaluation of the
    plain Taylor polynomial and diagonal Pade r_10 / r_26, all FP64 with the plain ||A||_1 rule,
    on the same kernels (orders above 256 run the tiled path for every method) and the same
    matrices: orders 384, 512 and 1024, dense N(0,1)/sqrt(n) scaled to ||A||_1 log-uniform in
    [1e-2, 1e2]."""
    cases = [(384, 64), (512, 64), (1024, 32)]
    g = np.random.default_rng(1710109890 + 10)
    stacks = []
    for n, count in cases:
        mats = [W.rescale(g.standard_normal((n, n)) / np.sqrt(n), float(np.exp(g.uniform(np.log(1e-2), np.log(1e2)))))
                for _ in range(count)]
        stacks.append(torch.from_numpy(np.stack(mats)).cuda())
    costs = {"reduced": {m: p for m, p in PRODUCTS.items()}, "ps": PS_PRODUCTS,
             "pade": {10: 3 + 4.0 / 3.0, 26: 6 + 4.0 / 3.0}}
    res = {}
    for mt in ("reduced", "ps", "pade"):
        ws = [torch.empty(P.workspace_bytes(A.shape[1], A.shape[0], method=mt), dtype=torch.uint8, device="cuda")
              for A in stacks]
        outs = [torch.empty_like(A) for A in stacks]

        def step():
            return [P.batched_uniform(A, workspace=w, out=o, method=mt) for A, w, o in zip(stacks, ws, outs)]

        ms = timed(torch, args, step)
        r = step()
        torch.cuda.synchronize()
        per = {}
        for (n, count), (_, m, s, st) in zip(cases, r):
            assert bool((st == 0).all())
            m, s = m.cpu().numpy(), s.cpu().numpy()
            per[n] = float(np.mean([costs[mt][int(a)] + int(b) for a, b in zip(m, s)]))
        res[mt] = {"ms": ms, "mean_products_plus_squarings": per, "outs": outs}
    # the three methods agree (each within its own truncation and rounding of e^A)
    dev = 0.0
    for i in range(len(cases)):
        for mt in ("ps", "pade"):
            X, R = res[mt]["outs"][i], res["reduced"]["outs"][i]
            dev = max(dev, float(((X - R).abs().sum(-2).amax(-1) / R.abs().sum(-2).amax(-1)).max()))
    total = sum(c for _, c in cases)
    config = {"workload": "orders 384 (64), 512 (64), 1024 (32): dense N(0,1)/sqrt(n), ||A||_1 log-uniform "
                          "[1e-2, 1e2]; three expm_batched_uniform calls per step per method, FP64, plain rule",
              "ms_per_step": {k: v["ms"] for k, v in res.items()},
              "matrices_per_s": {k: total / (v["ms"] * 1e-3) for k, v in res.items()},
              "mean_products_plus_squarings": {k: v["mean_products_plus_squarings"] for k, v in res.items()},
              "time_vs_pade": res["reduced"]["ms"] / res["pade"]["ms"],
              "time_vs_ps": res["reduced"]["ms"] / res["ps"]["ms"],
              "max_rel_diff_between_methods": dev}
    return line(args, "expm matrices/s (product-reduced Taylor vs Paterson-Stockmeyer vs Pade, FP64)",
                total / (res["reduced"]["ms"] * 1e-3), res["reduced"]["ms"], "f64", config, None, None)


def run_copy(args, torch, P, W):
    nbytes = 1 << 30
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(args.warmup):
        dst.copy_(src)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(args.steps):
        dst.copy_(src)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / args.steps
    return {"metric": "device copy GB/s (calibration)", "value": 2 * nbytes / (ms * 1e-3) / 1e9, "unit": "GB/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "copy of %d bytes (read %d + write %d per launch)" % (nbytes, nbytes, nbytes)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 50 for the sub-millisecond workloads batched, small and "
                         "magnus, else 20)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps before them (default: 50 for batched, small and magnus, whose "
                         "first few dozen calls run while the GPU's clocks are still rising; else 5)")
    ap.add_argument("--workload", default="batched", choices=["batched", "single", "precision", "complex", "learned",
                                                             "small", "magnus", "triangular", "comparison", "copy"])
    ap.add_argument("--selector", default="plain", choices=["plain", "alpha"])
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32", "bf16x3", "fp32all"])
    ap.add_argument("--method", default="reduced", choices=["reduced", "ps", "pade"],
                    help="the paper's T_m or a comparison method (ps: precision and small workloads; "
                         "pade: small workload)")
    ap.add_argument("--count", type=int, default=4096)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="ignore the autotuner's cache (library defaults)")
    ap.add_argument("--plain-passes", type=int, default=3,
                    help="timed passes of the plain one-launch-per-matrix form (batched workload; 0: skip it)")
    args = ap.parse_args()
    fast = args.workload in ("batched", "small", "magnus")
    if args.steps is None:
        args.steps = 50 if fast else 20
    if args.warmup is None:
        args.warmup = 50 if fast else 5
    if args.gpus != 1:
        print("bench.py measures one GPU: the method runs on a single MI355X (multi-GPU sharding "
              "is a design note, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1710_10989_amd as P
    from paper_1710_10989_amd import workloads as W
    from paper_1710_10989_amd import autotune as T
    # launch configuration: the autotuner's cache entry for this GPU architecture, if any
    installed = None if args.no_tune else T.install()
    args.tuning = {"source": "defaults (no cache entry for %s)" % T.arch() if installed is None and not args.no_tune
                   else "defaults (--no-tune)" if installed is None else "autotuner cache (%s)" % T.arch(),
                   "values": T.to_dict(T.get())}
    fn = {"batched": run_batched, "single": run_single, "precision": run_precision, "complex": run_complex,
          "learned": run_learned, "small": run_small, "magnus": run_magnus,
          "triangular": run_triangular, "comparison": run_comparison, "copy": run_copy}
    out = fn[args.workload](args, torch, P, W)
    if "config" in out:
        out["config"]["tuning"] = args.tuning
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
