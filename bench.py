#!/usr/bin/env python3
"""Time-to-tolerance of the accelerated farPCA loop (arXiv 2506.03859) on one
MI355X, through the C-ABI.

Workload (default): A = U diag(sigma) V^T, 20000 x 15000 FP32, sigma_i =
exp(-i/50) + 1e-6, U, V Haar (QR of seeded Gaussians); sparse sign test
matrix with zeta = 8 nonzeros per row (+-1/sqrt(8)), b = 64, P = 2, relative
tolerance 1e-3.  A step is one whole solve - every block of the loop and the
final decomposition - with A resident in HBM; block seeds 1000 + r.
Other workloads (--workload): the tall fixed-rank matrix, and the precision
form (the same matrix stored in BF16, sparse Gaussian density 0.05 or sparse
sign, tol 1e-2) beside its FP32 twin.

The JSON line carries the roofline of the dominant kernel (HIP events on the
library's stream around every launch of the kernel classes that stream A),
the sparse sketch's HBM rate, and the FP64 CPU oracle timed on a bounded
sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
PEAK_FP32_MFMA_TFLOPS = 157.3

WORKLOADS = {
    # name: (m, n, spectrum, seed, tol, b, P, sketch, zeta, p, storage of A)
    "exp50_20000x15000_ss8": (20000, 15000, "exp50", 2, 1e-3, 64, 2, "sparse_sign", 8, 0.0, "f32"),
    "tall_200000x4000_rank200": (200000, 4000, "tall", 4, 0.0, 50, 1, "sparse_sign", 4, 0.0, "f32"),
    # precision form: the same matrix stored in BF16 (round to nearest even),
    # sparse Gaussian test matrix of density 0.05, tol 1e-2; and its FP32 twin
    "bf16_exp50_20000x15000_sg05": (20000, 15000, "exp50", 2, 1e-2, 64, 2, "sparse_gaussian", 0,
                                    0.05, "bf16"),
    "exp50_20000x15000_sg05": (20000, 15000, "exp50", 2, 1e-2, 64, 2, "sparse_gaussian", 0, 0.05,
                               "f32"),
    "bf16_exp50_20000x15000_ss8_tol1e-2": (20000, 15000, "exp50", 2, 1e-2, 64, 2, "sparse_sign", 8,
                                           0.0, "bf16"),
    "exp50_20000x15000_ss8_tol1e-2": (20000, 15000, "exp50", 2, 1e-2, 64, 2, "sparse_sign", 8, 0.0,
                                      "f32"),
    # the paper's sparse regime (p = 1e-3, about 15 nonzeros per column of
    # Omega_j) with A stored column-major, so that the sketch gathers only the
    # columns Omega_j touches; and the same solve on row-major A
    "col_exp50_20000x15000_sg1e-3": (20000, 15000, "exp50", 2, 1e-2, 64, 2, "sparse_gaussian", 0,
                                     1e-3, "f32"),
    "exp50_20000x15000_sg1e-3": (20000, 15000, "exp50", 2, 1e-2, 64, 2, "sparse_gaussian", 0, 1e-3,
                                 "f32"),
}
# storage order of A (default row-major)
LAYOUTS = {"col_exp50_20000x15000_sg1e-3": "col"}


def counter_profiled():
    """True inside a rocprofv3 --pmc run (the profiler's counter settings are in the environment)."""
    v = os.environ.get("ROCPROF_COUNTER_COLLECTION", "")
    return v not in ("", "0", "false", "False") or bool(os.environ.get("ROCPROF_COUNTERS"))


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def make_matrix(name, device):
    import numpy as np
    import torch
    from paper_2506_03859_amd import synth
    m, n, spec, seed = WORKLOADS[name][:4]
    storage = WORKLOADS[name][10]
    if spec == "exp50":
        sigma = synth.exp_floor_sigma(min(m, n), decay=50.0, floor=1e-6)
        a64 = synth.spectral_torch(m, n, sigma, seed, device=device)
        a = a64.to(torch.float32).contiguous()
        del a64
    else:
        a = torch.from_numpy(synth.tall_lowrank(m, n, 100, 1e-6, seed, dtype=np.float32)).to(device)
    if storage == "bf16":
        a = a.to(torch.bfloat16).contiguous()     # round to nearest even
    if LAYOUTS.get(name, "row") == "col":
        a = a.t().contiguous().t()                # column-major view (A^T row-major in memory)
    torch.cuda.synchronize()
    return a


def source_hash(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


KERNEL_SOURCES = {
    "gemm_tn": ["paper_2506_03859_amd/csrc/gemm.hip"],
    "gemm_nn": ["paper_2506_03859_amd/csrc/gemm.hip"],
    "sketch": ["paper_2506_03859_amd/csrc/sketch.hip"],
    "gemm_tn_bf16": ["paper_2506_03859_amd/csrc/gemm_bf16.hip"],
    "gemm_tn_split": ["paper_2506_03859_amd/csrc/gemm_bf16.hip"],
    "gemm_nn_split": ["paper_2506_03859_amd/csrc/gemm_bf16.hip"],
    "gemm_nn_bf16": ["paper_2506_03859_amd/csrc/gemm_bf16.hip"],
    "sketch_bf16": ["paper_2506_03859_amd/csrc/sketch.hip"],
}


def measured_traffic(kernel):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha") != source_hash(KERNEL_SOURCES[kernel]):
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(a_dev, wl, blocks_gpu, min_seconds=10.0, max_solves=5):
    """The FP64 oracle on the same matrix (upcast), same parameters and seeds
    as the timed solves, run as whole solves until about `min_seconds` of CPU
    time have passed (a bounded sample of the workload)."""
    import numpy as np
    from oracle import FarpcaParams, farpca
    m, n, _, _, tol, b, P, sketch, zeta, p, _ = WORKLOADS[wl]
    a = a_dev.float().cpu().numpy().astype(np.float64)
    try:
        from threadpoolctl import threadpool_info
        cores = max(int(i.get("num_threads", 1)) for i in threadpool_info()) if threadpool_info() else 1
    except Exception:
        cores = len(os.sched_getaffinity(0))
    log(f"cpu baseline: oracle, whole solves of {m}x{n} in FP64 on {cores} threads")
    t0 = time.perf_counter()
    runs = []
    while len(runs) < max_solves and (time.perf_counter() - t0 < min_seconds or not runs):
        prm = FarpcaParams(tol=tol, rank=(200 if tol == 0.0 else 0), block=b, power=P, sketch=sketch,
                           p=p, zeta=zeta, seed=1000 + len(runs))
        res = farpca(a, prm)
        runs.append(res.blocks)
    dt = time.perf_counter() - t0
    per_solve = dt / len(runs)
    # one more solve on a single BLAS thread (the oracle's serial cost)
    single_ms, blas = None, None
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        blas = sorted({f"{i.get('internal_api')} {i.get('version')}" for i in threadpool_info()})
        with threadpool_limits(limits=1):
            t1 = time.perf_counter()
            farpca(a, FarpcaParams(tol=tol, rank=(200 if tol == 0.0 else 0), block=b, power=P,
                                   sketch=sketch, p=p, zeta=zeta, seed=1000))
            single_ms = (time.perf_counter() - t1) * 1e3
    except Exception as e:        # threadpoolctl missing or unable to limit: report none
        log(f"cpu baseline: no single-thread run ({e})")
    return {"value": len(runs) / dt, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(runs)} whole oracle solves (NumPy FP64, seeds 1000..) on the same {m}x{n} "
                      f"matrix upcast to FP64, {sorted(set(runs))} blocks each, {dt:.1f} s in total; "
                      f"{per_solve * 1e3:.0f} ms per solve (GPU solves: {blocks_gpu} blocks)",
            "ms_per_solve": per_solve * 1e3, "single_thread_ms_per_solve": single_ms, "blas": blas}


def time_solves(wl, A, steps, warmup, dev):
    """Whole solves of workload `wl` on the device matrix A: warm-up, then
    `steps` timed solves with HIP-event timing of the kernel classes.  Returns
    a summary (ms per solve, the A-pass and sketch rates, ranks)."""
    import torch
    from paper_2506_03859_amd import farpca as fp
    m, n, _, _, tol, b, P, sketch, zeta, p, storage = WORKLOADS[wl]
    rank = 200 if tol == 0.0 else 0
    plans = [fp.farpca_plan(fp.make_params(m, n, tol=tol, rank=rank, block=b, power=P, sketch=sketch,
                                           p=p, zeta=zeta, seed=1000 + r, a_dtype=storage,
                                           layout=LAYOUTS.get(wl, "row")))
             for r in range(warmup + steps)]
    work, U, S, V, eh = fp.alloc_outputs(plans[0], dev)
    for r in range(warmup):
        fp.farpca_run(plans[r], A, work, U, S, V, eh)
    torch.cuda.synchronize()
    fp.farpca_profile_enable(True)
    t0 = time.perf_counter()
    infos = []
    for r in range(steps):
        st, info = fp.farpca_run(plans[warmup + r], A, work, U, S, V, eh)
        infos.append((st, info.rank_l, info.blocks, info.eig_sweeps))
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    prof = {c: fp.farpca_profile_get(c) for c in fp.PROF_CLASSES}
    fp.farpca_profile_enable(False)
    for pl in plans:
        pl.free()
    elem = 2.0 if storage == "bf16" else 4.0
    out = {"workload": wl, "m": m, "n": n, "tol": tol, "rank": rank, "block": b, "power": P,
           "sketch": sketch, "zeta": zeta, "p": p, "a_storage": storage, "steps": steps,
           "ms_per_solve": ms, "solves_per_s": 1e3 / ms,
           "l": sorted({i[1] for i in infos}), "blocks": sorted({i[2] for i in infos}),
           "status": sorted({i[0] for i in infos})}
    for c in ("gemm_tn", "gemm_nn", "gemm_c", "sketch", "eig"):
        tot, cnt = prof[c]
        if not cnt:
            continue
        a_ms = tot / cnt
        rec = {"avg_launch_ms": a_ms, "total_ms_per_solve": tot / steps}
        if c.startswith("gemm"):
            rec["tflops"] = 2.0 * m * n * b / (a_ms * 1e-3) / 1e12
            rec["a_GBps"] = elem * m * n / (a_ms * 1e-3) / 1e9
            # FP32 matrix-core fraction only where the pass runs on them (column-
            # major FP32 A; row-major FP32 A runs every A-pass split on BF16)
            on_fp32 = storage == "f32" and LAYOUTS.get(wl, "row") == "col"
            rec["mfma_frac"] = rec["tflops"] / PEAK_FP32_MFMA_TFLOPS if on_fp32 else None
            rec["hbm_frac"] = rec["a_GBps"] / PEAK_HBM_GBPS
        elif c == "sketch":
            rec["GBps"] = (elem * m * n + 4.0 * m * b) / (a_ms * 1e-3) / 1e9
            rec["hbm_frac"] = rec["GBps"] / PEAK_HBM_GBPS
        out[c] = rec
    return out


def kernel_probe(wl, dev, reps=3):
    """The kernels that stream A, each launched `reps` times on a random matrix
    of the workload's shape, then a 1 GiB device-to-device copy (a plain read +
    write of known size for scaling FETCH_SIZE / WRITE_SIZE)."""
    import torch
    from paper_2506_03859_amd import farpca as fp
    m, n, _, _, tol, b, P, sketch, zeta, p, storage = WORKLOADS[wl]
    A = torch.randn(m, n, device=dev)
    if storage == "bf16":
        A = A.to(torch.bfloat16)
    skinny_n = torch.randn(n, 64, device=dev)
    skinny_m = torch.randn(m, 64, device=dev)
    Cm = torch.zeros(m, 64, device=dev)
    Cn = torch.zeros(n, 64, device=dev)
    layout = LAYOUTS.get(wl, "row")
    plan = fp.farpca_plan(fp.make_params(m, n, tol=tol, rank=(200 if tol == 0.0 else 0), block=b,
                                         power=P, sketch=sketch, p=p, zeta=zeta, seed=1000,
                                         a_dtype=storage, layout=layout))
    work, _, _, _, _ = fp.alloc_outputs(plan, dev)
    if storage == "bf16":
        nb = fp.farpca_gemm_bf16_scratch_bytes(max(m, n), max(m, n))
        buf = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
        off = (-buf.data_ptr()) % 256
        scratch = buf[off:off + nb]
        gemm_tn, gemm_nn = fp.farpca_gemm_bf16_tn, fp.farpca_gemm_bf16_nn
    elif layout == "row":
        # the solve's A-passes on row-major FP32 A run split on the BF16
        # matrix cores
        nb = max(fp.farpca_gemm_bf16_scratch_bytes(max(m, n), max(m, n)),
                 fp.farpca_gemm_scratch_bytes(max(m, n)))
        buf = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
        off = (-buf.data_ptr()) % 256
        scratch = buf[off:off + nb]
        gemm_tn, gemm_nn = fp.farpca_gemm_f32s_tn, fp.farpca_gemm_f32s_nn
    else:
        scratch = torch.empty(fp.farpca_gemm_scratch_bytes(max(m, n)) // 4, device=dev)
        gemm_tn, gemm_nn = fp.farpca_gemm_tn, fp.farpca_gemm_nn
    for r in range(reps):
        gemm_tn(A, skinny_m, Cn, n, b, m, scratch)
        gemm_nn(A, skinny_n, Cm, m, b, n, scratch)
        # column-major workloads: the sketch reads A^T row-major (same buffer, n x m)
        fp.farpca_sketch(plan, A if layout == "row" else A.reshape(n, m), r, work, Cm)
    torch.cuda.synchronize()
    plan.free()
    del A
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)      # an elementwise kernel: reads 1 GiB, writes 1 GiB
    torch.cuda.synchronize()
    log(f"kernel probe done ({reps} launches each, then a {src.numel() * 4 >> 20} MiB copy)")


def serve_trace(nreq=512, rate=200.0, seed=5, bank=24):
    """The serving workload: nreq requests with Poisson arrivals at `rate` per
    second; shapes m in [500, 8000], n in [300, 4000] log-uniform; spectra
    i^-1.5, exp(-i/30) or rank r + noise (r log-uniform in [5, min(m,n)/4],
    noise variance 1e-6 sigma_1^2); tol in {1e-2, 1e-3, 1e-4}; storage FP32 or
    BF16 (BF16 only where tol >= 4x the BF16 storage error, else FP32);
    sparse sign test matrix (zeta = 8), b by the default rule, P = 1.  The
    matrices come from a bank of `bank` seeded matrices drawn from the same
    distribution (generation cost); each request picks one, plus its own tol,
    storage and seed."""
    import numpy as np
    rng = np.random.default_rng(seed)
    mats = []
    for i in range(bank):
        m = int(round(math.exp(rng.uniform(math.log(500), math.log(8000)))))
        n = int(round(math.exp(rng.uniform(math.log(300), math.log(4000)))))
        kind = ("pow", "exp", "lowrank")[i % 3]
        r = int(round(math.exp(rng.uniform(math.log(5), math.log(max(6, min(m, n) // 4))))))
        mats.append((m, n, kind, r, 5000 + i))
    t = np.cumsum(rng.exponential(1.0 / rate, size=nreq))
    reqs = []
    for i in range(nreq):
        reqs.append(dict(t=float(t[i]), mat=int(rng.integers(0, bank)),
                         tol=float(rng.choice([1e-2, 1e-3, 1e-4])),
                         bf16=bool(rng.integers(0, 2)), seed=10000 + i))
    return mats, reqs


def serve_matrix(spec, device):
    import numpy as np
    import torch
    from paper_2506_03859_amd import synth
    m, n, kind, r, seed = spec
    k = min(m, n, 1024)
    if kind == "pow":
        a = synth.spectral_torch(m, n, np.arange(1, k + 1, dtype=np.float64) ** -1.5, seed, device)
    elif kind == "exp":
        a = synth.spectral_torch(m, n, np.exp(-np.arange(1, k + 1, dtype=np.float64) / 30.0), seed, device)
    else:
        a = synth.spectral_torch(m, n, np.ones(min(r, k)), seed, device)
        g = torch.Generator(device=device).manual_seed(seed)
        a += 1e-3 * torch.randn(m, n, generator=g, device=device, dtype=torch.float64)
    return a.to(torch.float32).contiguous()


def padded_rows(a, mult):
    """Row-major copy of a with its leading dimension rounded up to `mult`
    elements (zero padding), returned as the m x n view."""
    import torch
    m, n = a.shape
    ld = (n + mult - 1) // mult * mult
    buf = torch.zeros((m, ld), dtype=a.dtype, device=a.device)
    buf[:, :n] = a
    return buf[:, :n]


def serve_bench(args, dev, emit=True):
    """Open-loop replay of the serving trace through farpca_server_*: the
    mixed-storage trace (BF16 where eligible) and the same trace all in FP32,
    `serve_repeats` times each in alternation, and the BF16-eligible requests as
    one burst in each storage (alternating, the same number of times).  For the
    bursts every result's relative error ||A - U S V^T||_F / ||A||_F against the
    FP32 matrix is measured (torch FP64 on the device), so that the two forms
    are compared at their accuracy (served results against the FP64 oracle:
    tests/test_gpu_serve.py)."""
    import threading

    import numpy as np
    import torch
    from paper_2506_03859_amd import farpca as fp
    mats, reqs = serve_trace(nreq=args.serve_requests)
    log(f"serve: generating {len(mats)} matrices")
    # rows padded to 16 bytes (lda a multiple of 4 FP32 / 8 BF16 elements), the
    # layout the library's vector loads take for any width
    A32 = [padded_rows(serve_matrix(sp, dev), 4) for sp in mats]
    A16 = [padded_rows(a.to(torch.bfloat16), 8) for a in A32]
    floor = []
    for a, b16 in zip(A32, A16):
        floor.append(float(torch.linalg.norm(b16.float() - a) / torch.linalg.norm(a)))
    torch.cuda.synchronize()
    log("serve: matrices ready")
    pool = int(args.serve_pool_gb * (1 << 30))

    def eligible(q):
        return q["bf16"] and q["tol"] >= 4 * floor[q["mat"]]

    def replay(mode, sub=None, keep=False):
        # sub: (requests, storage) replayed as one burst (all submitted at once)
        rq = reqs if sub is None else sub[0]
        srv = fp.Server(pool, slots=args.serve_slots, starve_s=0.25)
        prms, store = [], []
        for q in rq:
            m, n = mats[q["mat"]][:2]
            bf = (mode == "mixed" and eligible(q)) if sub is None else sub[1] == "bf16"
            A = A16[q["mat"]] if bf else A32[q["mat"]]
            prms.append(fp.make_params(m, n, A.stride(0), tol=q["tol"], power=1, sketch="sparse_sign", zeta=8,
                                       seed=q["seed"], a_dtype="bf16" if bf else "f32"))
            store.append(bf)
        results, kept = {}, {}
        t_start = time.perf_counter()

        def submitter():
            for i, q in enumerate(rq):
                dt = t_start + q["t"] - time.perf_counter() if sub is None else 0.0
                if dt > 0:
                    time.sleep(dt)
                A = A16[q["mat"]] if store[i] else A32[q["mat"]]
                srv.submit(prms[i], A, i)

        th = threading.Thread(target=submitter)
        th.start()
        while len(results) < len(rq):
            for r in srv.poll(64, wait_ms=50):
                results[r.tag] = (r.status, r.t_submit, r.t_admit, r.t_done, r.info.rank_l)
                if keep and r.status >= 0 and r.info.rank_out > 0:
                    k = r.info.rank_out
                    U = torch.empty((r.m, k), dtype=torch.float32, device=dev)
                    S = torch.empty((k,), dtype=torch.float64, device=dev)
                    V = torch.empty((r.n, k), dtype=torch.float32, device=dev)
                    srv.fetch(r, U, S, V)
                    torch.cuda.synchronize()
                    kept[r.tag] = (U, S, V)
                srv.release(r.tag)
        th.join()
        mem = srv.memory()
        srv.close()
        lat = np.array([v[3] - v[1] for v in results.values()])
        t_first = min(v[1] for v in results.values())
        t_last = max(v[3] for v in results.values())
        st = [v[0] for v in results.values()]
        out = {"solves_per_s": len(rq) / (t_last - t_first), "wall_s": t_last - t_first,
               "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
               "mean_ms": float(lat.mean() * 1e3), "converged": int(sum(1 for x in st if x == 0)),
               "capped": int(sum(1 for x in st if x == 1)), "errors": int(sum(1 for x in st if x < 0)),
               "bf16_requests": int(sum(store)), "peak_pool_GiB": mem[1] / (1 << 30),
               "grows": mem[2], "preemptions": mem[3]}
        log(f"serve {mode}: {out}")
        return (out, kept, rq, store) if keep else out

    def spread(runs, key="solves_per_s"):
        v = [r[key] for r in runs]
        return {"runs": v, "mean": float(np.mean(v)), "min": float(np.min(v)), "max": float(np.max(v))}

    reps = max(1, args.serve_repeats)
    mixed, f32 = [], []
    for _ in range(reps):
        mixed.append(replay("mixed"))
        f32.append(replay("fp32"))
    elig = [q for q in reqs if eligible(q)]
    burst = {"requests": len(elig)}
    if elig:
        b16, b32 = [], []
        acc = {}
        for r in range(reps):
            keep = r == 0
            o16 = replay("burst_bf16", (elig, "bf16"), keep=keep)
            o32 = replay("burst_fp32", (elig, "f32"), keep=keep)
            if keep:
                acc = {"bf16": o16[1:], "fp32": o32[1:]}
                o16, o32 = o16[0], o32[0]
            b16.append(o16)
            b32.append(o32)
        burst["bf16"] = spread(b16)
        burst["fp32"] = spread(b32)
        burst["bf16_p99_ms"] = [x["p99_ms"] for x in b16]
        burst["fp32_p99_ms"] = [x["p99_ms"] for x in b32]
        # accuracy of each result: relative Frobenius error against the FP32 matrix
        errs = {}
        for form, (kept, rq, store) in acc.items():
            e = []
            for i, (U, S, V) in kept.items():
                a = A32[rq[i]["mat"]].double()
                rec = (U.double() * S) @ V.double().T
                e.append(float(torch.linalg.norm(a - rec) / torch.linalg.norm(a)))
            errs[form] = e
        burst["rel_error_vs_fp32_A"] = {form: {"median": float(np.median(e)), "max": float(np.max(e))}
                                        for form, e in errs.items() if e}
    line = {
        "metric": "served solves/s + p99 vs plain FP32",
        "value": float(np.mean([x["solves_per_s"] for x in mixed])), "unit": "solves/s", "n_gpus": 1,
        "higher_is_better": True, "dtype": "bf16+f32", "data": "synthetic",
        "config": {"workload": f"serve_{len(reqs)}req_poisson200", "slots": args.serve_slots,
                   "hw_queues": args.serve_hw_queues or None, "repeats": reps,
                   "pool_GiB": args.serve_pool_gb, "matrices": len(mats), "power": 1, "sketch": "sparse_sign",
                   "zeta": 8, "bf16_floor_median": float(np.median(floor))},
        "mixed": spread(mixed), "fp32": spread(f32),
        "mixed_p99_ms": [x["p99_ms"] for x in mixed], "fp32_p99_ms": [x["p99_ms"] for x in f32],
        "mixed_runs": mixed, "fp32_runs": f32,
        "eligible_burst": burst,
        "vs_baseline": None,
    }
    if emit:
        print(json.dumps(line), flush=True)
    return line


def serve_burst(args, dev):
    """The BF16-eligible requests of the serving trace submitted at once in one
    storage form, served `serve_repeats` times (the burst of serve_bench alone)."""
    import numpy as np
    import torch
    from paper_2506_03859_amd import farpca as fp
    mats, reqs = serve_trace(nreq=args.serve_requests)
    A32 = [padded_rows(serve_matrix(sp, dev), 4) for sp in mats]
    A16 = [padded_rows(a.to(torch.bfloat16), 8) for a in A32]
    floor = [float(torch.linalg.norm(b.float() - a) / torch.linalg.norm(a)) for a, b in zip(A32, A16)]
    torch.cuda.synchronize()
    elig = [q for q in reqs if q["bf16"] and q["tol"] >= 4 * floor[q["mat"]]]
    form = args.serve_burst
    rates = []
    for _ in range(max(1, args.serve_repeats)):
        srv = fp.Server(int(args.serve_pool_gb * (1 << 30)), slots=args.serve_slots, starve_s=0.25)
        t0 = time.perf_counter()
        for i, q in enumerate(elig):
            m, n = mats[q["mat"]][:2]
            A = A16[q["mat"]] if form == "bf16" else A32[q["mat"]]
            srv.submit(fp.make_params(m, n, A.stride(0), tol=q["tol"], power=1, sketch="sparse_sign", zeta=8,
                                      seed=q["seed"], a_dtype=form), A, i)
        done = 0
        while done < len(elig):
            for r in srv.poll(64, wait_ms=50):
                done += 1
                srv.release(r.tag)
        rates.append(len(elig) / (time.perf_counter() - t0))
        srv.close()
        log(f"serve burst {form}: {rates[-1]:.1f} solves/s")
    print(json.dumps({"metric": "served solves/s (burst of the BF16-eligible requests)", "unit": "solves/s",
                      "storage": form, "requests": len(elig), "runs": rates,
                      "value": float(np.mean(rates))}), flush=True)


def serve_summary(dev, nreq=512, slots=16):
    """The serving trace replayed once mixed (BF16 where eligible) and once all
    FP32, and the BF16-eligible requests as a burst in each storage: the figures
    of the serving half of the metric, for the default JSON line."""
    from types import SimpleNamespace
    args = SimpleNamespace(serve_requests=nreq, serve_slots=slots, serve_pool_gb=80.0,
                           serve_hw_queues=0, serve_repeats=1)
    line = serve_bench(args, dev, emit=False)
    burst = line["eligible_burst"]
    return {"workload": line["config"]["workload"], "slots": slots,
            "mixed_solves_per_s": line["mixed"]["mean"], "fp32_solves_per_s": line["fp32"]["mean"],
            "mixed_p50_ms": line["mixed_runs"][0]["p50_ms"], "mixed_p99_ms": line["mixed_p99_ms"][0],
            "fp32_p99_ms": line["fp32_p99_ms"][0],
            "bf16_eligible_requests": burst["requests"],
            "burst_bf16_solves_per_s": burst.get("bf16", {}).get("mean"),
            "burst_fp32_solves_per_s": burst.get("fp32", {}).get("mean"),
            "burst_rel_error_vs_fp32_A": burst.get("rel_error_vs_fp32_A")}


def stability_bench(args, dev):
    """Section 5.5 stability experiment: Matrix 1 form (sigma_j = j^-2, n x n)
    with block-diagonal right singular vectors (d Haar blocks of size n / d,
    d = 1, n / 10, n), tol 1e-4, b by the default rule, P = 1, at most
    ceil(n / 2b) blocks; for each test matrix and p in {ln(n)/n, 2e-3, 1e-2},
    `trials` solves with seeds 1..trials.  Two readings of a success: the
    solve stops with E < tol^2 ||A||^2 within the block cap (status 0), and
    that plus a true relative error ||A - U S V^T||_F / ||A||_F <= tol (formed
    in FP64 on the device).  One JSON line with both success rates (percent),
    the mean blocks per solve and the largest true error of a stopped solve."""
    import numpy as np
    import torch
    from paper_2506_03859_amd import farpca as fp
    from paper_2506_03859_amd import synth
    n, trials, tol = args.stability_n, args.stability_trials, 1e-4
    ds = [1, n // 10, n]
    ps = [("ln(n)/n", math.log(n) / n), ("2e-3", 2e-3), ("1e-2", 1e-2)]
    sketches = [("SB", "std_bernoulli"), ("SS", "sparse_sign"), ("SG", "sparse_gaussian"), ("B", "bernoulli")]
    table = {}
    table_q18 = {}
    blocks = {}
    worst = {}
    t_start = time.perf_counter()
    for d in ds:
        log(f"stability: generating {n} x {n}, d = {d}")
        A = synth.spectral_blockdiag_v_torch(n, synth.matrix1_sigma(n), d, seed=11, device=dev)
        A = A.to(torch.float32).contiguous()
        torch.cuda.synchronize()
        A64 = A.double()
        na = float(torch.linalg.norm(A64))
        for pname, pv in ps:
            for short, sk in sketches:
                ok, ok18, nb, emax = 0, 0, 0, 0.0
                for t in range(1, trials + 1):
                    res = fp.solve(A, tol=tol, power=1, sketch=sk, p=pv, seed=t)
                    rec = (res.U.double() * res.S) @ res.V.double().T
                    err = float(torch.linalg.norm(A64 - rec)) / na
                    del rec
                    ok += int(res.status == 0)
                    ok18 += int(res.status == 0 and err <= tol)
                    if res.status == 0:
                        emax = max(emax, err)
                    nb += res.info.blocks
                key = f"{short} p={pname} d={d}"
                table[key] = 100.0 * ok / trials
                table_q18[key] = 100.0 * ok18 / trials
                blocks[key] = nb / trials
                worst[key] = emax
                log(f"stability: {key}: {ok}/{trials} stopped below the tolerance, {ok18}/{trials} "
                    f"with true error <= tol, {nb / trials:.1f} blocks on average, largest error {emax:.3e}")
        del A64
        del A
        torch.cuda.empty_cache()
    line = {"metric": "success rate (stopped within ceil(n/2b) blocks; and with true error <= tol)",
            "unit": "percent",
            "n_gpus": 1, "data": "synthetic",
            "config": {"workload": f"stability_matrix1_{n}x{n}_blockdiagV", "tol": tol, "power": 1,
                       "trials": trials, "d": ds, "p": [pn for pn, _ in ps]},
            "success_percent": table, "success_true_error_percent": table_q18, "mean_blocks": blocks,
            "largest_true_error_of_stopped": worst,
            "wall_s": time.perf_counter() - t_start}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="exp50_20000x15000_ss8", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--serve", action="store_true",
                    help="replay the serving trace (Poisson arrivals, mixed shapes / tolerances / "
                         "storage) through farpca_server_* instead of the solve benchmark")
    ap.add_argument("--serve-burst", choices=["bf16", "f32"], default=None,
                    help="serve only the BF16-eligible requests of the trace as one burst in the "
                         "given storage (--serve-repeats times): the run a kernel trace is taken of")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--serve-repeats", type=int, default=3,
                    help="replays of each serving configuration (alternating), for the spread")
    ap.add_argument("--no-subrecords", action="store_true",
                    help="only the 20000 x 15000 solve line (no precision-form, tall and serving records)")
    ap.add_argument("--serve-pool-gb", type=float, default=80.0)
    ap.add_argument("--serve-hw-queues", type=int, default=0,
                    help="hardware queues of the process (GPU_MAX_HW_QUEUES, set before the HIP "
                         "runtime starts; 0 = the runtime's default)")
    ap.add_argument("--stability", action="store_true",
                    help="the Section 5.5 stability experiment (block-diagonal right singular "
                         "vectors, success rates per test matrix, p and d)")
    ap.add_argument("--stability-n", type=int, default=5000)
    ap.add_argument("--stability-trials", type=int, default=100)
    ap.add_argument("--kernel-probe", action="store_true",
                    help="only launch the kernels that stream A (A-pass products, sparse sketch) "
                         "on a random matrix of the workload's shape, plus a 1 GiB copy: the "
                         "input of the hardware-counter runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (--gpus must be 1)",
              file=sys.stderr)
        sys.exit(2)
    if counter_profiled() and not args.kernel_probe:
        # a hardware-counter run of this script once ended in a host segmentation
        # fault inside the FP64 QR that builds the workload's Haar factors; under
        # counter collection only the probe (random A, no factorisation) runs
        print("bench.py under hardware-counter collection: use --kernel-probe (the workload's "
              "input generation does not run in a counter-profiled process)", file=sys.stderr)
        sys.exit(2)
    if args.serve and args.serve_hw_queues > 0:
        # streams of concurrent slots map onto distinct hardware queues only up
        # to this count; must be set before the runtime initialises
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(32, args.serve_hw_queues))

    import torch
    from paper_2506_03859_amd import farpca as fp
    fp.load_library()
    dev = "cuda:0"
    torch.cuda.set_device(0)
    wl = args.workload
    if args.kernel_probe:
        kernel_probe(wl, dev)
        return
    if args.serve_burst:
        serve_burst(args, dev)
        return
    if args.serve:
        serve_bench(args, dev)
        return
    if args.stability:
        stability_bench(args, dev)
        return
    m, n, _, _, tol, b, P, sketch, zeta, p, storage = WORKLOADS[wl]
    rank = 200 if tol == 0.0 else 0
    log(f"generating {wl}")
    A = make_matrix(wl, dev)
    log("matrix ready")

    nruns = args.warmup + args.steps
    plans = [fp.farpca_plan(fp.make_params(m, n, tol=tol, rank=rank, block=b, power=P, sketch=sketch,
                                           p=p, zeta=zeta, seed=1000 + r, a_dtype=storage,
                                           layout=LAYOUTS.get(wl, "row")))
             for r in range(nruns)]
    work, U, S, V, eh = fp.alloc_outputs(plans[0], dev)
    if args.copy_probe:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    for r in range(args.warmup):
        fp.farpca_run(plans[r], A, work, U, S, V, eh)
        log(f"warmup {r + 1}/{args.warmup} done")
    torch.cuda.synchronize()

    fp.farpca_profile_enable(True)
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_done = []
    for r in range(args.steps):
        # farpca_run returns once the solve's results are on the device
        status, info = fp.farpca_run(plans[args.warmup + r], A, work, U, S, V, eh)
        t_done.append(time.perf_counter())
        infos.append((status, info.rank_l, info.blocks, info.err_indicator / info.norm_a2,
                      info.eig_sweeps))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per_solve_ms = [(b_ - a_) * 1e3 for a_, b_ in zip([t0] + t_done[:-1], t_done)]
    prof = {c: fp.farpca_profile_get(c) for c in fp.PROF_CLASSES}
    fp.farpca_profile_enable(False)
    log(f"timed {args.steps} solves")
    for pl in plans:
        pl.free()

    ms = (t1 - t0) * 1e3 / args.steps
    blocks = [i[2] for i in infos]
    ls = [i[1] for i in infos]

    # per-launch averages of the kernels that stream A
    def avg(c):
        tot, cnt = prof[c]
        return (tot / cnt if cnt else None), cnt

    gemm_flops = 2.0 * m * n * b
    elem = 2.0 if storage == "bf16" else 4.0
    a_bytes = elem * m * n
    cand = {}
    for c in ("gemm_tn", "gemm_nn", "gemm_c", "sketch"):
        a_ms, cnt = avg(c)
        if a_ms:
            cand[c] = (prof[c][0], a_ms, cnt)
    dom = max(cand, key=lambda c: cand[c][0])
    tot_ms, a_ms, cnt = cand[dom]
    layout = LAYOUTS.get(wl, "row")
    # row-major FP32 A: every A-pass runs split on the BF16 matrix cores
    split = storage == "f32" and layout == "row" and dom in ("gemm_tn", "gemm_nn", "gemm_c")
    pass_name = {"gemm_tn": "A^T Y", "gemm_nn": "A G", "gemm_c": "C_j^T = A^T Q_j"}.get(dom)
    if dom == "sketch":
        alg = a_bytes + 4.0 * m * b
        achieved = alg / (a_ms * 1e-3) / 1e9
        roof = {"kernel": "sketch_kernel", "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBPS,
                "unit": "GB/s", "frac": achieved / PEAK_HBM_GBPS}
    elif storage == "bf16":
        # BF16 A-passes: 2 m n bytes of A per launch against HBM (the exact
        # three-term products need 3 x 2 m n b flop of BF16 MFMA, under its peak)
        achieved = a_bytes / (a_ms * 1e-3) / 1e9
        kname = f"gemm_bf16_kernel<{'false' if dom == 'gemm_nn' else 'true'}, *, false> ({pass_name})"
        roof = {"kernel": kname, "bound": "hbm", "achieved": achieved,
                "peak": PEAK_HBM_GBPS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBPS}
    elif split:
        # FP32 A-passes on the BF16 matrix cores (both operands split in three,
        # 6 x 2 m n b flop of BF16 MFMA, far under its peak): 4 m n bytes of A
        # per launch against HBM
        achieved = a_bytes / (a_ms * 1e-3) / 1e9
        kname = ("gemm_f32s_nn_lds_kernel<true> (A G, FP32 A split)" if dom == "gemm_nn"
                 else f"gemm_bf16_kernel<true, true, true> ({pass_name}, FP32 A split)")
        roof = {"kernel": kname, "bound": "hbm",
                "achieved": achieved, "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBPS,
                "fp32_equivalent_tflops": gemm_flops / (a_ms * 1e-3) / 1e12}
    else:
        achieved = gemm_flops / (a_ms * 1e-3) / 1e12
        kname = f"gemm_kernel<{'false' if dom == 'gemm_nn' else 'true'}, *> ({pass_name}, FP32 matrix cores)"
        roof = {"kernel": kname, "bound": "mfma", "achieved": achieved,
                "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_MFMA_TFLOPS}
    if dom == "sketch":
        alg_per_launch = a_bytes + 4.0 * m * b
    else:
        alg_per_launch = a_bytes if (storage == "bf16" or split) else gemm_flops
    base_key = "gemm_tn" if dom == "gemm_c" else dom
    traffic_key = f"{base_key}_split" if split else (base_key if storage == "f32" else f"{base_key}_bf16")
    roof.update({"avg_launch_ms": a_ms, "launches": cnt, "algorithmic_per_launch": alg_per_launch,
                 "traffic": measured_traffic(traffic_key) if layout == "row" else None})
    if layout == "col" and dom != "sketch":
        # A^T row-major: the logical A^T Y runs on the NN kernel, A G on the TN one
        roof["kernel"] = f"{pass_name} as the {'TN' if dom == 'gemm_nn' else 'NN'} kernel on A^T"
    if layout == "col" and dom == "sketch":
        roof["kernel"] = "sketch_cols_kernel"
        alg_per_launch = 4.0 * m * (p * n * b) + 4.0 * m * b
        roof["algorithmic_per_launch"] = alg_per_launch
        roof["achieved"] = alg_per_launch / (a_ms * 1e-3) / 1e9
        roof["frac"] = roof["achieved"] / PEAK_HBM_GBPS
    classes = {}
    for c, (tot, cnt) in prof.items():
        classes[c] = {"total_ms_per_solve": tot / args.steps, "launches": cnt,
                      "avg_launch_ms": (tot / cnt if cnt else None)}
    sk_ms, _ = avg("sketch")
    # algorithmic bytes of one sketch: all of A row-major; column-major, the
    # columns Omega_j touches (expected nnz(Omega_j) = p n b for the i.i.d. kinds)
    if layout == "col" and zeta == 0 and sketch != "gaussian":
        sk_bytes = 4.0 * m * (p * n * b) + 4.0 * m * b
    else:
        sk_bytes = a_bytes + 4.0 * m * b
    sketch_gbps = sk_bytes / (sk_ms * 1e-3) / 1e9 if sk_ms else None
    for c in ("gemm_tn", "gemm_nn", "gemm_c"):
        if classes[c]["avg_launch_ms"]:
            classes[c]["tflops"] = gemm_flops / (classes[c]["avg_launch_ms"] * 1e-3) / 1e12
            classes[c]["a_GBps"] = a_bytes / (classes[c]["avg_launch_ms"] * 1e-3) / 1e9

    out = {
        "metric": "time-to-tolerance & sketch HBM GB/s per solve",
        "value": 1e3 / ms,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "time_to_tolerance_ms": ms,
        "solve_ms": {"median": float(sorted(per_solve_ms)[len(per_solve_ms) // 2]),
                     "min": min(per_solve_ms), "max": max(per_solve_ms)},
        "sketch_hbm_GBps": sketch_gbps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if storage == "f32" else "bf16",
        "data": "synthetic",
        "config": {"workload": wl, "m": m, "n": n, "tol": tol, "rank": rank, "block": b, "power": P,
                   "sketch": sketch, "zeta": zeta, "p": p, "a_storage": storage, "a_layout": layout,
                   "blocks": sorted(set(blocks)), "l": sorted(set(ls)),
                   "parallelism": "single GPU"},
        "roofline": roof,
        "kernels": classes,
        "runs": [{"status": s, "l": l, "blocks": bl, "rel_E": e, "eig_sweeps": sw}
                 for s, l, bl, e, sw in infos],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, wl, max(blocks))
    if not args.no_subrecords and wl == "exp50_20000x15000_ss8":
        # the other configurations of the metric, beside the headline: the
        # precision form (the same matrix stored in BF16) with its FP32 twin,
        # the tall fixed-rank matrix, and the serving trace
        import torch
        sub = {}
        log("subrecord: precision form")
        A16 = A.to(torch.bfloat16).contiguous()
        sub["bf16"] = time_solves("bf16_exp50_20000x15000_sg05", A16, 5, 1, dev)
        sub["fp32_twin"] = time_solves("exp50_20000x15000_sg05", A, 5, 1, dev)
        sub["bf16_speedup"] = sub["fp32_twin"]["ms_per_solve"] / sub["bf16"]["ms_per_solve"]
        out["precision_form"] = sub
        del A16, A
        torch.cuda.empty_cache()
        log("subrecord: tall fixed rank")
        At = make_matrix("tall_200000x4000_rank200", dev)
        out["tall_fixed_rank"] = time_solves("tall_200000x4000_rank200", At, 3, 1, dev)
        del At
        torch.cuda.empty_cache()
        log("subrecord: serving")
        out["serving"] = serve_summary(dev)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
