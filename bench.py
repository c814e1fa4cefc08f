#!/usr/bin/env python3
"""Benchmark of the forward-stable DPR1 eigensolver on one MI355X.

One step = all n eigenpairs (eigenvalues and the full eigenvector matrix V)
of one DPR1 matrix of order n = 32768 (d sorted-descending distinct draws from
U[-1, 1], z ~ N(0, 1)/sqrt(n), rho = 1; seed 2), inputs resident in HBM.
The JSON line also carries the eigenvalues-only variant, the batched mix
(2048 ragged problems, persistent launch vs one launch per problem), the
forward+backward batch (256 problems of n = 512), the roofline of the
dominant kernel and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6   # MI355X FP64 vector (and matrix) peak
HBM_PEAK_GBS = 8000.0

# Algorithmic FP64 flops per (eigenvalue k, inner index j) pair, counted as the
# peak counts them: a fused multiply-add is 2, an add, multiply or division 1
# (the Newton refinement of the hardware reciprocal is not counted).
FLOPS_SHIFT = 10          # (d_j - d_k) - tau (2), 1/den, t, t/den, 3 adds, fma for t/den^2 (2)
FLOPS_TIP = 19            # TwoSum d_j - sigma (6), 1/dl, quotient + residual (7), compensated add (5)
FLOPS_ROOT_MODEL = 14     # per pass: delta' (2), nu delta' - 1 (2), q, 1/q, t, 1/pp (2), tp, tp3, 3 adds
FLOPS_ROOT_BISECT = 7     # per pass: delta' (2), nu delta' - 1 (2), q, 1/q, add
FLOPS_FINAL = 20.375      # accurate last pass: delta', pp (4), q, 1/q, t, corrected quotient (4),
                          # 1/pp (2), tp, tp3, tp4, 3 adds, and the sum of t: a tree over blocks
                          # of eight (7/8) feeding a Neumaier sum (4/8)


def flops_per_pair(root, passes_mean):
    """Algorithmic flops per (k, j) pair done by the eigenvalue kernel (k_eig): the shift pass,
    the tip, `passes_mean` plain root-finder passes and the accurate last pass (which also gives
    ||x||)."""
    per = FLOPS_ROOT_MODEL if root == 1 else FLOPS_ROOT_BISECT
    return FLOPS_SHIFT + FLOPS_TIP + per * passes_mean + FLOPS_FINAL


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--root", type=int, default=1, help="0 bisection, 1 model iteration (default)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="target wall time of the oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip batched / fwd+bwd / eigenvalues-only lines")
    ap.add_argument("--no-tune", action="store_true",
                    help="default launch shape instead of the autotuned one (tuning cache or a fresh tuning run)")
    ap.add_argument("--tune-only", action="store_true",
                    help="fill the tuning cache for every solve this bench times, then exit")
    ap.add_argument("--launch", default=None,
                    help="SPLIT,WAVES_PER_SIMD,MAIN_PASSES: time this launch shape instead of the tuned one")
    ap.add_argument("--mode", default="solve", choices=["solve", "copy"],
                    help="copy: a plain device copy of known size, to calibrate HBM byte counters")
    ap.add_argument("--only", default=None, choices=["batched", "fwd_bwd", "general", "tridiag"],
                    help="run only this workload (for profiler runs); prints its JSON")
    args = ap.parse_args()
    if args.mode == "copy":
        return copy_calibration()
    if args.only:
        import torch
        import paper_1405_7537_amd.dpr1 as D
        from paper_1405_7537_amd import workloads as W
        dev = torch.device("cuda:0")
        fn = {"batched": bench_batched, "fwd_bwd": bench_fwd_bwd, "general": bench_general,
              "tridiag": bench_tridiag}[args.only]
        print(json.dumps(fn(D, W, torch, dev, args)), flush=True)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; shard eigenvalue blocks across GPUs "
                          "as described in the design notes", "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch
    import paper_1405_7537_amd.dpr1 as D
    from paper_1405_7537_amd import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = args.n
    d_h, z_h, rho = W.uniform(n, 2, zscale=1.0 / math.sqrt(n))
    d = torch.as_tensor(d_h, device=dev)
    z = torch.as_tensor(z_h, device=dev)
    lam = torch.empty(n, dtype=torch.float64, device=dev)
    Vt = torch.empty((n, n), dtype=torch.float64, device=dev)
    idx = torch.empty(n, dtype=torch.int32, device=dev)
    mu = torch.empty(n, dtype=torch.float64, device=dev)
    xn = torch.empty(n, dtype=torch.float64, device=dev)
    info = torch.empty(1, dtype=torch.int32, device=dev)
    work = torch.empty(D.workspace_bytes(n), dtype=torch.uint8, device=dev)
    out = (lam, Vt, idx, mu, xn, info)
    ev = [D.HipEvents() for _ in range(args.steps)]
    log(f"[bench] n={n} V {n * n * 8 / 1e9:.2f} GB, warmup {args.warmup}, steps {args.steps}")

    def step(o, vectors=True, want_stats=False):
        return D.eig(d, z, rho, vectors=vectors, opts=o, check=False, out=out if vectors else
                     (lam, None, idx, mu, xn, info), work=work, want_stats=want_stats)

    base, tune = tuned(D, args, d, z, rho, vectors=True)
    base_ev, tune_ev = tuned(D, args, d, z, rho, vectors=False)
    if args.tune_only:
        bench_batched(D, W, torch, dev, args)
        print(json.dumps({"mode": "tune-only", "n": n, "vectors": tune, "eigenvalues_only": tune_ev}), flush=True)
        return
    for _ in range(args.warmup):
        step(base)
    torch.cuda.synchronize()
    r = step(base, want_stats=True)
    torch.cuda.synchronize()
    st = r.stats_dict()
    assert int(info.item()) == 0
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(base)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = n / (ms_step / 1e3)
    # The same solves with the eigenvector write after the eigenvalue kernel (opts.vwrite = 1, the default),
    # timed with the library's events on the launch stream: the eigenvalue kernel is then one
    # launch (the roofline's duration) and the second phase (k_fixvec + k_fixout) writes V alone.
    seq = D.opts(root=args.root, split=base.split, main_passes=base.main_passes,
                 waves_per_simd=base.waves_per_simd, vwrite=1)
    step(seq)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(D.opts(root=args.root, split=base.split, main_passes=base.main_passes,
                    waves_per_simd=base.waves_per_simd, vwrite=1, events=ev[s].ptr))
    torch.cuda.synchronize()
    ms_seq = (time.perf_counter() - t0) * 1e3 / args.steps
    eig_ms = float(np.mean([e.eig_ms() for e in ev]))
    vec_ms = float(np.mean([e.vec_ms() for e in ev]))
    iters_mean = st["iters_sum"] / n
    fpp = flops_per_pair(args.root, iters_mean)
    achieved = fpp * n * n / (eig_ms / 1e3) / 1e12
    vec_gbs = n * n * 8 / (vec_ms / 1e3) / 1e9
    log(f"[bench] {ms_step:.3f} ms/step ({value:.4g} eigenpairs/s); with the write after the eigenvalue kernel "
        f"{ms_seq:.3f} ms/step: k_eig {eig_ms:.3f} ms, k_fixvec+k_fixout {vec_ms:.3f} ms ({vec_gbs:.0f} GB/s); "
        f"iters/eig {iters_mean:.2f}, stats {st}")

    # HBM bytes of one k_eig launch from the FETCH_SIZE / WRITE_SIZE counters,
    # scaled by the copy-kernel calibration; used only while the kernel
    # sources are the ones the counters were taken on
    # per launch shape (split, waves per SIMD, pass budget): the register
    # budget changes what stays in registers and so the bytes moved
    traffic = None
    shape = f"{int(base.split)},{int(base.waves_per_simd) or 4},{int(base.main_passes) or 2}"
    tf = os.path.join(ROOT, "profiles", f"k_eig_n{n}_traffic.txt")
    if os.path.exists(tf):
        try:
            tj = json.load(open(tf))
            if tj.get("source_sha") == source_sha() and tj.get("n") == n:
                traffic = tj.get("shapes", {}).get(shape, {}).get("k_eig_bytes")
        except Exception:
            traffic = None

    result = {
        "metric": "eigenpairs/s FP64 at n=32768 + batched mix; fwd+bwd/s; % FP64 peak",
        "value": value,
        "unit": "eigenpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"single DPR1 n={n}, all eigenvalues + full V (FP64), d~U[-1,1] sorted, "
                               f"z~N(0,1)/sqrt(n), rho=1, seed 2",
                   "n": n, "root": "model" if args.root == 1 else "bisection", "tuning": tune},
        "roofline": {"bound": "alu", "kernel": "k_eig", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic,
                     "flops_per_pair": fpp, "kernel_ms": eig_ms},
        "v_write": {"kernel": "k_fixvec+k_fixout (V written after the eigenvalue kernel, k_fix's work beside it)",
                    "ms": vec_ms, "GB/s": vec_gbs, "frac_hbm": vec_gbs / HBM_PEAK_GBS,
                    "ms_per_step_sequential": ms_seq,
                    "note": ("value is timed with the tuned write: " + (
                        "after the eigenvalue kernel (opts.vwrite = 0), as here" if int(base.vwrite) <= 1 else
                        f"the eigenvalue kernel in {int(base.vwrite)} chunks, each chunk's columns but the last "
                        f"written on a second stream while the next chunk is solved (opts.vwrite = "
                        f"{int(base.vwrite)}); k_eig and the write are timed here with the write after the "
                        "eigenvalue kernel, same launch shape"))},
        "stats": st,
    }

    # ---- CPU oracle on a bounded sample of the same matrix (eigenpairs with vectors)
    if not args.no_cpu:
        from oracle import oracle as O
        nth = O.max_threads()
        # calibrate: one eigenpair, then size the sample for ~cpu-seconds of wall time
        t = time.perf_counter()
        O.eig_some(d_h, z_h, rho, [n // 2], vectors=True, nthreads=1)
        per = time.perf_counter() - t
        nk = int(max(nth, min(n, args.cpu_seconds * nth / per)))
        ks = np.unique(np.linspace(0, n - 1, nk).astype(np.int64))
        log(f"[bench] oracle sample: {ks.size} eigenpairs with vectors on {nth} threads")
        t = time.perf_counter()
        lo, Vo, _ = O.eig_some(d_h, z_h, rho, ks, vectors=True, nthreads=nth)
        tc = time.perf_counter() - t
        lam_g = lam.cpu().numpy()[ks]
        Vs = Vt[torch.as_tensor(ks, device=dev)].cpu().numpy().T   # columns k of V
        el = float(np.max(np.abs(lam_g - lo) / np.abs(lo)))
        evv = float(np.max(np.abs(Vs - Vo) / np.abs(Vo)))
        cpu_model = "unknown"
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
        # the small configurations in full on one thread: n = 256 uniform (seed 0) and the graded
        # n = 4096 matrix (seed 1), all eigenpairs with eigenvectors
        one = {}
        for name, (dd_, zz_, rr_) in (("n256_uniform", W.uniform(256, 0)), ("n4096_graded", W.graded(4096, 1))):
            t = time.perf_counter()
            O.eig(dd_, zz_, rr_, nthreads=1)
            el_ = time.perf_counter() - t
            one[name] = {"s": el_, "eigenpairs/s": dd_.size / el_}
        result["cpu_baseline"] = {"value": ks.size / tc, "unit": "eigenpairs/s", "cores": nth, "kind": "oracle",
                                  "cpu_model": cpu_model,
                                  "sample": f"{ks.size} evenly spaced eigenpairs (eigenvalue + eigenvector) of "
                                            f"the n={n} matrix, {tc:.1f} s wall",
                                  "one_thread_full": one}
        result["max_rel_err_vs_oracle"] = {"lambda": el, "V": evv, "sample": int(ks.size)}
        log(f"[bench] oracle {ks.size / tc:.4g} eigenpairs/s, max rel err lambda {el:.2e} V {evv:.2e}")

    if not args.no_extra:
        # eigenvalues only
        for _ in range(2):
            step(base_ev, vectors=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(base_ev, vectors=False)
        torch.cuda.synchronize()
        ms_ev = (time.perf_counter() - t0) * 1e3 / args.steps
        result["eigenvalues_only"] = {"value": n / (ms_ev / 1e3), "ms_per_step": ms_ev, "tuning": tune_ev}
        del Vt, out
        torch.cuda.empty_cache()
        result["batched"] = bench_batched(D, W, torch, dev, args)
        fb = bench_fwd_bwd(D, W, torch, dev, args)
        if fb is not None:
            result["fwd_bwd"] = fb
        result["general"] = bench_general(D, W, torch, dev, args)
        result["tridiag"] = bench_tridiag(D, W, torch, dev, args)

    print(json.dumps(result), flush=True)


def copy_calibration(nbytes=1 << 30, reps=3):
    """y <- x for 1 GiB float64 buffers: each dispatch reads and writes exactly nbytes."""
    import torch
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    print(json.dumps({"mode": "copy", "bytes_read": nbytes, "bytes_written": nbytes, "reps": reps,
                      "ms": ms, "GB/s": 2 * nbytes / (ms / 1e3) / 1e9}), flush=True)


def source_sha():
    """Hash of the sources k_eig is compiled from (its file, the double-double header, the ABI
    header): the stored traffic record is used only while these are unchanged."""
    import hashlib
    h = hashlib.sha256()
    for f in ("paper_1405_7537_amd/csrc/dpr1_kernels.hip", "paper_1405_7537_amd/csrc/dd.h", "include/dpr1.h"):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def tuned(D, args, d, z, rho, vectors):
    """Options of the timed solves: the autotuned split and pass budget (tuning cache, else a tuning
    run before any timing), or the defaults with --no-tune.  Returns (opts, description)."""
    o = D.opts(root=args.root)
    if args.launch and vectors:
        sp, wps, mp = (int(x) for x in args.launch.split(","))
        o = D.opts(root=args.root, split=sp, waves_per_simd=wps, main_passes=mp)
        log(f"[bench] launch shape given: split {sp}, waves/SIMD {wps}, main_passes {mp}")
        return o, {"split": sp, "waves_per_simd": wps, "main_passes": mp, "from_cache": False, "given": True}
    if args.no_tune:
        return o, {"split": "default", "main_passes": "default"}
    from paper_1405_7537_amd import tuning
    o, entry, hit = tuning.tuned_opts(d, z, rho, vectors=vectors, opts=o)
    log(f"[bench] tuned (vectors={vectors}): split {o.split}, waves/SIMD {o.waves_per_simd}, "
        f"main_passes {o.main_passes}, vwrite {o.vwrite} ({'cache' if hit else 'tuned now'}, {entry['ms']:.3f} ms)")
    return o, {"split": int(o.split), "waves_per_simd": int(o.waves_per_simd), "main_passes": int(o.main_passes),
               "vwrite": int(o.vwrite), "from_cache": bool(hit)}


def bench_batched(D, W, torch, dev, args):
    d_h, z_h, rho_h, offs = W.batched(2048, 3)
    sizes = np.diff(offs)
    d = torch.as_tensor(d_h, device=dev)
    z = torch.as_tensor(z_h, device=dev)
    rho = torch.as_tensor(rho_h, device=dev)
    if args.no_tune:
        b = D.Batch(offs, opts=D.opts(root=args.root))
        tune = {"split": int(b.plan.split), "main_passes": "default"}
    else:
        from paper_1405_7537_amd import tuning
        b, entry, hit = tuning.tuned_batch(offs, d, z, rho, opts=D.opts(root=args.root))
        tune = {"split": int(b.plan.split), "waves_per_simd": int(b.plan.opts.waves_per_simd),
                "main_passes": int(b.plan.opts.main_passes), "from_cache": bool(hit)}
        log(f"[bench] batched tuned: split {tune['split']}, waves/SIMD {tune['waves_per_simd']}, main_passes "
            f"{tune['main_passes']} ({'cache' if hit else 'tuned now'}, {entry['ms']:.3f} ms)")
    if args.tune_only:
        return tune
    N = int(offs[-1])
    for _ in range(2):
        b.solve(d, z, rho)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.solve(d, z, rho)
    torch.cuda.synchronize()
    ms_p = (time.perf_counter() - t0) * 1e3 / args.steps
    b.check()
    # every 128th problem against the oracle (eigenvalues and every eigenvector component)
    err = {"lambda": 0.0, "V": 0.0, "sample": "16 problems (every 128th), all eigenpairs"}
    if not args.no_cpu:
        from oracle import oracle as O
        lam_all = b.lam.cpu().numpy()
        for p in range(0, 2048, 128):
            a, e = int(offs[p]), int(offs[p + 1])
            lo, Vo = O.eig(d_h[a:e], z_h[a:e], rho_h[p])
            Vg = b.vblock(p).cpu().numpy()
            err["lambda"] = max(err["lambda"], float(np.max(np.abs(lam_all[a:e] - lo) / np.abs(lo))))
            err["V"] = max(err["V"], float(np.max(np.abs(Vg - Vo) / np.abs(Vo))))
    # the same problems, one launch sequence per problem
    work = torch.empty(D.workspace_bytes(int(sizes.max())), dtype=torch.uint8, device=dev)
    info = torch.empty(1, dtype=torch.int32, device=dev)
    views = []
    for p in range(2048):
        a, e = int(offs[p]), int(offs[p + 1])
        np_ = e - a
        vo = int(b.voffs_host[p])
        views.append((d[a:e], z[a:e], float(rho_h[p]),
                      (b.lam[a:e], b.V[vo:vo + np_ * np_].view(np_, np_), b.shift_idx[a:e], b.mu[a:e],
                       b.xnorm[a:e], info)))
    o = D.opts(root=args.root)

    def each():
        for dd, zz, rr, out in views:
            D.eig(dd, zz, rr, opts=o, check=False, out=out, work=work)

    each()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = max(1, args.steps // 2)
    for _ in range(reps):
        each()
    torch.cuda.synchronize()
    ms_e = (time.perf_counter() - t0) * 1e3 / reps
    log(f"[bench] batched mix N={N}: persistent {ms_p:.3f} ms, one launch each {ms_e:.3f} ms")
    res = {"workload": "2048 DPR1 problems, sizes log-uniform in [16,2048] (seed 3), all eigenpairs + V",
           "ntotal": N, "sum_n2": int(np.sum(sizes ** 2)),
           "persistent": {"value": N / (ms_p / 1e3), "unit": "eigenpairs/s", "ms_per_step": ms_p, "tuning": tune},
           "max_rel_err_vs_oracle": err if not args.no_cpu else None,
           "one_launch_each": {"value": N / (ms_e / 1e3), "unit": "eigenpairs/s", "ms_per_step": ms_e}}
    del b, views
    torch.cuda.empty_cache()
    return res


def bench_fwd_bwd(D, W, torch, dev, args):
    r = fwd_bwd_timing(D, torch, dev, args.steps)
    log(f"[bench] fwd+bwd 256 x n=512: {r['ms_per_step']:.3f} ms (forward {r['forward_ms']:.3f} ms); "
        f"V not stored: {r['v_not_stored']['ms_per_step']:.3f} ms")
    return r


def bench_general(D, W, torch, dev, args):
    """The front end for reducible inputs (unsorted, repeated poles, zero z_j) at the same n: host
    reduction + reduced solve + assembly of V, one synchronising call per step."""
    n = args.n
    d_h, z_h, rho = W.reducible(n, 4, rho=1.0)
    d = torch.as_tensor(d_h, device=dev)
    z = torch.as_tensor(z_h, device=dev)
    r = D.eig_general(d, z, rho)
    del r
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = D.eig_general(d, z, rho, check=False)
        del r
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    # size of the reduced problem: distinct poles whose z part is not all zero
    nz = {}
    for dv, zv in zip(d_h.tolist(), z_h.tolist()):
        nz[dv] = nz.get(dv, False) or zv != 0.0
    m = int(sum(nz.values()))
    log(f"[bench] general n={n} (reduced m={m}): {ms:.3f} ms/step, {n / (ms / 1e3):.4g} eigenpairs/s")
    torch.cuda.empty_cache()
    # Hermitian: the same poles, z with uniform random phases; V complex128 (16 n^2 bytes)
    zc = torch.as_tensor(z_h * np.exp(1j * np.random.default_rng(4).uniform(0, 2 * np.pi, n)), device=dev)
    r = D.eig_hermitian(d, zc, rho)
    del r
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = D.eig_hermitian(d, zc, rho, check=False)
        del r
    torch.cuda.synchronize()
    ms_h = (time.perf_counter() - t0) * 1e3 / args.steps
    log(f"[bench] hermitian n={n}: {ms_h:.3f} ms/step, {n / (ms_h / 1e3):.4g} eigenpairs/s")
    torch.cuda.empty_cache()
    err = None
    if not args.no_cpu:
        err = general_error(D, W, 4096)
        log(f"[bench] general vs oracle (n=4096): {err}")
    return {"workload": f"n={n}, uniform poles in [-1,1] with n/10 repeated and n/10 zero z_j (seed 4), "
                        "all eigenpairs + V", "n": n, "reduced_n": m, "ms_per_step": ms,
            "value": n / (ms / 1e3), "unit": "eigenpairs/s", "max_rel_err_vs_oracle": err,
            "hermitian": {"workload": "the same poles and |z|, uniform random phases, complex128 V",
                          "ms_per_step": ms_h, "value": n / (ms_h / 1e3), "unit": "eigenpairs/s"}}


def fwd_bwd_timing(D, torch, dev, steps, nb=256, n=512, seed=4):
    """Forward + backward of nb problems of order n: L = sum(w * lam) + sum(W o V)."""
    from paper_1405_7537_amd import workloads as W
    d_h, z_h, rho_h = W.uniform_batch(nb, n, seed)
    rng = np.random.default_rng(seed + 100)
    d = torch.as_tensor(d_h, device=dev)
    z = torch.as_tensor(z_h, device=dev)
    rho = torch.as_tensor(rho_h, device=dev)
    w = torch.as_tensor(rng.standard_normal((nb, n)), device=dev)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    Wb = torch.randn((nb, n, n), generator=g, dtype=torch.float64, device=dev)   # column-major V_bar blocks
    offs = np.arange(nb + 1, dtype=np.int64) * n
    b = D.Batch(offs, device=dev)
    wb = int(D.lib().dpr1_backward_workspace_size(n, nb))
    work = torch.empty(wb, dtype=torch.uint8, device=dev)

    def one():
        b.solve(d, z, rho)
        return D.backward_batched(d, z, rho, b.shift_idx.view(nb, n), b.mu.view(nb, n), b.xnorm.view(nb, n),
                                b.V, w, Wb, work=work)

    import time
    for _ in range(2):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    t0 = time.perf_counter()
    for _ in range(steps):
        b.solve(d, z, rho)
    torch.cuda.synchronize()
    ms_f = (time.perf_counter() - t0) * 1e3 / steps
    flops = 2 * 2 * n ** 3 * nb
    # the same gradients with V never stored: eigenvalues-only forward, V rebuilt in the GEMM loads
    b2 = D.Batch(offs, vectors=False, device=dev)

    def one_recompute():
        b2.solve(d, z, rho)
        return D.backward_batched(d, z, rho, b2.shift_idx.view(nb, n), b2.mu.view(nb, n), b2.xnorm.view(nb, n),
                                None, w, Wb, work=work)

    for _ in range(2):
        one_recompute()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one_recompute()
    torch.cuda.synchronize()
    ms_r = (time.perf_counter() - t0) * 1e3 / steps
    # the sampled problems against the oracle's dense reverse mode, errors relative to the
    # magnitudes |V| |X| |V|^T (d_bar), rho |V| (|X| + |X|^T) |y| (z_bar), |y|^T |X| |y| (rho_bar),
    # |X| = |F| o (|V|^T |V_bar|): the scales of the rounding of the two products
    err = None
    try:
        from oracle import oracle as O
        b.solve(d, z, rho)
        db, zb, rb = D.backward_batched(d, z, rho, b.shift_idx.view(nb, n), b.mu.view(nb, n), b.xnorm.view(nb, n),
                                        b.V, w, Wb, work=work)
        db, zb, rb = db.cpu().numpy(), zb.cpu().numpy(), rb.cpu().numpy()
        wn = w.cpu().numpy()
        err = {"d_bar": 0.0, "z_bar": 0.0, "rho_bar": 0.0, "sample": "problems 0 and 255, each against the oracle's "
               "dense FP64 reverse mode, relative to the magnitude of the products"}
        for p in (0, nb - 1):
            lo, Vo, dg = O.eig(d_h[p], z_h[p], rho_h[p], diags=True)
            Vb = Wb[p].cpu().numpy().T
            do, zo, ro = O.backward(d_h[p], z_h[p], rho_h[p], [x["sigma"] for x in dg], [x["mu"] for x in dg], Vo,
                                    lam_bar=wn[p], V_bar=Vb)
            gap = lo[None, :] - lo[:, None]
            np.fill_diagonal(gap, 1.0)
            Xa = (np.abs(Vo).T @ np.abs(Vb)) / np.abs(gap)
            np.fill_diagonal(Xa, np.abs(wn[p]))
            Va = np.abs(Vo)
            y = np.abs(Vo.T @ z_h[p])
            Md = np.sum((Va @ Xa) * Va, axis=1)
            Mz = abs(rho_h[p]) * Va @ ((Xa + Xa.T) @ y)
            Mr = y @ Xa @ y
            err["d_bar"] = max(err["d_bar"], float(np.max(np.abs(db[p] - do) / Md)))
            err["z_bar"] = max(err["z_bar"], float(np.max(np.abs(zb[p] - zo) / Mz)))
            err["rho_bar"] = max(err["rho_bar"], float(abs(rb[p] - ro) / Mr))
    except Exception as ex:  # the timing stands without the check
        err = {"error": str(ex)}
    return {"workload": f"{nb} DPR1 problems of n={n} (seed {seed}), L = sum(w*lam) + sum(W o V)",
            "max_rel_err_vs_oracle": err,
            "value": nb / (ms / 1e3), "unit": "problems/s (forward+backward)", "ms_per_step": ms,
            "forward_ms": ms_f, "backward_ms": ms - ms_f,
            "gemm_TFLOPs": flops / ((ms - ms_f) / 1e3) / 1e12,
            "v_not_stored": {"value": nb / (ms_r / 1e3), "ms_per_step": ms_r,
                             "note": "forward without eigenvectors; the backward rebuilds V in its GEMM loads"}}


def general_error(D, W, n):
    """The front end on a reducible problem of order n (seed 4) against the oracle: eigenvalues
    relative; a simple eigenvalue that is not a pole componentwise relative; groups of equal
    eigenvalues (and deflated/reflected columns) by the projector onto their columns, absolute."""
    from oracle import oracle as O
    d, z, rho = W.reducible(n, 4, rho=1.0)
    r = D.eig_general(d, z, rho)
    lam, V = r.lam.cpu().numpy(), r.V.cpu().numpy()
    lo, Vo = O.eig_general(d, z, rho)
    el = float(np.max(np.abs(lam - lo) / np.where(lo == 0, 1.0, np.abs(lo))))
    poles = set(d.tolist())
    ev = ep = 0.0
    s = 0
    for k in range(1, n + 1):
        if k == n or abs(lo[k] - lo[k - 1]) > 1e-13 * max(abs(lo[k - 1]), 1e-300):
            if k - s == 1 and lo[s] not in poles:
                nz = Vo[:, s] != 0
                ev = max(ev, float(np.max(np.abs(V[nz, s] - Vo[nz, s]) / np.abs(Vo[nz, s]))))
            else:
                ep = max(ep, float(np.max(np.abs(V[:, s:k] @ V[:, s:k].T - Vo[:, s:k] @ Vo[:, s:k].T))))
            s = k
    return {"lambda": el, "V": ev, "projector_abs": ep,
            "sample": f"the same front end on a reducible problem of order {n} (seed 4), all eigenpairs"}


def tridiag_error(D, W, n):
    """The divide-and-conquer driver at order n (seed 5) against the oracle's: eigenvalues relative,
    columns up to sign (absolute: a divide and conquer is accurate to eps ||T||)."""
    from oracle import oracle as O
    a, b = W.tridiagonal(n, 5)
    r = D.tridiag_eig(a, b)
    lam, Q = r.lam.cpu().numpy(), r.Q.cpu().numpy()
    lo, Qo = O.tridiag_eig(a, b)
    el = float(np.max(np.abs(lam - lo) / np.abs(lo)))
    eq = float(np.max(np.minimum(np.abs(Q - Qo).max(axis=0), np.abs(Q + Qo).max(axis=0))))
    return {"lambda": el, "Q_abs": eq, "sample": f"the same driver at order {n} (seed 5), all eigenpairs"}


def dc_gemm_flops(n):
    """FP64 flops of the products diag(Q1, Q2) V over the whole split tree (2 m^2 s + 2 (s-m)^2 s
    per merge of size s split at m = s // 2)."""
    tot, stack = 0, [n]
    while stack:
        s = stack.pop()
        if s < 2:
            continue
        m = s // 2
        tot += 2 * (m * m + (s - m) * (s - m)) * s
        stack += [m, s - m]
    return tot


def bench_tridiag(D, W, torch, dev, args, n=8192):
    """Symmetric tridiagonal T (n = 8192, N(0,1) entries, seed 5) by divide and conquer over DPR1
    merges; the library dense symmetric eigensolver on the same T is timed beside it for context."""
    a_h, b_h = W.tridiagonal(n, 5)
    a = torch.as_tensor(a_h, device=dev)
    b = torch.as_tensor(b_h, device=dev)
    r = D.tridiag_eig(a, b)
    work = r.work
    del r
    torch.cuda.synchronize()
    reps = max(1, min(args.steps, 5))
    t0 = time.perf_counter()
    for _ in range(reps):
        r = D.tridiag_eig(a, b, work=work)
        del r
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    fl = dc_gemm_flops(n)
    T = torch.diag(a) + torch.diag(b, 1) + torch.diag(b, -1)
    torch.linalg.eigh(T)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    torch.linalg.eigh(T)
    torch.cuda.synchronize()
    ms_ref = (time.perf_counter() - t0) * 1e3
    del T
    torch.cuda.empty_cache()
    log(f"[bench] tridiag n={n}: {ms:.2f} ms per solve ({fl / 1e9:.0f} GFLOP of merge products); "
        f"dense symmetric library solver on the same T: {ms_ref:.1f} ms")
    err = tridiag_error(D, W, 2048) if not args.no_cpu else None
    return {"workload": f"symmetric tridiagonal n={n}, diagonal and off-diagonal N(0,1) (seed 5), all eigenpairs",
            "ms_per_step": ms, "value": n / (ms / 1e3), "unit": "eigenpairs/s", "gemm_flops": fl,
            "max_rel_err_vs_oracle": err,
            "dense_library_eigh_ms": ms_ref}


if __name__ == "__main__":
    main()
