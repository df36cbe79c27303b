#!/usr/bin/env python3
"""Throughput of the SIM-M indicator evaluation on one MI355X.

Workload: the n = 40,000 convection-diffusion pencil (5-point -Lap u + (20,10).grad u
+ (0.5+0.5i) u on a 200 x 200 grid, B = tridiag(0.05, 1, 0.05)), region
R = [120,1400] x [-310,330] (105 eigenvalues), 16 Gauss points per edge, m = 80,
4 levels, the column norms of X = V_m Y at every level.  One step = one full pass of
the hot path: every shift's banded LU and Arnoldi basis, the Schur forms, the shifted
solves / sums / decisions of every level, the projections and the subdivision.
The line also carries the metric's speedup clause (mixed precision over plain FP64 on
the n = 250,000 workload) and the CPU oracle's complete run of the same workload.

Prints one JSON line.  value = resolvent solves per second: quadrature-point
systems (A - z_j B) x_j = f solved in the Krylov spaces (12 g per square tested),
over the whole step.  The pencil and f are resident in HBM before timing starts.

  python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# Hardware queues of the process (read by the HIP runtime when it starts; its default
# is 4).  The driver computes one LU factor ahead per queue beyond the run's own (at
# most 11), and streams beyond the queue count share queues and serialise.  Each
# factor is a stream of short launches, and with more queues those launches slow the
# run stream's own kernels more.  Means of 6 steps on the n = 40,000 workload: 6 ahead
# with 8 queues 578-590 ms, 7 ahead 610 ms, 11 ahead with 12 queues 653 ms, 7 with 9
# queues 679 ms, 8 with 10 queues 682 ms.  The other workloads keep 12:
# their worker and spike streams share queues with 8 (adjoint gradient at n = 100,000:
# 430 against 340 ms).
def _workload_arg(argv):
    for i, a in enumerate(argv):
        if a == "--workload" and i + 1 < len(argv):
            return argv[i + 1]
        if a.startswith("--workload="):
            return a.split("=", 1)[1]
    return "cfg1"


HW_QUEUES = int(os.environ.get("SIMM_BENCH_HW_QUEUES", "8" if _workload_arg(sys.argv[1:]) == "cfg1" else "12"))
os.environ["GPU_MAX_HW_QUEUES"] = str(HW_QUEUES)

METRIC = "resolvent solves/s + indicators/s at n=40k; speedup vs plain FP64 at 1e-6"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


FP64_PEAK_TFLOPS = 78.6   # 256 CUs x 4 SIMDs x 16 FP64 FMA lanes x 2 flops x 2.4 GHz
FP32_MFMA_PEAK_TFLOPS = 157.3   # dense FP32 matrix cores
BF16_MFMA_PEAK_TFLOPS = 2500.0  # dense BF16 matrix cores
LU_PANEL = 16


def measured_traffic(profile: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or None when
    the kernel source has changed since the counters were taken (the summary names
    the source file and its sha256)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", profile)
    try:
        fields = {}
        with open(path) as fh:
            for line in fh:
                if ":" in line and not line.startswith(" "):
                    k, _, v = line.partition(":")
                    fields[k.strip()] = v.strip()
        src = os.path.join(ROOT, fields["source"])
        with open(src, "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != fields["source_sha256"]:
                return None
        return int(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def measured_profile_value(profile: str, key: str, sources):
    """An integer field of a committed rocprofv3 counter summary, or None when one of
    the kernel sources has changed since the counters were taken."""
    import hashlib
    try:
        text = open(os.path.join(ROOT, "profiles", profile)).read()
        for src in sources:
            digest = hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()
            if f"{src} {digest}" not in text:
                return None
        for line in text.splitlines():
            if line.startswith(key + ":"):
                return int(line.split(":", 1)[1])
    except (OSError, ValueError):
        return None
    return None


APPLY_SOURCES = ["paper_2006_16117_amd/csrc/band_spike.hip", "paper_2006_16117_amd/csrc/arnoldi.hip",
                 "paper_2006_16117_amd/csrc/band_sweep.hip"]


def apply_bytes(n: int, k: int, kb: int) -> int:
    """Algorithmic HBM bytes of one application of M = (A - sigma B)^{-1} B: the
    factor (3k+1 band rows), B (2 k_B + 1 rows), and about six n-vectors in and out,
    complex128: 16 n [(3k+1) + (2 k_B + 1) + 6]."""
    return 16 * n * ((3 * k + 1) + (2 * kb + 1) + 6)


def lu_flops_per_launch(kl: int, ku: int) -> int:
    """Algorithmic flops of one panel launch of the band LU: 16 columns, each a
    rank-1 update of kl rows by kl + ku columns (8 real flops per complex
    multiply-add)."""
    return LU_PANEL * 8 * kl * (kl + ku)


def cpu_baseline(pen, f, params, n_qp, threads=0):
    """The CPU oracle on the same workload: one complete SIM-M run (every shift's LU and
    Arnoldi basis, every level's squares, the association's and the fallbacks' extra
    evaluations), timed on the host.  value = the GPU step's resolvent solves over the
    oracle's wall time (the same squares, so the same solves).  threads: BLAS threads
    (0: the library default, normally one per core)."""
    import contextlib
    import oracle.simm as O
    from threadpoolctl import threadpool_info, threadpool_limits
    with (threadpool_limits(limits=threads) if threads > 0 else contextlib.nullcontext()):
        used = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
        t0 = time.perf_counter()
        res = O.simm(pen, f, params)
        t = time.perf_counter() - t0
    return {"value": n_qp / t, "unit": "resolvent solves/s", "cores": int(used), "kind": "oracle",
            "sample": (f"one complete oracle run of this workload on the host ({len(res.shifts)} shifts, K = {res.K}, "
                       f"{len(res.clusters)} clusters): {t:.1f} s, BLAS threads {int(used)}, host cores "
                       f"{os.cpu_count()}"),
            "seconds": t, "host_cpus": os.cpu_count()}


def bench_batch(args):
    """Batched form: every pencil of the batch run separately (one stream), then all
    together through simm_run_batch (up to --workers runs in flight).  value is the
    batched resolvent-solve rate summed over the pencils."""
    import torch
    from workloads import load_config, make_batch
    import paper_2006_16117_amd.simm as S

    assert torch.cuda.is_available(), "needs a ROCm GPU"
    os.environ.setdefault("SIMM_BATCH_PROGRESS", "1")   # the library prints a line per pencil and level
    batch = make_batch(args.workload)
    log("batch", args.workload, len(batch), "pencils, n =", sum(p.n for p, _, _ in batch))
    pencils = [S.Pencil.from_workload(p) for p, _, _ in batch]
    fs = [f for _, f, _ in batch]
    # results keep only levels, clusters and small per-shift data (a batch of large
    # pencils would otherwise hold every factor and Krylov basis of every run)
    prms = [S.params_from_dict(d, flags=S.SIMM_FLAG_RELEASE_FACTORS) for _, _, d in batch]
    bprms = [S.params_from_dict(d, flags=S.SIMM_FLAG_RELEASE_FACTORS, lookahead=args.batch_lookahead)
             for _, _, d in batch]
    torch.cuda.synchronize()
    for w in range(args.warmup):
        t0 = time.perf_counter()
        S.simm_run_batch(pencils, fs, bprms, workers=args.workers)
        log(f"batched warm-up {w + 1}/{args.warmup}: {time.perf_counter() - t0:.2f} s")
    t0 = time.perf_counter()
    n_qp = n_sq = 0
    for i, (P, f, prm) in enumerate(zip(pencils, fs, prms)):
        if args.no_sequential:
            break
        r = S.simm_run(P, f, prm)
        n_qp += r.counters["quadrature_systems"]
        n_sq += r.counters["squares"]
        del r
        if (i + 1) % 8 == 0:
            log(f"sequential: {i + 1}/{len(pencils)} runs, {time.perf_counter() - t0:.1f} s")
    t_seq = time.perf_counter() - t0
    log(f"sequential: {t_seq:.2f} s")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        bat = S.simm_run_batch(pencils, fs, bprms, workers=args.workers)
    t_bat = (time.perf_counter() - t0) / args.steps
    if args.no_sequential:
        n_qp = sum(r.counters["quadrature_systems"] for r in bat)
        n_sq = sum(r.counters["squares"] for r in bat)
        t_seq = float("nan")
    assert sum(r.counters["quadrature_systems"] for r in bat) == n_qp
    log(f"batched ({args.workers} in flight): {t_bat:.2f} s")
    cfg = load_config(args.workload)
    out = {
        "metric": "resolvent solves/s, batched form (all pencils of the batch, runs in flight together)",
        "value": n_qp / t_bat,
        "unit": "resolvent solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_bat * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "sequential_value": n_qp / t_seq,
        "sequential_ms": t_seq * 1e3,
        "speedup_vs_sequential": t_seq / t_bat,
        "indicators_per_s": n_sq / t_bat,
        "config": {"workload": cfg["description"], "pencils": len(batch),
                   "n_total": sum(p.n for p, _, _ in batch), "workers": args.workers,
                   "lookahead_per_run": args.batch_lookahead, "hw_queues": HW_QUEUES,
                   "resolvent_solves_per_step": n_qp, "squares_per_step": n_sq},
    }
    print(json.dumps(out))


def mixed_vs_fp64(S, P, fd, params, steps, warmup):
    """The mixed-precision form (FP32 band LU, every solve refined to a backward error of
    1e-12, BF16/FP32 projections) against the plain FP64 form on one pencil: wall time of
    `steps` runs of each after `warmup`, region sets of every level compared, and the FP64
    error of each eigenvalue (the Ritz value of the cluster's shift)."""
    import numpy as np
    import torch
    prm64 = S.params_from_dict(params, flags=S.SIMM_FLAG_PROJECT)
    prmmx = S.params_from_dict(params, flags=S.SIMM_FLAG_PROJECT, precision=S.SIMM_PREC_MIXED)
    out = {}
    res = {}
    for name, prm in (("fp64", prm64), ("mixed", prmmx)):
        for w in range(warmup):
            r = S.simm_run(P, fd, prm)
            log(f"{name} warmup {w + 1}/{warmup}: {r.ms['total']:.1f} ms")
            del r
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            r = S.simm_run(P, fd, prm)
            log(f"{name} step {k + 1}/{steps}: {r.ms['total']:.1f} ms (shift builds {r.ms['shift_builds']:.1f})")
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / steps
        res[name] = r
        out[name] = {"ms_per_step": t * 1e3, "shift_build_ms": r.ms["shift_builds"], "indicator_ms": r.ms["indicators"],
                     "projection_ms": r.ms["projection"], "resolvent_solves_per_s": r.counters["quadrature_systems"] / t,
                     "shifts": r.n_shifts, "levels": r.K, "clusters": int(len(r.lam))}
    a, b = res["fp64"], res["mixed"]
    same = a.K == b.K and all(np.array_equal(x.keys, y.keys) and np.array_equal(x.decision, y.decision)
                              and np.array_equal(x.shift, y.shift) for x, y in zip(a.levels, b.levels))
    ok = np.isfinite(a.lam_ritz) & np.isfinite(b.lam_ritz)
    err = (np.abs(b.lam_ritz[ok] - a.lam_ritz[ok]) / np.abs(a.lam_ritz[ok])) if same else np.array([np.inf])
    out["region_sets_equal"] = bool(same)
    out["clusters_equal"] = bool(same and np.array_equal(a.lam, b.lam))
    out["eigenvalue_fp64_rel_err"] = {"max": float(err.max()) if err.size else 0.0,
                                      "median": float(np.median(err)) if err.size else 0.0,
                                      "count": int(err.size),
                                      "per_eigenvalue": [float(e) for e in err]}
    out["refinement"] = b.refine
    out["speedup_vs_plain_fp64"] = out["fp64"]["ms_per_step"] / out["mixed"]["ms_per_step"]
    return out


def bench_mixed(args):
    """Mixed-precision workload: the metric's speedup clause (plain FP64 form over the
    mixed-precision form at h0 = 1e-6, equal region sets)."""
    import numpy as np
    import torch
    from workloads import load_config, make_workload
    import paper_2006_16117_amd.simm as S
    assert torch.cuda.is_available(), "needs a ROCm GPU"
    cfg = load_config(args.workload)
    pen, f, params = make_workload(args.workload)
    log("workload", args.workload, "n =", pen.n)
    P = S.Pencil.from_workload(pen)
    fd = torch.from_numpy(np.ascontiguousarray(f)).to("cuda:0")
    mx = mixed_vs_fp64(S, P, fd, params, args.steps, args.warmup)
    out = {
        "metric": "resolvent solves/s of the mixed-precision form at n=250k; speedup vs plain FP64 at 1e-6",
        "value": mx["mixed"]["resolvent_solves_per_s"],
        "unit": "resolvent solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mx["mixed"]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 factor + f64 refinement",
        "data": "synthetic",
        "speedup_vs_plain_fp64": mx["speedup_vs_plain_fp64"],
        "config": {"workload": cfg["description"], "n": pen.n, "kl": pen.kl_a, "m": params["m"],
                   "gauss_per_edge": params["gauss_per_edge"], "h0": params["h0"]},
        "mixed_vs_fp64": mx,
    }
    print(json.dumps(out))


def bench_gradient(args):
    """Differentiation workload: one SIM-M run of A(p) = A0 + p A1 fixes the squares
    (admissible squares of the last level) and their shifts; the timed step is one
    simm_gradient call (J, dJ/dp and the n values of dJ/d diag(A)).  The derivatives
    are checked against central differences of the library's J at the same shifts."""
    import numpy as np
    import torch
    from workloads import load_config, make_workload, random_band_matrix
    import paper_2006_16117_amd.simm as S

    assert torch.cuda.is_available(), "needs a ROCm GPU"
    cfg = load_config(args.workload)
    dcfg = cfg["differentiation"]
    pen0, f, params = make_workload(args.workload)
    n = pen0.n
    k1 = dcfg["k1"]
    a1 = random_band_matrix(n, k1, dcfg["seed"], 1.0 / np.sqrt(n))
    p0 = dcfg["p"]
    kl, ku, band = S._band_sum(n, [(pen0.kl_a, pen0.ku_a, pen0.a_band), (k1, k1, p0 * a1)])
    P = S.Pencil(n, kl, ku, band, pen0.kl_b, pen0.ku_b, pen0.b_band)
    prm = S.params_from_dict(params)
    t0 = time.perf_counter()
    res = S.simm_run(P, f, prm)
    t_run = time.perf_counter() - t0
    last = res.levels[-1]
    adm = np.nonzero(last.decision == S.ADMISSIBLE)[0]
    used = sorted(set(int(last.shift[i]) for i in adm))
    remap = {s: j for j, s in enumerate(used)}
    regions = np.array([(res.K, last.keys[i, 0], last.keys[i, 1], remap[int(last.shift[i])]) for i in adm],
                       dtype=np.int64).reshape(-1, 4)
    shifts = [res.shift(s) for s in used]
    sigmas = [sh.info()["sigma"] for sh in shifts]
    log(f"run: {t_run * 1e3:.0f} ms, K = {res.K}, {len(adm)} admissible squares, {len(used)} shifts")
    for w in range(args.warmup):
        S.simm_gradient(shifts, regions, prm, a1, k1, k1, n=n)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        J, dp, gd = S.simm_gradient(shifts, regions, prm, a1, k1, k1, n=n)
        log(f"gradient {s + 1}/{args.steps}: J = {J:.6e}, dJ/dp = {dp:.6e}")
    t_grad = (time.perf_counter() - t0) / args.steps
    if args.no_fd:
        print(json.dumps({"metric": "adjoint gradient evaluations/s", "value": 1.0 / t_grad, "unit": "gradients/s",
                          "ms_per_step": t_grad * 1e3, "forward_run_ms": t_run * 1e3, "J": J, "dJdp": dp}))
        return
    # central differences of J (same shifts, same squares)
    prob = S.ProjectedNorms(n, pen0.kl_a, pen0.ku_a, pen0.a_band, k1, k1, a1, f, sigmas, regions, prm, params["m"],
                            pen0.kl_b, pen0.ku_b, pen0.b_band)
    h = dcfg["fd_h"]
    z = np.zeros(n, dtype=np.complex128)
    fd_p = (prob.evaluate(p0 + h, z, derivatives=False)[0] - prob.evaluate(p0 - h, z, derivatives=False)[0]) / (2 * h)
    err_p = abs(dp - fd_p) / abs(fd_p)
    log(f"dJ/dp {dp:.10e}  central difference {fd_p:.10e}  rel {err_p:.2e}")
    # diagonal entries checked: the two largest |dJ/dA_ii| and the configured ones.  The
    # central difference has an O(h^2) truncation error, large at entries whose
    # eigenvalue sits near quadrature nodes of a small square; the Richardson
    # combination (4 D(h/2) - D(h)) / 3 of the steps h and h/2 removes it.
    scale = float(np.max(np.abs(gd)))
    top = [int(i) for i in np.argsort(-np.abs(gd))[:2]]
    err_d = err_r = 0.0

    def central(i, hh):
        e = np.zeros(n, dtype=np.complex128)
        e[i] = hh
        Jd = [prob.evaluate(p0, v, derivatives=False)[0] for v in (e, -e, 1j * e, -1j * e)]
        return complex((Jd[0] - Jd[1]) / (2 * hh), (Jd[2] - Jd[3]) / (2 * hh))

    for i in top + list(dcfg["fd_diag"]):
        d1 = central(i, h)
        d2 = central(i, h / 2)
        rich = (4 * d2 - d1) / 3
        err_d = max(err_d, abs(gd[i] - d1) / scale)
        err_r = max(err_r, abs(gd[i] - rich) / scale)
        log(f"grad_diag[{i}] {gd[i]:.10e}  central difference {d1:.10e} ({abs(gd[i] - d1) / scale:.2e})  "
            f"Richardson {rich:.10e} ({abs(gd[i] - rich) / scale:.2e})")
    out = {
        "metric": "adjoint gradient evaluations/s (J, dJ/dp and dJ/d diag(A) over the last level's squares)",
        "value": 1.0 / t_grad,
        "unit": "gradients/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_grad * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "forward_run_ms": t_run * 1e3,
        "J": J,
        "dJdp": dp,
        "fd_rel_err_dJdp": err_p,
        "fd_rel_err_diag": err_d,
        "fd_richardson_rel_err_diag": err_r,
        "fd_checked_diag": top + list(dcfg["fd_diag"]),
        "config": {"workload": cfg["description"], "n": n, "kl": kl, "ku": ku, "m": params["m"],
                   "squares": int(regions.shape[0]), "shifts": len(used), "levels": res.K},
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg1")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="BLAS threads of the CPU oracle baseline (0: the library default, one per core)")
    ap.add_argument("--no-fd", action="store_true", help="differentiation workload: skip the central differences")
    ap.add_argument("--mult-k", type=int, default=4, help="start vectors for the multiplicity step (0: skip)")
    ap.add_argument("--project-c", type=int, default=1600,
                    help="columns of the full-level projection measured after the steps (0: skip)")
    ap.add_argument("--workers", type=int, default=16, help="runs in flight in the batched form (at most 16)")
    ap.add_argument("--lookahead", type=int, default=0,
                    help="LU factors computed ahead in the timed run (0: the library default)")
    ap.add_argument("--batch-lookahead", type=int, default=2,
                    help="look-ahead of each run in the batched form (0: the batch default, one at a time)")
    ap.add_argument("--no-sequential", action="store_true", help="batched form only (no separate runs)")
    ap.add_argument("--no-speedup", action="store_true",
                    help="skip the metric's speedup clause (mixed precision vs plain FP64 on the n = 250,000 workload)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes (three times): the reference "
                         "for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE to HBM bytes")
    args = ap.parse_args()
    if args.copy_calibration > 0:
        import torch
        n = args.copy_calibration // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the shift-parallel multi-GPU "
              "layout is described in the design notes but not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from workloads import load_config, make_workload
    import paper_2006_16117_amd.simm as S

    if load_config(args.workload)["generator"]["kind"].endswith("_batch"):
        return bench_batch(args)
    if "differentiation" in load_config(args.workload):
        return bench_gradient(args)
    if args.workload.startswith("cfg3"):
        return bench_mixed(args)

    assert torch.cuda.is_available(), "needs a ROCm GPU"
    dev = torch.device("cuda:0")
    pen, f, params = make_workload(args.workload)
    log("workload", args.workload, "n =", pen.n)
    P = S.Pencil.from_workload(pen)
    fd = torch.from_numpy(np.ascontiguousarray(f)).to(dev)
    prm = S.params_from_dict(params, flags=S.SIMM_FLAG_PROJECT | S.SIMM_FLAG_KERNEL_TIMING, lookahead=args.lookahead)
    torch.cuda.synchronize()

    for w in range(args.warmup):
        res = S.simm_run(P, fd, prm)
        log(f"warmup {w + 1}/{args.warmup}: {res.ms['total']:.1f} ms")
        del res
    torch.cuda.synchronize()
    kms = {k: 0.0 for k in S.KERNEL_NAMES}
    kcnt = {k: 0 for k in S.KERNEL_NAMES}
    t0 = time.perf_counter()
    last = None
    for s in range(args.steps):
        res = S.simm_run(P, fd, prm)
        for k in S.KERNEL_NAMES:
            kms[k] += res.kernel_ms[k]
            kcnt[k] += res.kernel_launches[k]
        log(f"step {s + 1}/{args.steps}: {res.ms['total']:.1f} ms")
        last = res
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    n_qp = last.counters["quadrature_systems"]
    n_sq = last.counters["squares"]
    value = n_qp / (ms_per_step / 1e3)

    n = pen.n
    kl, ku = max(pen.kl_a, pen.kl_b), max(pen.ku_a, pen.ku_b)
    kb = max(pen.kl_b, pen.ku_b) if pen.b_band is not None else 0
    # dominant kernel: the band LU's panel step (one launch per 16 columns plus one)
    lu_launches = kcnt["band_lu"]   # panel launches (factors cancelled part-way included)
    lu_us_step = kms["band_lu"] * 1e3 / max(lu_launches, 1)
    # The step computes up to 11 factors at once (the level-1 association's look-ahead),
    # so its panel launches share the device; the roofline takes the launch alone: one
    # more run, untimed, that builds its shifts one at a time (HIP events around each
    # factor's launches on the run's stream).
    solo = S.simm_run(P, fd, S.params_from_dict(params, flags=S.SIMM_FLAG_KERNEL_TIMING, lookahead=1))
    lu_us = solo.kernel_ms["band_lu"] * 1e3 / max(solo.kernel_launches["band_lu"], 1)
    lu_solo_launches = solo.kernel_launches["band_lu"]
    del solo
    lu_tflops = lu_flops_per_launch(kl, ku) / (lu_us * 1e-6) / 1e12
    # K2: one application of M (B v + partitioned L and U sweeps)
    b_apply = apply_bytes(n, max(kl, ku), kb)
    apply_ms = kms["band_sweep"] / max(kcnt["band_sweep"], 1)
    apply_gbs = b_apply / (apply_ms / 1e3) / 1e9
    step_kernel_ms = {k: kms[k] / args.steps for k in kms}
    # shifted solves: the triangular system (I + (sigma - z) T) y = g of one quadrature
    # point is m^2 / 2 complex multiply-adds, 4 m^2 real flops (every shift of this
    # workload keeps m_eff = m)
    m = params["m"]
    ind_tflops = 4.0 * m * m * n_qp / (kms["indicators"] / args.steps * 1e-3) / 1e12 if kms["indicators"] > 0 else 0.0
    # X = V_m Y: 8 n m flops per column, two columns (s_c, s_f) per square
    proj_flops = 8.0 * n * m * 2 * n_sq
    proj_tflops = proj_flops / (kms["project"] / args.steps * 1e-3) / 1e12 if kms["project"] > 0 else 0.0
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "resolvent solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "indicators_per_s": n_sq / (ms_per_step / 1e3),
        "speedup_vs_plain_fp64": None,
        "config": {
            "workload": ("convection-diffusion pencil n=40000 (200x200 grid, h=1/201), B=tridiag(0.05,1,0.05), "
                         "R=[120,1400]x[-310,330], 16 Gauss points/edge, m=80, 4 levels, column norms of X=V_mY every level"),
            "n": pen.n, "kl": kl, "ku": ku, "m": params["m"], "gauss_per_edge": params["gauss_per_edge"],
            "levels": last.K, "shifts": last.n_shifts, "squares_per_step": n_sq,
            "resolvent_solves_per_step": n_qp, "clusters": len(last.lam),
            "hw_queues": HW_QUEUES,
        },
        "roofline": {
            "kernel": "k_band_lu_step (one 16-column panel of the banded LU)",
            "bound": "alu",
            "achieved": lu_tflops,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": lu_tflops / FP64_PEAK_TFLOPS,
            "traffic": measured_traffic("k_band_lu_step_convdiff_n40000_traffic.md"),
            "flops_per_launch": lu_flops_per_launch(kl, ku),
            "us_per_launch": lu_us,
            "launches_measured": lu_solo_launches,
            "measured_in": "a run building its shifts one at a time (no factor beside it), HIP events per factor",
            "us_per_launch_in_step": lu_us_step,
            "launches_per_step": lu_launches // args.steps,
        },
        "roofline_apply": {
            "kernel": "one application of M = U^-1 L^-1 P B (k_prepare_input; k_chunk_fwd, k_spike_chain x2, "
                      "k_spike_fix, k_spike_correct; k_chunk_bwd, k_spike_chain x2, k_spike_fix, k_spike_correct)",
            "bound": "hbm",
            "achieved": apply_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": apply_gbs / HBM_PEAK_GBS,
            "bytes_per_launch": b_apply,
            "traffic": measured_profile_value("apply_cgs2_convdiff_n40000_traffic.md", "apply_bytes_per_launch",
                                              APPLY_SOURCES),
            "ms_per_launch": apply_ms,
            "launches_per_step": kcnt["band_sweep"] // args.steps,
        },
        "roofline_indicators": {
            "kernel": "k_indicators (shifted solves, sums, residuals and decisions of a batch of squares)",
            "bound": "alu",
            "achieved": ind_tflops,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": ind_tflops / FP64_PEAK_TFLOPS,
            "flops_per_point": 4 * m * m,
            "points_per_step": n_qp,
            "ms_per_step": kms["indicators"] / args.steps,
        },
        "roofline_project": {
            "kernel": "k_vmy (column norms of X = V_m Y on the FP64 matrix cores, X not stored), per level and shift",
            "bound": "mfma",
            "achieved": proj_tflops,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": proj_tflops / FP64_PEAK_TFLOPS,
            "flops_per_step": proj_flops,
            "ms_per_step": kms["project"] / args.steps,
        },
        "kernel_ms_per_step": step_kernel_ms,
    }
    if args.project_c > 0:
        # X = V_m Y alone at a level's full width (c columns: s_c and s_f of c/2 squares)
        # on the first shift's basis, outside the timed step; HIP events on torch's stream.
        # FP64 with X written (the roofline), then each precision with only the column
        # norms formed (what a run needs), and the error of the reduced-precision norms.
        c = args.project_c
        sh = last.shift(0)
        me = sh.info()["m_eff"]
        g = torch.Generator(device="cpu").manual_seed(7)
        Yd = torch.randn((c, me), dtype=torch.complex128, generator=g).to(dev)    # column-major Y
        Xd = torch.empty((c, pen.n), dtype=torch.complex128, device=dev)
        pfl = 8.0 * pen.n * me * c

        def time_proj(X, prec, nd):
            for _ in range(2):
                S.simm_project(sh, Yd.T, X, nd, precision=prec)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 5
            e0.record()
            for _ in range(reps):
                S.simm_project(sh, Yd.T, X, nd, precision=prec)
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps

        nd64 = torch.empty(c, dtype=torch.float64, device=dev)
        pms = time_proj(Xd.T, S.SIMM_PROJ_FP64, nd64)
        out["roofline_project_full_level"] = {
            "kernel": f"k_vmy + column norms, n = {pen.n}, m = {me}, c = {c}, X written",
            "bound": "mfma", "achieved": pfl / (pms * 1e-3) / 1e12, "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": pfl / (pms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, "ms_per_launch": pms,
            "flops_per_launch": pfl,
        }
        log(f"projection c = {c} FP64 with X: {pms:.3f} ms")
        del Xd
        ref = None
        prec_out = {}
        for name, prec, peak in (("fp64", S.SIMM_PROJ_FP64, FP64_PEAK_TFLOPS),
                                 ("fp32", S.SIMM_PROJ_FP32, FP32_MFMA_PEAK_TFLOPS),
                                 ("bf16", S.SIMM_PROJ_BF16, BF16_MFMA_PEAK_TFLOPS)):
            nd = torch.empty(c, dtype=torch.float64, device=dev)
            ms = time_proj(None, prec, nd)
            nrm = nd.cpu().numpy()
            if ref is None:
                ref = nrm
            rel = float(np.max(np.abs(nrm - ref) / ref))
            prec_out[name] = {"ms_per_launch": ms, "achieved_tflops": pfl / (ms * 1e-3) / 1e12,
                              "peak_tflops": peak, "frac": pfl / (ms * 1e-3) / 1e12 / peak,
                              "max_rel_err_col_norms_vs_fp64": rel}
            log(f"projection c = {c} {name}, norms only: {ms:.3f} ms, max rel. error of the norms {rel:.2e}")
        out["project_norms_only_by_precision"] = prec_out
    if args.mult_k > 0:
        # multiplicities (Sec. 3.4) of the step's clusters from k further start vectors,
        # outside the timed step: k Krylov spaces per shift on the kept factors
        from workloads import start_vectors
        F = start_vectors(pen.n, args.mult_k, load_config(args.workload)["generator"]["seed"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mult, _ = S.simm_multiplicities(last, F)
        torch.cuda.synchronize()
        mms = (time.perf_counter() - t0) * 1e3
        shifts_used = len({int(s) for s in last.levels[-1].shift[last.levels[-1].decision != 0]})
        out["multiplicity"] = {
            "k": args.mult_k, "clusters": int(len(mult)), "ms": mms,
            "krylov_spaces": shifts_used * args.mult_k,
            "clusters_per_s": len(mult) / (mms / 1e3),
            "multiplicities": np.bincount(mult).tolist(),
        }
        log(f"multiplicities: k = {args.mult_k}, {len(mult)} clusters in {mms:.1f} ms")
    if not args.no_speedup:
        # the metric's third clause: plain FP64 form over the mixed-precision form at
        # h0 = 1e-6 on the n = 250,000 workload (one run of each after one warm-up)
        pen3, f3, params3 = make_workload("cfg3")
        log("speedup clause: workload cfg3, n =", pen3.n)
        P3 = S.Pencil.from_workload(pen3)
        fd3 = torch.from_numpy(np.ascontiguousarray(f3)).to(dev)
        mx = mixed_vs_fp64(S, P3, fd3, params3, 1, 1)
        out["speedup_vs_plain_fp64"] = mx["speedup_vs_plain_fp64"]
        mx["workload"] = load_config("cfg3")["description"]
        out["mixed_vs_fp64"] = mx
        del P3, fd3
    if not args.no_cpu_baseline:
        log("cpu baseline (one complete oracle run of the workload)")
        out["cpu_baseline"] = cpu_baseline(pen, f, params, n_qp, args.cpu_threads)
        log(f"cpu baseline: {out['cpu_baseline']['seconds']:.1f} s")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
