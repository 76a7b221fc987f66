"""Benchmark of the all-pairs CCM hot path on one MI355X.

One step = the whole hot path over one batch of synthetic input that is already resident
in HBM: simplex optE for every library (E = 1..20, Tp = 1, leave-one-out) -> neighbour
tables at each library's optE (Tp = 0) -> FP32 cross-map of every library against every
target, reduced to Pearson rho.  The workload is the 512-library x 101,729-target block at
L = 1600 (filtered-Poisson rates of a 101,729-unit sparse rate network, z-scored).

Prints ONE JSON line.  `value` = library x target cross-maps per second of the whole step.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cross-maps/s (library x target rho), FP32 gather vs BF16-MFMA, % HBM/MFMA peak"
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
# FP32 vector peak without packed FP32 (which every kernel here leaves out): 256 CUs x 4 SIMDs
# x 16 lanes x 2 flops x 2.4 GHz
FP32_FMA_PEAK_TFLOPS = 78.6


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def gather_model_bytes(lib_E, L: int, n_tgt: int) -> float:
    """Algorithmic bytes of one FP32 cross-map launch: per cross-map 4 n_E (target column
    read once) + 4 (rho), plus the library's table (8 k L bytes) read once."""
    lib_E = np.asarray(lib_E, dtype=np.int64)
    n = L - lib_E + 1
    k = lib_E + 1
    return float(np.sum(n_tgt * (4.0 * n + 4.0) + 8.0 * k * L))


def gather_fmas(lib_E, L: int, n_tgt: int) -> float:
    """Useful multiply-adds of one FP32 cross-map launch: k n_E per cross-map (the
    k-neighbour prediction of every query time)."""
    lib_E = np.asarray(lib_E, dtype=np.int64)
    n = L - lib_E + 1
    k = lib_E + 1
    return float(np.sum(k * n) * n_tgt)


def mfma_flops(lib_E, L: int, n_tgt: int) -> float:
    """Dense MFMA work of the BF16 densified form: 2 * n_E * L per cross-map."""
    lib_E = np.asarray(lib_E, dtype=np.int64)
    n = L - lib_E + 1
    return float(np.sum(2.0 * n * L) * n_tgt)


def source_hash(*names) -> str:
    """Hash of the code of the named kernel sources: comment-only lines and blank lines are
    left out, so editing a comment keeps the committed counter summary valid."""
    h = hashlib.sha1()
    for n in names:
        with open(os.path.join(ROOT, "paper_2011_11082_amd", "csrc", n), "rb") as f:
            for line in f:
                t = line.strip()
                if t and not t.startswith(b"//"):
                    h.update(t + b"\n")
    return h.hexdigest()[:12]


def load_traffic(kernel_src: str, launches_per_call: int = 1):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, if it was taken on
    the current kernel source (else None)."""
    p = os.path.join(ROOT, "profiles", "gather_fp32_brain101729_pmc.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("source_hash") != source_hash(kernel_src):
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_model() -> str:
    """The host CPU's model name (first 'model name' line of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or "unknown"


def cpu_baseline(panel, n_lib_total: int, n_tgt_total: int, L: int, n_tgt_sample: int = 256):
    """Time the CPU oracle on a bounded sample and scale to the metric's unit.

    One oracle process per library, each on its own core (at most 16, the host share of one
    GPU): optE E = 1..20 + the table at optE, then the cross-map of 256 evenly spaced
    targets.  The per-library and per-pair CPU times scale linearly to the full block
    (libraries are independent; a pair's cost does not depend on the target), spread over
    the same number of cores."""
    import shutil
    import subprocess
    import tempfile

    P = max(1, min(16, os.cpu_count() or 1))
    libs = list(range(min(P, n_lib_total)))
    tgt = np.arange(0, n_tgt_total, max(1, n_tgt_total // n_tgt_sample))[:n_tgt_sample]
    tmp = tempfile.mkdtemp(prefix="ccm_cpu_sample_")
    sample = os.path.join(tmp, "sample.npz")
    np.savez(sample, lib=np.ascontiguousarray(panel[:, libs]),
             tgt=np.ascontiguousarray(panel[:, tgt]))
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    t0 = time.perf_counter()
    procs = [subprocess.Popen([sys.executable, "-m", "oracle.sample_worker", sample, str(c),
                               os.path.join(tmp, f"out{c}.npz")], cwd=ROOT, env=env)
             for c in range(len(libs))]
    rcs = [p.wait() for p in procs]
    wall = time.perf_counter() - t0
    if any(rcs):
        raise RuntimeError(f"oracle sample workers failed: {rcs}")
    out = {}
    per_lib, per_pair = [], []
    for c, li in enumerate(libs):
        with np.load(os.path.join(tmp, f"out{c}.npz"), allow_pickle=False) as z:
            out[li] = (int(z["E"]), z["idx"], z["rho"])
            per_lib.append(float(z["t_lib"]))
            per_pair.append(float(z["t_pair"]))
    shutil.rmtree(tmp, ignore_errors=True)
    t_lib = float(np.mean(per_lib))
    t_pair = float(np.mean(per_pair))
    cores = len(libs)
    total = (n_lib_total * t_lib + n_lib_total * n_tgt_total * t_pair) / cores
    return {
        "value": n_lib_total * n_tgt_total / total,
        "unit": "cross-maps/s",
        "cores": cores,
        "cpu_model": cpu_model(),
        "host_cpus": os.cpu_count(),
        "host_cpus_usable": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
        "kind": "oracle",
        "sample": (f"{cores} libraries, one oracle process each on {cores} cores ({wall:.1f} s "
                   f"wall): optE E=1..20 + table ({t_lib:.2f} s per library), cross-map vs "
                   f"{len(tgt)} targets ({t_pair * 1e6:.0f} us per pair); scaled to "
                   f"{n_lib_total} x {n_tgt_total} over {cores} cores (extrapolated)"),
    }, out, tgt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="brain101729")
    ap.add_argument("--n-lib", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bf16", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint (gradient of rho over library-target pairs)")
    ap.add_argument("--no-convergence", action="store_true",
                    help="skip the CCM convergence test (tables over library subsamples)")
    ap.add_argument("--no-target-E", action="store_true",
                    help="skip the per-target-E form (optE of every series + all-E tables)")
    ap.add_argument("--no-long-series", action="store_true",
                    help="skip the step at the paper's recording lengths (L = 3,780 and 8,528)")
    ap.add_argument("--no-full-matrix", action="store_true",
                    help="skip the whole N x N matrices of the 1,024- and 8,192-series workloads")
    ap.add_argument("--profile-steps", action="store_true",
                    help="no timing extras (for runs under rocprofv3)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (a known-size "
                         "reference for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not "
                          "part of it (libraries would shard across GPUs with no exchange)"}))
        sys.exit(2)

    import torch

    import paper_2011_11082_amd as ccm
    import synth

    ccm.load_library()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")

    if args.copy_calibration_mib:
        nb = args.copy_calibration_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.copy_calibration_mib} MiB done")
        del src, dst

    t = time.perf_counter()
    wl = synth.make(args.workload)
    log(f"workload {args.workload} {wl.panel.shape} ready in {time.perf_counter() - t:.1f} s")
    panel = wl.panel
    L, N = panel.shape
    lib_ids_np = wl.lib_ids if args.n_lib is None else wl.lib_ids[: args.n_lib]
    n_lib = len(lib_ids_np)
    n_tgt = wl.n_tgt
    ts = torch.as_tensor(panel).to(dev)
    lib_ids = torch.as_tensor(lib_ids_np, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()

    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    def step(record=None):
        optE, rho_E = ccm.simplex_optE(ts, lib_ids, 1, wl.E_max, 1, 1, ccm.MODE_LOO)
        e1 = ev(); e1.record()
        idx, w, _ = ccm.knn(ts, lib_ids, optE, 1, 0, 21, want_d2=False)
        e2 = ev(); e2.record()
        rho = ccm.crossmap_rho(ts, idx, w, optE, 1, wl.tgt0, n_tgt, ccm.PRECISION_FP32)
        e3 = ev(); e3.record()
        if record is not None:
            record.append((e1, e2, e3))
        return optE, idx, w, rho

    for i in range(args.warmup):
        step()
        log(f"warmup step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()

    marks = []
    starts = []
    t0 = ev(); t0.record()
    wall0 = time.perf_counter()
    for i in range(args.steps):
        s = ev(); s.record(); starts.append(s)
        out = step(marks)
    t1 = ev(); t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t0.elapsed_time(t1)
    ms_step = total_ms / args.steps
    t_opt = np.mean([s.elapsed_time(m[0]) for s, m in zip(starts, marks)])
    t_knn = np.mean([m[0].elapsed_time(m[1]) for m in marks])
    t_cm = np.mean([m[1].elapsed_time(m[2]) for m in marks])
    log(f"timed {args.steps} steps: {ms_step:.2f} ms/step (optE {t_opt:.2f}, knn {t_knn:.2f}, "
        f"crossmap {t_cm:.2f}); wall {wall:.2f} s")
    optE, idx, w, rho = out
    optE_np = optE.cpu().numpy()
    cross = float(n_lib) * n_tgt
    value = cross / (ms_step * 1e-3)

    model_bytes = gather_model_bytes(optE_np, L, n_tgt)
    achieved = model_bytes / (t_cm * 1e-3) / 1e9
    traffic = load_traffic("crossmap.hip")
    fmas = gather_fmas(optE_np, L, n_tgt)
    fma_tflops = 2.0 * fmas / (t_cm * 1e-3) / 1e12
    roofline = {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
        "kernel": "ccm_crossmap_rho FP32 (table prep + gather)",
        "model_bytes_per_launch": model_bytes, "launch_ms": round(float(t_cm), 3),
        # the limits the call actually meets: FMA issue (the useful k n_E multiply-adds per
        # cross-map against the non-packed FP32 peak) and the HBM bytes the counters measured
        "fma_issue": {"useful_fmas_per_launch": fmas, "achieved": round(fma_tflops, 2),
                      "peak": FP32_FMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                      "frac": round(fma_tflops / FP32_FMA_PEAK_TFLOPS, 4)},
        "real_hbm": (None if traffic is None else
                     {"achieved": round(traffic / (t_cm * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                      "unit": "GB/s",
                      "frac": round(traffic / (t_cm * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}),
    }

    res = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "cross-maps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"{args.workload}: {n_lib} libraries x {n_tgt} targets, L={L}, "
                         "filtered-Poisson rates of a sparse rate network (z-scored); "
                         "optE E=1..20 (LOO, Tp=1) -> tables at optE (k=E+1) -> FP32 cross-map"),
            "n_lib": n_lib, "n_tgt": n_tgt, "L": L,
        },
        "breakdown_ms": {"simplex_optE": round(float(t_opt), 3), "knn": round(float(t_knn), 3),
                         "crossmap_fp32": round(float(t_cm), 3)},
        "crossmap_fp32_rate": round(cross / (t_cm * 1e-3), 1),
        "optE_hist": np.bincount(optE_np, minlength=21)[1:].tolist(),
        "roofline": roofline,
    }

    # BF16-MFMA form on the same tables (not part of the step; reported beside it)
    rho_bf = None
    if not args.no_bf16:
        for _ in range(1):
            ccm.crossmap_rho(ts, idx, w, optE, 1, wl.tgt0, n_tgt, ccm.PRECISION_BF16)
        torch.cuda.synchronize()
        eb0 = ev(); eb0.record()
        nb = max(1, min(3, args.steps))
        for _ in range(nb):
            rho_bf = ccm.crossmap_rho(ts, idx, w, optE, 1, wl.tgt0, n_tgt, ccm.PRECISION_BF16)
        eb1 = ev(); eb1.record()
        torch.cuda.synchronize()
        t_bf = eb0.elapsed_time(eb1) / nb
        flops = mfma_flops(optE_np, L, n_tgt)
        d = (rho_bf - rho).abs()
        d = d[~torch.isnan(d)].double()
        res["bf16"] = {
            "crossmap_ms": round(float(t_bf), 3),
            "rate": round(cross / (t_bf * 1e-3), 1),
            "speedup_vs_fp32": round(float(t_cm / t_bf), 4),
            "mfma": {"bound": "mfma", "achieved": round(flops / (t_bf * 1e-3) / 1e12, 1),
                     "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(flops / (t_bf * 1e-3) / 1e12 / BF16_PEAK_TFLOPS, 4),
                     "dense_flops_per_launch": flops},
            "max_abs_drho_vs_fp32": float(d.max()) if d.numel() else None,
            "abs_drho_vs_fp32": ({"max": float(d.max()),
                                  "p99": float(torch.quantile(d[:: max(1, d.numel() // 4000000)], 0.99)),
                                  "median": float(d.median()), "n": int(d.numel())}
                                 if d.numel() else None),
        }
        log(f"bf16 crossmap {t_bf:.2f} ms")

    # The paper's per-target-E form (not part of the step; reported beside it): optE of every
    # series (phase 1 at full N), each library's table at every E, then each target read
    # through the tables at its own E.
    if not args.no_target_E and not args.profile_steps:
        all_ids = torch.arange(N, dtype=torch.int32, device=dev)
        tE = {}
        for rep in range(2):   # one warm-up, one timed
            ea = ev(); ea.record()
            optE_all, _ = ccm.simplex_optE(ts, all_ids, 1, wl.E_max, 1, 1, ccm.MODE_LOO)
            eb = ev(); eb.record()
            tidx, tw, _ = ccm.knn_all_E(ts, lib_ids, 1, wl.E_max, 1, 21)
            ec = ev(); ec.record()
            rho_t = ccm.crossmap_rho_target_E(ts, tidx, tw, n_lib, optE_all[wl.tgt0: wl.tgt0 + n_tgt],
                                              E_lo=1, tgt0=wl.tgt0, n_tgt=n_tgt)
            ed = ev(); ed.record()
            torch.cuda.synchronize()
            tE = {"optE_all_series_ms": round(ea.elapsed_time(eb), 2),
                  "tables_all_E_ms": round(eb.elapsed_time(ec), 3),
                  "crossmap_ms": round(ec.elapsed_time(ed), 3)}
            del tidx, tw, rho_t
        # the paper's own phase-1 protocol (first half = library, second half = prediction)
        ea = ev(); ea.record()
        optE_half, _ = ccm.simplex_optE(ts, all_ids, 1, wl.E_max, 1, 1, ccm.MODE_HALF)
        eb = ev(); eb.record()
        torch.cuda.synchronize()
        tE["optE_all_series_half_split_ms"] = round(ea.elapsed_time(eb), 2)
        tE["optE_half_split_agrees_with_loo"] = round(
            float((optE_half == optE_all).float().mean()), 4)
        del optE_half
        tE["n_series"] = N
        tE["n_tables"] = n_lib * wl.E_max
        tE["crossmap_rate"] = round(cross / (tE["crossmap_ms"] * 1e-3), 1)
        tE["optE_hist_all_series"] = torch.bincount(optE_all.long(), minlength=21)[1:].tolist()
        res["per_target_E"] = tE
        log(f"per-target-E: optE of {N} series {tE['optE_all_series_ms']:.0f} ms "
            f"(half split {tE['optE_all_series_half_split_ms']:.0f} ms), "
            f"{tE['n_tables']} tables {tE['tables_all_E_ms']:.1f} ms, "
            f"cross-map {tE['crossmap_ms']:.1f} ms")
        del optE_all

    # The CCM convergence test (not part of the step; reported beside it): every library's
    # table at its optE over random library subsamples of growing size (7 sizes x 4 draws),
    # then the cross-map of 1,024 evenly spaced targets.
    if not args.no_convergence and not args.profile_steps:
        sizes = [25, 50, 100, 200, 400, 800, 1500]
        n_draw = 4
        n_cv_tgt = 1024
        masks = np.zeros((n_lib, len(sizes) * n_draw, L), dtype=bool)
        for E in sorted(set(optE_np.tolist())):
            rows = np.nonzero(optE_np == E)[0]
            masks[rows] = synth.library_samples(L, int(E), sizes, n_draw, int(E))[None]
        cols = np.arange(0, n_tgt, n_tgt // n_cv_tgt)[:n_cv_tgt] + wl.tgt0
        Ysub = ts[:, torch.as_tensor(cols, device=dev)].contiguous()
        m_dev = torch.as_tensor(masks, device=dev)
        ids_rep = lib_ids.repeat_interleave(masks.shape[1])
        E_rep = optE.repeat_interleave(masks.shape[1])
        panel_cv = torch.cat([ts[:, lib_ids.long()], Ysub], dim=1).contiguous()
        lib_cols = torch.arange(n_lib, dtype=torch.int32, device=dev).repeat_interleave(masks.shape[1])
        for rep in range(2):   # one warm-up, one timed
            ea = ev(); ea.record()
            cidx, cw, _ = ccm.knn(panel_cv, lib_cols, E_rep, 1, 0, 21, want_d2=False,
                                  cand_mask=m_dev.reshape(-1, L))
            eb = ev(); eb.record()
            crho = ccm.crossmap_rho(panel_cv, cidx, cw, E_rep, 1, n_lib, n_cv_tgt)
            ec = ev(); ec.record()
            torch.cuda.synchronize()
        curve = crho.reshape(n_lib, len(sizes), n_draw, n_cv_tgt).nanmean(dim=(0, 2, 3))
        cv = {"n_tables": int(cidx.shape[0]), "library_sizes": sizes, "draws_per_size": n_draw,
              "n_tgt": n_cv_tgt, "tables_ms": round(ea.elapsed_time(eb), 3),
              "crossmap_ms": round(eb.elapsed_time(ec), 3),
              "mean_rho_by_size": [round(float(v), 4) for v in curve.cpu()]}
        res["convergence"] = cv
        log(f"convergence: {cv['n_tables']} subsampled tables {cv['tables_ms']:.1f} ms, "
            f"cross-map {cv['crossmap_ms']:.1f} ms, mean rho by size {cv['mean_rho_by_size']}")
        del cidx, cw, crho, m_dev, panel_cv

    # The adjoint (not part of the step; reported beside it): d rho / d (targets, libraries)
    # with the neighbour sets fixed, for 4,096 seeded (library, target) pairs of this block.
    if not args.no_adjoint and not args.profile_steps:
        rng = np.random.default_rng(45)
        P = 4096
        prow = torch.as_tensor(rng.integers(0, n_lib, size=P).astype(np.int32), device=dev)
        ptgt = torch.as_tensor(rng.integers(0, n_tgt, size=P).astype(np.int32) + wl.tgt0,
                               device=dev)
        X = ts[:, lib_ids.long()].t().contiguous()
        grho = torch.ones(P, dtype=torch.float32, device=dev)
        gts = torch.zeros_like(ts)
        glib = torch.zeros_like(X)
        for rep in range(2):   # one warm-up, one timed
            ea = ev(); ea.record()
            ccm.crossmap_rho_backward(ts, X, idx, w, optE, prow, ptgt, grho, 1, gts, glib)
            eb = ev(); eb.record()
            torch.cuda.synchronize()
        res["adjoint"] = {"pairs": P, "backward_ms": round(ea.elapsed_time(eb), 3),
                          "us_per_pair": round(ea.elapsed_time(eb) * 1e3 / P, 2)}
        log(f"adjoint: {P} pairs backward {ea.elapsed_time(eb):.1f} ms")
        del X, gts, glib

    # The whole step at the recording lengths of the paper's Subject6 (3,780) and Subject11
    # (8,528) data, beyond the 16-target LDS tile (the gather then reads a global tile copy
    # through L2): 512 libraries x 8,192 filtered-Poisson targets, one timed step each.
    if not args.no_long_series and not args.profile_steps:
        long_res = []
        for Llong in (3780, 8528):
            wl2 = synth.make("poisson8192", T=Llong)
            ts2 = torch.as_tensor(wl2.panel, device=dev)
            ids2 = torch.arange(512, dtype=torch.int32, device=dev)
            for rep in range(2):   # one warm-up, one timed
                e0, e1, e2, e3 = ev(), ev(), ev(), ev()
                e0.record()
                oE2, _ = ccm.simplex_optE(ts2, ids2, 1, 20, 1, 1)
                e1.record()
                i2, w2, _ = ccm.knn(ts2, ids2, oE2, 1, 0, 21, want_d2=False)
                e2.record()
                r2 = ccm.crossmap_rho(ts2, i2, w2, oE2)
                e3.record()
                torch.cuda.synchronize()
            eb0, eb1 = ev(), ev()
            eb0.record()
            rb = ccm.crossmap_rho(ts2, i2, w2, oE2, precision=ccm.PRECISION_BF16)
            eb1.record()
            torch.cuda.synchronize()
            n2 = 512 * ts2.shape[1]
            t_step = e0.elapsed_time(e3)
            long_res.append({
                "L": Llong, "n_lib": 512, "n_tgt": int(ts2.shape[1]),
                "step_ms": round(t_step, 3), "rate": round(n2 / (t_step * 1e-3), 1),
                "optE_ms": round(e0.elapsed_time(e1), 3), "knn_ms": round(e1.elapsed_time(e2), 3),
                "crossmap_fp32_ms": round(e2.elapsed_time(e3), 3),
                "crossmap_bf16_ms": round(eb0.elapsed_time(eb1), 3),
                "max_abs_drho_bf16_vs_fp32": float((rb - r2).abs().nan_to_num(0.0).max())})
            log(f"long series L={Llong}: step {t_step:.1f} ms (optE {e0.elapsed_time(e1):.1f}, "
                f"tables {e1.elapsed_time(e2):.1f}, FP32 cross-map {e2.elapsed_time(e3):.1f}, "
                f"BF16 {eb0.elapsed_time(eb1):.1f})")
            del ts2, i2, w2, r2, rb
        res["long_series"] = long_res

    # The whole N x N matrix (phase 1 over every series, then blocks of 512 libraries) of the
    # 1,024-series rate network (L = 1,450) and the 8,192-series filtered-Poisson panel
    # (L = 1,600), one timed call each after a warm-up; the latter in both cross-map forms.
    if not args.no_full_matrix and not args.profile_steps:
        fm = []
        for name, precs in (("ratenet1024", (ccm.PRECISION_FP32,)),
                            ("poisson8192", (ccm.PRECISION_FP32, ccm.PRECISION_BF16))):
            wl3 = synth.make(name)
            ts3 = torch.as_tensor(wl3.panel, device=dev)
            N3 = int(ts3.shape[1])
            for prec in precs:
                for rep in range(2):   # one warm-up, one timed
                    e0, e1 = ev(), ev()
                    e0.record()
                    r3, _ = ccm.ccm_matrix(ts3, 1, wl3.E_max, block=512, precision=prec)
                    e1.record()
                    torch.cuda.synchronize()
                t3 = e0.elapsed_time(e1)
                fm.append({"workload": name, "N": N3, "L": int(ts3.shape[0]),
                           "precision": "bf16" if prec == ccm.PRECISION_BF16 else "fp32",
                           "ms": round(t3, 2), "rate": round(N3 * N3 / (t3 * 1e-3), 1)})
                log(f"full matrix {name} {fm[-1]['precision']}: {N3}x{N3} in {t3:.1f} ms")
                del r3
            del ts3
        res["full_matrix"] = fm

    if not args.no_cpu_baseline and not args.profile_steps:
        log("timing the CPU oracle on a bounded sample")
        cb, oracle_out, tgt = cpu_baseline(panel, n_lib, n_tgt, L)
        res["cpu_baseline"] = cb
        # parity on the same sample
        idx_np = idx.cpu().numpy()
        rho_np = rho.cpu().numpy()
        pe = {}
        exact = True
        d32, d16 = [], []
        rho_bf_np = rho_bf.cpu().numpy() if rho_bf is not None else None
        for li, (E, oidx, orho) in oracle_out.items():
            if int(optE_np[li]) != E:
                pe[f"optE_{li}"] = [int(optE_np[li]), E]
                continue
            exact &= bool(np.array_equal(idx_np[li], oidx))
            ok = ~np.isnan(orho)
            d32.append(np.abs(rho_np[li, tgt].astype(np.float64) - orho)[ok])
            if rho_bf_np is not None:
                d16.append(np.abs(rho_bf_np[li, tgt].astype(np.float64) - orho)[ok])

        def stats(parts):
            d = np.concatenate(parts) if parts else np.zeros(0)
            if d.size == 0:
                return None
            return {"max": float(d.max()), "p99": float(np.quantile(d, 0.99)),
                    "median": float(np.median(d)), "n": int(d.size)}

        pe["knn_bit_exact"] = exact
        pe["abs_drho_fp32_vs_fp64_oracle"] = stats(d32)
        pe["abs_drho_bf16_vs_fp64_oracle"] = stats(d16)
        pe["max_abs_drho"] = pe["abs_drho_fp32_vs_fp64_oracle"]["max"] if d32 else None
        res["parity_sample"] = pe
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
