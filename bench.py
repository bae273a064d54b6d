#!/usr/bin/env python3
"""Fragment CCSD(T) throughput on one MI355X.

One step = one complete fragment solve through the C ABI
(lnocc_fragment_ccsd: DF split, MP2 guess, CCSD iterations to the residual
threshold, then (T)) on the realistic synthetic fragment (nocc=16, nvir=160,
naux=528, seed 1), in the mixed mode (ladder and (T) products in FP32 on the
matrix cores, everything else FP64) and, for comparison, in plain FP64.
Inputs are resident in HBM before the timed region.

The timed steps run the library's default path (the residual evaluation of
each iteration replayed from a captured HIP graph, no per-launch events).  One
further solve, outside the timed region, runs with per-launch HIP events on
the solve's stream; it gives the per-class kernel times and the roofline
position of the dominant contraction kernel.

Three further legs are added to the same JSON line (each can be switched off):
  ladder_on_the_fly  the same fragment with the particle-particle ladder formed
                 on the fly from the dressed B~_vv in every iteration (the path of
                 fragments whose stored ladder does not fit in memory);
  large_triples  (T) at the large fragment's full size (nocc=32, nvir=400,
                 naux=1300, seed 4) on the MP1 amplitudes, mixed and FP64, with
                 the algorithmic rate 2 o^3 v^4 + 2 o^4 v^3 over the wall time;
  batch          the 64 uneven fragments of the batched workload through
                 lnocc_batch_solve in the mixed mode against the same fragments
                 solved one at a time in FP64, with parity against the stored
                 oracle values of a subset.

--workload batch times the batched workload alone (one step = the whole batch).

Prints one JSON line with solves/s, the (T) contraction rate, the roofline
position of the dominant contraction kernel and the FP64 CPU oracle timed on a
bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import pathlib
import sys
import time

import numpy as np

ROOT = pathlib.Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

METRIC = "fragment CCSD(T) solves/s + (T) TFLOP/s, mixed vs FP64, at |ΔE|≤1e-6 Eh"
PEAKS_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}
DTYPES = {"fp64": "f64", "fp32": "f32+f64", "bf16": "bf16+f64"}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_sources_hash() -> str:
    h = hashlib.sha256()
    for p in sorted((ROOT / "paper_2407_11258_amd" / "csrc").glob("*")):
        h.update(p.read_bytes())
    return h.hexdigest()[:16]


def cpu_baseline(frag, n_iter: int, budget_triples: int = 4) -> dict:
    """The oracle as it stands, on a bounded sample of the same fragment:
    one CCSD residual evaluation and a few unique (T) triples, scaled to one
    solve (n_iter residual evaluations plus every unique triple)."""
    from oracle import ccsd as occ, triples as otr
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        cores = max([i.get("num_threads", 1) for i in info if i.get("user_api") == "blas"] or [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    o, v = frag.nocc, frag.nvir
    t2, _ = occ.mp2(frag.B, frag.eps_occ, frag.eps_vir)
    t1 = np.zeros((o, v))
    t0 = time.perf_counter()
    occ.residuals(frag.B, frag.eps_occ, frag.eps_vir, t1, t2)
    t_res = time.perf_counter() - t0
    ints = otr.TriplesIntegrals(frag.B, o)
    triples = [(i, j, k) for i in range(o) for j in range(i, o) for k in range(j, o)
               if not (i == j == k)]
    t0 = time.perf_counter()
    for (i, j, k) in triples[:budget_triples]:
        otr.w_v(ints, t1, t2, i, j, k)
    t_trip = (time.perf_counter() - t0) / max(1, min(budget_triples, len(triples)))
    est = n_iter * t_res + len(triples) * t_trip
    return {"value": 1.0 / est, "unit": "solves/s", "cores": int(cores), "kind": "oracle",
            "sample": (f"1 CCSD residual ({t_res:.2f} s) x {n_iter} iterations + "
                       f"{min(budget_triples, len(triples))} of {len(triples)} unique (T) triples "
                       f"({t_trip:.2f} s each); estimated {est:.1f} s per solve")}


def parse_args():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="single_realistic")
    ap.add_argument("--precision", default="fp32", choices=sorted(PEAKS_TFLOPS))
    ap.add_argument("--compare-fp64", type=int, default=1,
                    help="also time the plain FP64 path (single: same steps; batch: 64 "
                         "sequential solves)")
    ap.add_argument("--autotune", type=int, default=1,
                    help="tune tile shapes and split counts during the warmup (plans kept for "
                         "the timed steps)")
    ap.add_argument("--batch-slots", type=int, default=4)
    ap.add_argument("--batch-streams", type=int, default=4)
    ap.add_argument("--batch-autotune", type=int, default=0,
                    help="batched workload: before timing, tune contraction plans on the first "
                         "iteration of every fragment (in each timed precision), one fragment "
                         "at a time")
    ap.add_argument("--conv-tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--level-shift", type=float, default=0.0)
    ap.add_argument("--diis-start", type=int, default=1)
    ap.add_argument("--diis-space", type=int, default=16)
    ap.add_argument("--max-iter", type=int, default=100)
    ap.add_argument("--triples-reps", type=int, default=2,
                    help="timed repetitions of (T) alone on the converged amplitudes")
    ap.add_argument("--large-triples", type=int, default=1,
                    help="add the large-fragment (T) leg (mixed and FP64, about 90 s)")
    ap.add_argument("--otf-leg", type=int, default=2, metavar="STEPS",
                    help="add the on-the-fly ladder leg (the single fragment solved with the "
                         "ladder formed from B~_vv every iteration) with this many timed steps; "
                         "0 = off")
    ap.add_argument("--ladder", default="auto", choices=["auto", "on_the_fly"],
                    help="ladder path of the single-fragment solves (auto: stored when it "
                         "fits; on_the_fly: formed from B~_vv every iteration)")
    ap.add_argument("--batch-leg", type=int, default=1,
                    help="add the batched-workload leg (mixed batch vs sequential FP64)")
    ap.add_argument("--plans", default="",
                    help="load contraction plans from this file before timing (if it exists)")
    ap.add_argument("--save-plans", default="",
                    help="save the contraction plans in use after the timed run to this file")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device (a plain copy of known size "
                         "that scales hardware byte counters)")
    return ap.parse_args()


def roofline(prof: dict, precision: str, workload: str) -> dict:
    """Position of the kernel class with the largest device time."""
    dominant = max(prof, key=lambda k: prof[k]["ms"])
    d = prof[dominant]
    achieved = d["flops"] / d["ms"] / 1e9 if d["ms"] > 0 else 0.0
    # ladder and (T) products run in the chosen precision; every other contraction in FP64;
    # split-bf16 products (their own class) against the bf16 matrix-core peak over the
    # six bf16 products that make one FP32-class product
    kprec = precision if dominant in ("ladder_build", "ladder_contract", "triples_w") else "fp64"
    if dominant == "mlp":
        kprec = "fp32"
    if dominant == "split":
        kprec = "split_bf16x6"
    peak = PEAKS_TFLOPS["bf16"] / 6.0 if kprec == "split_bf16x6" else PEAKS_TFLOPS[kprec]
    traffic = None
    tpath = ROOT / "profiles" / "traffic.json"
    if tpath.exists():
        ent = json.loads(tpath.read_text()).get(f"{workload}:{kprec}:{dominant}")
        if ent and ent.get("sources") == kernel_sources_hash():
            traffic = ent.get("bytes_per_launch")
    return {"bound": "mfma", "kernel": dominant, "precision": kprec, "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
            "flops_per_launch": d["flops"] / max(1, d["launches"]),
            "avg_launch_ms": d["ms"] / max(1, d["launches"])}


def kernel_table(prof: dict) -> dict:
    return {k: {"launches": p["launches"], "ms_total": p["ms"],
                "tflops": (p["flops"] / p["ms"] / 1e9) if p["ms"] > 0 else None}
            for k, p in prof.items()}


def run_single(args, L, torch) -> dict:
    from synth import CONFIG_SHAPES, make_fragment
    o, v, X, seed = CONFIG_SHAPES[args.workload]
    log(f"workload {args.workload}: nocc={o} nvir={v} naux={X} seed={seed}")
    frag = make_fragment(o, v, X, seed)
    dev = torch.device("cuda:0")
    B = torch.tensor(frag.B, device=dev)
    eo = torch.tensor(frag.eps_occ, device=dev)
    ev = torch.tensor(frag.eps_vir, device=dev)
    t1 = torch.empty((o, v), dtype=torch.float64, device=dev)
    t2 = torch.empty((o, o, v, v), dtype=torch.float64, device=dev)
    ws = L.Workspace(dev)

    def timed(precision: str, steps: int, warmup: int, ladder: str = "auto"):
        opt = L.make_options(precision=precision, level_shift=args.level_shift,
                             diis_start=args.diis_start, diis_space=args.diis_space,
                             max_iter=args.max_iter, ladder=ladder,
                             autotune=bool(args.autotune))
        fs = L.make_fragment_struct(B, eo, ev, t1, t2, args.conv_tol)
        ws.attach([fs], opt)

        def step():
            st = L.lnocc_fragment_ccsd(fs, opt)
            if st < 0:
                raise RuntimeError(f"{L.lnocc_status_string(st)}: {L.lnocc_last_error()}")

        for w in range(warmup):
            step()
            log(f"{precision} warmup {w + 1}/{warmup}: {fs.n_iter} iterations, "
                f"E_CCSD={fs.e_ccsd:.10f}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            step()
            log(f"{precision} step {k + 1}/{steps} done")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        # per-class launch times: one more solve with HIP events around every
        # contraction (this switches the graph replay off), outside the timed steps
        L.lnocc_profile_enable(True)
        step()
        torch.cuda.synchronize()
        L.lnocc_profile_enable(False)
        prof = L.lnocc_profile_collect()
        log(f"{precision} profiled solve done")
        return fs, opt, elapsed, prof

    if args.plans and pathlib.Path(args.plans).exists():
        log(f"loaded {L.lnocc_autotune_load(args.plans)} contraction plans")
    fs, opt, elapsed, prof = timed(args.precision, args.steps, args.warmup, ladder=args.ladder)
    # traffic entries are kept per ladder path (different kernels)
    wkey = args.workload + ("_otf" if args.ladder == "on_the_fly" else "")
    res = {"value": args.steps / elapsed, "ms_per_step": 1e3 * elapsed / args.steps,
           "config": {"workload": args.workload, "nocc": o, "nvir": v, "naux": X, "seed": seed,
                      "precision": args.precision, "ladder": args.ladder,
                      "conv_tol": args.conv_tol,
                      "level_shift": args.level_shift, "diis_start": args.diis_start,
                      "diis_space": args.diis_space,
                      "autotune": bool(args.autotune), "ccsd_iterations": fs.n_iter,
                      "status": fs.status},
           "e_ccsd": fs.e_ccsd}
    # (T) alone on the converged amplitudes (the solves above already warmed it up)
    ft = L.make_fragment_struct(B, eo, ev, t1, t2, args.conv_tol)
    nrep = max(1, args.triples_reps)
    t0 = time.perf_counter()
    for _ in range(nrep):
        L.lnocc_fragment_triples(ft, opt)
    torch.cuda.synchronize()
    t_triples = (time.perf_counter() - t0) / nrep
    f_t = 2.0 * o ** 3 * v ** 4 + 2.0 * o ** 4 * v ** 3
    log(f"(T): {t_triples * 1e3:.1f} ms, E_(T)={ft.e_t:.12f}")
    res.update(triples_tflops=f_t / t_triples / 1e12, triples_ms=t_triples * 1e3, e_t=ft.e_t,
               kernels=kernel_table(prof), roofline=roofline(prof, args.precision, wkey))
    gpath = ROOT / "tests" / "golden" / f"{args.workload}.json"
    golden = json.loads(gpath.read_text()) if gpath.exists() else None
    if golden and golden.get("input_sha256") != frag.sha256():
        golden = None
    if golden:
        res["parity_vs_oracle"] = {"d_e_ccsd": fs.e_ccsd - golden["e_ccsd"],
                                   "d_e_t": ft.e_t - golden["e_t"]}
    if args.compare_fp64 and args.precision != "fp64":
        f64, opt64, el64, prof64 = timed("fp64", args.steps, args.warmup, ladder=args.ladder)
    if args.save_plans:
        log(f"saved {L.lnocc_autotune_save(args.save_plans)} contraction plans")
    if args.compare_fp64 and args.precision != "fp64":
        ft64 = L.make_fragment_struct(B, eo, ev, t1, t2, args.conv_tol)
        st = L.lnocc_fragment_triples(ft64, opt64)
        torch.cuda.synchronize()
        if st < 0:
            raise RuntimeError(f"{L.lnocc_status_string(st)}: {L.lnocc_last_error()}")
        cmp = {"value": args.steps / el64, "unit": "solves/s", "ms_per_step": 1e3 * el64 / args.steps,
               "ccsd_iterations": f64.n_iter, "e_ccsd": f64.e_ccsd, "e_t": ft64.e_t,
               "roofline": roofline(prof64, "fp64", wkey)}
        if golden:
            cmp["parity_vs_oracle"] = {"d_e_ccsd": f64.e_ccsd - golden["e_ccsd"],
                                       "d_e_t": ft64.e_t - golden["e_t"]}
        res["fp64"] = cmp
        res["speedup_vs_fp64"] = res["value"] / cmp["value"]
    if args.otf_leg:
        # the same solve with the particle-particle ladder formed on the fly from
        # B~_vv every iteration (the path of fragments whose stored ladder does not fit)
        fo, _, elo, profo = timed(args.precision, args.otf_leg, 1, ladder="on_the_fly")
        leg = {"value": args.otf_leg / elo, "unit": "solves/s", "ladder": "on_the_fly",
               "ms_per_step": 1e3 * elo / args.otf_leg, "precision": args.precision,
               "ccsd_iterations": fo.n_iter, "e_ccsd": fo.e_ccsd, "e_t": fo.e_t,
               "kernels": kernel_table(profo),
               "roofline": roofline(profo, args.precision, args.workload + "_otf")}
        if golden:
            leg["parity_vs_oracle"] = {"d_e_ccsd": fo.e_ccsd - golden["e_ccsd"],
                                       "d_e_t": fo.e_t - golden["e_t"]}
        res["ladder_on_the_fly"] = leg
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample)")
        res["cpu_baseline"] = cpu_baseline(frag, fs.n_iter)
    del ws
    torch.cuda.empty_cache()
    if args.large_triples:
        res["large_triples"] = run_large_triples(args, L, torch)
        torch.cuda.empty_cache()
    if args.batch_leg:
        res["batch"] = run_batch(args, L, torch, leg=True)
        torch.cuda.empty_cache()
    return res


def run_large_triples(args, L, torch) -> dict:
    """(T) at the large fragment's full size on its MP1 amplitudes (T1 = 0), mixed
    and FP64.  CCSD itself does not converge on this synthetic input, so the
    amplitudes are the starting ones; the cost of (T) does not depend on them."""
    from synth import CONFIG_SHAPES, make_fragment
    o, v, X, seed = CONFIG_SHAPES["large"]
    log(f"large (T) leg: nocc={o} nvir={v} naux={X} seed={seed}")
    frag = make_fragment(o, v, X, seed)
    dev = torch.device("cuda:0")
    B = torch.tensor(frag.B, device=dev)
    eo = torch.tensor(frag.eps_occ, device=dev)
    ev = torch.tensor(frag.eps_vir, device=dev)
    t1 = torch.empty((o, v), dtype=torch.float64, device=dev)
    t2 = torch.empty((o, o, v, v), dtype=torch.float64, device=dev)
    ws = L.Workspace(dev)
    opt0 = L.make_options(precision="fp64", do_triples=False, max_iter=0)
    f0 = L.make_fragment_struct(B, eo, ev, t1, t2, args.conv_tol)
    ws.attach([f0], opt0)
    st = L.lnocc_fragment_ccsd(f0, opt0)   # MP1 amplitudes and E_MP2
    if st < 0:
        raise RuntimeError(f"{L.lnocc_status_string(st)}: {L.lnocc_last_error()}")
    del ws
    torch.cuda.empty_cache()
    f_t = 2.0 * o ** 3 * v ** 4 + 2.0 * o ** 4 * v ** 3
    out = {"workload": "large", "nocc": o, "nvir": v, "naux": X, "seed": seed,
           "amplitudes": "MP1 (T1 = 0)", "e_mp2": f0.e_mp2, "flops": f_t}
    for prec in ("fp32", "fp64"):
        ws = L.Workspace(dev)
        opt = L.make_options(precision=prec, autotune=bool(args.autotune))
        ft = L.make_fragment_struct(B, eo, ev, t1, t2, args.conv_tol)
        ws.attach([ft], opt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = L.lnocc_fragment_triples(ft, opt)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        if st < 0:
            raise RuntimeError(f"{L.lnocc_status_string(st)}: {L.lnocc_last_error()}")
        rate = f_t / el / 1e12
        out[prec] = {"seconds": el, "tflops": rate, "peak": PEAKS_TFLOPS[prec],
                     "frac": rate / PEAKS_TFLOPS[prec], "e_t": ft.e_t}
        log(f"large (T) {prec}: {el:.1f} s, {rate:.1f} TFLOP/s, E_(T)={ft.e_t:.12f}")
        del ws
        torch.cuda.empty_cache()
    out["d_e_t_mixed_vs_fp64"] = out["fp32"]["e_t"] - out["fp64"]["e_t"]
    return out


def run_batch(args, L, torch, leg: bool = False) -> dict:
    """The 64-fragment batched workload: mixed-precision lnocc_batch_solve against
    the same fragments solved one at a time in FP64.  With --batch-autotune, an
    untimed pass first tunes the contraction plans of every fragment (one CCSD
    iteration each, alone on the device, in the batch's precision and in FP64); the
    timed runs then use those plans without tuning."""
    from synth import batch_shapes, make_fragment
    shapes = batch_shapes()
    log(f"batch workload: {len(shapes)} fragments")
    precision = "fp32" if leg else args.precision
    steps = 1 if leg else args.steps
    warmup = 1 if leg else args.warmup
    dev = []
    for s in shapes:
        f = make_fragment(*s)
        dev.append(tuple(torch.tensor(x, dtype=torch.float64, device="cuda:0")
                         for x in (f.B, f.eps_occ, f.eps_vir)))
    torch.cuda.synchronize()
    ws = L.Workspace("cuda:0")
    kw = dict(conv_tol=args.conv_tol, level_shift=args.level_shift, diis_start=args.diis_start,
              diis_space=args.diis_space, max_iter=args.max_iter, workspace=ws)
    tune_s = None
    if args.batch_autotune:
        t0 = time.perf_counter()
        tk = dict(kw, max_iter=1)
        precs = [precision] + (["fp64"] if args.compare_fp64 and precision != "fp64" else [])
        for i, d in enumerate(dev):
            for pr in precs:
                L.solve(*d, precision=pr, autotune=True, **tk)
            if i % 16 == 15:
                log(f"plans tuned for {i + 1}/{len(dev)} fragments")
        torch.cuda.synchronize()
        tune_s = time.perf_counter() - t0
    for w in range(warmup):   # a few fragments: library and kernels loaded
        L.solve_batch(dev[:4], precision=precision, batch_slots=args.batch_slots,
                      batch_streams=args.batch_streams, **kw)
        log(f"warmup {w + 1}/{warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        res = L.solve_batch(dev, precision=precision, batch_slots=args.batch_slots,
                            batch_streams=args.batch_streams, **kw)
        log(f"batch step {k + 1}/{steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    n = len(shapes)
    out = {"value": n * steps / elapsed, "ms_per_step": 1e3 * elapsed / steps,
           "config": {"workload": "batch", "fragments": n, "precision": precision,
                      "conv_tol": args.conv_tol, "batch_slots": args.batch_slots,
                      "batch_streams": args.batch_streams,
                      "plans": (f"tuned before timing ({tune_s:.1f} s, first iteration of every "
                                f"fragment)" if tune_s is not None else "heuristic (not tuned)"),
                      "ccsd_iterations": sum(r.n_iter for r in res),
                      "statuses": {str(st): sum(r.status == st for r in res)
                                   for st in sorted({r.status for r in res})}}}
    if leg:
        out["unit"] = "fragments/s"
        out["seconds"] = elapsed
    gpath = ROOT / "tests" / "golden" / "batch_ccsd.json"
    if gpath.exists():
        gold = json.loads(gpath.read_text())
        dcc, dt = [], []
        for g in gold["fragments"]:
            k = g["index"]
            if shapes[k][3] == g["seed"]:
                dcc.append(abs(res[k].e_ccsd - g["e_ccsd"]))
                dt.append(abs(res[k].e_t - g["e_t"]))
        if dcc:
            out["parity_vs_oracle"] = {"fragments": len(dcc), "max_abs_d_e_ccsd": max(dcc),
                                       "max_abs_d_e_t": max(dt)}
    if args.compare_fp64:
        t0 = time.perf_counter()
        seq = []
        for i, d in enumerate(dev):
            seq.append(L.solve(*d, precision="fp64", **kw))
            if i % 16 == 15:
                log(f"sequential fp64: {i + 1}/{n}")
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        de = [abs(a.e_ccsd - b.e_ccsd) for a, b in zip(res, seq)]
        dt = [abs(a.e_t - b.e_t) for a, b in zip(res, seq)]
        out["fp64_sequential"] = {"value": n / el, "unit": "solves/s", "seconds": el,
                                  "max_abs_d_e_ccsd": max(de), "max_abs_d_e_t": max(dt)}
        out["speedup_vs_fp64_sequential"] = out["value"] / out["fp64_sequential"]["value"]
    if not leg:
        # per-class launch times from one more (untimed) batch with HIP events
        L.lnocc_profile_enable(True)
        L.solve_batch(dev, precision=precision, batch_slots=args.batch_slots,
                      batch_streams=args.batch_streams, **kw)
        torch.cuda.synchronize()
        L.lnocc_profile_enable(False)
        prof = L.lnocc_profile_collect()
        out["kernels"] = kernel_table(prof)
        out["roofline"] = roofline(prof, precision, "batch")
    return out


def main() -> int:
    args = parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(fragments would be sharded across GPUs with no exchange but the final "
              "energies); run with --gpus 1.", file=sys.stderr)
        return 2

    import torch
    from paper_2407_11258_amd import lnocc as L

    if args.copy_calibration > 0:
        n = args.copy_calibration << 20
        src = torch.empty(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.copy_calibration} MiB done")
        del src, dst

    torch.cuda.set_device(0)
    res = run_batch(args, L, torch) if args.workload == "batch" else run_single(args, L, torch)
    result = {
        "metric": METRIC,
        "value": res.pop("value"),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[args.precision],
        "data": "synthetic",
        "config": res.pop("config"),
    }
    result.update(res)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
