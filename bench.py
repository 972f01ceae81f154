#!/usr/bin/env python3
"""RI-PNOF7 J/K + gradient builds per second on one MI355X.

One step = one build: the half- and full-MO transforms, the MO J/K matrices,
the per-MO AO J^q/K^q matrices, the PNOF7 energy, the Lagrangian and the
orbital gradient, on inputs already resident in HBM.  The default workload is
the cyclohexane-like synthetic molecule (n_bf=348, n_aux=1044, 24 pairs,
Ncwo=4, n_mo=348) with 30 fixed small orbital rotations: step i rebuilds
everything for the i-th rotated C (cycling).

Prints ONE JSON line with builds/s, TFLOP/s, the roofline of the dominant
kernel (HIP events over the timed region) and the FP64 CPU oracle timed on a
bounded sample on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RI-PNOF7 J/K+gradient builds/s & TFLOP/s; split-prec vs FP64 at 1 µEh"
PEAK = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0, "f16": 2500.0}   # dense MFMA TFLOP/s
MODES = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3, "fp16x3": 4}
PRODUCTS = {"fp64": 1, "fp32": 1, "bf16x3": 3, "bf16x6": 6, "fp16x3": 3}   # MFMA products per multiply-add
MODE_PEAK = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16", "bf16x6": "bf16", "fp16x3": "f16"}
HBM_GBS = 8000.0

# HBM bytes per launch of the dominant kernel, from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each divided by what the same
# counter reads per byte of a 1 GiB device-to-device copy (FETCH_SIZE 0.5,
# WRITE_SIZE 1.0).  "src" is the sha256 of the GEMM kernel sources the counters
# were taken on: a figure is reported only while those sources are unchanged.
# The runs and their command lines are in profiles/.
TRAFFIC = {
    ("half_transform", "c6h12", "fp64"): {"src": "4eaded17099386bb", "fetch": 1173737881, "write": 348779520,
                                         "profile": "profiles/fp64_c6h12_counters.md"},
}


def kernel_src_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("mfma_engine.hpp", "kernels.hip"):
        with open(os.path.join(ROOT, "paper_2012_15662_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_of(kernel, workload, prec):
    t = TRAFFIC.get((kernel, workload, prec))
    if t is None or t["src"] != kernel_src_hash():
        return None, None
    return t["fetch"] + t["write"], {"fetch_bytes": t["fetch"], "write_bytes": t["write"], "profile": t["profile"]}


def kernel_flops(nb, na, nw, nmo):
    """Algorithmic flops per launch of each kernel (symmetric outputs counted once);
    the pre-split kernels (b stored pre-split) do the same arithmetic."""
    return {
        "half_transform": 2.0 * na * nb * nb * nw,
        "half_transform_presplit": 2.0 * na * nb * nb * nw,
        "jao_presplit": 1.0 * na * nw * nb * (nb + 1),
        "mo_transform": 2.0 * na * nb * nw * nw,
        "jk_mo_partial": 4.0 * na * nw * nw,
        "jao": 1.0 * na * nw * nb * (nb + 1),
        "kao": 1.0 * na * nw * nb * (nb + 1),
        "hc_gemm": 2.0 * nb * nb * nw,
        "fock": 4.0 * nw * nw * nb * nb,
        "lambda_gemm": 2.0 * nmo * nb * nw,
    }


def kernel_bytes(nb, na, nw):
    """Minimum HBM bytes per FP64 launch (operands read once, outputs written once)."""
    return {
        "half_transform": 8.0 * na * nb * nb + 8.0 * nw * na * nb,
        "mo_transform": 8.0 * nw * na * nb + 8.0 * na * nw * nw,
        "jao": 4.0 * na * nb * (nb + 1) + 8.0 * nw * nb * nb,
        "kao": 8.0 * nw * na * nb + 8.0 * nw * nb * nb,
    }


def build_flops(nb, na, nw, nmo):
    """Algorithmic flops of one build (the pre-split kernels' entries are the
    same work as their split-on-load kernels, so they are not added again)."""
    return sum(v for k, v in kernel_flops(nb, na, nw, nmo).items() if not k.endswith("_presplit"))


def cpu_baseline(inst, Cs, budget_s=20.0):
    """Time the FP64 oracle (as it stands) on this host's cores."""
    import numpy as np
    from oracle import pnof7_ri as ri
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    n, t0 = 0, time.perf_counter()
    while True:
        ri.build_instance(inst, C=Cs[n % len(Cs)])
        n += 1
        el = time.perf_counter() - t0
        if el > budget_s or n >= 200:
            break
    return {"value": n / el, "unit": "builds/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{n} full FP64 builds of the same workload (numpy oracle, rotated C), {el:.1f} s"}


def time_builds(ctx, b, Cd, H, occ, pm, inst, prec, steps, warmup, profile=False, direct=False, b_split=None):
    """Warm up (autotunes tiles on first use), then time `steps` builds
    (rif_build, or rif_build_direct with direct=True; b_split: b stored
    pre-split for this precision).  profile: False, True (event pairs around
    every launch) or one kernel's report name (pairs around that one only)."""
    import torch
    build = ctx.build_direct if direct else ctx.build
    out = None
    for i in range(max(warmup, 1)):
        out = build(b, Cd[i % len(Cd)], H, occ, pm, inst.n_pairs, inst.n_cwo, prec=prec, out=out, b_split=b_split)
    ctx.sync()
    if profile:
        # True: every launch; a name: only that kernel's launches (two event
        # records per launch of it, so the timed loop keeps its pace)
        ctx.profile(True, only=None if profile is True else profile)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        out = build(b, Cd[i % len(Cd)], H, occ, pm, inst.n_pairs, inst.n_cwo, prec=prec, out=out, b_split=b_split)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ctx.sync()
    prof = None
    if profile:
        prof = ctx.profile_report()
        ctx.profile(False)
    return el, out, prof


def oracle_errors(out, ref):
    """Energy (absolute, Eh) and gradient (normwise max|dG| / max|G|) errors of
    one build against the FP64 oracle's, and whether the reduced-precision
    target (1 uEh, 1e-6) holds."""
    e = float(out["energy"].cpu()[0])
    g = out["grad"].cpu().numpy()
    dE = e - ref["energy"]
    gerr = float(abs(g - ref["grad"]).max() / abs(ref["grad"]).max())
    return {"dE_vs_oracle": dE, "dE_rel_vs_oracle": abs(dE) / abs(ref["energy"]), "grad_err_vs_oracle": gerr,
            "within_1uEh_1e-6": bool(abs(dE) <= 1e-6 and gerr <= 1e-6)}


def fastest_within_target(modes, base_rate):
    """The fastest reduced-precision mode whose energy is within 1 uEh and
    gradient within 1e-6 (normwise) of the oracle's (b pre-split where faster)."""
    best = None
    for name, m in modes.items():
        if name == "fp64" or not m["within_1uEh_1e-6"]:
            continue
        for pre, rate in ((False, m["builds_s"]), (True, (m.get("presplit_b") or {}).get("builds_s"))):
            if rate and (best is None or rate > best["builds_s"]):
                best = {"mode": name, "b_presplit": pre, "builds_s": rate,
                        "speedup_vs_fp64": round(rate / base_rate, 3), "dE_vs_oracle": m["dE_vs_oracle"],
                        "grad_err_vs_oracle": m["grad_err_vs_oracle"]}
    return best


def precision_study(ctx, workload, steps):
    """Every mode at one more workload (the cyclodecane-like molecule): builds/s
    (b split on load and pre-split), error against the FP64 oracle, and the
    FP64 half transform's roofline (HIP events over its timed builds)."""
    import numpy as np
    import torch

    import synth
    from oracle import pnof7_ri as ri

    inst = synth.workload(workload)
    nb, na, nw, nmo = inst.n_bf, inst.n_aux, inst.n_omega, inst.n_mo
    t0 = time.perf_counter()
    ref = ri.build_instance(inst)
    t_oracle = time.perf_counter() - t0
    dev = "cuda:0"
    b = torch.from_numpy(inst.b).to(dev)
    Cd = [torch.from_numpy(inst.C).to(dev)]
    H, occ = torch.from_numpy(inst.H).to(dev), torch.from_numpy(inst.occ).to(dev)
    pm = torch.from_numpy(inst.pair_of.astype(np.int32)).to(dev)
    inst.b = None
    flops = build_flops(nb, na, nw, nmo)
    kf = kernel_flops(nb, na, nw, nmo)
    modes, base = {}, None
    roof = None
    for name, pv in MODES.items():
        prof = "half_transform" if name == "fp64" else False
        el, out, pr = time_builds(ctx, b, Cd, H, occ, pm, inst, pv, steps, 2, profile=prof)
        rate = steps / el
        if name == "fp64":
            base = rate
            n, ms = pr["half_transform"]
            ach = kf["half_transform"] / (ms / n * 1e-3) / 1e12
            roof = {"kernel": "half_transform", "bound": "mfma", "achieved": round(ach, 3), "peak": PEAK["f64"],
                    "unit": "TFLOP/s", "frac": round(ach / PEAK["f64"], 4)}
        o = ctx.build(b, Cd[0], H, occ, pm, inst.n_pairs, inst.n_cwo, prec=pv)
        ctx.sync()
        modes[name] = {"builds_s": round(rate, 2), "speedup": round(rate / base, 3),
                       "tflops": round(flops * rate / 1e12, 2), **oracle_errors(o, ref)}
        if name != "fp64":
            bs = ctx.presplit_b(b, pv)
            el4, _, _ = time_builds(ctx, b, Cd, H, occ, pm, inst, pv, steps, 2, b_split=bs)
            modes[name]["presplit_b"] = {"builds_s": round(steps / el4, 2), "speedup": round(steps / el4 / base, 3)}
            del bs
    del b
    torch.cuda.empty_cache()
    return {"config": f"{workload}: n_bf={nb} n_aux={na} pairs={inst.n_pairs} ncwo={inst.n_cwo} n_omega={nw} "
                      f"n_mo={nmo}, unrotated C", "steps": steps, "oracle_build_s": round(t_oracle, 2),
            "roofline_fp64": roof, "modes": modes, "fastest_within_1uEh": fastest_within_target(modes, base)}


def four_centre_study(ctx, sizes=(128, 192, 232, 288, 348), reps=4):
    """RI against the conventional four-centre path (Table 1) on the same
    integrals, FP64, one J/K build each: J, K, J^q and K^q for one C.
    RI = rif_transform + rif_jk_mo + rif_jk_ao_per_mo; four-centre =
    rif_jk_4c on integrals stored once (rif_eri4_from_b, timed apart as step
    0).  Shapes follow the cyclohexane-like molecule: n_aux = 3 n_bf, Ncwo 4,
    pairs = round(24 n_bf / 348).  Fits t ~ n_bf^k for both paths."""
    import numpy as np
    import torch

    import synth

    rows = []
    for nb in sizes:
        npair = max(1, int(round(24 * nb / 348)))
        inst = synth.make_instance(nb, 3 * nb, npair, 4, 500 + nb)
        w = inst.n_omega
        b = torch.from_numpy(inst.b).cuda()
        C = torch.from_numpy(inst.C).cuda()
        inst.b = None

        def ri_once(o):
            o["b_half"], o["b_mo"], o["d"] = ctx.transform(b, C, w, 0, o.get("b_half"), o.get("b_mo"), o.get("d"))
            o["J"], o["K"] = ctx.jk_mo(o["b_mo"], o["d"], 0, o.get("J"), o.get("K"))
            o["Jn"], o["Kn"] = ctx.jk_ao_per_mo(b, o["b_half"], o["d"], 0, o.get("Jn"), o.get("Kn"))
            return o

        def timed(f, n):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(n):
                f()
            e1.record()
            e1.synchronize()
            return e0.elapsed_time(e1) / n

        ro = {}
        for _ in range(2):
            ri_once(ro)
        t_ri = timed(lambda: ri_once(ro), 3 * reps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        eri = ctx.eri4_from_b(b)
        torch.cuda.synchronize()
        t_eri = (time.perf_counter() - t0) * 1e3
        fo = ctx.jk_4c(eri, C, w)
        t_4c = timed(lambda: ctx.jk_4c(eri, C, w, out=fo), reps)
        ctx.sync()
        diff = max(float((fo[k] - ro[k]).abs().max() / ro[k].abs().max()) for k in ("J", "K", "Jn", "Kn"))
        rows.append({"n_bf": nb, "n_aux": 3 * nb, "n_omega": w, "ri_ms": round(t_ri, 4), "fourc_ms": round(t_4c, 3),
                     "speedup": round(t_4c / t_ri, 2), "eri_step0_ms": round(t_eri, 1),
                     "eri_gb": round(eri.numel() * 8 / 1e9, 2), "max_rel_diff_ri_vs_4c": diff})
        print(f"four-centre n_bf={nb}: RI {t_ri:.3f} ms, 4c {t_4c:.2f} ms ({t_4c / t_ri:.1f}x)", file=sys.stderr,
              flush=True)
        del eri, fo, ro, b, C
        torch.cuda.empty_cache()
    def fit(rs):
        x = np.log([r["n_bf"] for r in rs])
        return {k: round(float(np.polyfit(x, np.log([r[k] for r in rs]), 1)[0]), 2) for k in ("ri_ms", "fourc_ms")}
    big = fit([r for r in rows if r["n_bf"] >= 192])
    every = fit(rows)
    return {"config": "J, K, J^q, K^q for one C (FP64); n_aux = 3 n_bf, Ncwo 4, pairs = round(24 n_bf/348)",
            "sizes": rows, "exponent_ri": big["ri_ms"], "exponent_fourc": big["fourc_ms"],
            "exponent_all_sizes": every,
            "exponent_note": "t ~ n_bf^k by least squares over n_bf >= 192 (below that the RI build is "
                             "launch-latency bound); formal: RI n_bf^2 n_aux n_Omega, four-centre n_bf^4 n_Omega "
                             "(n_aux, n_Omega proportional to n_bf here: 4 and 5)",
            "paper_context": "paper (24 Xeon threads, DoNOF): PNOF7-RI vs PNOF7 12x per outer iteration "
                             "(cyclopropane), 83x occupancy and 37x orbital optimisation (cyclononane)"}


def bench_fourc(args):
    """RI against the conventional four-centre path alone (the sweep of the
    default line's four_centre record), e.g. for a kernel trace."""
    import paper_2012_15662_amd as rif
    ctx = rif.Context(0)
    ctx.autotune(not args.no_tune)
    rec = four_centre_study(ctx)
    big = rec["sizes"][-1]
    line = {"metric": "RI vs four-centre J/K build time ratio (Table 1 path, same integrals)",
            "value": big["speedup"], "unit": "x (four-centre time / RI time) at the largest size", "n_gpus": 1,
            "higher_is_better": True, "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "fourc: " + rec["config"]}, **rec}
    ctx.close()
    print(json.dumps(line))


def bench_batch(args):
    """64 uneven molecules (n_bf ~ U{60..400}, n_aux = 3 n_bf, pairs = n_bf//12,
    Ncwo = 2): one grouped launch per step, captured in a hipGraph and replayed.
    Reports aggregate builds/s and the same molecules built one after another."""
    import numpy as np
    import torch

    import paper_2012_15662_amd as rif
    import synth

    prec = MODES[args.prec]
    ctx = rif.Context(0)
    ctx.autotune(not args.no_tune)
    # the molecules tests/test_gpu_batch64.py compares with the oracle
    items, flops = [], 0.0
    for inp, npair, ncwo in synth.make_batch_device(64):
        nb = inp["b"].shape[1]
        items.append((inp, npair, ncwo, None))
        flops += build_flops(nb, 3 * nb, npair * (1 + ncwo), nb)
    batch = ctx.batch(items, prec=prec)
    for _ in range(max(args.warmup, 1)):
        batch.run(use_graph=True)
    ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch.run(use_graph=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ctx.sync()
    # the same molecules one build call after another (no batching, no graph)
    for inp, npair, ncwo, out in zip([i[0] for i in items], [i[1] for i in items], [i[2] for i in items],
                                     batch.outs):
        ctx.build_instance(inp, npair, ncwo, out=out, prec=prec)
    ctx.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for inp, npair, ncwo, out in zip([i[0] for i in items], [i[1] for i in items], [i[2] for i in items],
                                     batch.outs):
        ctx.build_instance(inp, npair, ncwo, out=out, prec=prec)
    torch.cuda.synchronize()
    el_seq = time.perf_counter() - t1
    ctx.sync()
    per = el / args.steps
    presplit = None
    if prec != MODES["fp64"]:
        # the same batch with every b stored once in this mode's pieces
        # (rif_presplit_b; bitwise the same results)
        items2 = []
        for inp, npair, ncwo, _ in items:
            inp2 = dict(inp)
            inp2["b_split"] = ctx.presplit_b(inp["b"], prec)
            items2.append((inp2, npair, ncwo, None))
        batch2 = ctx.batch(items2, prec=prec)
        for _ in range(max(args.warmup, 1)):
            batch2.run(use_graph=True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for _ in range(args.steps):
            batch2.run(use_graph=True)
        torch.cuda.synchronize()
        per2 = (time.perf_counter() - t2) / args.steps
        batch2.close()
        del items2
        presplit = {"builds_s": round(64 / per2, 2), "ms_per_step": round(per2 * 1e3, 3),
                    "vs_split_on_load": round(per / per2, 3)}
    line = {
        "metric": METRIC, "value": round(64 / per, 2), "unit": "builds/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(per * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16", "bf16x6": "bf16", "fp16x3": "f16"}[args.prec],
        "data": "synthetic",
        "config": {"workload": "batch64: 64 molecules, n_bf ~ U{60..400} (seed 3), n_aux = 3 n_bf, "
                               "pairs = n_bf//12, Ncwo = 2, b drawn on the GPU (seeds 3000+i); "
                               "one step = all 64 builds",
                   "precision": args.prec},
        "tflops": round(flops / per / 1e12, 2), "flops_per_step": flops,
        "sequential_builds_s": round(64 / el_seq, 2), "batch_speedup": round(el_seq / per, 3),
        "presplit_b": presplit,
        "tiles": [t for t in ctx.tune_report().strip().splitlines() if t.startswith("g_")],
    }
    batch.close()
    ctx.close()
    print(json.dumps(line))


def batch_study(ctx, steps=10, warmup=2):
    """The 64-molecule uneven batch (the batch64 workload, the molecules
    tests/test_gpu_batch64.py compares with the oracle) inside the default
    run: FP64 and BF16x6, grouped launches replayed from a hipGraph; FP64
    also one build call after another."""
    import torch

    import synth

    items, flops = [], 0.0
    for inp, npair, ncwo in synth.make_batch_device(64):
        nb = inp["b"].shape[1]
        items.append((inp, npair, ncwo, None))
        flops += build_flops(nb, 3 * nb, npair * (1 + ncwo), nb)
    res = {"config": "64 molecules, n_bf ~ U{60..400} (seed 3), n_aux = 3 n_bf, pairs = n_bf//12, Ncwo = 2; "
                     "one step = all 64 builds"}
    for name in ("fp64", "bf16x6"):
        batch = ctx.batch(items, prec=MODES[name])
        for _ in range(warmup):
            batch.run(use_graph=True)
        ctx.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            batch.run(use_graph=True)
        torch.cuda.synchronize()
        per = (time.perf_counter() - t0) / steps
        ctx.sync()
        ent = {"builds_s": round(64 / per, 2), "ms_per_step": round(per * 1e3, 3),
               "tflops": round(flops / per / 1e12, 2)}
        if name == "fp64":
            outs = batch.outs
            for inp, npair, ncwo, _ in items:   # warm the single-build tiles
                ctx.build_instance(inp, npair, ncwo, out=None, prec=MODES[name])
            ctx.sync()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for (inp, npair, ncwo, _), out in zip(items, outs):
                ctx.build_instance(inp, npair, ncwo, out=out, prec=MODES[name])
            torch.cuda.synchronize()
            el_seq = time.perf_counter() - t1
            ctx.sync()
            ent["sequential_builds_s"] = round(64 / el_seq, 2)
            ent["batch_speedup"] = round(el_seq / per, 3)
        res[name] = ent
        batch.close()
    res["bf16x6"]["speedup_vs_fp64"] = round(res["bf16x6"]["builds_s"] / res["fp64"]["builds_s"], 3)
    del items
    torch.cuda.empty_cache()
    return res


def largest_study(ctx, steps=3):
    """The largest workload (n_bf 1000, n_aux 3000, 60 pairs, Ncwo 6; b is 24 GB
    in FP64, drawn on the GPU) inside the default run: FP64 and BF16x6
    builds/s, and BF16x6's energy and gradient against the FP64 build (which
    tests/test_gpu_largest.py holds to the oracle at 1e-10)."""
    import torch

    import synth

    size, seed = (1000, 3000, 60, 6), 31
    t, npair, ncwo = synth.make_instance_device(*size, seed)
    nb, na = size[0], size[1]
    nw = npair * (1 + ncwo)
    flops = build_flops(nb, na, nw, nb)
    res = {"config": f"n_bf={nb} n_aux={na} pairs={npair} ncwo={ncwo} n_omega={nw} n_mo={nb} (seed {seed})"}
    outs = {}
    for name in ("fp64", "bf16x6"):
        pv = MODES[name]
        out = ctx.build(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], npair, ncwo, prec=pv)   # tiles, warm-up
        ctx.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.build(t["b"], t["C"], t["H"], t["occ"], t["pair_of"], npair, ncwo, prec=pv, out=out)
        ctx.sync()
        torch.cuda.synchronize()
        per = (time.perf_counter() - t0) / steps
        res[name] = {"builds_s": round(1 / per, 3), "ms_per_build": round(per * 1e3, 2),
                     "tflops": round(flops / per / 1e12, 2)}
        outs[name] = (float(out["energy"].cpu()[0]), out["grad"].cpu().numpy())
        del out
    e64, g64 = outs["fp64"]
    e16, g16 = outs["bf16x6"]
    res["bf16x6"]["speedup_vs_fp64"] = round(res["bf16x6"]["builds_s"] / res["fp64"]["builds_s"], 3)
    res["bf16x6"]["dE_vs_fp64"] = e16 - e64
    res["bf16x6"]["grad_err_vs_fp64"] = float(abs(g16 - g64).max() / abs(g64).max())
    del t
    torch.cuda.empty_cache()
    return res


def bench_onwarm(args):
    print(json.dumps(onwarm_study(args)))


def onwarm_study(args):
    """Learned ON warm start at scale: 2000 training molecules (n_bf ~ U{48..200},
    n_aux = 3 n_bf, pairs = n_bf//12, Ncwo ~ U{1..6}) solved by the plain ON
    optimiser from the cold start; the MLP trains on their converged ONs on the
    GPU; 200 held-out molecules and one n_bf=1000 / n_aux=3000 / 60-pair /
    Ncwo=6 molecule are then solved cold and warm."""
    import numpy as np
    import torch

    import paper_2012_15662_amd as rif
    import synth
    from paper_2012_15662_amd import warmstart as ws

    ctx = rif.Context(0)
    rng = np.random.default_rng(10)

    def make(n, seed0):
        out = []
        for i in range(n):
            nb = int(rng.integers(48, 201))
            inp, npair, ncwo = synth.make_instance_device(nb, 3 * nb, nb // 12, int(rng.integers(1, 7)), seed0 + i)
            out.append(ws.jk_problem(ctx, inp, npair, ncwo))
            del inp
        torch.cuda.synchronize()
        return out

    t0 = time.perf_counter()
    train = make(args.n_train, 10000)
    test = make(args.n_test, 20000)
    t_data = time.perf_counter() - t0
    print(f"data: {len(train)} train / {len(test)} test molecules, {t_data:.1f} s", file=sys.stderr, flush=True)
    tr = rif.OnSet(ctx, train)
    it_tr, st_tr, t_tr = ws.solve(ctx, tr, ws.prior_rows(tr))
    X, T, M = ws.features(ctx, tr, with_targets=True)
    mu, sd = ws.standardisation(X)
    X, T, M = ws.features(ctx, tr, with_targets=True, mu=mu, sigma=sd)
    net = ws.WarmStartMLP(ctx, seed=0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    losses = net.fit(X, T, M, epochs=args.epochs, lr=args.lr, lr_final=args.lr_final)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    print(f"trained {args.epochs} epochs on {X.shape[0]} pairs in {t_train:.1f} s, loss "
          f"{losses[0]:.3e} -> {losses[-1]:.3e}", file=sys.stderr, flush=True)

    def cold_warm(probs):
        c = rif.OnSet(ctx, probs)
        ic, sc, tc = ws.solve(ctx, c, ws.prior_rows(c))
        w = rif.OnSet(ctx, probs)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        Xt, _, Mt = ws.features(ctx, w, mu=mu, sigma=sd)
        P = net.predict(Xt, Mt)
        torch.cuda.synchronize()
        t_inf = time.perf_counter() - ta
        iw, sw, tw = ws.solve(ctx, w, P)
        Ec, Ew = c.energy.cpu().numpy(), w.energy.cpu().numpy()
        # each molecule on its own, as the ON step of the Fig. 1 loop runs:
        # starting ONs (cold: the prior; warm: features + network), then the
        # optimiser; summed over the molecules
        per = {}
        for kind in ("cold", "warm"):
            tot = 0.0
            for prob in probs:
                one = rif.OnSet(ctx, [prob])
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if kind == "warm":
                    Xo, _, Mo = ws.features(ctx, one, mu=mu, sigma=sd)
                    Po = net.predict(Xo, Mo)
                else:
                    Po = ws.prior_rows(one)
                ctx.on_warmstart(one, Po)
                ctx.on_optimize(one)
                torch.cuda.synchronize()
                tot += time.perf_counter() - t0
            per[kind] = tot
        return {"iters_cold_mean": float(ic.mean()), "iters_warm_mean": float(iw.mean()),
                "iters_cold_median": float(np.median(ic)), "iters_warm_median": float(np.median(iw)),
                "iter_reduction": round(1.0 - float(iw.mean()) / float(ic.mean()), 4),
                "converged_cold": int((sc == 0).sum()), "converged_warm": int((sw == 0).sum()),
                "n": len(probs), "same_minimum": int((np.abs(Ec - Ew) <= 1e-9 * np.abs(Ec)).sum()),
                "warm_lower_energy": int((Ew < Ec - 1e-9 * np.abs(Ec)).sum()),
                "time_cold_s": round(tc, 5), "time_warm_s": round(tw + t_inf, 5), "time_inference_s": round(t_inf, 5),
                "time_note": "time_*: all molecules in one launch (its time follows the slowest problem); "
                             "per_molecule_*: each molecule's starting ONs and optimisation on its own, summed",
                "per_molecule_cold_s": round(per["cold"], 5), "per_molecule_warm_s": round(per["warm"], 5),
                "per_molecule_time_reduction": round(1.0 - per["warm"] / per["cold"], 4)}

    held = cold_warm(test)
    print("held-out:", held, file=sys.stderr, flush=True)
    inp, npair, ncwo = synth.make_instance_device(1000, 3000, 60, 6, 4)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    big_prob = ws.jk_problem(ctx, inp, npair, ncwo)
    torch.cuda.synchronize()
    t_big_jk = time.perf_counter() - tb
    del inp
    torch.cuda.empty_cache()
    big = cold_warm([big_prob])
    big["jk_build_s"] = round(t_big_jk, 4)
    line = {
        "metric": "ON iterations to max|dE/dgamma| <= 1e-8, learned warm start vs cold start",
        "value": held["iter_reduction"], "unit": "fractional reduction in mean ON iterations (held-out)",
        "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
        "config": {"workload": f"onwarm: {args.n_train} train / {args.n_test} held-out molecules "
                               "n_bf ~ U{48..200}, n_aux = 3 n_bf, pairs = n_bf//12, Ncwo ~ U{1..6}; "
                               "large: n_bf 1000, n_aux 3000, 60 pairs, Ncwo 6"},
        "train": {"iters_mean": float(it_tr.mean()), "converged": int((st_tr == 0).sum()),
                  "pairs": int(X.shape[0]), "epochs": args.epochs, "loss_first": losses[0],
                  "loss_last": losses[-1], "train_s": round(t_train, 2), "data_s": round(t_data, 1)},
        "held_out": held, "large": big,
    }
    ctx.close()
    return line


EIG_NAMES = {0: "auto (reduction + divide and conquer)", 1: "rocSOLVER dsyevd",
             2: "reduction + rocSOLVER dstedc", 3: "reduction + divide and conquer"}


def bench_orbopt(args):
    """Orbital optimisation by iterative diagonalisation of F^lambda (the inner
    iterations of Fig. 1) on the cyclohexane-like workload: one ON step, then
    `steps` inner iterations (build, max|G|, F^lambda, eigen-decomposition,
    rotation), timed as one rif_pnof_optimize call; plus a small molecule
    (n_bf=20, n_aux=40, 2 pairs, Ncwo=1) run to convergence."""
    import numpy as np
    import torch

    import paper_2012_15662_amd as rif
    import synth

    ctx = rif.Context(0)
    if not args.no_tune:
        ctx.autotune(True)
    ctx.set_eigensolver(args.eig, args.eig_groups)

    def upload(inst):
        d = {k: torch.from_numpy(np.ascontiguousarray(getattr(inst, k))).cuda() for k in ("b", "C", "H", "occ")}
        d["pair_of"] = torch.from_numpy(inst.pair_of.astype(np.int32)).cuda()
        d["gamma"] = torch.zeros(inst.n_pairs * inst.n_cwo, dtype=torch.float64, device="cuda")
        return d

    def run(inst, d, **kw):
        C, occ, gamma = d["C"].clone(), d["occ"].clone(), d["gamma"].clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res, he, hg = ctx.optimize(d["b"], C, d["H"], occ, gamma, d["pair_of"], inst.n_pairs, inst.n_cwo,
                                   hist_len=100000, **kw)
        torch.cuda.synchronize()
        return res, he, hg, time.perf_counter() - t0

    inst = synth.workload(args.orb_size)
    d = upload(inst)
    run(inst, d, max_outer=1, max_inner=3, tol_grad=1e-14)          # tile tuning, solver set-up
    res, he, hg, wall = run(inst, d, max_outer=1, max_inner=args.steps, tol_grad=1e-14)
    n = res["inner_total"]
    per_ms = (res["ms_build"] + res["ms_orbital"]) / n
    print(f"{args.orb_size}: {n} inner iterations, build {res['ms_build'] / n:.3f} ms, orbital step "
          f"{res['ms_orbital'] / max(1, n - 1):.3f} ms, ON step {res['ms_on']:.2f} ms; E {he[0]:.6f} -> {he[-1]:.6f}, "
          f"max|G| {hg[0]:.2e} -> {hg[-1]:.2e}", file=sys.stderr, flush=True)

    small_line = None
    if not args.no_small:
        small = synth.make_instance(20, 40, 2, 1, 31)
        ds = upload(small)
        rs, hes, _, wall_s = run(small, ds, max_outer=40, max_inner=4000, tol_grad=1e-6, tol_energy=1e-9)
        print(f"small: status {rs['status']} after {rs['outer']} outer / {rs['inner_total']} inner iterations, "
              f"{wall_s:.2f} s, E {rs['energy']:.10f}", file=sys.stderr, flush=True)
        small_line = {"status": rs["status"], "outer": rs["outer"], "inner": rs["inner_total"],
                      "wall_s": round(wall_s, 3), "energy": rs["energy"], "max_grad": rs["max_grad"],
                      "ms_build": round(rs["ms_build"], 1), "ms_orbital": round(rs["ms_orbital"], 1)}

    cpu = None
    if not args.no_cpu:
        from oracle import orbital as orb
        ts = time.perf_counter()
        k = orb.inner_loop(inst.b, inst.C, inst.H, inst.occ, inst.pair_of, inst.n_pairs, 30, 1e-14)
        tc = time.perf_counter() - ts
        cpu = {"value": round(len(k["energies"]) / tc, 3), "unit": "inner iterations/s",
               "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)), "kind": "oracle",
               "sample": f"{len(k['energies'])} inner iterations of the same workload at fixed ONs "
                         f"(numpy build + eigh), {tc:.1f} s"}

    line = {
        "metric": "orbital-optimisation inner iterations/s (build + F^lambda eigen-decomposition + rotation)",
        "value": round(1e3 / per_ms, 3), "unit": "inner iterations/s", "n_gpus": 1, "steps": n,
        "warmup": 3, "ms_per_step": round(per_ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"orbopt: {args.orb_size} n_bf={inst.n_bf} n_aux={inst.n_aux} pairs={inst.n_pairs} "
                               f"ncwo={inst.n_cwo} n_mo={inst.n_mo}, fixed ONs after one ON step",
                   "eigensolver": EIG_NAMES[args.eig]},
        "split_ms": {"build_with_maxG": round(res["ms_build"] / n, 4),
                     "orbital_step": round(res["ms_orbital"] / max(1, n - 1), 4),
                     "on_step_once": round(res["ms_on"], 3)},
        "wall_s": round(wall, 3), "energy_first": he[0], "energy_last": he[-1], "max_grad_first": hg[0],
        "max_grad_last": hg[-1], "max_grad_min": min(hg), "energy_min": min(he),
        "trajectory": [{"iteration": i, "energy": he[i], "max_grad": hg[i]}
                       for i in sorted(set([0, 9, 99, 499, 999, 1999, 4999, len(he) - 1])) if i < len(he)],
        "small_to_convergence": small_line,
        "cpu_baseline": cpu,
    }
    # release the context (its rocBLAS handle, streams, events and arena)
    # while the HIP runtime is fully up, not from a finaliser at exit
    del d
    ctx.close()
    torch.cuda.synchronize()
    print(json.dumps(line))


def bench_prep(args):
    """b from the three-centre integrals and the metric (rif_prepare_b) at the
    cyclohexane-like size: n_bf=348, n_aux=1044, an ill-conditioned metric
    (condition 1e10, three slightly negative eigenvalues).  Done once per
    molecule; reported per preparation, split into its phases."""
    import numpy as np
    import torch

    import paper_2012_15662_amd as rif
    import synth

    nb, na = 348, 1044
    G = synth.make_metric(na, 20, cond=1e10, n_negative=3)
    T = synth.make_three_centre(nb, na, 21)
    ctx = rif.Context(0)
    ctx.autotune(True)   # the solve GEMM's tile, measured in the warm-up
    Td, Gd = torch.from_numpy(T).cuda(), torch.from_numpy(G).cuda()
    b = torch.empty_like(Td)
    for _ in range(max(1, args.warmup)):
        ctx.prepare_b(Td, Gd, b=b)
    ctx.sync()
    steps = max(1, min(args.steps, 10))
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.prepare_b(Td, Gd, b=b)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = ctx.profile_report()
    ctx.profile(False)
    phases = {k: round(ms / n, 3) for k, (n, ms) in prof.items() if k.startswith("prep_")}
    # the solve runs on the packed upper triangles of the slabs with the
    # triangular factor's zeros skipped: n_aux^2 n_bf (n_bf + 1) / 2 flops
    # (phase time includes the packing and the mirrored unpacking)
    gemm_flops = 1.0 * na * na * nb * (nb + 1) / 2
    gemm_ms = phases.get("prep_solve_gemm")
    cpu = None
    if not args.no_cpu:
        from oracle import metric as mt
        ts = time.perf_counter()
        mt.prepare_b(T, G)
        tc = time.perf_counter() - ts
        cpu = {"value": round(1.0 / tc, 4), "unit": "preparations/s",
               "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)), "kind": "oracle",
               "sample": f"one preparation of the same inputs (numpy Bunch-Kaufman + triangular solve), {tc:.1f} s"}
    line = {
        "metric": "b preparations/s (pivoted metric factorisation, eigenvalue correction, solve)",
        "value": round(steps / el, 3), "unit": "preparations/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * el / steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "prep: n_bf=348 n_aux=1044, metric condition 1e10 with 3 negative eigenvalues"},
        "phases_ms": phases,
        "solve_gemm_tflops": round(gemm_flops / (gemm_ms * 1e-3) / 1e12, 2) if gemm_ms else None,
        "cpu_baseline": cpu,
    }
    ctx.close()
    torch.cuda.synchronize()
    print(json.dumps(line))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c6h12", choices=["tiny", "c6h12", "c10h20", "batch64", "onwarm", "orbopt", "prep", "fourc"])
    ap.add_argument("--n-train", type=int, default=2000)
    ap.add_argument("--n-test", type=int, default=200)
    ap.add_argument("--epochs", type=int, default=2000)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--lr-final", type=float, default=1e-4)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=12.0,
                    help="seconds of oracle builds for the CPU baseline (at most 200 builds)")
    ap.add_argument("--no-tune", action="store_true", help="heuristic tile shapes instead of autotuning")
    ap.add_argument("--prec", default="fp64", choices=list(MODES))
    ap.add_argument("--calib", action="store_true",
                    help="run one 1 GiB device-to-device copy first (reference for HBM counters)")
    ap.add_argument("--no-modes", action="store_true", help="skip timing the other precision modes")
    ap.add_argument("--presplit", action="store_true",
                    help="with a reduced-precision --prec: b stored pre-split (rif_presplit_b) in the timed builds")
    ap.add_argument("--no-direct", action="store_true", help="skip timing rif_build_direct")
    ap.add_argument("--no-4c", action="store_true", help="skip the RI vs four-centre comparison")
    ap.add_argument("--no-c10h20", action="store_true",
                    help="skip the precision study at the cyclodecane-like size")
    ap.add_argument("--no-batch64", action="store_true", help="skip the 64-molecule batch sub-record")
    ap.add_argument("--no-onwarm", action="store_true", help="skip the learned ON warm-start sub-record")
    ap.add_argument("--no-largest", action="store_true",
                    help="skip the largest workload (n_bf 1000, b 24 GB) sub-record")
    ap.add_argument("--eig", type=int, default=0, choices=[0, 1, 2, 3],
                    help="orbopt eigensolver: 0 automatic (3 where it fits), 1 rocSOLVER dsyevd, "
                         "2 one-launch reduction + rocSOLVER dstedc, 3 one-launch reduction + own divide and conquer")
    ap.add_argument("--eig-groups", type=int, default=0,
                    help="orbopt: workgroups of the one-launch tridiagonal reduction (0: default)")
    ap.add_argument("--orb-size", default="c6h12", choices=["tiny", "c6h12", "c10h20"],
                    help="orbopt: the molecule whose inner iterations are run")
    ap.add_argument("--no-small", action="store_true",
                    help="orbopt: skip the small molecule run to convergence")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path would shard over the orbitals of Omega; see the design notes)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch64":
        return bench_batch(args)
    if args.workload == "onwarm":
        return bench_onwarm(args)
    if args.workload == "orbopt":
        return bench_orbopt(args)
    if args.workload == "prep":
        return bench_prep(args)
    if args.workload == "fourc":
        return bench_fourc(args)

    import numpy as np
    import torch

    import paper_2012_15662_amd as rif
    import synth

    inst = synth.workload(args.workload)
    Cs = synth.rotation_sequence(inst.C, 30)
    nb, na, nw, nmo = inst.n_bf, inst.n_aux, inst.n_omega, inst.n_mo
    dev = "cuda:0"
    b = torch.from_numpy(inst.b).to(dev)
    Cd = [torch.from_numpy(c).to(dev) for c in Cs]
    H = torch.from_numpy(inst.H).to(dev)
    occ = torch.from_numpy(inst.occ).to(dev)
    pm = torch.from_numpy(inst.pair_of.astype(np.int32)).to(dev)
    if args.calib:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ctx = rif.Context(0)
    ctx.autotune(not args.no_tune)
    if args.presplit and args.prec == "fp64":
        raise SystemExit("--presplit needs a reduced-precision --prec")
    bsp = ctx.presplit_b(b, MODES[args.prec]) if args.presplit else None
    # per-kernel breakdown from its own untimed pass: event pairs around every
    # launch cost about 4% of a build, so the timed loop records only the
    # dominant kernel's launches, whose average the roofline uses
    n_prof = max(5, min(args.steps, 30))
    _, _, prof = time_builds(ctx, b, Cd, H, occ, pm, inst, MODES[args.prec], n_prof, args.warmup,
                             profile=True, b_split=bsp)
    dom = max(prof, key=lambda k: prof[k][1])
    el, out, prof_dom = time_builds(ctx, b, Cd, H, occ, pm, inst, MODES[args.prec], args.steps, 1,
                                    profile=dom, b_split=bsp)
    ref_out = ctx.build(b, Cd[0], H, occ, pm, inst.n_pairs, inst.n_cwo, prec=MODES[args.prec], b_split=bsp)
    ctx.sync()
    e_main = float(ref_out["energy"].cpu()[0])   # energy at the unrotated C

    kf = kernel_flops(nb, na, nw, nmo)
    per_kernel = {}
    for name, (n, ms) in prof.items():
        avg = ms / n
        ent = {"launches": n, "avg_ms": round(avg, 5)}
        if name in kf:
            ent["tflops"] = round(kf[name] / (avg * 1e-3) / 1e12, 2)
        per_kernel[name] = ent
    traffic, traffic_detail = traffic_of(dom, args.workload, args.prec)
    dom_avg_s = prof_dom[dom][1] / prof_dom[dom][0] * 1e-3   # over the timed region
    achieved = kf.get(dom, 0.0) / dom_avg_s / 1e12
    builds_s = args.steps / el
    flops = build_flops(nb, na, nw, nmo)
    line = {
        "metric": METRIC,
        "value": round(builds_s, 3),
        "unit": "builds/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(el / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16", "bf16x6": "bf16", "fp16x3": "f16"}[args.prec],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: n_bf={nb} n_aux={na} pairs={inst.n_pairs} "
                               f"ncwo={inst.n_cwo} n_omega={nw} n_mo={nmo}, 30 rotated C",
                   "precision": args.prec, **({"b_presplit": True} if args.presplit else {})},
        "tflops": round(flops * builds_s / 1e12, 3),
        "flops_per_build": flops,
        "roofline": {"kernel": dom, "bound": "mfma", "achieved": round(achieved, 3),
                     "peak": PEAK[MODE_PEAK[args.prec]], "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK[MODE_PEAK[args.prec]], 4),
                     "mfma_products_per_fma": PRODUCTS[args.prec],
                     "traffic": traffic, "traffic_detail": traffic_detail,
                     "algorithmic_bytes": kernel_bytes(nb, na, nw).get(dom)},
        "kernels": per_kernel,
        "kernels_note": ("avg_ms is event time on the stream each kernel runs on, from a separate "
                         "profiled pass of the same builds; jk_mo_partial, "
                         "jk_mo_reduce, energy and the H C_Omega small_gemm run on the side stream "
                         "overlapped with the main chain, so theirs is overlapped wall time"),
        "tiles": ctx.tune_report().strip().splitlines(),
        "energy_at_C0": e_main,
    }
    if not args.no_modes:
        # every arithmetic mode on the same workload: speed-up over this run,
        # and error against the FP64 oracle at the unrotated C (energy absolute,
        # gradient normwise), judged against the reduced-precision target
        from oracle import pnof7_ri as ri
        ref = ri.build_instance(inst, C=Cs[0])
        modes = {}
        for name, pv in MODES.items():
            if name == args.prec:
                rate, o2 = builds_s, ref_out
            else:
                n2 = max(5, args.steps // 2)
                el2, _, _ = time_builds(ctx, b, Cd, H, occ, pm, inst, pv, n2, 2)
                rate = n2 / el2
                o2 = ctx.build(b, Cd[0], H, occ, pm, inst.n_pairs, inst.n_cwo, prec=pv)
                ctx.sync()
            modes[name] = {"builds_s": round(rate, 2), "speedup": round(rate / builds_s, 3),
                           "tflops": round(flops * rate / 1e12, 2), **oracle_errors(o2, ref)}
            if name != "fp64" and MODES[args.prec] == MODES["fp64"]:
                # b stored once in this mode's pieces (rif_presplit_b); same results
                bs = ctx.presplit_b(b, pv)
                el4, _, _ = time_builds(ctx, b, Cd, H, occ, pm, inst, pv, n2, 2, b_split=bs)
                modes[name]["presplit_b"] = {"builds_s": round(n2 / el4, 2),
                                             "speedup": round((n2 / el4) / builds_s, 3),
                                             "bytes": int(bs.numel())}
                del bs
        line["modes"] = modes
        line["fastest_within_1uEh"] = fastest_within_target(modes, builds_s)
        if not args.no_c10h20:
            del ref
            line["c10h20"] = precision_study(ctx, "c10h20", max(6, args.steps // 3))
    if not args.no_direct:
        # the same energy, lambda and G without the per-MO AO matrices
        el3, o3, prof3 = time_builds(ctx, b, Cd, H, occ, pm, inst, MODES[args.prec], args.steps, args.warmup,
                                     profile="direct_gradient", direct=True)
        od = ctx.build_direct(b, Cd[0], H, occ, pm, inst.n_pairs, inst.n_cwo, prec=MODES[args.prec])
        om = ctx.build(b, Cd[0], H, occ, pm, inst.n_pairs, inst.n_cwo, prec=MODES[args.prec])
        ctx.sync()
        g_m = om["grad"].cpu().numpy()
        yd = prof3.get("direct_gradient")
        line["direct_gradient"] = {
            "builds_s": round(args.steps / el3, 2), "ms_per_build": round(1e3 * el3 / args.steps, 4),
            "speedup_vs_build": round((args.steps / el3) / builds_s, 3),
            "dE_vs_build": float(od["energy"].cpu()[0]) - float(om["energy"].cpu()[0]),
            "grad_rel_vs_build": float(abs(od["grad"].cpu().numpy() - g_m).max() / abs(g_m).max()),
            "contraction_ms": round(yd[1] / yd[0], 5) if yd else None,
            "contraction_tflops": round(2.0 * nb * nw * na * nw / (yd[1] / yd[0] * 1e-3) / 1e12, 2) if yd else None,
        }
    if not args.no_4c:
        line["four_centre"] = four_centre_study(ctx)
    if not args.no_batch64:
        line["batch64"] = batch_study(ctx)
    if not args.no_largest:
        line["largest"] = largest_study(ctx)
    if not args.no_onwarm:
        ow = onwarm_study(args)   # its own context
        line["onwarm"] = {"metric": ow["metric"], "iter_reduction_held_out": ow["value"], "config": ow["config"],
                          "train": ow["train"], "held_out": ow["held_out"], "large": ow["large"]}
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(inst, Cs, args.cpu_budget)
    ctx.close()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
