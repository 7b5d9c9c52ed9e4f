"""Benchmark: J/K build throughput (unique shell quartets / s) on one MI355X.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--no-cpu-baseline] [--no-mixed] [--no-grad]
                    [--no-batch]

Workload: 40 atoms on a jittered cubic lattice (2.5 bohr, +-0.3), shells
s, s, p, d per atom with 3 primitives each (440 Cartesian functions), Schwarz
screening at 1e-10, density C C^T with C of 440 x 80 N(0,1)/sqrt(N), seed 2.
A step is one mjk_build_jk: zero J/K, every class kernel (ERIs fused with the
J/K digestion), symmetrize.  The plan (pair tables, Schwarz factors, sort,
work lists) is built once before timing and reported separately as plan_ms.

Prints one JSON line.  `roofline` is for the costliest class kernel, timed
with HIP events on the launch stream during the timed steps; `cpu_baseline`
times the plain FP64 CPU oracle on a bounded sample of the same workload.
`mixed`: the 120-atom workload built in FP64 and in mixed precision (speedup,
E2 difference).  `grad`: the 60-atom workload's forward (J/K + E2) and
backward (nuclear gradient) times.  `batch`: 64 molecules of 8-12 atoms
(s, s, p, d, f shells, K ~ U{1..6}; the recipe's 8-96 atoms by option) built
one molecule at a time and as one batch with autotuned tiles; per-molecule times come from in-kernel wall-clock stamps.  `scf`:
RHF on the 40-atom workload around the library, per-iteration time and the
J/K share, with full and with incremental (density-screened) Fock builds.
"""
import argparse
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "J/K build ERI quartets/s + speedup vs FP64 GPU path at ≤1e-6 Eh error"
FP64_PEAK_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_jk_40atom_spd.json")
# per-(class, K-bucket) tiles that Algorithm 2 chose on the batched workload
TILE_CACHE = os.path.join(ROOT, "paper_2412_13203_amd", "tiles_gfx950.json")


def _cache_has(path, key):
    with open(path) as fh:
        return any(k.endswith("/" + key) for k in json.load(fh))


def kernel_source_hash(cls):
    """Hash of the sources a class kernel is built from (its generated class
    code, the kernel templates, the record layouts and the Boys table)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2412_13203_amd", "csrc")
    h = hashlib.sha256()
    for f in ("kernels.hpp", "mjk_types.hpp", os.path.join("gen", "boys_table.inc"),
              os.path.join("gen", f"cls_{cls}.inc")):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def kernel_name(cls):
    """Kernel template that runs J/K class `cls` ("dddp"): the per-lane k_jk or,
    for classes split into recurrence passes, k_jk_split."""
    try:
        recs = json.load(open(os.path.join(ROOT, "paper_2412_13203_amd", "csrc", "gen", "opcount.json")))
        split = {"".join("spdf"[l] for l in r["tuple"]): r["split"] for r in recs}[cls]
    except (OSError, KeyError, ValueError):
        return f"class {cls}"
    ls = ",".join(str("spdf".index(c)) for c in cls)
    return f"k_jk_split<{ls}>" if split else f"k_jk<{ls}>"


def measured_traffic(cls):
    """HBM bytes per launch of class `cls` from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE record, if it was taken on the current sources."""
    try:
        rec = json.load(open(TRAFFIC_FILE))["classes"][cls]
    except (OSError, KeyError, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_hash(cls):
        return None
    return rec["fetch_bytes"] + rec["write_bytes"]


def cpu_baseline(cfg, nbra=32):
    """Oracle quartets/s on a sample: nbra bra pairs at a fixed stride of the
    unique-quartet list, every kept ket of each (same screening rule).  The
    cost of one bra pair varies by orders of magnitude with its class, so the
    sample is a fixed, evenly spread set (~15 s on 16 host threads), not one
    sized from a timing probe."""
    import oracle
    b, D, tau = cfg["basis"], cfg["D"], cfg["tau"]
    ns = len(b["shell_l"])
    npair = ns * (ns + 1) // 2
    t0 = time.time()
    Q = oracle.schwarz(b)
    t_q = time.time() - t0
    stride = max(1, npair // nbra)
    rows = np.arange(stride // 2, npair, stride, dtype=np.int32)
    t0 = time.time()
    _, _, nq = oracle.jk_rows(b, D, tau, rows, Q)
    dt = time.time() - t0
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next(l.split(":", 1)[1].strip() for l in fh if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {
        "value": nq / dt, "unit": "quartets/s", "cores": oracle.nthreads(), "cpu_model": cpu, "kind": "oracle",
        "sample": f"{len(rows)} bra pairs (every {stride}th of {npair}), all kept kets: {nq} quartets in "
                  f"{dt:.2f} s; Schwarz table {t_q:.2f} s not included",
    }


def mixed_comparison(torch, mjk, inputs, dev, taus=(1e-4,), steps=1):
    """120-atom s,s,p,d workload: FP64 path vs mixed path (same plan inputs).
    E2 = 1/2 Tr(DJ) - 1/4 Tr(DK); the FP64 GPU path is the reference here
    (it matches the FP64 oracle to ~1e-13 relative on the parity tests)."""
    cfg = inputs.make_config(3)
    b = cfg["basis"]
    D = torch.as_tensor(cfg["D"], device=f"cuda:{dev}")
    res = {}
    runs = [("fp64", 0.0)] + [(f"mixed_{t:g}", t) for t in taus]
    for name, f32 in runs:
        plan = mjk.Plan(b, tau=cfg["tau"], fp32_tau=f32, device=dev)
        J = torch.empty_like(D)
        K = torch.empty_like(D)
        plan.build_jk(D, J, K)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            plan.build_jk(D, J, K)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        e2 = float(plan.e2(D, J, K).item())
        res[name] = {"ms": ms, "e2": e2, "quartets": plan.stats["nquartet_kept"],
                     "quartets_fp32": plan.stats["nquartet_fp32"], "J": J, "K": K}
        print(f"bench: 120-atom {name}: {ms:.1f} ms, E2 {e2:.10f}", file=sys.stderr, flush=True)
        del plan
    f = res["fp64"]
    out = {"workload": "120-atom jittered-lattice molecule, s,s,p,d x 3 primitives, nbf 1320, Schwarz 1e-10",
           "nbf": b["nbf"], "quartets_kept": f["quartets"], "fp64_ms": f["ms"],
           "fp64_quartets_per_s": f["quartets"] / (f["ms"] * 1e-3), "e2_fp64": f["e2"], "by_fp32_tau": []}
    for t in taus:
        m = res[f"mixed_{t:g}"]
        out["by_fp32_tau"].append({
            "fp32_tau": t, "quartets_fp32": m["quartets_fp32"], "mixed_ms": m["ms"],
            "speedup_vs_fp64": f["ms"] / m["ms"], "mixed_quartets_per_s": m["quartets"] / (m["ms"] * 1e-3),
            "e2_mixed": m["e2"], "e2_abs_err": abs(m["e2"] - f["e2"]),
            "max_abs_dJ": float(torch.max(torch.abs(m["J"] - f["J"]))),
            "max_abs_dK": float(torch.max(torch.abs(m["K"] - f["K"])))})
    ok = [r for r in out["by_fp32_tau"] if r["e2_abs_err"] <= 1e-6]
    out["best_within_1e-6_Eh"] = (max(ok, key=lambda r: r["speedup_vs_fp64"]) if ok else None)
    return out


def grad_comparison(torch, mjk, inputs, dev, steps=2, warmup=1):
    """60-atom s,s,p,d workload, no screening: forward (J/K build + E2) and
    backward (nuclear gradient at fixed D) times with HIP events on the launch
    stream, and the per-class gradient kernel times."""
    cfg = inputs.make_config(5)
    b = cfg["basis"]
    D = torch.as_tensor(cfg["D"], device=f"cuda:{dev}")
    t0 = time.time()
    plan = mjk.Plan(b, tau=cfg["tau"], device=dev, grad=True)
    torch.cuda.synchronize()
    plan_ms = (time.time() - t0) * 1e3
    J = torch.empty_like(D)
    K = torch.empty_like(D)
    e = torch.empty((), dtype=torch.float64, device=f"cuda:{dev}")
    g = torch.empty((b["xyz"].shape[0], 3), dtype=torch.float64, device=f"cuda:{dev}")
    for _ in range(warmup):
        plan.build_jk(D, J, K)
        plan.e2(D, J, K, e)
        plan.grad_e2(D, g)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    fwd = bwd = 0.0
    per_cls = {}
    for _ in range(steps):
        plan.set_timing(False)
        ev[0].record()
        plan.build_jk(D, J, K)
        plan.e2(D, J, K, e)
        ev[1].record()
        plan.set_timing(True)
        plan.grad_e2(D, g)
        ev[2].record()
        torch.cuda.synchronize()
        fwd += ev[0].elapsed_time(ev[1])
        bwd += ev[1].elapsed_time(ev[2])
        for t in plan.timings():
            acc = per_cls.setdefault(t["cls"], {"ms": 0.0, "nlaunch": 0, "flops": 0.0})
            acc["ms"] += t["ms"]
            acc["nlaunch"] += t["nlaunch"]
            acc["flops"] += t["flops"]
    fwd /= steps
    bwd /= steps
    print(f"bench: 60-atom gradient: forward {fwd:.1f} ms, backward {bwd:.1f} ms", file=sys.stderr, flush=True)
    gh = g.cpu().numpy()
    dom_cls, dom = max(per_cls.items(), key=lambda kv: kv[1]["ms"])
    gfl = plan.stats["grad_flops_kept"]
    return {
        "workload": "60-atom jittered-lattice molecule, s,s,p,d x 3 primitives, nbf 660, no screening, FP64",
        "nbf": b["nbf"], "quartets": plan.stats["nquartet_kept"], "plan_ms": plan_ms,
        "forward_ms": fwd, "backward_ms": bwd, "backward_over_forward": bwd / fwd,
        "e2": float(e.item()), "sum_rule_max_abs": float(np.max(np.abs(gh.sum(axis=0)))),
        "max_abs_grad": float(np.max(np.abs(gh))),
        "backward_algorithmic_tflops": gfl / (bwd * 1e-3) / 1e12,
        "dominant_kernel": {"kernel": f"k_grad<{dom_cls}>", "avg_launch_ms": dom["ms"] / dom["nlaunch"],
                            "achieved_tflops": dom["flops"] / (dom["ms"] * 1e-3) / 1e12,
                            "frac": dom["flops"] / (dom["ms"] * 1e-3) / 1e12 / FP64_PEAK_TFLOPS},
        "classes": {k: {"ms": round(v["ms"] / steps, 3),
                        "tflops": round(v["flops"] / (v["ms"] * 1e-3) / 1e12, 3) if v["ms"] > 0 else None}
                    for k, v in sorted(per_cls.items(), key=lambda kv: -kv[1]["ms"])},
    }


def scf_comparison(torch, inputs, dev, config=2, natom=None):
    """The SCF iteration around the library (Section 2.1): RHF on a lattice
    workload (charges and occupied orbitals from the recipe's density width),
    once with a full J/K build every iteration and once incremental (density
    changes with density-weighted screening, a full rebuild every 8
    iterations and to confirm convergence).  Per-iteration time and the J/K
    build's share of it, HIP events on the launch stream."""
    from paper_2412_13203_amd import scf
    cfg = inputs.make_config(config, natom=natom) if natom else inputs.make_config(config)
    Z, nocc = inputs.scf_system(cfg)
    out = {"workload": f"{cfg['natom']}-atom jittered-lattice molecule, s,s,p,d x 3 primitives, nbf {cfg['basis']['nbf']}, "
                       f"Schwarz {cfg['tau']}, Z = {Z[0]:g} per atom, {nocc} doubly occupied orbitals, RHF + DIIS",
           "nbf": cfg["basis"]["nbf"]}
    for mode in ("full", "incremental"):
        t0 = time.time()
        r = scf.RHF(cfg["basis"], Z, nocc, tau=cfg["tau"], device=dev)
        setup = time.time() - t0
        res = r.run(e_tol=1e-9, err_tol=1e-7, incremental=mode == "incremental",
                    log=lambda m: print(f"bench: SCF {mode}: {m}", file=sys.stderr, flush=True))
        it_ms = float(np.sum(res["ms_per_iter"]))
        jk_ms = float(np.sum(res["ms_jk"]))
        print(f"bench: SCF {mode}: {res['iterations']} iterations, E = {res['energy']:.10f}, "
              f"{it_ms / res['iterations']:.1f} ms/iteration, J/K share {jk_ms / it_ms:.3f}", file=sys.stderr,
              flush=True)
        out[mode] = {"converged": res["converged"], "iterations": res["iterations"], "energy": res["energy"],
                     "setup_s": setup, "ms_per_iteration": it_ms / res["iterations"],
                     "jk_ms_per_iteration": jk_ms / res["iterations"], "jk_share": jk_ms / it_ms,
                     "total_s": it_ms * 1e-3, "kept_quartets": res["kept_quartets"]}
    out["incremental_speedup"] = out["full"]["total_s"] / out["incremental"]["total_s"]
    out["energy_difference"] = abs(out["full"]["energy"] - out["incremental"]["energy"])
    return out


def ablation(torch, mjk, inputs, dev, steps=3):
    """Component ablation on the 40-atom workload (the paper breaks its gain
    down by component):
      * binning by primitive-pair count off (MJK_FLAG_NO_KBINS): the pairs of
        a class share one bin, so a wave mixes loop trip counts;
      * Algorithm 1 off: a library whose generator took the fixed textbook
        recurrence order (build: MJK_FIXED_PATH=1 python -m
        paper_2412_13203_amd.build --variant fixedpath), timed in a child
        process of this script;
      * the two generators' recurrence flops per class (their opcount.json)
        and the time to construct every class's recurrence path."""
    import subprocess
    cfg = inputs.make_config(2)
    b = cfg["basis"]
    D = torch.as_tensor(cfg["D"], device=f"cuda:{dev}")
    out = {"workload": "40-atom s,s,p,d workload as the headline, FP64, per-build times (HIP events)"}

    def time_plan(flags):
        plan = mjk.Plan(b, tau=cfg["tau"], device=dev, flags=flags)
        J, K = plan.build_jk(D)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            plan.build_jk(D, J, K)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps, plan.stats["nquartet_kept"]

    out["full_ms"], nq = time_plan(0)
    out["no_kbins_ms"], nq2 = time_plan(mjk.FLAG_NO_KBINS)
    assert nq2 == nq
    print(f"bench: ablation: full {out['full_ms']:.1f} ms, no K-bins {out['no_kbins_ms']:.1f} ms", file=sys.stderr,
          flush=True)
    # every pair of the 40-atom workload has K_A K_B = 9, so the binning by
    # primitive count only matters where K varies: a 32-atom molecule of the
    # batched recipe (s, s, p, d shells, K ~ U{1..6})
    m = inputs.make_batch(nmol=1, seed=4, atom_range=(32, 32), shells=(0, 0, 1, 2))[0]
    b, D = m["basis"], torch.as_tensor(m["D"], device=f"cuda:{dev}")
    out["varK_workload"] = f"32-atom molecule of the batched recipe, s,s,p,d, K ~ U{{1..6}}, nbf {b['nbf']}"
    out["varK_full_ms"], nq = time_plan(0)
    out["varK_no_kbins_ms"], nq2 = time_plan(mjk.FLAG_NO_KBINS)
    assert nq2 == nq
    print(f"bench: ablation (K ~ U{{1..6}}): full {out['varK_full_ms']:.1f} ms, no K-bins "
          f"{out['varK_no_kbins_ms']:.1f} ms", file=sys.stderr, flush=True)
    variant = os.path.join(ROOT, "paper_2412_13203_amd", "_lib", "libmjk_fixedpath.so")
    if os.path.exists(variant):
        r = subprocess.run([sys.executable, "-u", os.path.abspath(__file__), "--steps", str(steps), "--no-mixed",
                            "--no-grad", "--no-batch", "--no-scf", "--no-cpu-baseline"],
                           env={**os.environ, "MJK_LIBRARY": variant}, capture_output=True, text=True, timeout=600)
        if r.returncode == 0:
            child = json.loads(r.stdout.strip().splitlines()[-1])
            out["fixed_path_ms"] = child["ms_per_step"]
            out["fixed_path_classes_ms"] = {k: v["ms_per_step"] for k, v in child["classes"].items()}
        else:
            out["fixed_path_error"] = r.stderr[-2000:]
        print(f"bench: ablation: fixed recurrence order {out.get('fixed_path_ms')} ms", file=sys.stderr, flush=True)
    flops = {}
    for tag, sub in (("greedy", "gen"), ("fixed", "gen_fixedpath")):
        try:
            recs = json.load(open(os.path.join(ROOT, "paper_2412_13203_amd", "csrc", sub, "opcount.json")))
        except OSError:
            continue
        for rec in recs:
            if rec.get("forward"):
                name = "".join("spdf"[l] for l in rec["tuple"])
                flops.setdefault(name, {})[tag] = {"single_pass": rec["vrr_flops"],
                                                    "passes": rec.get("split_vrr_flops") or rec["vrr_flops"]}
    out["vrr_flops_per_primitive_quartet"] = flops
    sys.path.insert(0, os.path.join(ROOT, "paper_2412_13203_amd", "gen"))
    import eri_gen
    for tag, fixed in (("greedy", False), ("fixed", True)):
        eri_gen.FIXED_PATH = fixed
        t0 = time.time()
        for c in eri_gen.quartet_classes(2):
            eri_gen.best_vrr(*c)
        out[f"path_construction_s_{tag}"] = time.time() - t0
    eri_gen.FIXED_PATH = False
    return out


def batch_comparison(torch, mjk, inputs, dev, nmol=64, atom_range=(8, 12), steps=1, tune_reps=1):
    """Many molecules of uneven size: sequential single-molecule FP64 builds
    (default tiles) vs one batch (one launch per class over all molecules),
    with default tiles and with the tiles Algorithm 2 picks on this batch."""
    shells = (0, 0, 1, 2, 3) if mjk.lib().mjk_lmax() >= 3 else (0, 0, 1, 2)
    mols = inputs.make_batch(nmol=nmol, seed=4, atom_range=atom_range, shells=shells)
    tau = mols[0]["tau"]
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    # sequential: one plan per molecule, plans built before timing
    plans = [mjk.Plan(m["basis"], tau=tau, device=dev) for m in mols]
    print(f"bench: {nmol} single-molecule plans bound", file=sys.stderr, flush=True)
    Ds = [torch.as_tensor(m["D"], device=f"cuda:{dev}") for m in mols]
    outs = [(torch.empty_like(D), torch.empty_like(D)) for D in Ds]
    def seq_pass(what):
        # a progress line every 16 molecules (the full atom range takes minutes)
        for i, (p, D, (J, K)) in enumerate(zip(plans, Ds, outs)):
            p.build_jk(D, J, K)
            if (i + 1) % 16 == 0:
                torch.cuda.synchronize()
                print(f"bench: {what}, molecule {i + 1} of {nmol}", file=sys.stderr, flush=True)

    # warm-up: the largest molecule (every class kernel of the batch is loaded)
    big = max(range(nmol), key=lambda i: mols[i]["basis"]["nbf"])
    plans[big].build_jk(Ds[big], *outs[big])
    torch.cuda.synchronize()
    ev0.record()
    for s_ in range(steps):
        seq_pass(f"sequential pass {s_ + 1} of {steps}")
    ev1.record()
    torch.cuda.synchronize()
    seq_ms = ev0.elapsed_time(ev1) / steps
    nq = sum(p.stats["nquartet_kept"] for p in plans)
    del plans, outs
    t0 = time.time()
    bt = mjk.Batch([m["basis"] for m in mols], tau=tau, device=dev)
    torch.cuda.synchronize()
    plan_ms = (time.time() - t0) * 1e3
    print(f"bench: sequential {seq_ms:.1f} ms; batch plan bound in {plan_ms:.0f} ms", file=sys.stderr, flush=True)
    D = bt.pack([m["D"] for m in mols])
    J = torch.empty_like(D)
    K = torch.empty_like(D)

    def timed():
        bt.build_jk(D, J, K)
        torch.cuda.synchronize()
        print("bench: batch warm-up build done", file=sys.stderr, flush=True)
        ev0.record()
        for _ in range(steps):
            bt.build_jk(D, J, K)
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / steps

    default_ms = timed()
    print(f"bench: batch with default tiles {default_ms:.1f} ms", file=sys.stderr, flush=True)
    nkb = mjk.lib().mjk_num_kbuckets()
    cached_s = None
    t0 = time.time()
    wl_key = f"batch{nmol}_atoms{atom_range[0]}-{atom_range[1]}_seed4"
    tiles_from = "autotuned in this run"
    if tune_reps == 0 and os.path.exists(TILE_CACHE):
        # tiles an earlier autotune run stored for this workload (no tuning here)
        qpl = bt.autotune(D, per_bucket=True, cache=TILE_CACHE, key=wl_key, reps=1) \
            if _cache_has(TILE_CACHE, wl_key) else None
        if qpl is not None:
            tiles_from = f"{os.path.relpath(TILE_CACHE, ROOT)} (an earlier autotune run on this workload)"
            tuned_ms = timed()
            tune_s = time.time() - t0
        else:
            qpl = [1] * (mjk.num_classes() * nkb)
            tuned_ms = default_ms
            tune_s = 0.0
            tiles_from = "default (one quartet per lane)"
    elif tune_reps > 0:
        # Algorithm 2 over (class, bra K-bucket) units; the table goes to a
        # cache file, and a second call finds it there instead of tuning
        cache = os.path.join(tempfile.mkdtemp(), "mjk_tiles.json")
        qpl = bt.autotune(D, reps=tune_reps, per_bucket=True, cache=cache, key=wl_key,
                          log=lambda m: print(f"bench: {m}", file=sys.stderr, flush=True))
        tune_s = time.time() - t0
        bt.set_tiles([1] * len(qpl))
        t1 = time.time()
        again = bt.autotune(D, reps=tune_reps, per_bucket=True, cache=cache, key=wl_key)
        cached_s = time.time() - t1
        assert again == qpl
        tuned_ms = timed()
    else:
        qpl = [1] * (mjk.num_classes() * nkb)
        tuned_ms = default_ms
        tune_s = 0.0
        tiles_from = "default (one quartet per lane)"
    bt.set_stamps(True)
    bt.build_jk(D, J, K)
    torch.cuda.synchronize()
    times = [t for t, n in zip(bt.mol_times(), bt.nq_per_mol) if n > 0]
    dur = sorted(t1 - t0_ for t0_, t1 in times)
    ends = sorted(t1 for _, t1 in times)
    names = mjk.class_names()
    print(f"bench: batch of {nmol}: sequential {seq_ms:.1f} ms, batch {default_ms:.1f} ms, tuned {tuned_ms:.1f} ms",
          file=sys.stderr, flush=True)
    return {
        "workload": f"{nmol} jittered-lattice molecules, atoms ~ U{{{atom_range[0]}..{atom_range[1]}}}, shells "
                    f"{','.join('spdf'[l] for l in shells)}, K ~ U{{1..6}}, Schwarz {tau:g}, FP64",
        "nmol": nmol, "nbf_total": int(sum(bt.nbf)), "quartets": bt.stats["nquartet_kept"],
        "prim_quartets": bt.stats["nprim_quartet_kept"], "plan_ms": plan_ms,
        "sequential_ms": seq_ms, "sequential_quartets_per_s": nq / (seq_ms * 1e-3),
        "batch_default_ms": default_ms, "batch_tuned_ms": tuned_ms,
        "batch_quartets_per_s": bt.stats["nquartet_kept"] / (tuned_ms * 1e-3),
        "speedup_vs_sequential": seq_ms / tuned_ms, "autotune_s": tune_s, "autotuned": tune_reps > 0,
        "autotune_cached_s": cached_s, "tiles_from": tiles_from,
        "tuned_quartets_per_lane": {f"{names[u // nkb]}/kbucket{u % nkb}": v for u, v in enumerate(qpl) if v != 1},
        "per_molecule_ms": {"min": dur[0], "median": dur[len(dur) // 2], "max": dur[-1]},
        "finish_spread_ms": ends[-1] - ends[0],
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the 120-atom mixed-precision comparison (FP32 below Q_AB Q_CD = fp32_tau: "
                         "speedup over the FP64 path and E2 difference)")
    ap.add_argument("--no-grad", action="store_true",
                    help="skip the 60-atom nuclear-gradient timing (backward / forward ratio)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-molecule batched build (one launch per class, autotuned tiles)")
    ap.add_argument("--batch-atoms", type=int, nargs=2, default=[8, 12], metavar=("LO", "HI"),
                    help="atom-count range of the batch's molecules (the full recipe is 8 96)")
    ap.add_argument("--batch-steps", type=int, default=1, help="timed builds per batch measurement")
    ap.add_argument("--batch-tune-reps", type=int, default=0,
                    help="builds per autotuner trial (0: no tuning in this run; the batch then uses the "
                         "tiles an earlier autotune run stored for its workload, if any)")
    ap.add_argument("--ablation", action="store_true",
                    help="also run the component ablation on the 40-atom workload (binning off, fixed "
                         "recurrence order if its variant library is built, generator flops)")
    ap.add_argument("--no-scf", action="store_true",
                    help="skip the SCF driver timing (RHF on the 40-atom workload, full and incremental)")
    ap.add_argument("--scf-config", type=int, default=2, help="workload of the SCF timing (2: 40 atoms, 3: 120)")
    ap.add_argument("--fp32-tau", type=float, nargs="+", default=[1e-4, 1e-5, 1e-6],
                    help="mixed-precision thresholds for --mixed (first one is the headline)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="also run one device-to-device copy of MB MiB (known-size kernel for scaling "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (asked for --gpus {args.gpus}); "
              "the J/K work would shard by class-pair tiles with one all-reduce of J and K, "
              "which is not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2412_13203_amd import inputs, mjk
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = 0
    torch.cuda.set_device(dev)
    cfg = inputs.make_config(2)
    b, D_host = cfg["basis"], cfg["D"]
    print(f"bench: workload 40-atom s,s,p,d lattice, nbf={b['nbf']}, tau={cfg['tau']}", file=sys.stderr, flush=True)

    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=f"cuda:{dev}")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"bench: calibration copy of {n * 8} bytes done", file=sys.stderr, flush=True)
        del src, dst

    torch.cuda.synchronize()
    t0 = time.time()
    plan = mjk.Plan(b, tau=cfg["tau"], device=dev)
    torch.cuda.synchronize()
    plan_ms = (time.time() - t0) * 1e3
    st = plan.stats
    D = torch.as_tensor(D_host, device=f"cuda:{dev}")
    J = torch.empty_like(D)
    K = torch.empty_like(D)
    for _ in range(args.warmup):
        plan.build_jk(D, J, K)
    torch.cuda.synchronize()
    print(f"bench: plan {plan_ms:.1f} ms, {st['nquartet_kept']} quartets kept, warmup done", file=sys.stderr,
          flush=True)

    # timed steps, per-class events on the launch stream (torch's current stream)
    plan.set_timing(True)
    per_cls = {}
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.time()
    ev0.record()
    total_ms_events = 0.0
    for _ in range(args.steps):
        plan.build_jk(D, J, K)
        torch.cuda.synchronize()
        for t in plan.timings():
            acc = per_cls.setdefault(t["cls"], {"ms": 0.0, "nlaunch": 0, "flops": 0.0, "nquartet": 0,
                                                "nprim_quartet": 0})
            acc["ms"] += t["ms"]
            acc["nlaunch"] += t["nlaunch"]
            acc["flops"] += t["flops"]
            acc["nquartet"] += t["nquartet"]
            acc["nprim_quartet"] += t["nprim_quartet"]
    ev1.record()
    torch.cuda.synchronize()
    wall = time.time() - t0
    total_ms_events = ev0.elapsed_time(ev1)
    ms_per_step = total_ms_events / args.steps
    value = st["nquartet_kept"] / (ms_per_step * 1e-3)

    # parity spot check against the stored oracle blocks
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "config2_jk_blocks.json")))
    Jh, Kh = J.cpu().numpy(), K.cpu().numpy()
    off = inputs.ao_offsets(b)
    dj = dk = 0.0
    for (A, Bs), jv, kv in zip(gold["blocks"], gold["J"], gold["K"]):
        sa, sb = slice(off[A], off[A + 1]), slice(off[Bs], off[Bs + 1])
        dj = max(dj, float(np.max(np.abs(Jh[sa, sb].ravel() - np.array(jv)))))
        dk = max(dk, float(np.max(np.abs(Kh[sa, sb].ravel() - np.array(kv)))))

    # dominant kernel roofline (FP64 VALU bound)
    dom_cls, dom = max(per_cls.items(), key=lambda kv: kv[1]["ms"])
    avg_ms = dom["ms"] / dom["nlaunch"]
    flops_per_launch = dom["flops"] / dom["nlaunch"]
    achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12
    total_flops = sum(v["flops"] for v in per_cls.values()) / args.steps
    classes = {k: {"ms_per_step": round(v["ms"] / args.steps, 4),
                   "tflops": round(v["flops"] / (v["ms"] * 1e-3) / 1e12, 3) if v["ms"] > 0 else None,
                   "quartets": v["nquartet"] // args.steps}
               for k, v in sorted(per_cls.items(), key=lambda kv: -kv[1]["ms"])}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "quartets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "40-atom jittered-lattice molecule, s,s,p,d shells x 3 primitives, nbf 440, "
                               "Schwarz 1e-10, plain FP64 J/K build",
                   "nbf": b["nbf"], "shell_pairs": st["npair"], "quartets_kept": st["nquartet_kept"],
                   "quartets_total": st["nquartet_total"], "prim_quartets_kept": st["nprim_quartet_kept"],
                   "schwarz_tau": cfg["tau"], "seed": cfg["seed"]},
        "plan_ms": plan_ms,
        "wall_s_timed": wall,
        "prim_quartets_per_s": st["nprim_quartet_kept"] / (ms_per_step * 1e-3),
        "cart_eris_per_s": st["ncart_eri_kept"] / (ms_per_step * 1e-3),
        "algorithmic_tflops": total_flops / (ms_per_step * 1e-3) / 1e12,
        "fp64_frac_whole_step": total_flops / (ms_per_step * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
        "roofline": {"bound": "alu", "kernel": kernel_name(dom_cls), "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": measured_traffic(dom_cls),
                     "avg_launch_ms": avg_ms, "flops_per_launch": flops_per_launch},
        "classes": classes,
        "parity_vs_stored_oracle_blocks": {"max_abs_dJ": dj, "max_abs_dK": dk},
    }
    if not args.no_mixed:
        out["mixed"] = mixed_comparison(torch, mjk, inputs, dev, taus=args.fp32_tau)
    if not args.no_grad:
        out["grad"] = grad_comparison(torch, mjk, inputs, dev)
    if not args.no_batch:
        out["batch"] = batch_comparison(torch, mjk, inputs, dev, atom_range=tuple(args.batch_atoms),
                                        steps=args.batch_steps, tune_reps=args.batch_tune_reps)
    if not args.no_scf:
        out["scf"] = scf_comparison(torch, inputs, dev, config=args.scf_config)
    if args.ablation:
        out["ablation"] = ablation(torch, mjk, inputs, dev)
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
