"""Benchmark of the ray-tracing step on one MI355X.

Default workload: 256^3 grid, density exp of a k^-2.5 Gaussian random field
(ln-sigma 1.5), 2000 sources on its highest peaks, highly ionized start
(x_HI = 1e-4), packets finishing inside each step, 4 blackbody bins, flux
floor 1e-3, distance cap 50 cMpc/h, level cap 12, FP32 march with FP64
chemistry.  A step is one pass of the whole path: casting, every march
round, chemistry and ledger.  Inputs are resident in HBM before timing.

Prints one JSON line: crossings/s over the timed steps, the march kernel's
roofline figures from HIP-event timing of its launches, and the FP64 oracle
timed on a bounded sample of the same workload on the host's cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, published
# one VALU operation per lane per cycle: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# (the published 157.3 TFLOP/s counts an FMA as two and packed FP32 as two
# lanes, which this build does not emit)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
VALU_SIMDS, CLOCK_HZ = 256 * 4, 2.4e9
ALG_OPS_PER_CROSSING = 120          # FP32 operations of one crossing at 4 bins
ALG_BYTES_PER_CROSSING = 12         # opacity gather 8 B + one FP32 deposit 4 B
def alg_bytes_per_visit(nb):        # the packet record read and written
    return 2 * (36 + 8 * nb)
METRIC = "cell crossings/s at 256^3 + p50/p99 solve latency, batched vs plain per-solve"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("frt_kernels.hip", "frt_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2409_04521_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_valu(workload: str):
    """VALU figures of the march from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"march_{workload}_valu.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return {k: d[k] for k in ("lane_instr_per_crossing", "wave_instr_per_crossing", "lane_utilisation",
                              "valu_issue_frac", "trans_per_crossing")}


def valu_summary(db_dir: str, crossings_per_step: float, out_path: str):
    """VALU instructions of the march per crossing and the share of the
    SIMDs' issue cycles they take (4 cycles per wave64 instruction, 16 per
    transcendental one, over 1024 SIMDs at 2.4 GHz for the kernels' own
    duration), over the march launches of the last step of a rocprofv3 run
    with SQ_INSTS_VALU, SQ_THREAD_CYCLES_VALU and SQ_INSTS_VALU_TRANS_F32."""
    import glob
    import sqlite3
    dbs = glob.glob(os.path.join(db_dir, "**", "*.db"), recursive=True)
    con = sqlite3.connect(dbs[0])
    q = ("select dispatch_id, kernel_name, counter_name, sum(value), min(start), max(end) from counters_collection "
         "group by dispatch_id, counter_name order by dispatch_id")
    per = {}
    for did, name, cname, val, t0, t1 in con.execute(q):
        d = per.setdefault(did, {"name": name, "t0": t0, "t1": t1, "c": {}})
        d["c"][cname] = val
    ds = [per[k] for k in sorted(per)]
    last_seed = max(i for i, d in enumerate(ds) if "k_seed<" in d["name"])
    brick = [d for d in ds[last_seed:] if "k_brick" in d["name"]]
    tot = {c: sum(d["c"].get(c, 0.0) for d in brick) for c in ("SQ_INSTS_VALU", "SQ_THREAD_CYCLES_VALU",
                                                                  "SQ_INSTS_VALU_TRANS_F32")}
    secs = sum((d["t1"] - d["t0"]) * 1e-9 for d in brick)
    cycles = (tot["SQ_INSTS_VALU"] - tot["SQ_INSTS_VALU_TRANS_F32"]) * 4 + tot["SQ_INSTS_VALU_TRANS_F32"] * 16
    out = {"kernel": "k_brick (march)", "kernel_source_hash": kernel_source_hash(), "launches": len(brick),
           "crossings_per_step": crossings_per_step, "kernel_seconds": secs,
           "sq_insts_valu": tot["SQ_INSTS_VALU"], "sq_thread_cycles_valu": tot["SQ_THREAD_CYCLES_VALU"],
           "sq_insts_valu_trans_f32": tot["SQ_INSTS_VALU_TRANS_F32"],
           "lane_instr_per_crossing": tot["SQ_THREAD_CYCLES_VALU"] / crossings_per_step,
           "wave_instr_per_crossing": tot["SQ_INSTS_VALU"] * 64 / crossings_per_step,
           "lane_utilisation": tot["SQ_THREAD_CYCLES_VALU"] / (64 * tot["SQ_INSTS_VALU"]),
           "trans_per_crossing": tot["SQ_INSTS_VALU_TRANS_F32"] * 64 / crossings_per_step,
           "valu_issue_frac": cycles / (VALU_SIMDS * CLOCK_HZ * secs)}
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def measured_atomics(workload: str):
    """The march's L2 atomic requests against the atomic microbenchmark's, from
    the committed rocprofv3 counter summary, if it was taken on the current
    kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"march_{workload}_atomics.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return {k: d[k] for k in ("march_l2_atomics_per_launch", "march_l2_atomics_per_s", "microbench_l2_atomics_per_s",
                              "frac", "march_lds_atomic_instr_per_crossing")}


def atomics_summary(db_dir: str, crossings_per_step: float, out_path: str):
    """The march's atomic co-roofline from a rocprofv3 --pmc run of
    TCC_ATOMIC_sum and SQ_INSTS_LDS_ATOMIC over this benchmark: L2 atomic
    requests per second of the march launches of the last step against those
    of the random-address FP32 atomic microbenchmark run before timing (its
    best dispatch), and the march's LDS atomic wave-instructions per
    crossing (times 64)."""
    import glob
    import sqlite3
    dbs = glob.glob(os.path.join(db_dir, "**", "*.db"), recursive=True)
    con = sqlite3.connect(dbs[0])
    q = ("select dispatch_id, kernel_name, counter_name, sum(value), min(start), max(end) from counters_collection "
         "group by dispatch_id, counter_name order by dispatch_id")
    per = {}
    for did, name, cname, val, t0, t1 in con.execute(q):
        d = per.setdefault(did, {"name": name, "t0": t0, "t1": t1, "c": {}})
        d["c"][cname] = val
    ds = [per[k] for k in sorted(per)]
    mb = [d for d in ds if "k_mb_atomic" in d["name"]]
    mb_rate = max(d["c"].get("TCC_ATOMIC_sum", 0.0) / ((d["t1"] - d["t0"]) * 1e-9) for d in mb)
    last_seed = max(i for i, d in enumerate(ds) if "k_seed<" in d["name"])
    brick = [d for d in ds[last_seed:] if "k_brick" in d["name"]]
    tcc = sum(d["c"].get("TCC_ATOMIC_sum", 0.0) for d in brick)
    lds = sum(d["c"].get("SQ_INSTS_LDS_ATOMIC", 0.0) for d in brick)
    secs = sum((d["t1"] - d["t0"]) * 1e-9 for d in brick)
    out = {"kernel": "k_brick (march)", "kernel_source_hash": kernel_source_hash(), "launches": len(brick),
           "march_l2_atomics_per_launch": tcc / max(len(brick), 1), "march_l2_atomics_per_s": tcc / secs,
           "microbench_l2_atomics_per_s": mb_rate, "frac": (tcc / secs) / mb_rate,
           "march_lds_atomic_instr_per_crossing": lds * 64 / crossings_per_step,
           "kernel_seconds": secs}
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def measured_traffic(workload: str):
    """HBM bytes per march launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"march_{workload}_traffic.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def _pmc_per_dispatch(db_dir: str):
    """(kernel name, {counter: value}) per dispatch, in dispatch order, from
    a rocprofv3 --pmc run's SQLite output."""
    import glob
    import sqlite3
    dbs = glob.glob(os.path.join(db_dir, "**", "*.db"), recursive=True)
    if not dbs:
        raise FileNotFoundError(f"no rocprofv3 database under {db_dir}")
    con = sqlite3.connect(dbs[0])
    per = {}
    q = "select dispatch_id, name, counter_name, counter_value from pmc_events order by dispatch_id"
    for did, name, cname, val in con.execute(q):
        d = per.setdefault(did, [name, {}])
        d[1][cname] = d[1].get(cname, 0.0) + val
    return [per[k] for k in sorted(per)]


def pmc_summary(fetch_dir: str, write_dir: str, copy_mib: int, out_path: str):
    """HBM bytes per march launch of the last timed step, from FETCH_SIZE and
    WRITE_SIZE runs (KiB per dispatch) scaled by what the same counters read
    for the plain copy of copy_mib MiB made before timing."""
    res = {}
    for tag, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        ds = _pmc_per_dispatch(d)
        copies = [c[counter] for n, c in ds if "copyBuffer" in n and counter in c]
        if not copies:
            raise RuntimeError(f"{d}: no calibration copy found")
        scale = copy_mib * 1024.0 / max(copies)
        last_seed = max(i for i, (n, _) in enumerate(ds) if "k_seed<" in n)
        brick = [c[counter] for n, c in ds[last_seed:] if "k_brick" in n]
        res[tag] = {"kib_per_step": sum(brick), "launches": len(brick), "scale": scale}
    n = res["fetch"]["launches"]
    per_launch = (res["fetch"]["kib_per_step"] * res["fetch"]["scale"]
                  + res["write"]["kib_per_step"] * res["write"]["scale"]) * 1024.0 / max(n, 1)
    out = {"kernel": "k_brick (march)", "kernel_source_hash": kernel_source_hash(),
           "bytes_per_launch": per_launch, "launches_per_step": n,
           "fetch_kib_per_step": res["fetch"]["kib_per_step"], "write_kib_per_step": res["write"]["kib_per_step"],
           "fetch_scale": res["fetch"]["scale"], "write_scale": res["write"]["scale"]}
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def cpu_baseline(prob, n_sample: int, threads: int):
    from oracle import oracle as O
    from paper_2409_04521_amd import workloads as W

    o = O.Oracle(**prob.oracle_kwargs(), n_chunks=max(threads, 1))
    o.set_sources(prob.src_pos_cm[:n_sample], prob.ndot_bins[:n_sample])
    t0 = time.perf_counter()
    o.step(prob.dt_s, W.rotation_uniforms(prob.seed, 0, n_sample), threads=threads)
    dt = time.perf_counter() - t0
    cross = o.last_crossings()
    out = {"value": cross / dt, "unit": "crossings/s", "cores": threads, "kind": "oracle",
           "sample": f"first {n_sample} of {prob.n_src} sources, full {prob.shape[2]}^3 grid, 1 step, "
                     f"{cross} crossings in {dt:.1f} s (FP64 C oracle, OpenMP)"}
    # the same oracle on one thread, over a sixteenth of the sample
    n1 = max(1, n_sample // 16)
    o1 = O.Oracle(**prob.oracle_kwargs(), n_chunks=1)
    o1.set_sources(prob.src_pos_cm[:n1], prob.ndot_bins[:n1])
    t0 = time.perf_counter()
    o1.step(prob.dt_s, W.rotation_uniforms(prob.seed, 0, n1), threads=1)
    dt1 = time.perf_counter() - t0
    c1 = o1.last_crossings()
    out["single_thread"] = {"value": c1 / dt1, "unit": "crossings/s", "cores": 1,
                            "sample": f"first {n1} sources, same grid, 1 step, {c1} crossings in {dt1:.1f} s"}
    return out


def cpu_baseline_configs(threads: int, c4_boxes: int = 8):
    """The CPU-baseline leg per configuration: the FP64 oracle on `threads`
    host threads and on one, beside the GPU, on C1 (32^3 Stromgren box,
    50 steps, the GPU in FP64 and FP32), C2 (128^3 lognormal box, 64
    sources, 100 steps), C3a (256^3 GRF, 2000 sources from neutral at c, 20
    steps) and the first `c4_boxes` boxes of C4 one at a time (50 steps
    each).  Each row: ms per step and crossings per step of each side, whose
    crossing counts agree up to FP32 face ties.  With host threads the
    oracle keeps one rate field per source chunk (a deterministic sum),
    whose clearing and reduction dominate a step whose packets die near
    their sources; on one thread it keeps one."""
    from oracle import oracle as O
    from paper_2409_04521_amd import frt
    from paper_2409_04521_amd import workloads as W

    ctx = frt.Context(0)

    def gpu(probs, precision, steps):
        t, c = 0.0, 0
        for p in probs:
            g = frt.solve_from_problem(ctx, p, precision=precision)
            g.sync()
            t0 = time.perf_counter()
            for _ in range(steps):
                g.step(p.dt_s)
            g.sync()
            t += time.perf_counter() - t0
            c += g.ledger()["crossings"]
            g.close()
        n = steps * len(probs)
        return {"ms_per_step": 1e3 * t / n, "crossings_per_step": c / n, "steps": n, "precision": precision}

    def oracle(probs, steps, nthreads):
        t, c = 0.0, 0
        for p in probs:
            o = O.Oracle(**p.oracle_kwargs(), n_chunks=max(nthreads, 1))
            o.set_sources(p.src_pos_cm, p.ndot_bins)
            for k in range(steps):
                t0 = time.perf_counter()
                o.step(p.dt_s, p.uniforms(k), threads=nthreads)
                t += time.perf_counter() - t0
                c += o.last_crossings()
            o.close()
        n = steps * len(probs)
        return {"ms_per_step": 1e3 * t / n, "crossings_per_step": c / n, "steps": n, "threads": nthreads}

    rows = []
    cases = [("C1", "32^3 Stromgren, corner source, 1 bin, dt 2 Myr, FP64 oracle", [W.stromgren_c1()], 50,
              ("f64", "f32")),
             ("C2", "128^3 lognormal, 64 sources, 4 bins, sub-grid kappa, c, dt 1 Myr", [W.lognormal_c2()], 100,
              ("f32",)),
             ("C3a", "256^3 GRF, 2000 peak sources, 4 bins, from neutral at c, dt 1 Myr",
              [W.grf_c3(throughput=False)], 20, ("f32",)),
             (f"C4 (first {c4_boxes} boxes)", "uneven boxes 32-128^3, 1-256 sources, 3 bins, c, dt 1 Myr, one at a time",
              W.batch_c4()[:c4_boxes], 50, ("f32",))]
    for name, what, probs, steps, precs in cases:
        row = {"config": name, "workload": what}
        for pr in precs:
            row[f"gpu_{pr}"] = gpu(probs, pr, steps)
        row["oracle"] = oracle(probs, steps, threads)
        row["oracle_1_thread"] = oracle(probs, steps, 1)
        g = row[f"gpu_{precs[0]}"]
        row["oracle_over_gpu_time"] = row["oracle"]["ms_per_step"] / g["ms_per_step"]
        log(f"{name}: GPU {g['ms_per_step']:.2f} ms/step, oracle {row['oracle']['ms_per_step']:.1f} ms/step on "
            f"{threads} threads, {row['oracle_1_thread']['ms_per_step']:.1f} on one; crossings/step "
            f"{g['crossings_per_step']:.4g} vs {row['oracle']['crossings_per_step']:.4g}")
        rows.append(row)
    return rows


def avgchem_leg(frt, W, K: int, steps: int, warmup: int, stream):
    """Standard Mode with the time-averaged chemistry (K marches per step)
    against backward Euler (one march) on the same evolving 128^3 box with
    finite c and sub-grid opacity: ms per step of both, and the HBM rate of
    the chemistry kernels (per cell: 28 B before the first march, 44 B after
    each later one: Gamma f32, n_H, x and <x> f64, opacity f32)."""
    import numpy as np
    import torch

    prob = W.lognormal_c2(n_steps=warmup + steps)
    out = {"workload": f"{prob.name}: {prob.shape[2]}^3, {prob.n_src} sources, 4 bins, kappa_sub, c, dt 1 Myr",
           "iterations": K, "steps": steps, "warmup": warmup}
    xs = {}
    for k in (0, K):
        prob.chem_iterations = k
        ctx = frt.Context(0)
        s = frt.solve_from_problem(ctx, prob, stream=stream.cuda_stream)
        for _ in range(warmup):
            s.step(prob.dt_s)
        s.sync()
        s.set_timing(True)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            s.step(prob.dt_s)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        tm = s.timing()
        tag = "avg" if k else "be"
        out[f"{tag}_ms_per_step"] = ms
        out[f"{tag}_march_ms_per_step"] = tm["march_ms"] / steps
        out[f"{tag}_chem_ms_per_step"] = tm["chem_ms"] / steps
        if k:
            chem_bytes = prob.ncell * (28 + 44 * k)
            out["avg_chem_bytes_per_step"] = chem_bytes
            out["avg_chem_GBps"] = chem_bytes / (tm["chem_ms"] / steps * 1e-3) / 1e9
            out["avg_chem_hbm_frac"] = out["avg_chem_GBps"] / HBM_PEAK_GBS
        L = s.ledger()
        out[f"{tag}_ledger_closure"] = abs(L["emitted"] - L["absorbed_HI"] - L["absorbed_sub"] - L["escaped"]
                                           - L["dropped"] - L["in_flight"] - L["lost"]) / L["emitted"]
        xs[k] = s.fields()[0]
        s.close()
        ctx.close()
    out["cost_ratio"] = out["avg_ms_per_step"] / out["be_ms_per_step"]
    out["mean_x_HI"] = {"be": float(np.mean(xs[0])), "avg": float(np.mean(xs[K]))}
    return out


def temperature_leg(frt, W, steps: int, warmup: int, stream):
    """The cost of the temperature evolution (§4.1, §4.2) on the C2 box
    (128^3, 64 sources, 4 bins, sub-grid kappa, finite c), each opacity mode
    with the temperature off and on: gas from 1e4 K; in Standard Mode the
    heat per photon of a 5e4 K blackbody, in the Generalized Opacity Mode
    T_reion 2e4 K and spectral index 1.5; Hubble (3.3e-17 /s) and Compton
    (z = 8) cooling.  ms per step, and the march's and the chemistry
    kernels' ms per step, of each."""
    import numpy as np
    import torch

    out = {"steps": steps, "warmup": warmup}
    for mode in (0, 1):
        for temp in (False, True):
            prob = W.lognormal_c2(n_steps=warmup + steps)
            prob.opacity_mode, prob.he_chi = mode, (0.08 if mode else 0.0)
            if temp:
                prob.temperature = True
                prob.heat_ev = W.blackbody_heat(prob.n_bins, T_bb=5e4)
                prob.T = np.full(prob.shape, 1e4, np.float32)
                prob.hubble_s, prob.cmb_z = 3.3e-17, 8.0
            ctx = frt.Context(0)
            s = frt.solve_from_problem(ctx, prob, stream=stream.cuda_stream)
            for _ in range(warmup):
                s.step(prob.dt_s)
            s.sync()
            s.set_timing(True)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                s.step(prob.dt_s)
            e1.record(stream)
            torch.cuda.synchronize()
            tm = s.timing()
            tag = f"{'generalized' if mode else 'standard'}_{'T' if temp else 'fixed_T'}"
            out[tag] = {"ms_per_step": e0.elapsed_time(e1) / steps, "march_ms_per_step": tm["march_ms"] / steps,
                        "chem_ms_per_step": tm["chem_ms"] / steps}
            if temp:
                T = s.temperature()
                out[tag]["T_range_K"] = [float(T.min()), float(T.max())]
                out["workload"] = (f"{prob.name}: {prob.shape[2]}^3, {prob.n_src} sources, 4 bins, kappa_sub, c, "
                                   "dt 1 Myr")
            s.close()
            ctx.close()
    for m in ("standard", "generalized"):
        out[f"{m}_cost_ratio"] = out[f"{m}_T"]["ms_per_step"] / out[f"{m}_fixed_T"]["ms_per_step"]
    return out


def genopacity_leg(frt, W, steps: int, warmup: int, stream):
    """The Generalized Opacity Mode on the C2 box (128^3, 64 sources, 4 bins,
    finite c): every cell starts neutral behind its moving screen, the
    ionized gas absorbs with the box's sub-grid kappa.  Against Standard Mode
    with the same kappa as sub-grid opacity on the same box (both run the
    16^3 sub-grid march): ms per step, crossings/s, the share of photons
    stopped at fronts, and the chemistry kernel's HBM rate (48 B per cell:
    front count, x, n_H read; x, the staged ionized fraction, the cleared
    front count and rate written)."""
    import torch

    out = {"steps": steps, "warmup": warmup}
    for mode in (0, 1):
        prob = W.lognormal_c2(n_steps=warmup + steps)
        prob.opacity_mode, prob.he_chi = mode, (0.08 if mode else 0.0)
        ctx = frt.Context(0)
        s = frt.solve_from_problem(ctx, prob, stream=stream.cuda_stream)
        for _ in range(warmup):
            s.step(prob.dt_s)
        s.sync()
        L0 = s.ledger()
        s.set_timing(True)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            s.step(prob.dt_s)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        tm = s.timing()
        L = s.ledger()
        tag = "generalized" if mode else "standard"
        if mode:
            out["workload"] = (f"{prob.name}: {prob.shape[2]}^3, {prob.n_src} sources, 4 bins, c, dt 1 Myr, "
                               f"all cells neutral at the start, ionized-gas kappa from the sub-grid recipe, chi 0.08")
            out["front_share_of_emitted"] = (L["absorbed_front"] - L0["absorbed_front"]) / (L["emitted"] - L0["emitted"])
            out["front_excess_share_of_emitted"] = ((L["front_excess"] - L0["front_excess"])
                                                    / (L["emitted"] - L0["emitted"]))
            out["chem_GBps"] = prob.ncell * 48 / (tm["chem_ms"] / steps * 1e-3) / 1e9
            out["chem_hbm_frac"] = out["chem_GBps"] / HBM_PEAK_GBS
            out["mean_x_ion"] = float(1.0 - s.fields()[0].mean())
        out[f"{tag}_ms_per_step"] = ms
        out[f"{tag}_crossings_per_s"] = (L["crossings"] - L0["crossings"]) / (ms * steps * 1e-3)
        out[f"{tag}_ledger_closure"] = abs(L["emitted"] - L["absorbed_HI"] - L["absorbed_sub"] - L["absorbed_front"]
                                           - L["front_excess"] - L["escaped"] - L["dropped"] - L["in_flight"]
                                           - L["lost"]) / L["emitted"]
        s.close()
        ctx.close()
    return out


def merge_leg(frt, W, steps: int, stream):
    """Ray merging (§3.3) where it pays: packets carried at c for many steps
    through ionized gas lit by many sources, so that every cell sees packets
    of many sources.  The C3 density field and source recipe at 128^3 with
    the C3 cell size and 2000 sources, x_HI = 1e-4 at the start, c_hat = c
    and dt = dx / c (one cell per step, the paper's stepping), N_min = 2, and
    the paper's merging-test parameters l_merge = 0, N_ex = 4.  Without and
    with merging: time of the whole run (the merge included) once a first
    pass has grown every queue (the run is repeated from a bookmark), packets
    carried and the largest pass at the end, the peak device memory of the
    library, and the change of the global means of x_HI and Gamma."""
    import numpy as np
    import torch

    out = {"steps": steps}
    res = {}
    for merge in (False, True):
        prob = W.grf_c3(n=128, n_src=2000, throughput=True, n_steps=steps, box_cmpc_h=50.0)
        prob.c_ray = W.C_LIGHT
        prob.dt_s = prob.dx_cm / W.C_LIGHT
        prob.n_ray_min = 2.0
        prob.merge, prob.merge_level, prob.merge_exempt = merge, 0, 4.0
        out["workload"] = (f"C3 field and sources at 128^3, 50 cMpc/h, 2000 sources, 4 bins, x_HI 1e-4 at the start, "
                           f"c, dt = dx/c = {prob.dt_s / 3.15576e13:.2f} Myr, N_min 2, l_merge 0, N_ex 4")
        # the library's device memory through torch's allocator, so that
        # torch's peak counter sees every buffer it holds
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        torch.cuda.reset_peak_memory_stats()
        base = torch.cuda.memory_allocated()
        ctx = frt.Context(0, allocator=frt.TorchAllocator(0))
        s = frt.solve_from_problem(ctx, prob, stream=stream.cuda_stream)
        # a first, untimed pass over the run grows every queue to its size;
        # the timed pass repeats it from the bookmarked start
        s.mark()
        t0 = time.perf_counter()
        for _ in range(steps):
            s.step(prob.dt_s)
        s.sync()
        first_s = time.perf_counter() - t0
        L0 = s.ledger()
        s.rewind()
        s.set_timing(True)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            s.step(prob.dt_s)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        tm = s.timing()
        L = s.ledger()
        x, g = s.fields()
        tag = "merged" if merge else "plain"
        out[f"{tag}_ms"] = ms
        out[f"{tag}_first_pass_ms"] = first_s * 1e3
        out[f"{tag}_march_ms"] = tm["march_ms"]
        out[f"{tag}_chem_ms"] = tm["chem_ms"]
        out[f"{tag}_other_ms"] = tm["emit_ms"] + tm["other_ms"]
        out[f"{tag}_carried_at_end"] = L["n_in_flight"]
        out[f"{tag}_largest_pass"] = L["max_items"]
        out[f"{tag}_ray_visits"] = L["ray_visits"] - L0["ray_visits"]
        out[f"{tag}_crossings"] = L["crossings"] - L0["crossings"]
        out[f"{tag}_device_peak_GB"] = (torch.cuda.max_memory_allocated() - base) / 1e9
        # the ledger of the first pass (it keeps counting across the rewind)
        out[f"{tag}_ledger_closure"] = abs(L0["emitted"] - L0["absorbed_HI"] - L0["absorbed_sub"] - L0["escaped"]
                                           - L0["dropped"] - L0["in_flight"] - L0["lost"]
                                           - L0["merge_residual"]) / L0["emitted"]
        if merge:
            out["merge_ms"] = tm["merge_ms"]
            out["merges"] = L["merges"] - L0["merges"]
            out["rays_merged"] = L["rays_merged"] - L0["rays_merged"]
        res[merge] = (float(np.mean(x)), float(np.mean(g.astype(np.float64))))
        s.close()
        ctx.close()
    out["speedup"] = out["plain_ms"] / out["merged_ms"]
    out["carried_ratio"] = out["plain_carried_at_end"] / max(1, out["merged_carried_at_end"])
    out["memory_ratio"] = out["plain_device_peak_GB"] / max(1e-9, out["merged_device_peak_GB"])
    out["mean_x_HI_rel_change"] = res[True][0] / res[False][0] - 1.0
    out["mean_gamma_rel_change"] = res[True][1] / res[False][1] - 1.0
    return out


def batched_leg(frt, W, n_boxes: int, steps: int, warmup: int, stream):
    """The uneven-box batch: the same boxes stepped one solve at a time (the
    plain per-solve path, once step by step with a host wait per step and
    once with each solve's steps replayed from its own HIP graph and checked
    only at the end) and as one batch replayed from a HIP graph with the
    autotuned launch shape, also checked only at the end.  Returns whole-run
    crossings/s of each and the largest x_HI difference between them."""
    import numpy as np
    import torch

    boxes = W.batch_c4(n_boxes=n_boxes, n_steps=warmup + steps)
    dts = [b.dt_s for b in boxes]

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    ctx = frt.Context(0)
    plain = [frt.solve_from_problem(ctx, b, stream=stream.cuda_stream) for b in boxes]
    for s, dt in zip(plain, dts):
        for _ in range(warmup):
            s.step(dt)
    c0 = sum(s.ledger()["crossings"] for s in plain)

    def run_plain():
        for s, dt in zip(plain, dts):
            for _ in range(steps):
                s.step(dt)
            s.sync()
    t_plain = timed(run_plain)
    c_plain = sum(s.ledger()["crossings"] for s in plain) - c0
    x_plain = [s.fields()[0] for s in plain]
    for s in plain:
        s.close()
    del plain

    ctx_g = frt.Context(0)
    plain_g = [frt.solve_from_problem(ctx_g, b, stream=stream.cuda_stream) for b in boxes]
    for s, dt in zip(plain_g, dts):
        frt.batch_run([s], [dt], warmup, graph=True)
    c0 = sum(s.ledger()["crossings"] for s in plain_g)

    def run_plain_graph():
        for s, dt in zip(plain_g, dts):
            frt.batch_run([s], [dt], steps, graph=True, check_every=steps)
    t_plain_g = timed(run_plain_graph)
    c_plain_g = sum(s.ledger()["crossings"] for s in plain_g) - c0
    dx_g = max(float(np.abs(a - s.fields()[0]).max()) for a, s in zip(x_plain, plain_g))
    for s in plain_g:
        s.close()
    del plain_g

    ctx_b = frt.Context(0)
    batch = [frt.solve_from_problem(ctx_b, b, stream=stream.cuda_stream) for b in boxes]
    frt.batch_run(batch, dts, warmup, graph=True)
    tuning = frt.autotune(batch, dts)
    c0 = sum(s.ledger()["crossings"] for s in batch)
    t_batch = timed(lambda: frt.batch_run(batch, dts, steps, graph=True, check_every=steps))
    c_batch = sum(s.ledger()["crossings"] for s in batch) - c0
    dx = max(float(np.abs(a - s.fields()[0]).max()) for a, s in zip(x_plain, batch))
    cells = sum(int(np.prod(b.shape)) for b in boxes)
    srcs = sum(b.n_src for b in boxes)
    for s in batch:
        s.close()
    return {"workload": f"{n_boxes} boxes, edges 32-128, {cells} cells, {srcs} sources, 3 bins, c, dt 1 Myr",
            "steps": steps, "warmup": warmup,
            "plain_crossings_per_s": c_plain / t_plain, "plain_s": t_plain,
            "plain_form": "one solve at a time, frt_step per step (waits on the host every step)",
            "plain_graph_crossings_per_s": c_plain_g / t_plain_g, "plain_graph_s": t_plain_g,
            "plain_graph_form": "one solve at a time, its steps replayed from its own HIP graph, "
                                "queue counters read once at the end of the run",
            "batched_crossings_per_s": c_batch / t_batch, "batched_s": t_batch,
            "speedup": (c_batch / t_batch) / (c_plain / t_plain) if c_plain else None,
            "speedup_vs_plain_graph": (c_batch / t_batch) / (c_plain_g / t_plain_g) if c_plain_g else None,
            "crossings": c_batch, "max_abs_dx_HI_batched_vs_plain": dx,
            "max_abs_dx_HI_plain_graph_vs_plain": dx_g,
            "batched_form": "one launch sequence per step over all boxes, replayed from a HIP graph, "
                            "queue counters read once at the end of the run",
            "tuning": tuning}


def served_leg(frt, W, n_req: int, steps: int, rate: float, budget_bytes: int, slots: int):
    """The Poisson request trace served two ways on one GPU: the plain
    per-solve path taking requests one at a time in arrival order (FIFO), and
    the continuous-batching server.  Latency = finish - arrival."""
    import numpy as np

    reqs = W.served_c5(n_requests=n_req, rate_per_s=rate, n_steps=steps)

    def pct(v, q):
        return float(np.percentile(np.asarray(v), q))

    def fifo(arrivals):
        ctx = frt.Context(0)
        lat = []
        t0 = time.perf_counter()
        for r, a in zip(reqs, arrivals):
            wait = a - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            s = frt.solve_from_problem(ctx, r.problem)
            for _ in range(steps):
                s.step(r.problem.dt_s)
            s.fields()
            s.close()
            lat.append(time.perf_counter() - t0 - a)
        t = time.perf_counter() - t0
        ctx.close()
        return lat, t

    def served(arrivals):
        ctx = frt.Context(0)
        srv = frt.Server(ctx, budget_bytes, slots)
        t0 = time.perf_counter()
        ids = []
        for r, a in zip(reqs, arrivals):
            wait = a - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            ids.append(srv.submit(r.problem, steps))
        lat = []
        for rid in ids:
            if srv.wait(rid, 600.0) != frt.REQ_DONE:
                raise RuntimeError(f"served request {rid} did not finish")
            ts = srv.times(rid)
            lat.append(ts[2] - ts[0])
            srv.take(rid)
        t = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        ctx.close()
        return lat, t, st

    out = {"workload": f"{n_req} Poisson requests at {rate}/s, edges 64-256, 16-2000 sources, {steps} steps each, "
                       "4 bins, sub-grid opacity, c", "budget_bytes": budget_bytes, "slots": slots}
    for tag, arrivals in (("trace", [r.arrival_s for r in reqs]), ("burst", [0.0] * len(reqs))):
        lf, tf = fifo(arrivals)
        ls, ts, st = served(arrivals)
        out[tag] = {"fifo_p50_s": pct(lf, 50), "fifo_p99_s": pct(lf, 99), "fifo_solves_per_s": n_req / tf,
                    "served_p50_s": pct(ls, 50), "served_p99_s": pct(ls, 99), "served_solves_per_s": n_req / ts,
                    "max_in_flight": st["max_in_flight"], "peak_bytes": st["peak_bytes"], "ticks": st["ticks"]}
    out["burst"]["arrivals"] = "all requests at t = 0"
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--sources", type=int, default=2000)
    ap.add_argument("--cpu-sample", type=int, default=128)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the uneven-box batch leg")
    ap.add_argument("--batched-boxes", type=int, default=64)
    ap.add_argument("--batched-steps", type=int, default=49)
    ap.add_argument("--batched-warmup", type=int, default=1)
    ap.add_argument("--no-avgchem", action="store_true", help="skip the time-averaged chemistry leg")
    ap.add_argument("--avgchem-iterations", type=int, default=3)
    ap.add_argument("--avgchem-steps", type=int, default=10)
    ap.add_argument("--no-genopacity", action="store_true", help="skip the Generalized Opacity Mode leg")
    ap.add_argument("--no-merge", action="store_true", help="skip the ray-merging leg")
    ap.add_argument("--no-temperature", action="store_true", help="skip the temperature-evolution leg")
    ap.add_argument("--merge-steps", type=int, default=60)
    ap.add_argument("--no-served", action="store_true", help="skip the served (request trace) leg")
    ap.add_argument("--served-requests", type=int, default=128)
    ap.add_argument("--served-steps", type=int, default=50)
    ap.add_argument("--served-rate", type=float, default=4.0)
    ap.add_argument("--served-budget-gb", type=float, default=64.0)
    ap.add_argument("--served-slots", type=int, default=64)
    ap.add_argument("--copy-calibration-mib", type=int, default=1024,
                    help="size of a plain device copy run before timing; its hardware byte counters "
                         "calibrate the march kernel's (0 = skip)")
    ap.add_argument("--pmc-valu", nargs=2, metavar=("DB_DIR", "CROSSINGS_PER_STEP"),
                    help="write profiles/march_c3b_valu.json from a rocprofv3 --pmc run of the VALU counters")
    ap.add_argument("--pmc-atomics", nargs=2, metavar=("DB_DIR", "CROSSINGS_PER_STEP"),
                    help="write profiles/march_c3b_atomics.json from a rocprofv3 --pmc run of TCC_ATOMIC_sum and "
                         "SQ_INSTS_LDS_ATOMIC")
    ap.add_argument("--config-table", action="store_true",
                    help="time the FP64 oracle (host threads and one thread) beside the GPU on C1, C2, C3a and "
                         "a C4 sample, print one JSON line and exit")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/march_c3b_traffic.json from two rocprofv3 --pmc runs of this "
                         "benchmark (FETCH_SIZE, WRITE_SIZE) and exit")
    args = ap.parse_args()
    if args.pmc_valu:
        valu_summary(args.pmc_valu[0], float(args.pmc_valu[1]), os.path.join(ROOT, "profiles", "march_c3b_valu.json"))
        return
    if args.pmc_atomics:
        atomics_summary(args.pmc_atomics[0], float(args.pmc_atomics[1]),
                        os.path.join(ROOT, "profiles", "march_c3b_atomics.json"))
        return
    if args.pmc_summary:
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.copy_calibration_mib,
                    os.path.join(ROOT, "profiles", "march_c3b_traffic.json"))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU form "
              "(sources sharded over GPUs, one reduction of the rate field per step) is not built.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2409_04521_amd import frt
    from paper_2409_04521_amd import workloads as W

    if args.config_table:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        rows = cpu_baseline_configs(threads)
        print(json.dumps({"config_table": rows, "host_threads": threads, "gpu": torch.cuda.get_device_name(0)}),
              flush=True)
        return

    log("building inputs")
    prob = W.grf_c3(n=args.n, n_src=args.sources, throughput=True, box_cmpc_h=100.0 * args.n / 256)
    torch.cuda.init()
    stream = torch.cuda.Stream()          # default priority; the library enqueues on it
    torch.cuda.set_stream(stream)
    ctx = frt.Context(0)
    # achievable device rates, the denominators beside the published peaks:
    # a 2 GiB streaming copy and random FP32 atomics over 2^24 slots (the
    # size of this workload's rate field)
    mb = frt.microbench(ctx, 2 << 30, 1 << 24)
    log(f"microbench: copy {mb['copy_GBps']:.0f} GB/s, FP32 atomics {mb['atomic_per_s']:.3e}/s at random addresses")
    # first size of the pass queues: the largest pass of this workload holds
    # 2.72e8 packets (reported as max_pass_packets); with a third more the
    # warm-up step never overflows and re-runs (64-byte records: 23 GB per queue)
    hint = int(3.6e8 * (args.n / 256) ** 3 * args.sources / 2000)
    s = frt.solve_from_problem(ctx, prob, stream=stream.cuda_stream, queue_hint=hint)
    # Every step starts from the configured state (rewound on the device):
    # from x_HI = 1e-4 the dense source cells recombine within one step
    # (their Stromgren radii are below a tenth of a cell), after which every
    # packet dies in its source cell, so only the first step from this state
    # carries the workload's crossings.
    s.mark()
    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    log(f"loaded {prob.name}; warmup {args.warmup} step(s)")
    for _ in range(args.warmup):
        s.rewind()
        s.step(prob.dt_s)
        log(f"warmup step done: {s.ledger()['step_crossings']} crossings")
    s.sync()
    L0 = s.ledger()
    s.set_timing(True)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for k in range(args.steps):
        s.rewind()
        s.step(prob.dt_s)
    ev1.record(stream)
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    L1 = s.ledger()
    tm = s.timing()
    cross = L1["crossings"] - L0["crossings"]
    log(f"timed {args.steps} steps: {total_ms:.1f} ms, {cross} crossings, march {tm['march_ms']:.1f} ms "
        f"over {tm['march_launches']} launches, chem {tm['chem_ms']:.2f} ms")
    value = cross / (total_ms * 1e-3)

    nb = prob.n_bins
    d_visits = L1["ray_visits"] - L0["ray_visits"]
    # per crossing: opacity gather and one FP32 deposit; per visit: the packet
    # record read and written (2 (36 + 8 n_b) B)
    march_bytes = ALG_BYTES_PER_CROSSING * cross + alg_bytes_per_visit(nb) * d_visits
    closure = abs(L1["emitted"] - L1["absorbed_HI"] - L1["absorbed_sub"] - L1["escaped"] - L1["dropped"]
                  - L1["in_flight"] - L1["lost"]) / L1["emitted"]
    launches = max(tm["march_launches"], 1)
    per_launch = march_bytes / launches
    avg_launch_s = tm["march_ms"] * 1e-3 / launches
    hbm_achieved = per_launch / avg_launch_s / 1e9
    # the march issues vector ALU work, not memory traffic, at its limit: the
    # roofline is the ALU one, with the algorithmic operations per crossing
    ops_per_launch = ALG_OPS_PER_CROSSING * cross / launches
    achieved = ops_per_launch / avg_launch_s / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 2), "unit": "TFLOP/s",
            "frac": round(achieved / VALU_PEAK_TOPS, 4), "traffic": measured_traffic("c3b"),
            "kernel": "k_brick", "avg_launch_ms": round(avg_launch_s * 1e3, 4), "launches": tm["march_launches"],
            "algorithmic_ops_per_crossing": ALG_OPS_PER_CROSSING, "algorithmic_ops_per_launch": round(ops_per_launch),
            "hbm": {"achieved": round(hbm_achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(hbm_achieved / HBM_PEAK_GBS, 5), "algorithmic_bytes_per_launch": round(per_launch),
                    "bytes": f"{ALG_BYTES_PER_CROSSING} B per crossing + {alg_bytes_per_visit(nb)} B per visit",
                    "achievable": round(mb["copy_GBps"], 1),
                    "frac_of_achievable": round(hbm_achieved / mb["copy_GBps"], 5)},
            "valu": measured_valu("c3b"),
            "atomic": {"microbench_fp32_random_per_s": mb["atomic_per_s"], "counters": measured_atomics("c3b")}}

    out = {"metric": METRIC, "value": value, "unit": "crossings/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": total_ms / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{prob.name}: GRF k^-2.5 ln-sigma 1.5, peaks as sources, x_HI=1e-4, "
                                  f"c=inf, {nb} bins, floor 1e-3, cap 50 cMpc/h, l_max 12",
                      "cells": prob.ncell, "sources": prob.n_src, "crossings_per_step": cross / args.steps,
                      "visits_per_step": d_visits / args.steps,
                      "splits_per_step": (L1["splits"] - L0["splits"]) / args.steps,
                      "escapes_per_step": (L1["n_escaped"] - L0["n_escaped"]) / args.steps,
                      "drops_per_step": (L1["n_dropped"] - L0["n_dropped"]) / args.steps,
                      "ledger_closure": closure,
                      "max_pass_packets": L1["max_items"],
                      "steps_start_from": "the configured state, rewound on the device before each step",
                      "parallelism": "single GPU"},
           "roofline": roof,
           "kernel_ms": {k: round(v, 3) for k, v in tm.items() if k.endswith("_ms")}}
    s.close()
    ctx.close()
    if not args.no_batched:
        log(f"batched leg: {args.batched_boxes} boxes, {args.batched_steps} steps")
        out["batched"] = batched_leg(frt, W, args.batched_boxes, args.batched_steps, args.batched_warmup, stream)
        bt = out["batched"]
        log(f"batched: {bt['batched_crossings_per_s']:.3e} crossings/s vs plain {bt['plain_crossings_per_s']:.3e} "
            f"(x{bt['speedup']:.2f}) and plain from per-solve graphs {bt['plain_graph_crossings_per_s']:.3e} "
            f"(x{bt['speedup_vs_plain_graph']:.2f})")
    if not args.no_avgchem:
        log(f"time-averaged chemistry leg: K = {args.avgchem_iterations}, {args.avgchem_steps} steps")
        out["avg_chem"] = avgchem_leg(frt, W, args.avgchem_iterations, args.avgchem_steps, 2, stream)
        ac = out["avg_chem"]
        log(f"time-averaged chemistry: {ac['avg_ms_per_step']:.2f} ms/step vs backward Euler "
            f"{ac['be_ms_per_step']:.2f} (x{ac['cost_ratio']:.2f}); chemistry kernels {ac['avg_chem_GBps']:.0f} GB/s")
    if not args.no_genopacity:
        log("generalized opacity leg: 10 steps")
        out["gen_opacity"] = genopacity_leg(frt, W, 10, 2, stream)
        go = out["gen_opacity"]
        log(f"generalized opacity: {go['generalized_ms_per_step']:.2f} ms/step, "
            f"{go['generalized_crossings_per_s']:.3e} crossings/s (standard mode on the same box "
            f"{go['standard_ms_per_step']:.2f} ms/step); {go['front_share_of_emitted']:.2f} of photons stopped "
            f"at fronts, mean x_ion {go['mean_x_ion']:.3f}")
    if not args.no_temperature:
        log("temperature leg: 10 steps per mode, temperature fixed and evolving")
        out["temperature"] = temperature_leg(frt, W, 10, 2, stream)
        te = out["temperature"]
        log("temperature: " + "; ".join(
            f"{m} {te[m + '_fixed_T']['ms_per_step']:.2f} -> {te[m + '_T']['ms_per_step']:.2f} ms/step (chemistry "
            f"{te[m + '_fixed_T']['chem_ms_per_step']:.3f} -> {te[m + '_T']['chem_ms_per_step']:.3f}, march "
            f"{te[m + '_fixed_T']['march_ms_per_step']:.2f} -> {te[m + '_T']['march_ms_per_step']:.2f})"
            for m in ("standard", "generalized")))
    if not args.no_merge:
        log(f"ray-merging leg: {args.merge_steps} steps without and with merging")
        out["merge"] = merge_leg(frt, W, args.merge_steps, stream)
        mg = out["merge"]
        log(f"ray merging: {mg['merged_ms']:.0f} ms vs {mg['plain_ms']:.0f} ms without (x{mg['speedup']:.2f}); "
            f"carried {mg['merged_carried_at_end']} vs {mg['plain_carried_at_end']}, device "
            f"{mg['merged_device_peak_GB']:.1f} vs {mg['plain_device_peak_GB']:.1f} GB at peak; mean x_HI {mg['mean_x_HI_rel_change']:+.1e}, "
            f"mean Gamma {mg['mean_gamma_rel_change']:+.1e}")
    if not args.no_served:
        log(f"served leg: {args.served_requests} requests, {args.served_steps} steps each")
        out["served"] = served_leg(frt, W, args.served_requests, args.served_steps, args.served_rate,
                                   int(args.served_budget_gb * (1 << 30)), args.served_slots)
        for tag in ("trace", "burst"):
            sv = out["served"][tag]
            log(f"served ({tag}) p50/p99 {sv['served_p50_s']:.2f}/{sv['served_p99_s']:.2f} s, "
                f"{sv['served_solves_per_s']:.2f} solves/s vs FIFO {sv['fifo_p50_s']:.2f}/{sv['fifo_p99_s']:.2f} s, "
                f"{sv['fifo_solves_per_s']:.2f} solves/s")
    if not args.no_cpu:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        log(f"cpu baseline: oracle on {args.cpu_sample} sources with {threads} threads")
        out["cpu_baseline"] = cpu_baseline(prob, min(args.cpu_sample, prob.n_src), threads)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
