#!/usr/bin/env python3
"""Benchmark: MCPT(2) solves per second on the 1000-monomer HF-lattice workload.

One step = one complete solve of the resident problem (initial guess, sweeps
of Eqs. 58-59 until max|dT| < 1e-10, final Eq. 59 energy pass, Eqs. 54-56).
Inputs are uploaded to HBM before the timed region.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MCPT(2) solves/s + pair-contraction GB/s at 1000 monomers; p50/p99 served latency"
PEAK = {"fp64": (78.6, "TFLOP/s"), "fp32": (157.3, "TFLOP/s"), "bf16": (2500.0, "TFLOP/s")}   # MI355X dense
HBM_PEAK_GBS = 8000.0
MEASURED = {}   # the device's measured FP64 pipe rates (mcpt_device_rates), set once by main


def pipe_roof(w_bytes, ms, o):
    """The ladder's other roof: each streamed 8-byte integral meets round16(o^2) amplitude columns on
    v_mfma_f64_16x16x4, so its padded MFMA work per launch is 2 round16(o^2) flops per element; the
    fraction of the matrix pipe's measured rate that this work reaches."""
    padded = w_bytes / 8.0 * 2.0 * ((o * o + 15) // 16 * 16)
    rate = MEASURED.get("mfma_f64_tflops")
    return {"padded_mfma_flops_per_launch": padded,
            "min_ms_at_measured_mfma_rate": padded / (rate * 1e12) * 1e3 if rate else None,
            "frac_of_measured_mfma_f64": padded / (ms * 1e-3) / (rate * 1e12) if rate else None}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def counted_traffic(sweeps: int):
    """HBM-side bytes per pair-kernel launch from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE passes (calibrated by a plain copy), averaged over
    the timed launch mix (`sweeps` coupled launches and one energy pass); None
    once the kernel sources differ from the ones the counters were taken on."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "pair_fp64_counters_hf-10x10x10-c3.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    for name, digest in re.findall(r"sha256 (\S+) ([0-9a-f]{64})", text):
        src = os.path.join(ROOT, "paper_1409_2700_amd", "csrc", name)
        if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != digest:
            return None
    c = re.search(r"coupled_bytes_per_launch: ([0-9.e+]+)", text)
    e = re.search(r"energy_bytes_per_launch: ([0-9.e+]+)", text)
    if not (c and e):
        return None
    return (sweeps * float(c.group(1)) + float(e.group(1))) / (sweeps + 1)


def cpu_baseline(prob, sweeps: int, budget_s: float = 12.0) -> dict:
    """The FP64 oracle as it stands, on a bounded sample of the same workload:
    bulk monomers and every pair touching them; Eq. 59 timed per pair and the
    Eq. 58 update timed per (monomer, neighbour), scaled to one full solve
    (sweeps + the final energy pass)."""
    from oracle import mcpt_oracle
    threads = oracle_threads()
    orc = mcpt_oracle.Oracle(prob)
    T = orc.first_order()
    deg = [len(nb) for nb in orc.nb]
    order = sorted(range(prob.n_mono), key=lambda x: -deg[x])
    t_pairs = t_monos = 0.0
    n_pairs = n_sides = 0
    monos = []
    done_pairs = {}
    start = time.perf_counter()
    for x in order:
        if time.perf_counter() - start > budget_s:
            break
        todo = [q for q, _ in orc.nb[x] if q not in done_pairs]
        t0 = time.perf_counter()
        for q, tau in zip(todo, orc.pair_phase(T, todo)):
            done_pairs[q] = tau
        t_pairs += time.perf_counter() - t0
        n_pairs += len(todo)
        t0 = time.perf_counter()
        orc.monomer_phase(done_pairs, [x])
        t_monos += time.perf_counter() - t0
        n_sides += deg[x]
        monos.append(x)
    per_pair = t_pairs / max(n_pairs, 1)
    per_side = t_monos / max(n_sides, 1)
    sweep_s = prob.n_pair * per_pair + 2 * prob.n_pair * per_side
    solve_s = sweeps * sweep_s + prob.n_pair * per_pair
    return {
        "value": 1.0 / solve_s, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
        "sample": (f"{len(monos)} bulk monomers and their {n_pairs} pairs: Eq. 59 per pair "
                   f"{per_pair * 1e3:.2f} ms, Eq. 58 per monomer-neighbour {per_side * 1e3:.2f} ms, "
                   f"scaled to {prob.n_pair} pairs x {sweeps} sweeps + final pass "
                   f"({solve_s:.0f} s per solve)"),
        "cpu": cpu_model(), "host_cores": os.cpu_count(),
        "seconds_measured": t_pairs + t_monos,
    }


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo), else the machine type."""
    fields = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                key, _, val = line.partition(":")
                key = key.strip()
                if key in ("model name", "cpu family", "model", "stepping", "cpu MHz") and key not in fields:
                    fields[key] = val.strip()
                if not line.strip() and fields:
                    break
    except OSError:
        pass
    if "model name" not in fields:
        return platform.processor() or platform.machine()
    extra = ", ".join(f"{k} {fields[k]}" for k in ("cpu family", "model", "stepping", "cpu MHz") if k in fields)
    return f"{fields['model name']} ({extra})" if extra else fields["model name"]


def oracle_threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        return int(max([i.get("num_threads", 1) for i in threadpool_info()] or [1]))
    except Exception:
        return os.cpu_count() or 1


def small_configs(tol, with_cpu: bool) -> dict:
    """The 8- and 125-monomer crystals: FP64 GPU solves (median of 5, inputs
    resident) and, beside them, one full solve of the oracle as it stands on the
    host cores, with the agreement of the two."""
    import numpy as np
    import paper_1409_2700_amd as mc
    from oracle import mcpt_oracle
    from synth import make_workload
    out = {}
    for name in ("hf-2x2x2", "hf-5x5x5-c2"):
        prob = make_workload(name)
        with mc.Context(0) as ctx:
            pid = ctx.upload(prob)
            ctx.run(pid, tol=tol)
            times = []
            for _ in range(5):
                t0 = time.perf_counter()
                s = ctx.run(pid, tol=tol)
                times.append(time.perf_counter() - t0)
            ctx.release(pid)
        g = {"n_mono": prob.n_mono, "n_pair": prob.n_pair, "sweeps": s["sweeps"], "e_total": s["e_total"],
             "gpu_fp64_solves_per_s": 1.0 / float(np.median(times))}
        if with_cpu:
            t0 = time.perf_counter()
            r = mcpt_oracle.solve(prob, tol=tol)
            secs = time.perf_counter() - t0
            g["cpu_oracle"] = {"value": 1.0 / secs, "unit": "solves/s", "seconds": secs, "cores": oracle_threads(),
                               "kind": "oracle", "sample": "one full solve", "cpu": cpu_model()}
            g["rel_diff_vs_oracle"] = abs(s["e_total"] - r.e_total) / abs(r.e_total)
            g["sweeps_equal"] = s["sweeps"] == r.sweeps
            g["gpu_vs_oracle"] = g["gpu_fp64_solves_per_s"] / g["cpu_oracle"]["value"]
        log(f"[small] {name}: GPU {g['gpu_fp64_solves_per_s']:.1f} solves/s"
            + (f", oracle {g['cpu_oracle']['seconds']:.2f} s per solve" if with_cpu else ""))
        out[name] = g
    return out


MODES = {   # name: (precision, polish)
    "fp64": (0, 1),
    "bf16+polish": (2, 1),
    "fp32+polish": (1, 1),
}


def time_mode(ctx, pid, name, steps, warmup, tol, check_every, golden, graph=0):
    import numpy as np
    prec, polish = MODES[name]
    opts = dict(tol=tol, max_sweeps=200, check_every=check_every, precision=prec, polish=polish, graph=graph,
                autotune=1)
    for w in range(warmup):
        s = ctx.run(pid, **opts)
        log(f"[bench] {name} warmup {w}: {s['sweeps']} sweeps ({s['polish_sweeps']} FP64) "
            f"{s['seconds'] * 1e3:.1f} ms E={s['e_total']:.10f}")
    ctx.set_timing(True)
    t0 = time.perf_counter()
    runs = [ctx.run(pid, **opts) for _ in range(steps)]
    elapsed = time.perf_counter() - t0
    if graph:   # replayed graphs carry no per-launch events: one eager solve gives the kernel times
        ctx.set_timing(False)
        ctx.set_timing(True)
        ctx.run(pid, **dict(opts, graph=0))
        steps_timed = 1
    else:
        steps_timed = steps
    tm = ctx.timing()
    ctx.set_timing(False)
    s = runs[-1]
    for k, r in enumerate(runs):
        log(f"[bench] {name} step {k}: {r['sweeps']} sweeps {r['seconds'] * 1e3:.1f} ms")
    out = {
        "solves_per_s": steps / elapsed, "ms_per_solve": elapsed / steps * 1e3, "sweeps": s["sweeps"],
        "fp64_sweeps": s["sweeps"] if prec == 0 else s["polish_sweeps"], "e_total": s["e_total"],
        "fp64_pair_avg_ms": tm["pair_ms"] / max(tm["pair_launches"], 1),
        "fp64_pair_launches_per_solve": tm["pair_launches"] / steps_timed,
        "lowp_pair_avg_ms": tm["lowp_ms"] / max(tm["lowp_launches"], 1) if tm["lowp_launches"] else None,
        "lowp_pair_launches_per_solve": tm["lowp_launches"] / steps_timed,
        "monomer_avg_ms": tm["mono_ms"] / max(tm["mono_launches"], 1),
        "timing": tm,
    }
    if golden is not None:
        e = ctx.energy(pid, want_t=False)
        out["error_vs_oracle_Eh"] = {
            "e_total": abs(s["e_total"] - golden["e_total"]),
            "e_mono": abs(s["e_mono"] - golden["e_mono"]),
            "e_dimer": abs(s["e_dimer"] - golden["e_dimer"]),
            "max_e_m2": float(np.max(np.abs(e["e_m2"] - np.asarray(golden["e_m2"])))),
            "max_e_d2_sampled": float(np.max(np.abs(np.asarray(e["e_d2"])[golden["pair_index"]]
                                                    - np.asarray(golden["e_d2"])))),
        }
        out["relative_error_e_total"] = out["error_vs_oracle_Eh"]["e_total"] / abs(golden["e_total"])
    return out


def pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else None


def _served_pass(ctx, stream, n_req, arrivals, max_inflight, tol, alone_e):
    """Submit requests 0..n_req-1 (at the given arrival times, or as fast as the
    in-flight limit lets them: closed loop), collect them on a polling thread, and
    return latencies (the library's, from submission to result), completion and
    submission times, statuses and the relative difference from the alone energy."""
    import threading
    cv = threading.Condition()
    outstanding = {}
    lat, err, status = [None] * n_req, [None] * n_req, [None] * n_req
    done_t, sub_t = [None] * n_req, [None] * n_req
    state = {"done": 0, "submit_s": 0.0}

    def poller():
        while True:
            with cv:
                if state["done"] == n_req:
                    return
                items = list(outstanding.items())
            progressed = False
            for t, r in items:
                s = ctx.poll(t)
                if s is None:
                    continue
                done_t[r] = time.perf_counter()
                lat[r], status[r] = s["seconds"], s["status"]
                err[r] = abs(s["e_total"] - alone_e[r]) / abs(alone_e[r])
                ctx.release(t)
                with cv:
                    del outstanding[t]
                    state["done"] += 1
                    cv.notify_all()
                progressed = True
            if not progressed:
                time.sleep(0.0005)

    th = threading.Thread(target=poller)
    th.start()
    start = time.perf_counter()
    for r in range(n_req):
        if arrivals is not None:
            delay = start + arrivals[r] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
        with cv:
            cv.wait_for(lambda: len(outstanding) < max_inflight)
        sub_t[r] = time.perf_counter() - start
        with stream.lend(r) as p:
            t = ctx.submit(p, tol=tol)
        state["submit_s"] += time.perf_counter() - start - sub_t[r]
        with cv:
            outstanding[t] = r
    th.join()
    return start, lat, err, status, done_t, sub_t, state["submit_s"]


def serving(base, n_req, loads, workers, max_batch, tol, max_inflight=32, staging_bytes=64 << 30, mode=None,
            compare=(0,)):
    """Served stream (synth.ServedStream: requests cut from the resident crystal,
    sizes log-uniform in [8, N], one monomer displaced), first solved alone one at
    a time on the plain FP64 path (upload + solve), then submitted in a closed
    loop with at most max_inflight requests in flight (capacity: requests over
    the makespan), then with Poisson arrivals at the given fractions of that
    measured capacity.  Requests are lent as views of the relabelled crystal, so
    host memory holds only the in-flight copies the library makes at submission,
    in pinned staging blocks up to staging_bytes (mcpt_serve_staging)."""
    import numpy as np
    import paper_1409_2700_amd as mc
    from synth import ServedStream, SEED_ROOT

    t0 = time.time()
    stream = ServedStream(base)
    draws = [stream.draw(r) for r in range(n_req)]
    sizes = [d[0] for d in draws]
    pairs = [int(stream.pairs_below[n]) for n in sizes]
    log(f"[serve] {n_req} requests, monomers {min(sizes)}..{max(sizes)} (mean {np.mean(sizes):.0f}), "
        f"pairs mean {np.mean(pairs):.0f}, stream prepared in {time.time() - t0:.1f}s")
    alone = []
    with mc.Context(0) as ctx:
        with stream.lend(0) as p:   # untimed warm-up
            pid, _ = ctx.solve(p, tol=tol)
        ctx.release(pid)
        for r in range(n_req):
            with stream.lend(r) as p:
                t1 = time.perf_counter()
                pid, s = ctx.solve(p, tol=tol)
                alone.append((time.perf_counter() - t1, s["e_total"], s["sweeps"]))
            ctx.release(pid)
    alone_lat = [a[0] for a in alone]
    alone_e = [a[1] for a in alone]
    mean_alone = float(np.mean(alone_lat))
    out = {
        "requests": n_req, "monomers": {"min": int(min(sizes)), "mean": float(np.mean(sizes)),
                                         "max": int(max(sizes))},
        "pairs": {"mean": float(np.mean(pairs)), "max": int(max(pairs))},
        "workload": f"cut from the {base.n_mono}-monomer crystal: the n monomers nearest its centre, n "
                    f"log-uniform in [8, {base.n_mono}], every pair among them, one monomer displaced +-0.01 A",
        "alone": {"p50_s": pct(alone_lat, 50), "p99_s": pct(alone_lat, 99), "mean_s": mean_alone,
                  "solves_per_s": 1.0 / mean_alone, "samples": n_req,
                  "path": "mcpt_solve, one at a time (upload + FP64 solve)"},
        "workers": workers, "max_batch": max_batch, "loads": {},
    }
    log(f"[serve] alone: mean {mean_alone * 1e3:.1f} ms, p50 {pct(alone_lat, 50) * 1e3:.1f} ms")
    capacity = None

    def scheduler(mode):
        # one scheduler for several passes, so the pinned staging blocks made for the first requests are
        # reused; an untimed closed-loop pass over the first max_inflight requests makes them
        c = mc.Context(0)
        c.serve_config(workers=workers, max_batch=max_batch)
        c.serve_staging(staging_bytes)
        c.serve_tick_mode(mode)
        t0 = time.perf_counter()
        _served_pass(c, stream, min(n_req, max_inflight), None, max_inflight, tol, alone_e)
        return c, time.perf_counter() - t0

    modes = {mc.MCPT_SERVE_BATCH_END: "batch_end", mc.MCPT_SERVE_RETIRE_AT_TICKS: "retire_at_ticks",
             mc.MCPT_SERVE_JOIN_AT_TICKS: "join_at_ticks"}
    if mode is None:
        mode = mc.MCPT_SERVE_RETIRE_AT_TICKS   # the library's default
    ctx, warm_s = scheduler(mode)
    out["staging"] = {"cap_bytes": staging_bytes, "warmup_s": warm_s,
                      "pinned_bytes": ctx.serve_stats()["staging_pinned_bytes"]}
    out["tick_mode"] = modes[mode]
    out["tick_modes"] = ("batch_end: a batch's requests are reported when its last one stops; retire_at_ticks: "
                         "each request retires at the sweep tick where its solve stops; join_at_ticks: also "
                         "admits queued requests into running batches at ticks (below saturation)")
    extra = {f"capacity_{modes[m]}": m for m in modes if m != mode and m in compare}
    for load in ["capacity"] + [x for x in loads if x != "burst"] + list(extra):
        if load in extra:
            ctx.close()
            ctx, _ = scheduler(extra[load])
        if isinstance(load, str):
            arrivals, cap = None, max_inflight
        else:
            rng = np.random.default_rng([SEED_ROOT, 5, int(round(load * 1000))])
            arrivals, cap = np.cumsum(rng.exponential(1.0 / (load * capacity), n_req)), 2 * max_inflight
        st0 = ctx.serve_stats()
        start, lat, err, status, done_t, sub_t, sub_s = _served_pass(ctx, stream, n_req, arrivals, cap, tol, alone_e)
        st = ctx.serve_stats()
        makespan = max(done_t) - start
        key = load if isinstance(load, str) else f"{load:.2f}"
        entry = {"completed_solves_per_s": n_req / makespan, "p50_s": pct(lat, 50), "p99_s": pct(lat, 99),
                 "mean_s": float(np.mean(lat)), "batches": st["batches"] - st0["batches"],
                 "joined_at_ticks": st["joined_at_ticks"] - st0["joined_at_ticks"], "samples": n_req,
                 "all_ok": all(w == 0 for w in status), "max_rel_err_vs_alone": float(max(err)),
                 "submit_s": sub_s, "submit_share_of_makespan": sub_s / makespan,
                 "staging_pinned_bytes": st["staging_pinned_bytes"], "staged_pageable": st["staged_pageable"]}
        if load in extra:
            entry["max_in_flight"] = cap
            entry["vs_default_capacity"] = (n_req / makespan) / capacity
        elif load == "capacity":
            capacity = n_req / makespan
            out["capacity_solves_per_s"] = capacity
            out["capacity_vs_alone"] = capacity * mean_alone
            entry["max_in_flight"] = cap
        else:
            late = [max(0.0, sub_t[r] - arrivals[r]) for r in range(n_req)]
            entry.update({"offered_solves_per_s": load * capacity, "submission_delay_p99_s": pct(late, 99)})
        out["loads"][key] = entry
        log(f"[serve] {key}: {n_req / makespan:.2f} solves/s, p50 {pct(lat, 50) * 1e3:.1f} ms, "
            f"p99 {pct(lat, 99) * 1e3:.1f} ms, {entry['batches']} batches, {entry['joined_at_ticks']} joined at "
            f"ticks, max rel err {max(err):.1e}, submit {sub_s:.1f} s of {makespan:.1f} s")
    ctx.close()
    return out


def batched(n_clusters, tol):
    """Batching form: uneven cubic-lattice clusters (27..512 monomers, o5v27 /
    o8v56 half and half) uploaded as one batch; tile shape autotuned, sweeps
    graph-captured; FP32 polish and plain FP64 timed on the same batch, the
    stored oracle clusters (tests/golden/batch-64.json) compared."""
    import numpy as np
    import paper_1409_2700_amd as mc
    from synth import make_cluster_batch

    t0 = time.time()
    probs = make_cluster_batch(n_clusters, workers=min(16, os.cpu_count() or 1))
    n_mono = sum(p.n_mono for p in probs)
    n_pair = sum(p.n_pair for p in probs)
    vbytes = sum(p.v.nbytes for p in probs)
    log(f"[batch] {n_clusters} clusters, {n_mono} monomers, {n_pair} pairs, V {vbytes / 1e9:.1f} GB "
        f"made in {time.time() - t0:.0f}s")
    golden = None
    gpath = os.path.join(ROOT, "tests", "golden", "batch-64.json")
    if n_clusters == 64 and os.path.exists(gpath):
        with open(gpath) as f:
            golden = json.load(f)
    # algorithmic flops of one coupled sweep: 4 nX nY (nX + nY) per pair
    flops = 0.0
    for p in probs:
        nxv = p.n_occ.astype(np.float64) * p.n_vir
        if p.n_pair:
            a, b = nxv[p.pairs[:, 0]], nxv[p.pairs[:, 1]]
            flops += float(np.sum(4.0 * a * b * (a + b)))
    out = {"workload": "64 cubic-lattice clusters, 27-512 monomers (log-uniform), o5v27 / o8v56 half and half, "
                       "cutoff 2 spacings" if n_clusters == 64 else f"first {n_clusters} of the 64 clusters",
           "clusters": n_clusters, "monomers": n_mono, "pairs": n_pair, "v_fp64_GB": vbytes / 1e9,
           "coupled_sweep_TFLOP": flops / 1e12, "generate_s": time.time() - t0,
           "sizes": [p.n_mono for p in probs], "forms": {}}
    with mc.Context(0) as ctx:
        t0 = time.time()
        pid = ctx.upload_batch(probs)
        out["upload_s"] = time.time() - t0
        t0 = time.time()
        out["tuning"] = ctx.autotune(pid, mc.MCPT_FP32)
        out["tuning"]["seconds"] = time.time() - t0
        log(f"[batch] tuned: " + ", ".join(f"{v['sb']}x{v['nw']}/{v['pd']}:{v['ms']:.1f}ms"
                                          for v in out["tuning"]["variants"]))
        sl = ctx.cluster_slices(pid)
        for name, prec in (("fp32+polish", mc.MCPT_FP32), ("fp64", mc.MCPT_FP64)):
            # one eager solve per form with HIP-event kernel timing on (a solve takes tens of seconds,
            # so graph replay would save nothing measurable; the tests cover the graph path)
            opts = dict(tol=tol, precision=prec, polish=1, graph=0, autotune=1)
            ctx.set_timing(True)
            ctx.timing()
            t1 = time.perf_counter()
            s = ctx.run(pid, **opts)
            secs = time.perf_counter() - t1
            tm = ctx.timing()
            ctx.set_timing(False)
            per = ctx.cluster_results(pid)
            e = ctx.energy(pid, want_t=False)
            f = {"seconds": secs, "clusters_per_s": n_clusters / secs, "sweeps": s["sweeps"],
                 "fp64_sweeps": s["polish_sweeps"] if prec else s["sweeps"], "e_total": s["e_total"],
                 "all_ok": all(c["status"] == 0 for c in per)}
            if tm["lowp_launches"]:
                ms = tm["lowp_ms"] / tm["lowp_launches"]
                tf = tm["lowp_flops"] / (tm["lowp_ms"] * 1e-3) / 1e12
                f["lowp_pair"] = {"kernel": "pair_lowp_kernel (FP32)", "bound": "mfma", "avg_launch_ms": ms,
                                  "flops_per_launch": tm["lowp_flops"] / tm["lowp_launches"],
                                  "achieved_TFLOPs": tf, "peak_TFLOPs": PEAK["fp32"][0],
                                  "frac": tf / PEAK["fp32"][0], "launches": tm["lowp_launches"]}
            if tm["pair_launches"]:
                tf = tm["pair_flops"] / (tm["pair_ms"] * 1e-3) / 1e12
                f["fp64_pair"] = {"kernel": "pair_fp64_lds_kernel + pair_fp64_glb_kernel", "bound": "mfma",
                                  "avg_launch_ms": tm["pair_ms"] / tm["pair_launches"], "achieved_TFLOPs": tf,
                                  "peak_TFLOPs": PEAK["fp64"][0], "frac": tf / PEAK["fp64"][0],
                                  "launches": tm["pair_launches"]}
            if golden is not None:
                worst, sweeps_equal = 0.0, True
                for key, g in golden["clusters"].items():
                    c = int(key)
                    worst = max(worst, abs(per[c]["e_total"] - g["e_total"]) / abs(g["e_total"]),
                                float(np.max(np.abs(e["e_m2"][sl[c][0]] - g["e_m2"]))) /
                                float(np.max(np.abs(g["e_m2"]))))
                    if prec == 0:
                        sweeps_equal &= per[c]["sweeps"] == g["sweeps"]
                f["oracle_clusters"] = {"clusters": sorted(int(k) for k in golden["clusters"]),
                                        "max_rel_error": worst, "file": "tests/golden/batch-64.json"}
                if prec == 0:
                    f["oracle_clusters"]["sweeps_equal"] = bool(sweeps_equal)
            out["forms"][name] = f
            f["per_cluster_e"] = [c["e_total"] for c in per]
            log(f"[batch] {name}: {secs:.2f}s per batch solve ({n_clusters / secs:.2f} clusters/s), "
                f"{s['sweeps']} sweeps" + (f", oracle clusters max rel err {f['oracle_clusters']['max_rel_error']:.1e}"
                                          if golden is not None else ""))
        ctx.release(pid)
        a = np.asarray(out["forms"]["fp32+polish"].pop("per_cluster_e"))
        b = np.asarray(out["forms"]["fp64"].pop("per_cluster_e"))
        out["max_rel_diff_fp32polish_vs_fp64"] = float(np.max(np.abs(a - b) / np.abs(b)))
    return out


def pmc_pass(workload: str, precision: int = 0, sweeps: int = 2, singles: bool = False, lccd: bool = False,
             dimer: bool = False):
    """Counter pass for rocprofv3 --pmc: one device copy of a known size
    (the calibration kernel), then `sweeps` fixed sweeps of the resident
    workload in the given precision (no polish) and the final FP64 energy
    pass; nothing else is launched."""
    import torch
    import paper_1409_2700_amd as mc
    from synth import make_workload
    prob = make_workload(workload)
    n = 1 << 27   # 1 GiB of FP64
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"[pmc] calibration copy: {n * 8} bytes read and written")
    del src, dst
    with mc.Context(0) as ctx:
        if dimer:
            p, ints, dints = dimer_problem()
            pid = ctx.upload(p)
            ctx.lccd_attach(pid, ints)
            ctx.dimer_attach(pid, dints)
            s = ctx.run(pid, tol=0.0, max_sweeps=sweeps)
            log(f"[pmc] {DIMER_WORKLOAD}: {sweeps} fixed sweeps of step 5 and of step 6 with the dimer-internal "
                f"terms, E={s['e_total']:.10f}")
            return
        if lccd:
            from synth import LCCD_K_SCALE, lccd_integrals
            prob.k *= LCCD_K_SCALE
            pid = ctx.upload(prob)
            ctx.lccd_attach(pid, lccd_integrals(prob))
            s = ctx.run(pid, tol=0.0, max_sweeps=sweeps)
            log(f"[pmc] {workload}: {sweeps} fixed sweeps of step 5 and of step 6 (full monomer equation), "
                f"E={s['e_total']:.10f}")
            return
        pid = ctx.upload(prob)
        if singles:
            from synth import singles_source
            s = ctx.singles(pid, singles_source(prob), tol=0.0, max_sweeps=sweeps)
            log(f"[pmc] {workload}: {s['sweeps']} fixed singles sweeps, E_M1={s['e_m1']:.10f}")
            return
        s = ctx.run(pid, tol=0.0, max_sweeps=sweeps, precision=precision, polish=0)
        log(f"[pmc] {workload}: {s['sweeps']} fixed sweeps (precision {precision}) + final pass, "
            f"E={s['e_total']:.10f}")


def singles_mode(ctx, pid, prob, steps, warmup, tol):
    """Singles solves (Eq. 57 pair coupling, Eq. 53 energy) of the resident
    workload from the seeded source w: solves/s, the pair kernel against the
    HBM roofline (algorithmic bytes = the V stream, 8 nX nY per pair), the
    error against the stored singles-oracle result, and the oracle's own cost
    on a sample of pairs scaled to one solve."""
    import numpy as np
    from synth import singles_source
    w = singles_source(prob)
    gpath = os.path.join(ROOT, "tests", "golden", f"singles-{prob.meta.get('name', '')}.json")
    golden = json.load(open(gpath)) if os.path.exists(gpath) else None
    for _ in range(warmup):
        ctx.singles(pid, w, tol=tol)
    ctx.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        s = ctx.singles(pid, w, tol=tol)
    dt = (time.perf_counter() - t0) / max(steps, 1)
    tm = ctx.timing()
    ctx.set_timing(False)
    kl = max(tm["singles_launches"], 1)
    ms = tm["singles_ms"] / kl
    vb = tm["singles_v_bytes"] / kl
    out = {
        "solves_per_s": 1.0 / dt, "ms_per_solve": dt * 1e3, "sweeps": s["sweeps"], "e_m1": s["e_m1"],
        "pair_kernel": {"kernel": "singles_pair_kernel", "bound": "hbm", "avg_launch_ms": ms,
                        "algorithmic_bytes_per_launch": vb, "achieved_GBps": vb / (ms * 1e-3) / 1e9,
                        "peak_GBps": HBM_PEAK_GBS, "frac": vb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "launches": tm["singles_launches"]},
    }
    if golden is not None:
        e = ctx.singles_result(pid)
        out["oracle_reference"] = {"e_m1": golden["e_m1_total"], "sweeps": golden["sweeps"],
                                   "file": os.path.relpath(gpath, ROOT)}
        out["relative_error_e_m1"] = abs(s["e_m1"] - golden["e_m1_total"]) / abs(golden["e_m1_total"])
        out["max_rel_error_per_monomer"] = float(np.max(np.abs(e["e_m1"] - np.asarray(golden["e_m1"]))) /
                                                 np.max(np.abs(golden["e_m1"])))
    log(f"[bench] singles: {s['sweeps']} sweeps, {dt * 1e3:.1f} ms per solve, pair kernel {ms:.3f} ms = "
        f"{vb / (ms * 1e-3) / 1e9:.0f} GB/s")
    return out


def singles_cpu(prob, sweeps: int, sample_pairs: int = 4096) -> dict:
    """The singles oracle's pair sum timed on the first sample_pairs pairs,
    scaled to one solve (sweeps x all pairs)."""
    import numpy as np
    from oracle import mcpt_singles
    from synth import singles_source
    w = singles_source(prob)
    t, off = [], 0
    for x in range(prob.n_mono):
        n = prob.n_ov(x)
        t.append(w[off:off + n].reshape(int(prob.n_occ[x]), int(prob.n_vir[x])))
        off += n
    k = min(sample_pairs, prob.n_pair)
    sub = prob.subset_pairs(np.arange(prob.n_pair) < k)
    t0 = time.perf_counter()
    mcpt_singles.coupling(sub, t)
    per_pair = (time.perf_counter() - t0) / max(k, 1)
    solve_s = per_pair * prob.n_pair * sweeps
    return {"value": 1.0 / solve_s, "unit": "solves/s", "kind": "oracle",
            "sample": f"pair sum of the first {k} pairs ({per_pair * 1e6:.0f} us per pair), scaled to "
                      f"{prob.n_pair} pairs x {sweeps} sweeps ({solve_s:.0f} s per solve)"}


def fd_mode(ctx, pid, prob, tol, step=0.01, with_singles=True):
    """Finite-displacement workflow (Sec. IV.A): the four stretch modes of the
    central 2 x 2 x 1 cell, five-point grid at 0.01 A, unit energy of Eq. 66
    (E_M2 + E_M1 over the cell); 16 displaced geometries built on the device
    from the resident crystal and solved from its converged amplitudes."""
    from synth import central_cell, singles_source, stretch_modes
    cell = central_cell(prob)
    modes = stretch_modes(prob, cell, step_angstrom=step)
    w = singles_source(prob) if with_singles else None
    ctx.fd_stencil(pid, [(a, f) for _, a, f in modes[:1]], cell, step, w=w, tol=tol)   # warm-up
    t0 = time.perf_counter()
    res = ctx.fd_stencil(pid, [(a, f) for _, a, f in modes], cell, step, w=w, tol=tol)
    secs = time.perf_counter() - t0
    n_solves = 1 + 4 * len(modes)
    out = {"seconds": secs, "geometries": n_solves, "geometries_per_s": n_solves / secs,
           "step_angstrom": step, "tol": tol, "cell": [int(c) for c in cell], "singles": with_singles,
           "modes": {n: {"d2e_Eh_per_A2": r["d2e"], "sweeps": r["sweeps"], "pairs_rescaled": int(len(a))}
                     for (n, a, _), r in zip(modes, res)}}
    log(f"[fd] {n_solves} geometries in {secs:.2f}s: " +
        ", ".join(f"{n} {r['d2e']:.6f}" for (n, _, _), r in zip(modes, res)))
    return out


def lccd_mode(ctx, prob, steps, warmup, tol, cpu_budget: float = 8.0, with_cpu: bool = True):
    """Full monomer equation (Eq. 58 with its intramonomer terms; step 5 then
    step 6) on the same crystal with K and the (vv|vv), (oo|oo), (oo|vv)
    classes at the workload's scale: solves/s, the ladder kernel against the
    HBM roofline (algorithmic bytes = the packed <ab|cd> stream, 8 v^2 x
    round16(v^2) per monomer), the error against the stored oracle result, and
    the oracle's intramonomer terms timed on a sample of monomers."""
    import numpy as np
    from synth import LCCD_K_SCALE, Problem, lccd_integrals
    t0 = time.time()
    pl = Problem(prob.n_occ, prob.n_vir, prob.eps, prob.k * LCCD_K_SCALE, prob.pairs, prob.v, prob.sites,
                 dict(prob.meta, k_scale=LCCD_K_SCALE))
    ints = lccd_integrals(pl)
    log(f"[lccd] integrals {ints.nbytes() / 1e9:.2f} GB made in {time.time() - t0:.1f}s")
    pid = ctx.upload(pl)
    t0 = time.time()
    ctx.lccd_attach(pid, ints)
    attach_s = time.time() - t0
    gpath = os.path.join(ROOT, "tests", "golden", f"lccd-{prob.meta.get('name', '')}.json")
    golden = json.load(open(gpath)) if os.path.exists(gpath) else None
    # check_every = 1: no sweep is issued past convergence, so every timed ladder launch does full work
    opts = dict(tol=tol, max_sweeps=400, check_every=1)
    for _ in range(warmup):
        ctx.run(pid, **opts)
    ctx.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        s = ctx.run(pid, **opts)
    dt = (time.perf_counter() - t0) / max(steps, 1)
    tm = ctx.timing()
    ctx.set_timing(False)
    e_fp64 = ctx.energy(pid, want_t=False)
    kl = max(tm["lccd_launches"], 1)
    ms = tm["lccd_ladder_ms"] / kl
    # the mixed-precision form on the same problem: BF16 pair products, FP64 polish (and FP64 intramonomer terms)
    ob = dict(opts, precision=2, polish=1, autotune=1)
    ctx.run(pid, **ob)
    t0 = time.perf_counter()
    for _ in range(steps):
        sb = ctx.run(pid, **ob)
    dtb = (time.perf_counter() - t0) / max(steps, 1)
    wb = tm["lccd_w_bytes"] / kl
    fl = tm["lccd_ladder_flops"] / kl
    out = {
        "solves_per_s": 1.0 / dt, "ms_per_solve": dt * 1e3, "iso_sweeps": s["iso_sweeps"], "sweeps": s["sweeps"],
        "e_total": s["e_total"], "e_lccd_total": s["e_mono0"], "attach_s": attach_s,
        "workload": f"{prob.meta.get('name', '')} with K x {LCCD_K_SCALE} and intramonomer classes at sigma 0.01",
        "ladder_kernel": {"kernel": "lccd_ladder_lds_kernel", "bound": "hbm", "avg_launch_ms": ms,
                          "algorithmic_bytes_per_launch": wb, "achieved_GBps": wb / (ms * 1e-3) / 1e9,
                          "peak_GBps": HBM_PEAK_GBS, "frac": wb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                          "ladder_TFLOPs": fl / (ms * 1e-3) / 1e12, "launches": tm["lccd_launches"],
                          **pipe_roof(wb, ms, int(prob.n_occ[0]))},
        "ring_kernel_avg_ms": tm["lccd_ring_ms"] / kl,
        "pair_kernel_avg_ms": tm["pair_ms"] / max(tm["pair_launches"], 1),
        "monomer_avg_ms": tm["mono_ms"] / max(tm["mono_launches"], 1),
        "bf16_polish": {"solves_per_s": 1.0 / dtb, "ms_per_solve": dtb * 1e3, "sweeps": sb["sweeps"],
                        "fp64_sweeps": sb["polish_sweeps"], "e_total": sb["e_total"],
                        "rel_diff_vs_fp64": abs(sb["e_total"] - s["e_total"]) / abs(s["e_total"])},
    }
    if golden is not None:
        e = e_fp64
        out["oracle_reference"] = {"e_total": golden["e_total"], "iso_sweeps": golden["iso_sweeps"],
                                   "sweeps": golden["sweeps"], "file": os.path.relpath(gpath, ROOT)}
        out["relative_error_e_total"] = abs(s["e_total"] - golden["e_total"]) / abs(golden["e_total"])
        out["max_abs_error_e_m2_Eh"] = float(np.max(np.abs(e["e_m2"] - np.asarray(golden["e_m2"]))))
        out["max_abs_error_e_lccd_Eh"] = float(np.max(np.abs(e["e_m2"] - e["de_m2"] - np.asarray(golden["e_lccd"]))))
    ctx.release(pid)
    log(f"[lccd] {s['iso_sweeps']} + {s['sweeps']} sweeps, {dt * 1e3:.1f} ms per solve, ladder {ms:.3f} ms = "
        f"{wb / (ms * 1e-3) / 1e9:.0f} GB/s, ring {out['ring_kernel_avg_ms']:.3f} ms; BF16 + polish "
        f"{dtb * 1e3:.1f} ms ({sb['sweeps']} sweeps, {sb['polish_sweeps']} FP64)")
    if with_cpu:
        from oracle import mcpt_lccd
        orc = mcpt_lccd.LccdOracle(pl.subset_pairs(np.zeros(pl.n_pair, dtype=bool)), ints)
        T = orc.first_order()
        k, t0 = 0, time.perf_counter()
        while k < pl.n_mono and time.perf_counter() - t0 < cpu_budget:
            mcpt_lccd.intramonomer_terms(orc.v[k], T[k])
            k += 1
        per = (time.perf_counter() - t0) / max(k, 1)
        sweeps = (golden["iso_sweeps"] + golden["sweeps"]) if golden else s["iso_sweeps"] + s["sweeps"]
        out["cpu_oracle_intramonomer"] = {
            "seconds_per_solve": per * pl.n_mono * sweeps, "unit": "s", "kind": "oracle",
            "sample": f"intramonomer terms of {k} monomers ({per * 1e3:.1f} ms each), scaled to "
                      f"{pl.n_mono} monomers x {sweeps} sweeps (the pair part is cpu_baseline's)"}
    return out


DIMER_WORKLOAD = "hf-10x10x10-c1"
DIMER_WORKLOADS = {
    "hf-10x10x10-c1": "1000 monomers, their 2,700 nearest-neighbour pairs",
    "hf-10x10x10-c1.5": "1000 monomers, their 7,560 nearest and face-diagonal pairs",
}


def dimer_problem(name=DIMER_WORKLOAD):
    """A 1000-monomer crystal (the c3 crystal's blocks of its pairs), K at
    LCCD_K_SCALE, with the intramonomer and the dimer classes: the dimer class
    (vv|vv) alone is 4.25 MB per pair."""
    from synth import make_dimer_workload
    return make_dimer_workload(name, workers=min(16, os.cpu_count() or 1))


def dimer_mode(ctx, steps, warmup, tol, cpu_budget: float = 8.0, with_cpu: bool = True, name=DIMER_WORKLOAD):
    """Full equations with the dimer-internal terms of Eq. 59 (Tau iterated):
    solves/s, the pair-ladder launch against the HBM roofline (algorithmic
    bytes = the packed <a b|a1 b1> stream, 8 round16(v^2) round32(v^2) per
    pair), the ring launch, and the oracle's dimer-internal terms timed on a
    sample of pairs."""
    import numpy as np
    t0 = time.time()
    p, ints, dints = dimer_problem(name)
    log(f"[dimer] {name}: N={p.n_mono} P={p.n_pair}, dimer classes {dints.nbytes() / 1e9:.2f} GB "
        f"made in {time.time() - t0:.1f}s")
    pid = ctx.upload(p)
    ctx.lccd_attach(pid, ints)
    t0 = time.time()
    ctx.dimer_attach(pid, dints)
    attach_s = time.time() - t0
    opts = dict(tol=tol, max_sweeps=400, check_every=1)
    for _ in range(warmup):
        ctx.run(pid, **opts)
    ctx.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        s = ctx.run(pid, **opts)
    dt = (time.perf_counter() - t0) / max(steps, 1)
    tm = ctx.timing()
    ctx.set_timing(False)
    e = ctx.energy(pid, want_t=False)
    ctx.release(pid)
    kl = max(tm["dimer_launches"], 1)
    ms = tm["dimer_ladder_ms"] / kl
    wb = tm["dimer_w_bytes"] / kl
    fl = tm["dimer_ladder_flops"] / kl
    o, v = int(p.n_occ[0]), int(p.n_vir[0])
    npad = (o * v + 15) // 16 * 16
    ring_flops = 4 * 2.0 * (o * v) ** 3 * p.n_pair
    rms = tm["dimer_ring_ms"] / kl
    out = {
        "workload": f"{name}: {DIMER_WORKLOADS[name]}, K x 0.2, intramonomer classes at sigma 0.01, dimer "
                    f"classes at sigma 0.01 (R_nn / R)^3",
        "dimer_classes_GB": dints.nbytes() / 1e9,
        "solves_per_s": 1.0 / dt, "ms_per_solve": dt * 1e3, "iso_sweeps": s["iso_sweeps"], "sweeps": s["sweeps"],
        "e_total": s["e_total"], "attach_s": attach_s,
        "pair_ladder_kernel": {"kernel": "lccd_ladder_lds_kernel (on pairs)", "bound": "hbm", "avg_launch_ms": ms,
                               "algorithmic_bytes_per_launch": wb, "achieved_GBps": wb / (ms * 1e-3) / 1e9,
                               "peak_GBps": HBM_PEAK_GBS, "frac": wb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                               "ladder_TFLOPs": fl / (ms * 1e-3) / 1e12, "launches": tm["dimer_launches"],
                               **pipe_roof(wb, ms, o)},
        "ring_kernel": {"kernel": "dimer_ring_kernel", "bound": "mfma", "avg_launch_ms": rms,
                        "flops_per_launch": ring_flops, "achieved_TFLOPs": ring_flops / (rms * 1e-3) / 1e12,
                        "peak_TFLOPs": PEAK["fp64"][0],
                        "frac": ring_flops / (rms * 1e-3) / 1e12 / PEAK["fp64"][0], "padded_edge": npad},
        # HIP events around the whole pair phase: the two launches above and the pair kernel
        "pair_phase_avg_ms": tm["pair_ms"] / max(tm["pair_launches"], 1),
    }
    gpath = os.path.join(ROOT, "tests", "golden", f"dimer-{name}.json")
    if os.path.exists(gpath):
        g = json.load(open(gpath))
        out["oracle_reference"] = {"e_total": g["e_total"], "sweeps": g["sweeps"], "file": os.path.relpath(gpath, ROOT)}
        out["relative_error_e_total"] = abs(s["e_total"] - g["e_total"]) / abs(g["e_total"])
        out["max_abs_error_e_m2_Eh"] = float(np.max(np.abs(e["e_m2"] - np.asarray(g["e_m2"]))))
        out["max_abs_error_e_d2_Eh"] = float(np.max(np.abs(e["e_d2"][g["pair_index"]] - np.asarray(g["e_d2"]))))
    log(f"[dimer] {s['iso_sweeps']} + {s['sweeps']} sweeps, {dt * 1e3:.1f} ms per solve, pair ladder {ms:.3f} ms = "
        f"{wb / (ms * 1e-3) / 1e9:.0f} GB/s, ring {rms:.3f} ms")
    if with_cpu:
        from oracle import mcpt_dimer
        orc = mcpt_dimer.DimerOracle(p, ints, dints)
        rng = np.random.default_rng(0)
        k, t0 = 0, time.perf_counter()
        while k < p.n_pair and time.perf_counter() - t0 < cpu_budget:
            orc.internal(k, rng.standard_normal(orc.D_pair(k).shape) * 1e-3)
            k += 1
        per = (time.perf_counter() - t0) / max(k, 1)
        sweeps = s["sweeps"] + 1
        out["cpu_oracle_dimer_terms"] = {
            "seconds_per_solve": per * p.n_pair * sweeps, "unit": "s", "kind": "oracle",
            "sample": f"dimer-internal terms of {k} pairs ({per * 1e3:.1f} ms each), scaled to {p.n_pair} pairs x "
                      f"{sweeps} Eq. 59 steps (the rest of the solve is not included)"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="hf-10x10x10-c3")
    ap.add_argument("--headline", default="fp64", choices=list(MODES))
    ap.add_argument("--modes", default=",".join(MODES), help="comma-separated forms to time")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--check-every", type=int, default=1)
    ap.add_argument("--graph", type=int, default=0, help="1: replay HIP-graph captured sweeps")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--serve-requests", type=int, default=256, help="served-stream sample (0: skip)")
    ap.add_argument("--serve-workers", type=int, default=4)
    ap.add_argument("--serve-batch", type=int, default=16)
    ap.add_argument("--serve-mode", type=int, default=None,
                    help="tick mode of the served passes (0 batch end, 1 retire at ticks, 2 join at ticks; "
                         "default: the library's)")
    ap.add_argument("--serve-compare", default="0",
                    help="comma-separated other tick modes that get one capacity pass each ('' for none)")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="only launch a calibration copy and two fixed sweeps (for rocprofv3 --pmc)")
    ap.add_argument("--pmc-precision", type=int, default=0, help="0 FP64, 1 FP32, 2 BF16 sweeps in --pmc-pass")
    ap.add_argument("--pmc-singles", action="store_true", help="--pmc-pass runs two singles sweeps instead")
    ap.add_argument("--pmc-lccd", action="store_true",
                    help="--pmc-pass runs two sweeps of step 5 and two of step 6 of the full monomer equation")
    ap.add_argument("--pmc-dimer", action="store_true",
                    help="--pmc-pass runs two sweeps of each step with the dimer-internal terms")
    ap.add_argument("--singles-steps", type=int, default=3, help="timed singles solves (0: skip)")
    ap.add_argument("--fd", type=int, default=1, help="1: time the finite-displacement workflow (0: skip)")
    ap.add_argument("--lccd-steps", type=int, default=2,
                    help="timed solves of the full monomer equation (0: skip)")
    ap.add_argument("--dimer-steps", type=int, default=1,
                    help="timed solves with the dimer-internal terms of Eq. 59 (0: skip)")
    ap.add_argument("--small-configs", type=int, default=1,
                    help="1: time the 8- and 125-monomer crystals on the GPU and the oracle (0: skip)")
    ap.add_argument("--batched", type=int, default=64,
                    help="time the batching form on this many uneven clusters (64 = full set, 0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the MCPT(2) path is built and measured on a single "
              f"MI355X (requested --gpus {args.gpus}); multi-GPU sharding is a design note only.",
              file=sys.stderr)
        sys.exit(2)

    if args.pmc_pass:
        pmc_pass(args.workload, args.pmc_precision, singles=args.pmc_singles, lccd=args.pmc_lccd,
                 dimer=args.pmc_dimer)
        return
    import paper_1409_2700_amd as mc
    from synth import make_workload, DEFAULT_COUPLING_SCALE

    golden = None
    gpath = os.path.join(ROOT, "tests", "golden", f"{args.workload}.json")
    if os.path.exists(gpath):
        with open(gpath) as f:
            golden = json.load(f)
    t0 = time.time()
    prob = make_workload(args.workload)
    log(f"[bench] inputs {args.workload}: N={prob.n_mono} P={prob.n_pair} "
        f"({prob.nbytes() / 1e9:.2f} GB) in {time.time() - t0:.1f}s")
    ctx = mc.Context(0)
    rates = mc.device_rates(0)
    MEASURED.update(rates)
    log(f"[bench] device FP64 pipes: MFMA {rates['mfma_f64_tflops']:.1f} TFLOP/s, "
        f"VALU {rates['valu_f64_tflops']:.1f} TFLOP/s, clock {rates['clock_ghz']:.2f} GHz")
    t0 = time.time()
    pid = ctx.upload(prob)
    log(f"[bench] upload {time.time() - t0:.1f}s")
    modes = [m for m in args.modes.split(",") if m]
    if args.headline not in modes:
        modes.insert(0, args.headline)
    results = {}
    for name in modes:
        results[name] = time_mode(ctx, pid, name, args.steps, args.warmup, args.tol, args.check_every, golden,
                                  args.graph)
    singles = None
    if args.singles_steps > 0:
        singles = singles_mode(ctx, pid, prob, args.singles_steps, 1, args.tol)
    fd = fd_mode(ctx, pid, prob, 1e-12) if args.fd else None
    ctx.release(pid)
    lccd = None
    if args.lccd_steps > 0:
        lccd = lccd_mode(ctx, prob, args.lccd_steps, 1, args.tol, with_cpu=not args.no_cpu_baseline)
    dimer = None
    if args.dimer_steps > 0:
        dimer = dimer_mode(ctx, args.dimer_steps, 1, args.tol, with_cpu=not args.no_cpu_baseline)
        dimer["larger_crystal"] = dimer_mode(ctx, 1, 1, args.tol, with_cpu=False, name="hf-10x10x10-c1.5")
    ctx.close()
    served = None
    if args.serve_requests > 0:
        served = serving(prob, args.serve_requests, [0.5, 0.8], args.serve_workers, args.serve_batch,
                         args.tol, mode=args.serve_mode,
                         compare=tuple(int(m) for m in args.serve_compare.split(",") if m.strip()))

    h = results[args.headline]
    tm = h["timing"]
    prec = MODES[args.headline][0]
    if prec == 0 or tm["pair_ms"] >= tm["lowp_ms"]:
        kname, kms, kl, kfl, kvb, kpeak = ("pair_fp64_lds_kernel", tm["pair_ms"], tm["pair_launches"],
                                           tm["pair_flops"], tm["pair_v_bytes"], PEAK["fp64"][0])
        dtype = "f64"
    else:
        kname, kms, kl, kfl, kvb = ("pair_lowp_kernel", tm["lowp_ms"], tm["lowp_launches"], tm["lowp_flops"],
                                    tm["lowp_v_bytes"])
        kpeak = PEAK["bf16" if prec == 2 else "fp32"][0]
        dtype = "bf16+f64" if prec == 2 else "f32+f64"
    avg_ms = kms / max(kl, 1)
    flops_per_launch = kfl / max(kl, 1)
    achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12
    # monomer phase (Eq. 58 update, elementwise): reads K, G, T and writes T, M and the cleared G buffer,
    # 6 n^2 doubles per monomer (algorithmic, unpadded n)
    mono_bytes = 6.0 * 8.0 * float(sum(int(o) * int(v) * int(o) * int(v) for o, v in zip(prob.n_occ, prob.n_vir)))
    mono_ms = results["fp64"]["monomer_avg_ms"] if "fp64" in results else None
    out = {
        "metric": METRIC, "value": h["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": h["ms_per_solve"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {
            "workload": args.workload, "n_mono": prob.n_mono, "n_pair": prob.n_pair, "o": 5, "v": 27,
            "lattice": "simple cubic 3.4 A, open boundaries", "coupling_scale": DEFAULT_COUPLING_SCALE,
            "tol": args.tol, "form": args.headline, "sweeps": h["sweeps"],
        },
        "pair_contraction_GBps": kvb / (kms * 1e-3) / 1e9,
        "e_total": h["e_total"],
        "roofline": {
            "bound": "mfma", "achieved": achieved, "peak": kpeak, "unit": "TFLOP/s",
            "frac": achieved / kpeak,
            "traffic": counted_traffic(h["sweeps"]) if kname == "pair_fp64_lds_kernel" and args.workload == "hf-10x10x10-c3" else None,
            "traffic_unit": "bytes per launch (L2-fabric, counters calibrated by a 1 GiB copy)",
            "kernel": kname, "avg_launch_ms": avg_ms,
            "flops_per_launch": flops_per_launch, "launches": kl,
            # the sustained rate of the FP64 matrix pipe measured on this device at the kernel's occupancy
            "device_rates": rates,
            "frac_of_measured_mfma_f64": achieved / rates["mfma_f64_tflops"] if prec == 0 else None,
        },
        "monomer_phase": None if not mono_ms else {
            "bound": "hbm", "algorithmic_bytes_per_launch": mono_bytes, "avg_launch_ms": mono_ms,
            "achieved_GBps": mono_bytes / (mono_ms * 1e-3) / 1e9, "peak_GBps": HBM_PEAK_GBS,
            "frac": mono_bytes / (mono_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "forms": {k: {kk: vv for kk, vv in v.items() if kk != "timing"} for k, v in results.items()},
    }
    if singles is not None:
        out["singles"] = singles
    if lccd is not None:
        out["full_monomer_equation"] = lccd
    if dimer is not None:
        out["dimer_internal_terms"] = dimer
    if fd is not None:
        out["finite_displacement"] = fd
    if served is not None:
        out["serving"] = served
    if args.batched > 0:
        out["batched"] = batched(args.batched, args.tol)
    if args.small_configs:
        out["small_configs"] = small_configs(args.tol, with_cpu=not args.no_cpu_baseline)
    if golden is not None:
        out["oracle_reference"] = {"e_total": golden["e_total"], "sweeps": golden["sweeps"],
                                   "file": f"tests/golden/{args.workload}.json"}
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a sample ...")
        out["cpu_baseline"] = cpu_baseline(prob, golden["sweeps"] if golden else h["sweeps"], args.cpu_budget)
        log(f"[bench] cpu_baseline {out['cpu_baseline']['value']:.3e} solves/s")
        if fd is not None:
            # the oracle's cost of the same geometries: each an FP64 solve at the cpu_baseline rate
            fd["cpu_oracle_estimate_s"] = fd["geometries"] / out["cpu_baseline"]["value"]
        if singles is not None:
            singles["cpu_oracle"] = singles_cpu(prob, singles["sweeps"])
            log(f"[bench] singles cpu oracle {singles['cpu_oracle']['value']:.3e} solves/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
