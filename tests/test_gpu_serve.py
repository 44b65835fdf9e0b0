"""Serving form: requests submitted while others run, fused into batches by the
scheduler, admitted by HBM footprint.  Each served result must be the one the
same problem gives alone (mcpt_run on the caller's stream): sweep counts equal,
energies within 1e-12 relative (the atomics order of G aside, the arithmetic
is the same), and the FP64 oracle within 1e-10 relative.
"""
import time

import numpy as np
import pytest

from oracle import mcpt_oracle
from synth import make_served_request, make_workload
import paper_1409_2700_amd as mc

pytestmark = pytest.mark.gpu

SAME_RTOL = 1e-12


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b))) / max(float(np.max(np.abs(b))), 1e-300)


@pytest.fixture(scope="module")
def requests():
    return [make_served_request(r, max_mono=40) for r in range(10)]


def alone(prob, **opts):
    with mc.Context(0) as c:
        pid, s = c.solve(prob, raise_on_error=False, **opts)
        e = c.energy(pid) if s["status"] != mc.MCPT_ERR_DIVERGED else None
    return s, e


def wait_all(ctx, tickets, timeout_s=120.0):
    out = {}
    t0 = time.time()
    for t in tickets:
        left = max(1, int((timeout_s - (time.time() - t0)) * 1000))
        s = ctx.wait(t, left)
        assert s is not None, f"ticket {t} did not finish"
        out[t] = s
    return out


def check_served(ctx, probs, tickets, done, **opts):
    for p, t in zip(probs, tickets):
        s = done[t]
        s1, e1 = alone(p, **opts)
        assert s["status"] == s1["status"], (p.meta["name"], s, s1)
        assert s["sweeps"] == s1["sweeps"] and s["polish_sweeps"] == s1["polish_sweeps"]
        if s["status"] == mc.MCPT_ERR_DIVERGED:
            with pytest.raises(mc.MCPTError):
                ctx.energy(t)
            continue
        for k in ("e_total", "e_mono", "e_dimer", "e_mono0"):
            assert abs(s[k] - s1[k]) <= SAME_RTOL * abs(s1[k]), (p.meta["name"], k)
        e = ctx.energy(t)
        assert rel(e["e_m2"], e1["e_m2"]) <= SAME_RTOL
        assert rel(e["e_d2"], e1["e_d2"]) <= 1e-11
        assert rel(e["t"], e1["t"]) <= 1e-10
        assert s["seconds"] > 0.0


@pytest.mark.parametrize("prec", [mc.MCPT_FP64, mc.MCPT_FP32], ids=["fp64", "fp32polish"])
def test_served_mix_equals_alone(requests, prec):
    opts = dict(tol=1e-10, precision=prec, polish=1)
    with mc.Context(0) as ctx:
        ctx.serve_config(workers=3, max_batch=4)
        print(f"[gpu] serve {len(requests)} requests sizes {[p.n_mono for p in requests]} prec={prec}", flush=True)
        tickets = []
        for k, p in enumerate(requests):   # arrivals spread out: later ones land while earlier ones run
            tickets.append(ctx.submit(p, **opts))
            if k % 3 == 2:
                time.sleep(0.01)
        done = wait_all(ctx, tickets)
        st = ctx.serve_stats()
        assert st["completed"] == len(requests)
        assert st["batches"] <= len(requests)
        check_served(ctx, requests, tickets, done, **opts)
        for t in tickets:
            ctx.release(t)
        assert ctx.serve_stats()["tickets"] == 0


def test_served_against_oracle(requests):
    p = requests[0]
    with mc.Context(0) as ctx:
        t = ctx.submit(p, tol=1e-10)
        s = ctx.wait(t, 60000)
        r = mcpt_oracle.solve(p, tol=1e-10, max_sweeps=200)
        assert s["status"] == mc.MCPT_OK and s["sweeps"] == r.sweeps
        assert abs(s["e_total"] - r.e_total) <= 1e-10 * abs(r.e_total)
        e = ctx.energy(t)
        assert rel(e["e_m2"], r.e_m2) <= 1e-10


def test_late_small_requests_overtake_a_large_one():
    """Small requests submitted while a large one is on the GPU are admitted by
    another worker and finish first."""
    big = make_served_request(1000, min_mono=300, max_mono=300, cutoff=2.0)
    small = [make_served_request(1001 + k, min_mono=8, max_mono=8) for k in range(3)]
    with mc.Context(0) as ctx:
        ctx.serve_config(workers=2, max_batch=8)
        tb = ctx.submit(big, tol=0.0, max_sweeps=200)   # fixed sweeps: on the device for a while
        t0 = time.time()
        while ctx.serve_stats()["running_batches"] == 0 and ctx.poll(tb) is None and time.time() - t0 < 10:
            time.sleep(0.0005)
        ts = [ctx.submit(p, tol=1e-10) for p in small]
        done_small = wait_all(ctx, ts)
        assert ctx.poll(tb) is None, "the large request finished before the small ones"
        sb = ctx.wait(tb, 120000)
        assert sb["status"] == mc.MCPT_OK
        for t, p in zip(ts, small):
            assert done_small[t]["status"] == mc.MCPT_OK
            s1, _ = alone(p, tol=1e-10)
            assert abs(done_small[t]["e_total"] - s1["e_total"]) <= SAME_RTOL * abs(s1["e_total"])


def settled(ctx, timeout_s=30.0):
    """Serving counters once no batch is on the device (a batch frees its memory
    just after reporting its last request)."""
    t0 = time.time()
    st = ctx.serve_stats()
    while st["running_batches"] and time.time() - t0 < timeout_s:
        time.sleep(0.002)
        st = ctx.serve_stats()
    return st


def test_admission_waits_for_memory():
    """Admission prices a request at its footprint beside the results finished
    requests hold (their batch stays on the device until their tickets are released)."""
    probs = [make_served_request(2000, min_mono=30, max_mono=30)] * 3
    with mc.Context(0) as probe:
        t = probe.submit(probs[0], tol=1e-10)
        probe.wait(t, 60000)
        one = settled(probe)["bytes_in_use"]
    assert one > 0
    with mc.Context(0, hbm_budget=int(2.5 * one)) as ctx:
        ctx.serve_config(workers=3, max_batch=1)
        ts = [ctx.submit(p, tol=1e-10) for p in probs]
        a = ctx.wait(ts[0], 60000)
        b = ctx.wait(ts[1], 60000)
        assert a["status"] == b["status"] == mc.MCPT_OK
        # both results are held: the third request cannot be admitted
        assert ctx.wait(ts[2], 300) is None
        st = settled(ctx)
        assert st["queued"] == 1 and st["bytes_in_use"] <= st["budget"]
        ctx.release(ts[0])
        c = ctx.wait(ts[2], 60000)
        assert c is not None and c["status"] == mc.MCPT_OK
        assert abs(c["e_total"] - a["e_total"]) <= SAME_RTOL * abs(a["e_total"])
        assert settled(ctx)["bytes_in_use"] <= ctx.serve_stats()["budget"]


@pytest.mark.parametrize("mode", [mc.MCPT_SERVE_JOIN_AT_TICKS, mc.MCPT_SERVE_RETIRE_AT_TICKS,
                                  mc.MCPT_SERVE_BATCH_END], ids=["join", "retire", "batch-end"])
def test_requests_join_a_running_batch(mode):
    """With the only worker busy and a short queue, a request submitted while a
    batch runs joins it at a sweep tick: it is uploaded and merged with the
    batch's unfinished clusters, whose iteration continues where it stopped, and
    each request retires at the tick where its own solve stops.  Every sweep
    count and result equals the alone solve's; with admission at ticks off, the
    request waits for the batch to end."""
    ticks = mode == mc.MCPT_SERVE_JOIN_AT_TICKS
    # fixed sweeps keep the first request on the device while the others are copied in; the
    # joiner is larger than it (a join copies the unfinished clusters, so it needs that)
    first = make_served_request(3000, min_mono=40, max_mono=40, cutoff=2.0)
    late = [make_served_request(3001 + k, min_mono=50, max_mono=60, cutoff=2.0) for k in range(4)]
    opts = dict(tol=0.0, max_sweeps=400, check_every=1)
    with mc.Context(0) as ctx:
        ctx.serve_config(workers=1, max_batch=8)
        ctx.serve_tick_mode(mode)
        print(f"[gpu] join mode={mode} sizes {first.n_mono} {[p.n_mono for p in late]}", flush=True)
        t0 = ctx.submit(first, **opts)
        t_start = time.time()
        while ctx.serve_stats()["running_batches"] == 0 and time.time() - t_start < 10:
            time.sleep(0.0002)
        ts = [ctx.submit(late[0], **opts)]
        first_running = ctx.poll(t0) is None
        t_start = time.time()
        while ticks and ctx.serve_stats()["queued"] and time.time() - t_start < 0.5:
            time.sleep(0.0002)   # taken by a join at the next tick
        ts += [ctx.submit(p, **opts) for p in late[1:]]
        done = wait_all(ctx, [t0] + ts)
        st = settled(ctx)
        assert st["completed"] == 5
        assert first_running, "the first request ended before the second was submitted"
        if ticks:
            assert st["joined_at_ticks"] >= 1
        else:
            assert st["joined_at_ticks"] == 0
            assert st["batches"] >= 2
        check_served(ctx, [first] + late, [t0] + ts, done, **opts)
        for t in [t0] + ts:
            ctx.release(t)
        assert settled(ctx)["bytes_in_use"] == 0


def test_joined_requests_retire_one_by_one():
    """Requests of one batch that stop at different sweeps retire at their own
    ticks (a converged one does not wait for the others), with results readable
    while the batch goes on and after it has ended."""
    probs = [make_served_request(3100 + k, min_mono=60, max_mono=90) for k in range(6)]
    opts = dict(tol=1e-11, check_every=1)
    with mc.Context(0) as ctx:
        ctx.serve_config(workers=1, max_batch=3)
        ts = [ctx.submit(p, **opts) for p in probs]
        done = wait_all(ctx, ts)
        st = settled(ctx)
        assert st["completed"] == len(probs) and st["tickets"] == len(probs)
        check_served(ctx, probs, ts, done, **opts)
        with pytest.raises(mc.MCPTError):
            ctx.serve_tick_mode(mc.MCPT_SERVE_BATCH_END)   # the scheduler is running


def test_submit_errors_and_cancel(requests):
    p = requests[1]
    with mc.Context(0, hbm_budget=1 << 20) as small:
        with pytest.raises(mc.MCPTError) as ei:
            small.submit(p, tol=1e-10)
        assert ei.value.status == mc.MCPT_ERR_ADMISSION
    with mc.Context(0) as ctx:
        bad_eps = make_workload("hf-2x2x2")
        bad_eps.eps = bad_eps.eps.copy()
        bad_eps.eps[3] = np.inf
        with pytest.raises(mc.MCPTError) as ei:
            ctx.submit(bad_eps, tol=1e-10)
        assert ei.value.status == mc.MCPT_ERR_NONFINITE
        with pytest.raises(mc.MCPTError) as ei:
            ctx.submit(p, tol=1e-10, deterministic=2)
        assert ei.value.status == mc.MCPT_ERR_INVALID
        with pytest.raises(mc.MCPTError) as ei:
            ctx.poll(123456789)
        assert ei.value.status == mc.MCPT_ERR_UNKNOWN_ID
        t = ctx.submit(p, tol=1e-10)
        s = ctx.wait(t, 60000)
        assert s["status"] == mc.MCPT_OK
        ctx.release(t)
        with pytest.raises(mc.MCPTError):
            ctx.energy(t)


def test_diverging_request_does_not_disturb_the_mix(requests):
    bad = make_workload("hf-2x2x2", coupling_scale=1.0)
    probs = [requests[2], bad, requests[3]]
    opts = dict(tol=1e-10, max_sweeps=60)
    with mc.Context(0) as ctx:
        ctx.serve_config(workers=1, max_batch=8)
        ts = [ctx.submit(p, **opts) for p in probs]
        done = wait_all(ctx, ts)
        assert done[ts[1]]["status"] == mc.MCPT_ERR_DIVERGED
        check_served(ctx, probs, ts, done, **opts)


def test_nonfinite_request_fails_alone(requests):
    """A NaN in one request's dimer blocks is found on the device: that request
    fails with MCPT_ERR_NONFINITE, the requests batched with it are unaffected."""
    bad = make_workload("hf-2x2x2")
    bad.v = bad.v.copy()
    bad.v[5] = np.nan
    probs = [requests[4], bad, requests[5]]
    opts = dict(tol=1e-10)
    with mc.Context(0) as ctx:
        ctx.serve_config(workers=1, max_batch=8)
        ts = [ctx.submit(p, **opts) for p in probs]
        done = wait_all(ctx, ts)
        assert done[ts[1]]["status"] == mc.MCPT_ERR_NONFINITE
        with pytest.raises(mc.MCPTError):
            ctx.energy(ts[1])
        check_served(ctx, [probs[0], probs[2]], [ts[0], ts[2]], done, **opts)


@pytest.mark.parametrize("cap", [0, 2 << 20, 1 << 34], ids=["pageable", "cap-2MiB", "pinned"])
def test_staging_cap_keeps_results(requests, cap):
    """Requests copied to pinned staging blocks, to pageable memory, or some of
    each (a cap below the larger requests) all give the alone results; the
    counters say which memory the copies went to, and pinned blocks are reused."""
    opts = dict(tol=1e-10)
    with mc.Context(0) as ctx:
        ctx.serve_config(workers=2, max_batch=4)
        ctx.serve_staging(cap)
        print(f"[gpu] serve staging cap {cap}", flush=True)
        tickets = [ctx.submit(p, **opts) for p in requests]
        done = wait_all(ctx, tickets)
        st = ctx.serve_stats()
        check_served(ctx, requests, tickets, done, **opts)
        # every request has two arrays (k_intra, v_dimer)
        if cap == 0:
            assert st["staging_pinned_bytes"] == 0 and st["staged_pageable"] == 2 * len(requests)
        elif cap == 2 << 20:
            assert 0 < st["staging_pinned_bytes"] <= cap and 0 < st["staged_pageable"] < 2 * len(requests)
        else:
            assert st["staged_pageable"] == 0 and st["staging_pinned_bytes"] > 0
            for t in tickets:
                ctx.release(t)
            held = ctx.serve_stats()["staging_pinned_bytes"]
            for p in requests[:3]:   # one at a time: each is served from blocks freed earlier
                wait_all(ctx, [ctx.submit(p, **opts)])
            assert ctx.serve_stats()["staging_pinned_bytes"] == held
        with pytest.raises(mc.MCPTError):
            ctx.serve_staging(cap)   # the scheduler is running


def test_retired_result_read_while_its_batch_runs():
    """A request that retires while a slower request of its batch is still
    sweeping can be read at once (its results stay in the batch, which goes on
    skipping its clusters), and it equals its alone solve; so does the slower one."""
    fast = make_served_request(3200, min_mono=100, max_mono=100, cutoff=2.0, coupling_scale=0.05)
    slow = make_served_request(3201, min_mono=100, max_mono=100, cutoff=2.0, coupling_scale=0.35)
    opts = dict(tol=1e-13, max_sweeps=400, check_every=1)
    with mc.Context(0) as ctx:
        ctx.serve_config(workers=1, max_batch=4)
        tf, ts = ctx.submit(fast, **opts), ctx.submit(slow, **opts)
        sf = ctx.wait(tf, 60000)
        slow_running = ctx.poll(ts) is None
        ef = ctx.energy(tf)   # while the slow request sweeps, most likely
        print(f"[gpu] retired read: fast {sf['sweeps']} sweeps, slow still running: {slow_running}", flush=True)
        ss = ctx.wait(ts, 60000)
        assert ss["sweeps"] > sf["sweeps"]
        s1, e1 = alone(fast, **opts)
        assert sf["sweeps"] == s1["sweeps"] and abs(sf["e_total"] - s1["e_total"]) <= SAME_RTOL * abs(s1["e_total"])
        assert rel(ef["e_m2"], e1["e_m2"]) <= SAME_RTOL and rel(ef["t"], e1["t"]) <= 1e-10
        assert rel(ef["e_d2"], e1["e_d2"]) <= 1e-11
        check_served(ctx, [fast, slow], [tf, ts], {tf: sf, ts: ss}, **opts)


def test_nonfinite_joiner_fails_alone():
    """A request with a NaN in its dimer blocks that joins a running batch at a
    sweep tick fails by itself with MCPT_ERR_NONFINITE; the batch it joined and
    a later good joiner are unaffected."""
    first = make_served_request(3300, min_mono=40, max_mono=40, cutoff=2.0)
    bad = make_served_request(3301, min_mono=55, max_mono=55, cutoff=2.0)
    bad.v = bad.v.copy()
    bad.v[7] = np.nan
    good = make_served_request(3302, min_mono=55, max_mono=55, cutoff=2.0)
    opts = dict(tol=0.0, max_sweeps=400, check_every=1)
    with mc.Context(0) as ctx:
        ctx.serve_config(workers=1, max_batch=8)
        ctx.serve_tick_mode(mc.MCPT_SERVE_JOIN_AT_TICKS)
        t0 = ctx.submit(first, **opts)
        t_start = time.time()
        while ctx.serve_stats()["running_batches"] == 0 and time.time() - t_start < 10:
            time.sleep(0.0002)
        tb = ctx.submit(bad, **opts)
        t_start = time.time()
        while ctx.serve_stats()["queued"] and time.time() - t_start < 0.5:
            time.sleep(0.0002)
        tg = ctx.submit(good, **opts)
        done = wait_all(ctx, [t0, tb, tg])
        assert ctx.serve_stats()["joined_at_ticks"] >= 1
        assert done[tb]["status"] == mc.MCPT_ERR_NONFINITE
        with pytest.raises(mc.MCPTError):
            ctx.energy(tb)
        check_served(ctx, [first, good], [t0, tg], done, **opts)
