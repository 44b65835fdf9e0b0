"""Tile autotuner of the reduced-precision pair kernel: every tile shape is a
correct kernel (FP32 / BF16 polished solves within 1e-10 relative of the FP64
oracle, and equal to each other to rounding), the tuner picks one of them, and
its table round-trips through text."""
import json
import os

import numpy as np
import pytest

from synth import make_cluster_batch, make_workload
import paper_1409_2700_amd as mc

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def golden125():
    with open(os.path.join(GOLDEN, "hf-5x5x5-c2.json")) as f:
        return json.load(f)


def forced(ctx, pid, prec, sb, nw, pd):
    """Point the context's table entry for this problem at one tile shape."""
    ctx.autotune(pid, prec)   # creates the entry (and times every shape)
    lines = [l for l in ctx.tune_table().splitlines() if l]
    key = [l.split()[0] for l in lines if l.startswith("fp32/" if prec == mc.MCPT_FP32 else "bf16/")]
    assert len(key) == 1
    ctx.load_tune_table(f"{key[0]} {sb} {nw} {pd}\n")


@pytest.mark.parametrize("prec", [mc.MCPT_FP32, mc.MCPT_BF16], ids=["fp32", "bf16"])
def test_every_tile_shape_is_exact_after_polish(golden125, prec):
    prob = make_workload("hf-5x5x5-c2")
    with mc.Context(0) as ctx:
        pid = ctx.upload(prob)
        rep = ctx.autotune(pid, prec)
        assert rep["variants"] and 0 <= rep["best"] < len(rep["variants"])
        assert all(v["ms"] > 0.02 for v in rep["variants"])   # every shape did the whole pair phase
        print(f"[gpu] tune prec={prec}: " + ", ".join(f"{v['sb']}x{v['nw']}/{v['pd']}={v['ms']:.3f}ms"
                                                      for v in rep["variants"]), flush=True)
        energies = []
        for v in rep["variants"]:
            forced(ctx, pid, prec, v["sb"], v["nw"], v["pd"])
            s = ctx.run(pid, tol=1e-10, precision=prec, polish=1)
            assert s["status"] == mc.MCPT_OK
            assert abs(s["e_total"] - golden125["e_total"]) <= 1e-10 * abs(golden125["e_total"]), v
            e = ctx.energy(pid, want_t=False)
            assert np.max(np.abs(e["e_m2"] - np.asarray(golden125["e_m2"]))) <= 1e-10 * np.max(np.abs(e["e_m2"]))
            energies.append(s["e_total"])
        assert max(energies) - min(energies) <= 1e-12 * abs(energies[0])


def test_shapes_agree_without_polish_on_uneven_batch():
    """No polish: the reduced-precision iterate itself must not depend on the tile shape."""
    probs = make_cluster_batch(4, min_mono=4, max_mono=16, first=300)
    with mc.Context(0) as ctx:
        pid = ctx.upload_batch(probs)
        rep = ctx.autotune(pid, mc.MCPT_FP32)
        ref = None
        for v in rep["variants"]:
            forced(ctx, pid, mc.MCPT_FP32, v["sb"], v["nw"], v["pd"])
            s = ctx.run(pid, tol=0.0, max_sweeps=6, precision=mc.MCPT_FP32, polish=0)
            e = ctx.energy(pid)
            if ref is None:
                ref = (s, e)
                continue
            assert abs(s["e_total"] - ref[0]["e_total"]) <= 1e-10 * abs(ref[0]["e_total"]), v
            assert np.max(np.abs(e["t"] - ref[1]["t"])) <= 1e-9 * np.max(np.abs(ref[1]["t"])), v


def test_autotune_option_and_table_round_trip():
    prob = make_workload("hf-2x2x2")
    with mc.Context(0) as ctx:
        assert ctx.tune_table() == ""
        pid = ctx.upload(prob)
        s = ctx.run(pid, tol=1e-10, precision=mc.MCPT_FP32, polish=1, autotune=1)
        assert s["status"] == mc.MCPT_OK
        table = ctx.tune_table()
        assert table.count("\n") == 1 and table.startswith("fp32/")
        s2 = ctx.run(pid, tol=1e-10, precision=mc.MCPT_FP32, polish=1, autotune=1)   # uses the entry
        assert s2["sweeps"] == s["sweeps"]
        assert abs(s2["e_total"] - s["e_total"]) <= 1e-12 * abs(s["e_total"])
    with mc.Context(0) as other:
        other.load_tune_table(table)
        assert other.tune_table() == table
        for bad in ("fp32/x 7 7 1\n", "fp32/x 3 8\n", "nonsense\n"):
            with pytest.raises(mc.MCPTError) as ei:
                other.load_tune_table(bad)
            assert ei.value.status == mc.MCPT_ERR_INVALID
        pid = other.upload(prob)
        with pytest.raises(mc.MCPTError) as ei:
            other.autotune(pid, mc.MCPT_FP64)
        assert ei.value.status == mc.MCPT_ERR_INVALID
