"""Chunk batches on the GPU (MI355X only).

A batch of uneven crops of one uint16 phantom (with mask and axis), mixed
integration scales rho in {2, 3, 4}, one crop thinner than its filter radius:
every chunk's outputs equal, bitwise, those of st_compute on the same crop, and
match the FP64 oracle run on the crop (each crop is its own volume, reflected at
its faces; its origin places it in the axis' frame).  Graph replays with eager
work in between, direct multi-stream enqueue and every autotuned configuration
(tile shapes, chains, split targets, graph or direct) give the same bits;
graph replays of an untuned batch (lanes = 0: 8 chains) are checked on their
own.
"""

import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2508_07476_amd as st
from phantom import helix

from _parity import assert_parity, compare, summary

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SIGMA = 1.0
OUTS = ("e3", "evals", "fa", "ha", "ia", "flags")
# (origin (z, y, x), shape, rho)
CROPS = [((10, 20, 30), (40, 52, 36), 2.0), ((0, 0, 0), (64, 40, 48), 3.0),
         ((30, 5, 8), (33, 47, 70), 4.0), ((20, 30, 2), (50, 50, 50), 2.0),
         ((60, 40, 10), (28, 60, 44), 3.0), ((5, 60, 40), (72, 33, 29), 4.0),
         ((40, 70, 90), (12, 9, 35), 4.0)]


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def phantom():
    spec = helix.PhantomSpec(shape=(96, 112, 128), annuli=(helix.Annulus(16.0, 44.0),), period=4.0,
                             noise=(0.05,), dtype="u16", seed=4, with_mask=True)
    ph = helix.generate(spec)
    return ph


def _crop(t, org, shp):
    return t[org[0]:org[0] + shp[0], org[1]:org[1] + shp[1], org[2]:org[2] + shp[2]].contiguous()


def _chunks(ph):
    out = []
    for i, (org, shp, rho) in enumerate(CROPS):
        c = {"volume": _crop(ph["volume"], org, shp).to(DEV), "rho": rho, "origin": org}
        if i % 2 == 0:
            c["mask"] = _crop(ph["mask"], org, shp).to(DEV)
        out.append(c)
    return out


def _snapshot(batch):
    torch.cuda.synchronize()
    return [{k: v.clone() for k, v in r.items()} for r in batch.results]


def _same(a, b):
    return all(torch.equal(x[k], y[k]) for x, y in zip(a, b) for k in x)


def test_batch_matches_single_calls_and_oracle(phantom):
    chunks = _chunks(phantom)
    _log("case: batch of", len(chunks), "chunks, lanes=3")
    b = st.Batch(chunks, SIGMA, axis_center=phantom["center"], axis_direction=phantom["direction"],
                 outputs=OUTS, lanes=3)
    b.launch()
    torch.cuda.synchronize()
    for i, (c, res) in enumerate(zip(chunks, b.results)):
        org, shp, rho = CROPS[i]
        center = [phantom["center"][d] - org[d] for d in range(3)]
        single = st.st_compute(c["volume"], SIGMA, rho, mask=c.get("mask"), axis_center=center,
                               axis_direction=phantom["direction"], outputs=OUTS)
        torch.cuda.synchronize()
        for k in OUTS:
            assert torch.equal(res[k], single[k]), (i, k)
        g = {k: v.cpu().numpy() for k, v in res.items()}
        o = oracle.compute(c["volume"].cpu().numpy(), None if "mask" not in c else c["mask"].cpu().numpy(),
                           SIGMA, rho, axis_center=phantom["center"], axis_direction=phantom["direction"],
                           origin=org)
        stats = compare(g, o, shp, phantom["center"], phantom["direction"], origin=org)
        _log(f"chunk {i} {shp} rho {rho}:", summary(stats))
        assert_parity(stats, f"chunk {i}")
    b.close()


def test_batch_replays_tuning_and_direct_enqueue_are_bitwise_stable(phantom):
    chunks = _chunks(phantom)
    b = st.Batch(chunks, SIGMA, axis_center=phantom["center"], axis_direction=phantom["direction"],
                 outputs=OUTS, lanes=0)
    _log("case: lanes=0 batch, initial config", b.config())
    b.launch()
    ref = _snapshot(b)
    for rep in range(3):  # replays with eager work (clearing the outputs) in between
        for r in b.results:
            for v in r.values():
                v.zero_()
        torch.cuda.synchronize()
        b.launch()
        assert _same(_snapshot(b), ref), rep
    for t in range(2):  # tuning twice: the second call replaces the first call's graph
        cfg = b.tune(reps=1)
        _log("tuned config", cfg, "tiles", [b.tiles(i) for i in range(len(chunks))])
        # every configuration the tuner ran wrote the same bits
        assert _same(_snapshot(b), ref), t
        assert 1 <= cfg["lanes"] <= st.ST_BATCH_MAX_LANES and cfg["best_ms"] > 0
        for i in range(len(chunks)):
            rows, lanes = b.tiles(i)
            assert rows in (4, 8) and lanes in (16, 64), (i, rows, lanes)
        for r in b.results:
            for v in r.values():
                v.zero_()
        torch.cuda.synchronize()
        b.launch()
        assert _same(_snapshot(b), ref), t
    b.close()


def test_grouped_batch_matches_chains_bitwise(phantom):
    """Grouped launches (each pass one kernel over a round of chunks, geometry
    from a device table) give the same bits as the chains, replayed and direct;
    with a workspace of two slots the chunks fall into several rounds."""
    chunks = _chunks(phantom)
    ref = st.Batch(chunks, SIGMA, axis_center=phantom["center"], axis_direction=phantom["direction"],
                   outputs=OUTS, lanes=3)
    ref.launch()
    want = _snapshot(ref)
    ref.close()
    shapes = [tuple(c["volume"].shape) for c in chunks]
    for ws_lanes in (0, 2):
        ws = torch.empty(st.Batch.workspace_bytes(shapes, lanes=ws_lanes or st.ST_BATCH_MAX_LANES),
                         dtype=torch.uint8, device=DEV)
        b = st.Batch(chunks, SIGMA, axis_center=phantom["center"], axis_direction=phantom["direction"],
                     outputs=OUTS, lanes=st.ST_BATCH_GROUPED, workspace=ws)
        plan = b.plan()
        _log("case: grouped batch, workspace of", ws_lanes or st.ST_BATCH_MAX_LANES, "slots, plan", plan)
        assert plan["grouped"] and plan["rounds"] >= 1
        if ws_lanes == 2:
            assert plan["rounds"] >= 2
        for rep in range(2):
            for r in b.results:
                for v in r.values():
                    v.zero_()
            torch.cuda.synchronize()
            b.launch()
            got = _snapshot(b)
            for i, (x, y) in enumerate(zip(got, want)):
                for k in OUTS:
                    assert torch.equal(x[k], y[k]), (ws_lanes, rep, i, k)
        b.close()
        del ws


# small integration scales (rho radius 2 and 4) on narrow rows: the 16-lane
# final-pass segments of those radii, in chains and in grouped launches
CROPS_SMALL_RHO = [((10, 20, 30), (40, 52, 36), 0.5), ((0, 0, 0), (64, 40, 48), 1.0),
                   ((30, 5, 8), (33, 47, 70), 1.0), ((20, 30, 2), (20, 25, 50), 0.5)]


def test_small_rho_chunks_chains_grouped_and_single_calls_agree(phantom):
    chunks = []
    for i, (org, shp, rho) in enumerate(CROPS_SMALL_RHO):
        c = {"volume": _crop(phantom["volume"], org, shp).to(DEV), "rho": rho, "origin": org}
        if i % 2 == 1:
            c["mask"] = _crop(phantom["mask"], org, shp).to(DEV)
        chunks.append(c)
    kw = dict(axis_center=phantom["center"], axis_direction=phantom["direction"], outputs=OUTS)
    _log("case: small-rho chunks, chains / grouped / single calls")
    chains = st.Batch(chunks, SIGMA, lanes=2, **kw)
    chains.launch()
    a = _snapshot(chains)
    chains.close()
    grouped = st.Batch(chunks, SIGMA, lanes=st.ST_BATCH_GROUPED, **kw)
    assert grouped.plan()["grouped"]
    grouped.launch()
    b = _snapshot(grouped)
    grouped.close()
    for i, c in enumerate(chunks):
        center = tuple(phantom["center"][d] - c["origin"][d] for d in range(3))
        one = st.st_compute(c["volume"], SIGMA, c["rho"], mask=c.get("mask"), axis_center=center,
                            axis_direction=phantom["direction"], outputs=OUTS)
        torch.cuda.synchronize()
        for k in OUTS:
            assert torch.equal(a[i][k], one[k]), (i, k, "chains")
            assert torch.equal(b[i][k], one[k]), (i, k, "grouped")


def test_batch_graph_replays_are_bitwise_stable(phantom):
    chunks = _chunks(phantom)
    b = st.Batch(chunks, SIGMA, axis_center=phantom["center"], axis_direction=phantom["direction"],
                 outputs=OUTS, lanes=0)
    cfg = b.config()
    _log("case: lanes=0 batch replays, config", cfg)
    assert cfg["lanes"] == st.ST_BATCH_MAX_LANES and cfg["graph"]
    b.launch()
    ref = _snapshot(b)
    for rep in range(3):  # replays with eager work (clearing the outputs) in between
        for r in b.results:
            for v in r.values():
                v.zero_()
        torch.cuda.synchronize()
        b.launch()
        assert _same(_snapshot(b), ref), rep
    assert all(b.tiles(i) == (0, 0) for i in range(len(chunks)))  # untuned: library defaults
    b.close()


def test_batch_completion_record(phantom):
    """The completion record (read without waiting for the GPU): no chunk is
    done before the first launch, every chunk once a launch has finished, and
    the launch count follows the launches (the tuner's timing runs included),
    for chains and grouped launches."""
    chunks = _chunks(phantom)
    for lanes in (0, st.ST_BATCH_GROUPED):
        b = st.Batch(chunks, SIGMA, axis_center=phantom["center"], axis_direction=phantom["direction"],
                     outputs=OUTS, lanes=lanes)
        _log("case: completion record, lanes", lanes)
        done, launches = b.progress()
        assert launches == 0 and not any(done)
        b.launch()
        torch.cuda.synchronize()
        done, launches = b.progress()
        assert launches == 1 and all(done), done
        b.tune(reps=1)  # its timing runs are launches too, and leave every chunk complete
        done, tuned = b.progress()
        assert tuned > 1 and all(done), (tuned, done)
        for _ in range(2):
            b.launch()
        torch.cuda.synchronize()
        done, launches = b.progress()
        assert launches == tuned + 2 and all(done), (launches, done)
        b.close()
