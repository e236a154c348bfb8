"""The 200-chunk batch at its full size on the GPU (MI355X only): the crops of
``helix.batch_crops()`` (interior sides uniform in 64..384 per axis, halo
3 rho, rho in {2, 3, 4}, sigma 1) of the 512^3 uint16 phantom with its mask,
3.0 G voxels in all, run as one batch of 8 graph-replayed chains.

* Every chunk's outputs equal, bitwise, those of st_compute on the same crop,
  and the grouped launches (one kernel per pass over a round of chunks) give
  the same bits.
* Each padded chunk is its own volume, reflected at its faces (the halo of
  3 rho is below R_sigma + R_rho, so a chunk is compared with the oracle run on
  the same padded crop, not with the whole volume).  The FP64 oracle checks the
  smallest chunk of every rho whole, and four 32^3 blocks of the largest chunk
  that reach into its mask: against its low z face, against its high z face,
  in its middle z plane and against one y or x face (each block padded by
  R_sigma + R_rho inside the chunk, clipped at the chunk's faces, which keeps
  the block's values exact).
"""

import multiprocessing
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest
import torch

import oracle
import paper_2508_07476_amd as st
from phantom import helix

from _oracle_worker import oracle_cut
from _parity import assert_parity, compare, summary

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SIGMA = 1.0
OUTS = ("e3", "evals", "fa", "ha", "ia", "flags")
SHAPE = (512, 512, 512)


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _workers():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _blocks_in_mask(mask, B):
    """Four B^3 blocks of a chunk that reach into its mask: one at the low corner
    and one against the far z face (corners first, then face centres), one at
    the middle z plane (the centre first, then points a quarter of the way in y
    and x) and one at the middle of a y or x face, each the first candidate of
    its kind with at least a tenth of its voxels inside."""
    n = mask.shape
    lo = lambda d: 0  # noqa: E731
    hi = lambda d: n[d] - B  # noqa: E731
    mid = lambda d: (n[d] - B) // 2  # noqa: E731

    def inside(bo):
        return float(mask[bo[0]:bo[0] + B, bo[1]:bo[1] + B, bo[2]:bo[2] + B].float().mean()) >= 0.1

    corners = [(f(0), g(1), h(2)) for f in (lo, hi) for g in (lo, hi) for h in (lo, hi)]
    kinds = [
        [c for c in corners if c[0] == 0] + [(0, mid(1), mid(2))],
        [c for c in corners if c[0] == hi(0)] + [(hi(0), mid(1), mid(2))],
        [(mid(0), int(f * hi(1)), int(g * hi(2))) for f in (0.5, 0.25, 0.75) for g in (0.5, 0.25, 0.75)],
        [(mid(0), 0, mid(2)), (mid(0), hi(1), mid(2)), (mid(0), mid(1), 0), (mid(0), mid(1), hi(2))],
    ]
    out = []
    for cand in kinds:
        pick = next((c for c in cand if inside(c)), None)
        assert pick is not None, cand
        out.append(pick)
    return out


def _host(res, box=None):
    s = (slice(None),) * 3 if box is None else tuple(slice(a, b) for a, b in box)
    return {k: (v[(slice(None),) + s] if v.dim() == 4 else v[s]).cpu().numpy() for k, v in res.items()}


def test_batch_of_200_chunks_bitwise_and_against_the_oracle():
    ph = helix.generate(helix.spec_headline_u16(shape=SHAPE), device=DEV)
    crops = helix.batch_crops(SHAPE)
    assert len(crops) == 200 and {r for _, _, r in crops} == {2.0, 3.0, 4.0}
    chunks = []
    for org, shp, rho in crops:
        sl = tuple(slice(org[d], org[d] + shp[d]) for d in range(3))
        chunks.append({"volume": ph["volume"][sl].contiguous(), "mask": ph["mask"][sl].contiguous(),
                       "rho": rho, "origin": org})
    nvox = sum(c["volume"].numel() for c in chunks)
    _log(f"case: batch of {len(chunks)} chunks, {nvox} voxels, lanes=0")
    b = st.Batch(chunks, SIGMA, axis_center=ph["center"], axis_direction=ph["direction"], outputs=OUTS,
                 lanes=0)
    b.launch()
    torch.cuda.synchronize()

    # oracle jobs first, so the workers run while the GPU compares the chunks
    sizes = [int(np.prod(s)) for _, s, _ in crops]
    picks = {}
    for i, (_, _, rho) in enumerate(crops):
        if rho not in picks or sizes[i] < sizes[picks[rho]]:
            picks[rho] = i
    big = int(np.argmax(sizes))
    B = 32
    jobs = []  # (chunk index, block origin inside the chunk or None for whole, shape)
    for rho, i in sorted(picks.items()):
        jobs.append((i, None, crops[i][1]))
    for bo in _blocks_in_mask(chunks[big]["mask"], B):
        jobs.append((big, bo, (B, B, B)))
    pool = ProcessPoolExecutor(max_workers=_workers(), mp_context=multiprocessing.get_context("spawn"))
    futs = []
    for i, bo, shp in jobs:
        org, cshp, rho = crops[i]
        vol = chunks[i]["volume"].cpu().numpy()
        msk = chunks[i]["mask"].cpu().numpy()
        if bo is None:
            futs.append(pool.submit(oracle_cut, vol, msk, SIGMA, rho, ph["center"], ph["direction"], org,
                                    tuple((0, s) for s in cshp)))
            continue
        halo = oracle.radius(SIGMA) + oracle.radius(rho)
        lo = [max(0, bo[d] - halo) for d in range(3)]
        hi = [min(cshp[d], bo[d] + B + halo) for d in range(3)]
        sl = tuple(slice(lo[d], hi[d]) for d in range(3))
        cut = tuple((bo[d] - lo[d], bo[d] - lo[d] + B) for d in range(3))
        futs.append(pool.submit(oracle_cut, vol[sl], msk[sl], SIGMA, rho, ph["center"], ph["direction"],
                                tuple(org[d] + lo[d] for d in range(3)), cut))

    # every chunk bitwise equal to st_compute on its crop
    ws = torch.empty(max(st.st_workspace_bytes(tuple(c["volume"].shape)) for c in chunks), dtype=torch.uint8,
                     device=DEV)
    for i, (c, res) in enumerate(zip(chunks, b.results)):
        center = [ph["center"][d] - c["origin"][d] for d in range(3)]
        single = st.st_compute(c["volume"], SIGMA, c["rho"], mask=c["mask"], axis_center=center,
                               axis_direction=ph["direction"], outputs=OUTS, workspace=ws)
        for k in OUTS:
            assert torch.equal(res[k], single[k]), (i, crops[i], k)
        del single
    del ws
    _log("all 200 chunks bitwise equal to st_compute")
    # the same chunks as grouped launches: bitwise equal to the chains
    g = st.Batch(chunks, SIGMA, axis_center=ph["center"], axis_direction=ph["direction"], outputs=OUTS,
                 lanes=st.ST_BATCH_GROUPED)
    _log("grouped plan", g.plan())
    g.launch()
    torch.cuda.synchronize()
    for i, (x, y) in enumerate(zip(g.results, b.results)):
        for k in OUTS:
            assert torch.equal(x[k], y[k]), ("grouped", i, k)
    g.close()
    del g
    torch.cuda.empty_cache()
    _log("grouped launches bitwise equal to the chains")

    try:
        for (i, bo, shp), f in zip(jobs, futs):
            org, cshp, rho = crops[i]
            o = f.result()
            if bo is None:
                g = _host(b.results[i])
                gorg = org
            else:
                g = _host(b.results[i], tuple((bo[d], bo[d] + B) for d in range(3)))
                gorg = tuple(org[d] + bo[d] for d in range(3))
            stats = compare(g, o, shp, ph["center"], ph["direction"], origin=gorg)
            _log(f"chunk {i} {cshp} rho {rho} block {bo}:", summary(stats))
            assert stats["n_checked"] > 0, (i, bo)
            assert_parity(stats, f"chunk {i} block {bo}")
    finally:
        pool.shutdown(wait=True, cancel_futures=True)
    b.close()
