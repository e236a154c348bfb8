"""HIP path vs the oracle at the widths where the layout changes (MI355X only).

The workspace rows are padded to a multiple of 32 floats above 32 (else 4),
and the final pass covers a row with 256-output segments or, for narrow rows
and radii up to 16, with 64-output segments of four consecutive rows.  These
cases sit on both sides of each boundary, with a row count (nz * ny = 35) that
is not a multiple of four, so the last wave of 64-output segments holds rows
past the end; the radius-20 cases must take 256-output segments (one row
narrower than a segment, the others on both sides of two segments' width,
with rows that start off 16 bytes).
"""

import sys
import zlib

import numpy as np
import pytest
import torch

import oracle
import paper_2508_07476_amd as st

from _parity import assert_parity, compare, summary

pytestmark = pytest.mark.gpu

ALL = ("e3", "evals", "fa", "ha", "ia", "flags")


@pytest.mark.parametrize("nx,rho", [(31, 2.0), (32, 2.0), (33, 2.0), (63, 2.0), (64, 3.0), (65, 3.0),
                                    (255, 2.0), (256, 4.0), (257, 2.0), (97, 5.0),
                                    (511, 5.0), (512, 5.0), (513, 5.0)])
def test_widths_at_layout_boundaries(nx, rho):
    shape = (5, 7, nx)
    print(f"case: shape={shape} rho={rho}", file=sys.stderr, flush=True)
    gen = torch.Generator().manual_seed(zlib.crc32(repr(shape).encode()))
    vol = torch.rand(shape, generator=gen, dtype=torch.float64).to(torch.float32)
    mask = (torch.rand(shape, generator=gen) > 0.2).to(torch.uint8)
    center, direction = (2.0, 3.25, (nx - 1) / 2 + 0.4), (0.3, 1.0, 0.2)
    g = st.st_compute(vol.cuda(), 1.0, rho, mask=mask.cuda(), axis_center=center, axis_direction=direction,
                      outputs=ALL)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in g.items()}
    o = oracle.compute(vol.numpy(), mask.numpy(), 1.0, rho, axis_center=center, axis_direction=direction)
    stats = compare(g, o, shape, center, direction, mask=mask.numpy())
    print(summary(stats), file=sys.stderr, flush=True)
    assert stats["n_checked"] > 0
    assert_parity(stats, f"nx={nx}")
    out = mask.numpy() == 0
    assert np.all(g["flags"][out] == st.ST_FLAG_OUTSIDE_MASK)
    assert np.all(g["e3"][:, out] == 0)
