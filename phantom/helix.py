"""Rod-lattice helical phantoms with a known fibre field.

The paper applies its method to cardiac volumes whose myocyte helix angle
rotates across the wall (Fig. 1 and the Summary); no such data is available
here, so these synthetic volumes stand in for them.

Geometry (all lengths in voxels, arrays in (z, y, x) order, axis = +z through
``center``):

* For every annulus ``[r_in, r_out]`` the helix angle varies linearly with the
  radius, ``alpha(r) = alpha_in + (alpha_out - alpha_in) * (r - r_in) / (r_out - r_in)``.
* Fibres are rods on cylindrical layers ``r_m = r_in + P/2 + m P``.  On layer m
  the coordinate ``u = zeta cos(alpha_m) - r_m theta sin(alpha_m)`` is constant
  along a helix of angle ``alpha_m``; rods repeat in ``u`` with a period ``p_m``
  close to ``P`` that divides the layer's circumference in ``u`` (so the
  pattern closes around the cylinder).
* ``d`` is the distance to the nearest rod centre line (in the (u, r) plane) and
  the intensity is ``0.5 + 0.4 sin(2 pi d / P)`` plus Gaussian noise inside the
  annuli, exactly 0 outside.
* The true fibre direction is ``cos(alpha) e_theta + sin(alpha) e_z``: helix
  angle ``alpha(r)``, intrusion angle 0.

A single 1-D sinusoid perpendicular to the fibre would give a locally
one-dimensional texture (two equal small eigenvalues, an undetermined fibre);
the rod lattice gives the two-dimensional cross-fibre texture that makes the
fibre the unique smallest-eigenvalue direction.

Noise is drawn from ``torch.Generator`` seeded per call, in fixed slabs of
``SLAB`` z-planes, so a given (spec, device) pair always yields the same bytes.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional, Sequence

import torch

SLAB = 8  # z-planes generated per step (part of the noise stream definition)


@dataclass(frozen=True)
class Annulus:
    r_in: float
    r_out: float
    alpha_in_deg: float = 60.0   # helix angle at r_in (endocardium)
    alpha_out_deg: float = -60.0  # helix angle at r_out (epicardium)


@dataclass(frozen=True)
class PhantomSpec:
    shape: tuple                      # (nz, ny, nx)
    annuli: tuple                     # Annulus, ...
    period: float = 4.0               # rod spacing P (voxels)
    noise: tuple = (0.05,)            # noise std per z-band (equal bands), fraction of full range
    dtype: str = "f32"                # "f32" or "u16"
    seed: int = 0
    with_mask: bool = False           # also return the binary annulus mask (u8)
    center: Optional[tuple] = None    # (cz, cy, cx); default: volume centre

    def centre(self):
        if self.center is not None:
            return tuple(float(c) for c in self.center)
        return tuple((n - 1) / 2.0 for n in self.shape)


def spec_small_f32(seed: int = 0) -> PhantomSpec:
    """64^3 float32, one annulus r in [12, 28], +60 deg endo to -60 deg epi, noise 0.05."""
    return PhantomSpec(shape=(64, 64, 64), annuli=(Annulus(12.0, 28.0),), period=4.0,
                       noise=(0.05,), dtype="f32", seed=seed, with_mask=False)


def spec_headline_u16(seed: int = 1, shape=(512, 512, 512)) -> PhantomSpec:
    """512^3 uint16: the 64^3 geometry scaled x8 (r in [96, 224]), same rod period
    and noise, 16-bit quantised, with the binary annulus mask."""
    return PhantomSpec(shape=tuple(shape), annuli=(Annulus(96.0, 224.0),), period=4.0,
                       noise=(0.05,), dtype="u16", seed=seed, with_mask=True)


def spec_two_annuli_u16(seed: int = 2, shape=(2048, 1024, 1024)) -> PhantomSpec:
    """Two nested annuli with opposite helix trends and noise 0.02 / 0.1 / 0.2 by z-thirds."""
    s = max(shape[1], shape[2]) / 1024.0
    return PhantomSpec(shape=tuple(shape),
                       annuli=(Annulus(128.0 * s, 256.0 * s, 60.0, -60.0),
                               Annulus(320.0 * s, 480.0 * s, -60.0, 60.0)),
                       period=4.0, noise=(0.02, 0.1, 0.2), dtype="u16", seed=seed,
                       with_mask=False)


def spec_surrogate_u16(seed: int = 3, shape=(1024, 1024, 1024)) -> PhantomSpec:
    """Surrogate inference volume: one annulus (r in [0.1875, 0.4375] x the
    in-plane size, 192..448 at 1024), helix +70 deg endo to -50 deg epi (inside
    the surrogate's training range of +-[30, 80] deg), rod period 5, noise
    0.02 / 0.06 / 0.12 by z-thirds (inside the training range 0.01..0.2),
    16-bit quantised, with the annulus mask."""
    s = max(shape[1], shape[2])
    return PhantomSpec(shape=tuple(shape), annuli=(Annulus(0.1875 * s, 0.4375 * s, 70.0, -50.0),),
                       period=5.0, noise=(0.02, 0.06, 0.12), dtype="u16", seed=seed, with_mask=True)


def helix_angle(spec: PhantomSpec, r):
    """True helix angle (radians) at cylindrical radius ``r`` (tensor), NaN outside every annulus."""
    r = torch.as_tensor(r, dtype=torch.float64)
    out = torch.full_like(r, float("nan"))
    for a in spec.annuli:
        t = (r - a.r_in) / (a.r_out - a.r_in)
        alpha = math.radians(a.alpha_in_deg) + (math.radians(a.alpha_out_deg) - math.radians(a.alpha_in_deg)) * t
        inside = (r >= a.r_in) & (r <= a.r_out)
        out = torch.where(inside, alpha, out)
    return out


def _layers(spec: PhantomSpec):
    P = spec.period
    layers = []
    for a in spec.annuli:
        n_layers = int(math.floor((a.r_out - a.r_in) / P))
        a_in, a_out = math.radians(a.alpha_in_deg), math.radians(a.alpha_out_deg)
        for m in range(n_layers):
            rm = a.r_in + P / 2.0 + m * P
            am = a_in + (a_out - a_in) * (rm - a.r_in) / (a.r_out - a.r_in)
            L = 2.0 * math.pi * rm * abs(math.sin(am))
            pm = P if L < P else L / max(1, round(L / P))
            layers.append((rm, math.cos(am), math.sin(am), pm))
    return layers


def generate(spec: PhantomSpec, device="cpu"):
    """Return ``{"volume": tensor, "mask": tensor|None, "center": (cz,cy,cx), "direction": (1,0,0)}``.

    ``volume`` is float32 or uint16 (C-order (z, y, x)) on ``device``; ``mask`` is
    uint8 (1 inside an annulus) when ``spec.with_mask``.
    """
    nz, ny, nx = spec.shape
    dev = torch.device(device)
    cz, cy, cx = spec.centre()
    P = spec.period
    layers = _layers(spec)
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(spec.seed))

    out_dtype = torch.float32 if spec.dtype == "f32" else torch.uint16
    vol = torch.empty((nz, ny, nx), dtype=out_dtype, device=dev)
    mask = torch.empty((nz, ny, nx), dtype=torch.uint8, device=dev) if spec.with_mask else None

    y = torch.arange(ny, dtype=torch.float64, device=dev).view(1, ny, 1) - cy
    x = torch.arange(nx, dtype=torch.float64, device=dev).view(1, 1, nx) - cx
    r = torch.sqrt(y * y + x * x)            # (1, ny, nx)
    theta = torch.atan2(y, x)                # (1, ny, nx)
    inside = torch.zeros_like(r, dtype=torch.bool)
    for a in spec.annuli:
        inside |= (r >= a.r_in) & (r <= a.r_out)
    bands = len(spec.noise)

    for z0 in range(0, nz, SLAB):
        z1 = min(nz, z0 + SLAB)
        zeta = torch.arange(z0, z1, dtype=torch.float64, device=dev).view(-1, 1, 1) - cz
        d = torch.full((z1 - z0, ny, nx), float("inf"), dtype=torch.float64, device=dev)
        for rm, ca, sa, pm in layers:
            u = zeta * ca - (rm * sa) * theta
            du = torch.remainder(u + 0.5 * pm, pm) - 0.5 * pm
            d = torch.minimum(d, torch.sqrt(du * du + (r - rm) ** 2))
        val = 0.5 + 0.4 * torch.sin((2.0 * math.pi / P) * d)
        noise = torch.randn((z1 - z0, ny, nx), generator=gen, dtype=torch.float64, device=dev)
        zi = torch.arange(z0, z1, device=dev).view(-1, 1, 1)
        band = torch.clamp((zi * bands) // nz, max=bands - 1)
        sig = torch.tensor(spec.noise, dtype=torch.float64, device=dev)[band]
        val = torch.where(inside, val + sig * noise, torch.zeros_like(val))
        if spec.dtype == "u16":
            q = torch.round(torch.clamp(val, 0.0, 1.0) * 65535.0)
            vol[z0:z1] = q.to(torch.int32).to(torch.uint16)
        else:
            vol[z0:z1] = val.to(torch.float32)
        if mask is not None:
            mask[z0:z1] = inside.expand(z1 - z0, ny, nx).to(torch.uint8)
    return {"volume": vol, "mask": mask, "center": (cz, cy, cx), "direction": (1.0, 0.0, 0.0)}


def cylindrical_radius(spec: PhantomSpec, shape: Optional[Sequence[int]] = None, origin=(0, 0, 0)):
    """Distance of each voxel (of a block at ``origin``) from the phantom axis, float64 (1, ny, nx)."""
    nz, ny, nx = shape if shape is not None else spec.shape
    cz, cy, cx = spec.centre()
    y = torch.arange(origin[1], origin[1] + ny, dtype=torch.float64).view(1, ny, 1) - cy
    x = torch.arange(origin[2], origin[2] + nx, dtype=torch.float64).view(1, 1, nx) - cx
    return torch.sqrt(y * y + x * x)


def batch_crops(volume_shape=(512, 512, 512), n: int = 200, seed: int = 4, inner=(64, 384),
                rhos=(2.0, 3.0, 4.0), halo_per_rho: float = 3.0):
    """Uneven halo-padded chunks of one volume: for each of ``n`` chunks an
    integration scale rho drawn from ``rhos``, interior sides drawn uniformly
    from [inner[0], inner[1]] per axis, a halo of round(halo_per_rho * rho) on
    every side, and a uniform position where the padded chunk fits.  Returns a
    list of ((z, y, x) origin, (nz, ny, nx) padded shape, rho)."""
    import numpy as np

    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        rho = float(rng.choice(rhos))
        h = int(round(halo_per_rho * rho))
        shp = tuple(int(s) + 2 * h for s in rng.integers(inner[0], inner[1] + 1, size=3))
        org = tuple(int(rng.integers(0, volume_shape[d] - shp[d] + 1)) for d in range(3))
        out.append((org, shp, rho))
    return out
