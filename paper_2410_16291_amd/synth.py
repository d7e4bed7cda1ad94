"""Seeded synthetic inputs shaped like the paper's workloads.

The paper measures on immunofluorescence images of whole tumor sections (Sec. IV-A), which are not
available here; these generators stand in for them.  This module holds input generation only: no
step of the integral-image method lives here, so the oracle and the HIP path can both draw their
inputs from it.  Everything is numpy and deterministic in its seed.

  poisson_counts  per-pixel cell counts, Poisson(lam), uint8            (512x512, lam = 0.05)
  lognormal_u16   stained intensities, rint(lognormal(mu, sigma)) clipped to uint16
  thomas_mask     binary cell-centroid mask from a Thomas cluster process, uint8
  uneven_batch    a list of uneven-sized lognormal uint16 images
  request_stream  Poisson arrivals of build / query requests for the serving loop
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np


def poisson_counts(H: int, W: int, lam: float = 0.05, seed: int = 0) -> np.ndarray:
    """Per-pixel Poisson(lam) cell counts as uint8 (counts above 255 are clipped)."""
    rng = np.random.default_rng(seed)
    return np.minimum(rng.poisson(lam, (H, W)), 255).astype(np.uint8)


def lognormal_u16(H: int, W: int, mu: float = 6.0, sigma: float = 1.0, seed: int = 1,
                  rng: Optional[np.random.Generator] = None) -> np.ndarray:
    """Log-normal intensities, rounded to nearest and clipped to 0..65535, as uint16."""
    rng = rng if rng is not None else np.random.default_rng(seed)
    out = np.empty((H, W), np.uint16)
    rows = max(1, (1 << 24) // max(W, 1))          # generate in bands to bound temporaries
    for y in range(0, H, rows):
        band = rng.lognormal(mu, sigma, (min(rows, H - y), W))
        np.clip(np.rint(band), 0, 65535, out=band)
        out[y:y + band.shape[0]] = band.astype(np.uint16)
    return out


def thomas_points(H: int, W: int, parent_density: float = 2e-6, children: int = 200,
                  sigma: float = 40.0, seed: int = 2):
    """Child positions (ys, xs) of a Thomas cluster process inside an H x W image.

    Parents: Poisson(parent_density * H * W) of them, uniform over the image.  Each parent has
    exactly `children` children displaced by independent N(0, sigma^2) offsets per axis; a child
    lands on pixel floor(parent + offset) and is dropped if that pixel is outside the image.
    """
    rng = np.random.default_rng(seed)
    n_par = rng.poisson(parent_density * H * W)
    py = rng.uniform(0.0, H, n_par)
    px = rng.uniform(0.0, W, n_par)
    ys = np.floor(np.repeat(py, children) + rng.normal(0.0, sigma, n_par * children)).astype(np.int64)
    xs = np.floor(np.repeat(px, children) + rng.normal(0.0, sigma, n_par * children)).astype(np.int64)
    keep = (ys >= 0) & (ys < H) & (xs >= 0) & (xs < W)
    return ys[keep], xs[keep]


def thomas_mask(H: int, W: int, parent_density: float = 2e-6, children: int = 200,
                sigma: float = 40.0, seed: int = 2, out: Optional[np.ndarray] = None) -> np.ndarray:
    """Binary uint8 centroid mask (1 where at least one child landed) of a Thomas process."""
    ys, xs = thomas_points(H, W, parent_density, children, sigma, seed)
    if out is None:
        out = np.zeros((H, W), np.uint8)
    else:
        out[...] = 0
    out[ys, xs] = 1
    return out


def uneven_sizes(n: int = 64, lo: int = 1000, hi: int = 12000, seed: int = 3):
    """n (H, W) pairs with each side uniform on the integers lo..hi."""
    rng = np.random.default_rng(seed)
    return [tuple(int(v) for v in rng.integers(lo, hi + 1, 2)) for _ in range(n)]


def uneven_batch(n: int = 64, lo: int = 1000, hi: int = 12000, seed: int = 3,
                 mu: float = 6.0, sigma: float = 1.0) -> List[np.ndarray]:
    """n lognormal uint16 images with sides uniform on lo..hi (one generator stream)."""
    rng = np.random.default_rng(seed)
    sizes = [tuple(int(v) for v in rng.integers(lo, hi + 1, 2)) for _ in range(n)]
    return [lognormal_u16(h, w, mu, sigma, rng=rng) for (h, w) in sizes]


@dataclasses.dataclass
class Request:
    """One serving request: build a new image's tables, or query windows of a resident one."""
    t_arrival: float            # seconds from stream start
    kind: str                   # "build" or "query"
    image_seed: int = 0         # build: seed of the image; query: index among earlier builds
    H: int = 0
    W: int = 0
    win_h: int = 0
    win_w: int = 0
    stride: int = 1
    op: str = "sum"             # "sum" or "mean_std"


def request_stream(rate: float = 50.0, duration: float = 120.0, seed: int = 4,
                   build_frac: float = 0.2, side_lo: int = 2000, side_hi: int = 16000,
                   win_lo: int = 16, win_hi: int = 512, stride_hi: int = 8,
                   mean_std_frac: float = 0.25) -> List[Request]:
    """Poisson arrivals at `rate` per second mixing image builds and window queries.

    The first request is always a build, so queries always have a resident image to name.
    Query windows are uniform on win_lo..win_hi per side, clamped to the image later by the
    server; strides are uniform on 1..stride_hi.
    """
    rng = np.random.default_rng(seed)
    t, reqs, n_built = 0.0, [], 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        if n_built == 0 or rng.random() < build_frac:
            H, W = (int(v) for v in rng.integers(side_lo, side_hi + 1, 2))
            reqs.append(Request(t, "build", image_seed=1000 + n_built, H=H, W=W))
            n_built += 1
        else:
            reqs.append(Request(t, "query", image_seed=int(rng.integers(0, n_built)),
                                win_h=int(rng.integers(win_lo, win_hi + 1)),
                                win_w=int(rng.integers(win_lo, win_hi + 1)),
                                stride=int(rng.integers(1, stride_hi + 1)),
                                op="mean_std" if rng.random() < mean_std_frac else "sum"))
    return reqs


# ---------------------------------------------------------------- device-side generators
# Large inputs are drawn on the GPU with torch's seeded Philox generator (same distributions as
# above, float32 draws; not the same numbers as the numpy streams).  Tests that compare such an
# input with the oracle copy the generated image to the host first.

def lognormal_u16_device(H: int, W: int, seed: int, device, mu: float = 6.0, sigma: float = 1.0,
                         pitch: Optional[int] = None):
    """Log-normal intensities rounded to nearest and clipped to 0..65535, as a uint16 tensor
    (`pitch`: row pitch in elements of a wider buffer the image is a view of)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    z = torch.randn((H, W), generator=g, device=device, dtype=torch.float32)
    v = torch.exp_(z.mul_(sigma).add_(mu)).round_().clamp_(0, 65535).to(torch.int32)
    del z
    v -= (v >= 32768).to(torch.int32) * 65536          # two's-complement wrap into int16 range
    img = v.to(torch.int16)
    if pitch is not None and pitch != W:
        if pitch < W:
            raise ValueError("pitch must be >= W")
        buf = torch.zeros((H, pitch), dtype=torch.int16, device=device)
        buf[:, :W] = img
        img = buf[:, :W]
    return img.view(torch.uint16)


def thomas_mask_device(H: int, W: int, seed: int, device, parent_density: float = 2e-6, children: int = 200,
                       sigma: float = 40.0, out=None):
    """thomas_mask drawn on the host (the same points) and scattered into a device uint8 image:
    a new contiguous one, or `out` (an H x W uint8 device view of any row pitch, overwritten)."""
    import torch
    ys, xs = thomas_points(H, W, parent_density, children, sigma, seed)
    if out is None:
        img = torch.zeros((H, W), dtype=torch.uint8, device=device)
        img.view(-1)[torch.from_numpy(ys * W + xs).to(device)] = 1
        return img
    if tuple(out.shape) != (H, W) or out.dtype != torch.uint8:
        raise ValueError("out must be an H x W uint8 tensor")
    out.zero_()
    out[torch.from_numpy(ys).to(out.device), torch.from_numpy(xs).to(out.device)] = 1
    return out
