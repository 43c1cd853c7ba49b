"""Seeded Tucker + sparse tensors drawn directly on the GPU with torch.

Same recipe as ``generators.tucker_workload`` (Haar factors, N(0, 1) core,
unit-RMS or unscaled low-rank part, exact count of corrupted positions drawn
without replacement, additive uniform values) but with torch's generator, so
that the serving trace's hundreds of tensors are produced on the device in
milliseconds.  Holds none of the solver's arithmetic.
"""

from __future__ import annotations

from typing import Optional, Sequence, Tuple

import numpy as np


def tucker_on_device(dims: Sequence[int], ranks: Sequence[int], frac: float, seed: int,
                     value_range: Tuple[float, float] = (-10.0, 10.0), device="cuda",
                     dtype=None, scale: Optional[str] = "rms"):
    """Return (T, L, mask) as torch tensors on `device`; T in `dtype` (float32
    by default), L in float64, mask boolean.  ``scale``: ``"rms"`` scales the
    low-rank part to unit root-mean-square, None leaves the Tucker product as
    drawn (Section 5.1's synthetic tensors)."""
    import torch
    from .generators import haar_stiefel

    dtype = torch.float32 if dtype is None else dtype
    rng = np.random.default_rng(seed)
    factors = [torch.from_numpy(haar_stiefel(rng, int(d), int(r))).to(device)
               for d, r in zip(dims, ranks)]
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    L = torch.randn(tuple(int(r) for r in ranks), generator=g, device=device, dtype=torch.float64)
    for n, u in enumerate(factors):
        L = torch.movedim(torch.tensordot(u, L, dims=([1], [n])), 0, n)
    if scale == "rms":
        L = L / torch.sqrt(torch.mean(L * L))
    elif scale is not None:
        raise ValueError(f"unknown scale {scale!r}")
    numel = L.numel()
    count = int(round(frac * numel))
    pos = torch.randperm(numel, generator=g, device=device)[:count]
    lo, hi = value_range
    vals = torch.rand(count, generator=g, device=device, dtype=torch.float64) * (hi - lo) + lo
    T = L.reshape(-1).clone()
    T[pos] += vals
    mask = torch.zeros(numel, dtype=torch.bool, device=device)
    mask[pos] = True
    return T.reshape(L.shape).to(dtype).contiguous(), L.contiguous(), mask.reshape(L.shape)
