"""Seeded generators for the synthetic TRPCA workloads.

Every tensor is drawn on the host in float64 with ``numpy.random.default_rng``
from an explicit seed, so the oracle and the GPU path read identical bytes.
Nothing here computes any step of the solver.

Recipes (low-rank part ``L``, sparse part ``S``, observed ``T = L + S`` unless
stated otherwise):

* Tucker model of Section 5.1: a core with N(0, 1) entries multiplied along
  every mode by a column-orthonormal factor drawn from the Haar measure
  (QR of a Gaussian matrix with the signs of R's diagonal folded into Q).
* Sparse corruption: an exact count ``round(frac * numel)`` of positions drawn
  without replacement; values either added (``additive``) or substituted
  (``replace``) according to the recipe.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class Workload:
    """One synthetic TRPCA instance.

    ``T`` is the observed tensor (float64, C order).  ``L`` is the planted
    low-rank part, ``S`` the planted sparse part and ``mask`` the planted
    support (``S != 0`` positions chosen by the generator).
    """

    name: str
    T: np.ndarray
    L: np.ndarray
    S: np.ndarray
    mask: np.ndarray
    ranks: Tuple[int, ...]
    tol: float
    max_iter: int
    precision: str  # "fp64", "fp32" or "bf16"
    meta: Dict[str, object] = dataclasses.field(default_factory=dict)

    @property
    def dims(self) -> Tuple[int, ...]:
        return tuple(int(d) for d in self.T.shape)

    def observed(self, dtype=np.float64) -> np.ndarray:
        """``T`` rounded to ``dtype``; float32 runs give both sides these bytes."""
        return np.ascontiguousarray(self.T.astype(dtype))


def haar_stiefel(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    """A rows x cols matrix with orthonormal columns, Haar distributed."""
    g = rng.standard_normal((rows, cols))
    q, r = np.linalg.qr(g)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d


def tucker(core: np.ndarray, factors: Sequence[np.ndarray]) -> np.ndarray:
    """``core x_1 U_1 x_2 U_2 ... x_N U_N`` (mode products of Section 2.1)."""
    out = core
    for n, u in enumerate(factors):
        out = np.moveaxis(np.tensordot(u, out, axes=(1, n)), 0, n)
    return np.ascontiguousarray(out)


def _positions(rng: np.random.Generator, numel: int, frac: float) -> np.ndarray:
    count = int(round(frac * numel))
    return rng.choice(numel, size=count, replace=False)


def tucker_workload(
    name: str,
    dims: Sequence[int],
    core_ranks: Sequence[int],
    frac: float,
    seed: int,
    *,
    value_range: Tuple[float, float] = (-1.0, 1.0),
    mode: str = "additive",
    scale: Optional[str] = None,
    ranks: Optional[Sequence[int]] = None,
    tol: float = 1e-5,
    max_iter: int = 1000,
    precision: str = "fp64",
) -> Workload:
    """Tucker low-rank tensor plus sparse corruption.

    ``scale``: None (leave the Tucker product as drawn), ``"rms"`` (scale the
    low-rank part to unit root-mean-square), ``"minmax"`` (map it affinely
    onto [0, 1]) or ``"minmax255"`` (onto [0, 255], an 8-bit image range).
    ``mode``: ``"additive"`` adds U(value_range) at the chosen positions;
    ``"impulse"`` replaces them by 0 or 1 with equal probability; ``"replace"``
    replaces them by U(value_range).
    """
    rng = np.random.default_rng(seed)
    dims = tuple(int(d) for d in dims)
    core = rng.standard_normal(tuple(core_ranks))
    factors = [haar_stiefel(rng, d, r) for d, r in zip(dims, core_ranks)]
    L = tucker(core, factors)
    if scale == "rms":
        L = L / math.sqrt(float(np.mean(L * L)))
    elif scale == "minmax":
        L = (L - L.min()) / (L.max() - L.min())
    elif scale == "minmax255":
        L = 255.0 * (L - L.min()) / (L.max() - L.min())
    elif scale is not None:
        raise ValueError(f"unknown scale {scale!r}")
    numel = L.size
    pos = _positions(rng, numel, frac)
    mask = np.zeros(numel, dtype=bool)
    mask[pos] = True
    T = L.reshape(-1).copy()
    S = np.zeros(numel)
    if mode == "additive":
        vals = rng.uniform(value_range[0], value_range[1], size=pos.size)
        T[pos] += vals
        S[pos] = vals
    elif mode == "impulse":
        vals = rng.integers(0, 2, size=pos.size).astype(np.float64)
        S[pos] = vals - T[pos]
        T[pos] = vals
    elif mode == "replace":
        vals = rng.uniform(value_range[0], value_range[1], size=pos.size)
        S[pos] = vals - T[pos]
        T[pos] = vals
    else:
        raise ValueError(f"unknown corruption mode {mode!r}")
    return Workload(
        name=name,
        T=T.reshape(dims),
        L=L,
        S=S.reshape(dims),
        mask=mask.reshape(dims),
        ranks=tuple(int(r) for r in (ranks if ranks is not None else core_ranks)),
        tol=tol,
        max_iter=max_iter,
        precision=precision,
        meta={"seed": seed, "frac": frac, "core_ranks": tuple(core_ranks),
              "value_range": value_range, "mode": mode, "scale": scale},
    )


def mri_standin(rho: float, seed: int = 17127000, core_ranks=(30, 30, 30),
                precision: str = "fp64") -> Workload:
    """Stand-in for the brain-MRI restoration of Section 5.2, whose data is not
    available: a 181 x 217 x 181 tensor, here a Tucker tensor of rank
    ``core_ranks`` (N(0, 1) core, Haar factors) mapped onto [0, 255], with a
    fraction ``rho`` of the voxels replaced by U(0, 255); solved with
    R_n = 40, epsilon 1e-5, maxiter 1000 as in the paper."""
    return tucker_workload("mri", (181, 217, 181), core_ranks, rho, seed, value_range=(0.0, 255.0),
                           mode="replace", scale="minmax255", ranks=(40, 40, 40), tol=1e-5,
                           max_iter=1000, precision=precision)


def psnr(X: np.ndarray, L: np.ndarray, peak: float = 255.0) -> float:
    """Peak signal-to-noise ratio 10 log10(peak^2 / mean((X - L)^2)) in dB."""
    mse = float(np.mean((np.asarray(X, dtype=np.float64) - L) ** 2))
    return float("inf") if mse == 0 else 10.0 * math.log10(peak * peak / mse)


def video_workload(
    name: str,
    dims: Sequence[int] = (144, 176, 400),
    bg_ranks: Sequence[int] = (8, 8, 3),
    blocks: int = 5,
    block: int = 12,
    seed: int = 17120302,
    *,
    tol: float = 1e-6,
    max_iter: int = 1000,
    precision: str = "bf16",
) -> Workload:
    """Video-shaped tensor (rows x cols x frames).

    Background: Tucker model of multilinear rank ``bg_ranks`` scaled to unit
    RMS.  Foreground: ``blocks`` square patches of ``block`` x ``block`` pixels,
    each a fixed U(0, 1) texture, starting at a uniform position and moving one
    pixel per frame with a velocity drawn from {-1, 0, 1}^2 minus the origin,
    reflecting at the borders; later patches overwrite earlier ones.  The
    patches are added to the background.
    """
    rng = np.random.default_rng(seed)
    h, w, f = (int(d) for d in dims)
    core = rng.standard_normal(tuple(bg_ranks))
    factors = [haar_stiefel(rng, d, r) for d, r in zip((h, w, f), bg_ranks)]
    L = tucker(core, factors)
    L = L / math.sqrt(float(np.mean(L * L)))
    S = np.zeros((h, w, f))
    vel_choices = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1) if (dy, dx) != (0, 0)]
    for _ in range(blocks):
        tex = rng.uniform(0.0, 1.0, size=(block, block))
        y = int(rng.integers(0, h - block + 1))
        x = int(rng.integers(0, w - block + 1))
        dy, dx = vel_choices[int(rng.integers(0, len(vel_choices)))]
        for t in range(f):
            S[y:y + block, x:x + block, t] = tex
            ny, nx = y + dy, x + dx
            if ny < 0 or ny > h - block:
                dy = -dy
                ny = y + dy
            if nx < 0 or nx > w - block:
                dx = -dx
                nx = x + dx
            y, x = ny, nx
    mask = S != 0
    T = L + S
    return Workload(
        name=name, T=T, L=L, S=S, mask=mask, ranks=tuple(bg_ranks), tol=tol,
        max_iter=max_iter, precision=precision,
        meta={"seed": seed, "blocks": blocks, "block": block,
              "nonzero_frac": float(mask.mean())},
    )


# Configuration recipes.  c1..c4 are single solves; "srv" is the serving trace.
CONFIGS = {
    # 50^3, Tucker core 5^3, unit-RMS low-rank part, 10% additive U(-10, 10).
    "c1": dict(kind="tucker", dims=(50, 50, 50), core_ranks=(5, 5, 5), frac=0.10,
               value_range=(-10.0, 10.0), scale="rms", tol=1e-8, max_iter=200,
               precision="fp64", seed=17120001),
    # 200^3, Tucker core 10^3 (no scaling stated), 20% additive U(-20, 20).
    "c2": dict(kind="tucker", dims=(200, 200, 200), core_ranks=(10, 10, 10), frac=0.20,
               value_range=(-20.0, 20.0), scale=None, tol=1e-6, max_iter=1000,
               precision="fp32", seed=17120002),
    # Video-shaped 144 x 176 x 400, background rank (8, 8, 3), moving blocks.
    "c3": dict(kind="video", dims=(144, 176, 400), core_ranks=(8, 8, 3), tol=1e-6,
               max_iter=1000, precision="bf16", seed=17120003),
    # 64^4, Tucker core 6^4 min-max normalised, 15% impulse (0 or 1).
    "c4": dict(kind="tucker", dims=(64, 64, 64, 64), core_ranks=(6, 6, 6, 6), frac=0.15,
               mode="impulse", scale="minmax", tol=1e-6, max_iter=1000,
               precision="fp32", seed=17120004),
}


def make_config(name: str, *, dims: Optional[Sequence[int]] = None,
                seed: Optional[int] = None) -> Workload:
    """Build a named configuration; ``dims``/``seed`` override for small variants."""
    spec = dict(CONFIGS[name])
    kind = spec.pop("kind")
    if dims is not None:
        spec["dims"] = tuple(dims)
    if seed is not None:
        spec["seed"] = seed
    if kind == "video":
        return video_workload(
            name, dims=spec["dims"], bg_ranks=spec["core_ranks"], seed=spec["seed"],
            tol=spec["tol"], max_iter=spec["max_iter"], precision=spec["precision"])
    return tucker_workload(
        name, spec["dims"], spec["core_ranks"], spec["frac"], spec["seed"],
        value_range=spec.get("value_range", (-1.0, 1.0)), mode=spec.get("mode", "additive"),
        scale=spec.get("scale"), tol=spec["tol"], max_iter=spec["max_iter"],
        precision=spec["precision"])


def serving_trace(count: int = 512, qps: float = 100.0, seed: int = 17120005,
                  dim_range: Tuple[int, int] = (32, 256),
                  rank_range: Tuple[int, int] = (3, 15),
                  frac_range: Tuple[float, float] = (0.05, 0.20)) -> List[dict]:
    """Request specs for the serving workload.

    Each request is a 3-way tensor with dims uniform in ``dim_range``, per-mode
    Tucker ranks uniform in ``rank_range`` (redrawn until every r_n is at most
    the product of the other two, so a Tucker core of that rank exists and
    every r_n <= I_n), unit-RMS low-rank part and a corruption fraction uniform
    in ``frac_range`` with values U(-10, 10).  Arrival times follow a Poisson
    process of rate ``qps``.  Tensors are drawn lazily by ``materialise``.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / qps))
        dims = tuple(int(d) for d in rng.integers(dim_range[0], dim_range[1] + 1, size=3))
        while True:
            r = [int(x) for x in rng.integers(rank_range[0], rank_range[1] + 1, size=3)]
            if all(r[n] <= r[(n + 1) % 3] * r[(n + 2) % 3] and r[n] <= dims[n] for n in range(3)):
                break
        frac = float(rng.uniform(*frac_range))
        out.append(dict(index=i, arrival=t, dims=dims, ranks=tuple(r), frac=frac,
                        seed=int(seed * 1000 + i)))
    return out


def materialise(spec: dict, precision: str = "fp32", tol: float = 1e-6,
                max_iter: int = 1000) -> Workload:
    """Draw the tensor of one serving request."""
    return tucker_workload(
        f"srv{spec['index']}", spec["dims"], spec["ranks"], spec["frac"], spec["seed"],
        value_range=(-10.0, 10.0), scale="rms", tol=tol, max_iter=max_iter,
        precision=precision)
