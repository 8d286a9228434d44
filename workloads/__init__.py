"""Seeded synthetic inputs shared by the tests, the bench and the smoke check.

This module holds no arithmetic of the transform: only random images of the
shapes and value distributions of the benchmark workloads.  Both the CPU oracle
and the HIP library receive the arrays it returns.

Recipes (seed ``2411_07351 + k`` for workload k):

* uniform uint8: ``integers(0, 256)``;
* edge maps: uint8 in {0, 1}, Bernoulli(p = 0.05) background plus 20 straight
  segments with endpoints uniform over the image, rasterised by Bresenham's
  algorithm and drawn with value 1;
* ragged sizes: rows and columns independent, ``round(exp(U[ln lo, ln hi]))``;
* float images: ``standard_normal`` in float32;
* serving stream: sides log-uniform in [64, 4096], 70 % edge maps and 30 %
  float images, arrivals a Poisson process (exponential gaps of mean 1/QPS).
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 2411_07351


def rng_for(k: int, salt: int = 0) -> np.random.Generator:
    """Generator of workload k (salt picks an independent stream for tests)."""
    return np.random.default_rng(SEED_BASE + k + 1000 * salt)


def uniform_u8(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    return rng.integers(0, 256, size=(rows, cols), dtype=np.uint8)


def normal_f32(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    return rng.standard_normal(size=(rows, cols)).astype(np.float32)


def _segment(img: np.ndarray, r0: int, c0: int, r1: int, c1: int) -> None:
    """Bresenham rasterisation of the segment (r0, c0)-(r1, c1), value 1."""
    dr, dc = abs(r1 - r0), abs(c1 - c0)
    sr = 1 if r1 >= r0 else -1
    sc = 1 if c1 >= c0 else -1
    err = dc - dr
    r, c = r0, c0
    while True:
        img[r, c] = 1
        if r == r1 and c == c1:
            break
        e2 = 2 * err
        if e2 > -dr:
            err -= dr
            c += sc
        if e2 < dc:
            err += dc
            r += sr


def edge_map_segments(rng: np.random.Generator, rows: int, cols: int, p: float = 0.05,
                      segments: int = 20) -> tuple[np.ndarray, np.ndarray]:
    """An edge map and its planted segments, (segments, 4) rows (r0, c0, r1, c1)."""
    img = (rng.random(size=(rows, cols)) < p).astype(np.uint8)
    ends = rng.integers(0, [rows, cols, rows, cols], size=(segments, 4))
    for r0, c0, r1, c1 in ends:
        _segment(img, int(r0), int(c0), int(r1), int(c1))
    return img, ends


def edge_map(rng: np.random.Generator, rows: int, cols: int, p: float = 0.05,
             segments: int = 20) -> np.ndarray:
    return edge_map_segments(rng, rows, cols, p, segments)[0]


def edge_maps(rng: np.random.Generator, n: int, rows: int, cols: int) -> np.ndarray:
    return np.stack([edge_map(rng, rows, cols) for _ in range(n)])


def ragged_shapes(rng: np.random.Generator, n: int, lo: int, hi: int) -> list[tuple[int, int]]:
    u = rng.uniform(np.log(lo), np.log(hi), size=(n, 2))
    sizes = np.clip(np.rint(np.exp(u)).astype(np.int64), lo, hi)
    return [(int(r), int(c)) for r, c in sizes]


def ragged_edge_maps(rng: np.random.Generator, n: int, lo: int, hi: int) -> list[np.ndarray]:
    return [edge_map(rng, r, c) for r, c in ragged_shapes(rng, n, lo, hi)]


def serving_requests(rng: np.random.Generator, n: int, lo: int = 64, hi: int = 4096,
                     u8_share: float = 0.7) -> list[tuple[str, np.ndarray]]:
    """n requests of the serving stream: (kind, image) with kind "u8" (edge
    map) or "f32" (standard normal)."""
    reqs = []
    for r, c in ragged_shapes(rng, n, lo, hi):
        if rng.random() < u8_share:
            reqs.append(("u8", edge_map(rng, r, c)))
        else:
            reqs.append(("f32", normal_f32(rng, r, c)))
    return reqs


def poisson_arrivals(rng: np.random.Generator, n: int, qps: float) -> np.ndarray:
    """Arrival times (seconds from 0) of n requests of a Poisson process of rate
    qps; all zero when qps is infinite (a closed burst)."""
    if not np.isfinite(qps):
        return np.zeros(n)
    return np.cumsum(rng.exponential(1.0 / qps, size=n))
