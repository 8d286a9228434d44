"""CPU oracle for the dyadic-pattern fast Hough transform (FHT2DS / FHT2DT).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or runs
this module: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code, table or
helper with the HIP library under ``paper_2411_07351_amd/``.

Everything here is written for obviousness, not speed: exact integer rounding,
int64 accumulation for integer images and float64 accumulation for floating
ones.  The paper is Kazimirov, Nikolaev, Rybakova, Terekhin, "Generalization of
Brady-Yong Algorithm for Fast Hough Transform to Arbitrary Image Size"
(arXiv 2411.07351).  Citations below name its sections, algorithms, equations
and theorems.

Readings of the paper taken here (each is also listed in the design notes):

* ``[.]`` (Alg. 1 and Alg. 2) is round-to-nearest with ties to even, evaluated
  exactly on the rational ``t (n_P - 1) / (n - 1)``.  Floor would break the
  coincidence with Brady-Yong at n = 2^q (Sec. 3); the tie rule is fixed by the
  statistics of Sec. 5 (36.38 %, the peak sequence 23, 45, ..., 1451).
* ``Rotate(v, r)[s] = v[(s + r) mod h]`` (Alg. 1): the only direction under
  which Alg. 1 sums along Alg. 2's patterns lifted by ``+(t - t_1)``.
* Four quadrants.  The paper defines one family (mostly horizontal lines,
  slope t/(n-1) in [0, 1], Sec. 3).  A row-major R x C image gives four
  lane-major views A[x][y]: q0 = V+ (lanes are image rows, sign +1),
  q1 = V- (image rows, sign -1), q2 = H+ (lanes are image columns, +1),
  q3 = H- (image columns, -1).  Output q is ``out_q[t][s]`` with t over the
  lanes and s over the positions.
* Lines wrap around: positions are taken mod h (Alg. 1, ``mod h``).
"""
from __future__ import annotations

import functools
from fractions import Fraction

import numpy as np

SPLIT_S = 0  # FHT2DS: floor half on the left (Sec. 3)
SPLIT_T = 1  # FHT2DT: largest power of two below w on the left (Sec. 3)

QUADRANT_NAMES = ("V+", "V-", "H+", "H-")


# ---------------------------------------------------------------------------
# Split rules and rounding (Sec. 3, Alg. 1 and Alg. 2)
# ---------------------------------------------------------------------------

def rhe(num: int, den: int) -> int:
    """Nearest integer to num/den for num >= 0, den > 0, ties to even.

    This is the ``[.]`` of Alg. 1 (``[t k_P]``) and Alg. 2
    (``[t (n_P - 1)/(n - 1)]``), computed on the exact rational.
    """
    if den <= 0 or num < 0:
        raise ValueError("rhe expects num >= 0 and den > 0")
    q, r = divmod(num, den)
    if 2 * r > den:
        return q + 1
    if 2 * r < den:
        return q
    return q + (q & 1)


def split_s(w: int) -> tuple[int, int]:
    """Split_S(w) = <floor(w/2), ceil(w/2)> (Sec. 3, the FHT2DS rule)."""
    return w // 2, w - w // 2


def split_t(w: int) -> tuple[int, int]:
    """Split_T(w) = <2^(ceil(log2 w) - 1), w - 2^(ceil(log2 w) - 1)> (Sec. 3).

    For w >= 2, ceil(log2 w) equals the bit length of w - 1.
    """
    if w < 2:
        raise ValueError("Split_T is only applied to w >= 2")
    p = 1 << ((w - 1).bit_length() - 1)
    return p, w - p


def split_fn(split: int):
    if split == SPLIT_S:
        return split_s
    if split == SPLIT_T:
        return split_t
    raise ValueError(f"unknown split {split}")


# ---------------------------------------------------------------------------
# Generating patterns (Alg. 2)
# ---------------------------------------------------------------------------

def pattern(n: int, t: int, split: int) -> list[int]:
    """FHT2D_Pattern(n, t, Split) of Alg. 2: y = pat(x) for x in [0, n).

    For n > 1 the width is split into <n0, n1>, each child slope is
    t_P = [t (n_P - 1) / (n - 1)], the right child's pattern is lifted by
    t - t_1, and the two are concatenated.  For n = 1 the pattern is <0>.
    """
    if not 0 <= t < n:
        raise ValueError("need 0 <= t < n")
    if n == 1:
        return [0]
    n0, n1 = split_fn(split)(n)
    t0 = rhe(t * (n0 - 1), n - 1)
    t1 = rhe(t * (n1 - 1), n - 1)
    left = pattern(n0, t0, split)
    right = [y + (t - t1) for y in pattern(n1, t1, split)]
    return left + right


@functools.lru_cache(maxsize=64)
def _patterns_cached(n: int, split: int) -> np.ndarray:
    p = np.array([pattern(n, t, split) for t in range(n)], dtype=np.int64)
    p.setflags(write=False)
    return p


def patterns(n: int, split: int) -> np.ndarray:
    """All generating patterns for width n: an n x n array P[t][x] (Alg. 2)."""
    return _patterns_cached(int(n), int(split))


# ---------------------------------------------------------------------------
# The transform as plain sums along patterns (Sec. 3: every summed pattern is
# a vertical shift of a generating pattern)
# ---------------------------------------------------------------------------

def hough_lanes(A: np.ndarray, split: int, sigma: int = 1, absolute: bool = False):
    """Hough image of a lane-major array A[x][y], x in [0, W), y in [0, H).

    ``J[t][s] = sum_x A[x][(s + sigma * pat_{W,t}(x)) mod H]``.

    Integer input accumulates in int64, floating input in float64.  With
    ``absolute`` the same sums are taken over |A|; that is the per-line scale
    for floating-point tolerances.
    """
    A = np.asarray(A)
    if A.ndim != 2 or A.shape[0] < 1 or A.shape[1] < 1:
        raise ValueError("A must be a non-empty 2-D array")
    if sigma not in (1, -1):
        raise ValueError("sigma must be +1 or -1")
    W, H = A.shape
    acc = np.int64 if np.issubdtype(A.dtype, np.integer) else np.float64
    src = A.astype(acc)
    if absolute:
        src = np.abs(src)
    P = patterns(W, split)
    s = np.arange(H)
    lane = np.arange(W)[:, None]
    out = np.empty((W, H), dtype=acc)
    for t in range(W):
        cols = (s[None, :] + sigma * P[t][:, None]) % H
        out[t] = src[lane, cols].sum(axis=0)
    return out


def quadrant_views(img: np.ndarray):
    """The four lane-major views (A, sigma) of a row-major R x C image."""
    img = np.asarray(img)
    return ((img, 1), (img, -1), (img.T, 1), (img.T, -1))


def hough4(img: np.ndarray, split: int, absolute: bool = False):
    """All four quadrant Hough images of a row-major image, in q order."""
    return [hough_lanes(A, split, sig, absolute) for A, sig in quadrant_views(img)]


# ---------------------------------------------------------------------------
# Alg. 1 written as the paper's recursion (a second formulation of the same
# numbers; the direct sums above are the definition)
# ---------------------------------------------------------------------------

def rotate(v: np.ndarray, r: int) -> np.ndarray:
    """Rotate(v, r): circular shift with Rotate(v, r)[s] = v[(s + r) mod h]."""
    h = v.shape[0]
    return v[(np.arange(h) + r) % h]


def fht2d(I: np.ndarray, split: int, sigma: int = 1) -> np.ndarray:
    """FHT2D(w, h, I, Split) of Alg. 1 for a lane-major I[x][y].

    sigma = -1 rotates the right half the other way, which is the mirrored
    (negative-slope) family.
    """
    I = np.asarray(I)
    w, h = I.shape
    acc = np.int64 if np.issubdtype(I.dtype, np.integer) else np.float64
    if w == 1:
        return I.astype(acc).copy()
    w0, w1 = split_fn(split)(w)
    J0 = fht2d(I[:w0], split, sigma)
    J1 = fht2d(I[w0:], split, sigma)
    J = np.zeros((w, h), dtype=acc)
    for t in range(w):
        t0 = rhe(t * (w0 - 1), w - 1)
        t1 = rhe(t * (w1 - 1), w - 1)
        J[t] = J0[t0] + rotate(J1[t1], (sigma * (t - t1)) % h)
    return J


# ---------------------------------------------------------------------------
# Classic Brady-Yong (1992) for W = 2^q, written without Split or [.]
# (Sec. 3: both FHT2DS and FHT2DT coincide with it at n = 2^q)
# ---------------------------------------------------------------------------

def brady_yong(A: np.ndarray, sigma: int = 1) -> np.ndarray:
    """Radix-2 dyadic Hough transform of a lane-major A[x][y], W a power of 2.

    Blocks of 2m lanes are built from two blocks of m lanes: slope t takes
    slope floor(t/2) from both halves and shifts the right half by ceil(t/2).
    """
    A = np.asarray(A)
    W, H = A.shape
    if W & (W - 1):
        raise ValueError("Brady-Yong needs a power-of-two lane count")
    acc = np.int64 if np.issubdtype(A.dtype, np.integer) else np.float64
    J = A.astype(acc).copy()
    s = np.arange(H)
    m = 1
    while m < W:
        nxt = np.empty_like(J)
        for b in range(0, W, 2 * m):
            for t in range(2 * m):
                half, up = t // 2, (t + 1) // 2
                nxt[b + t] = J[b + half] + J[b + m + half][(s + sigma * up) % H]
        J = nxt
        m *= 2
    return J


# ---------------------------------------------------------------------------
# Explicit operator (tiny shapes): the transform as a 0/1 count matrix
# ---------------------------------------------------------------------------

def explicit_matrix(W: int, H: int, split: int, sigma: int = 1) -> np.ndarray:
    """M with J.ravel() = M @ A.ravel() for lane-major A of shape (W, H)."""
    P = patterns(W, split)
    M = np.zeros((W * H, W * H), dtype=np.int64)
    for t in range(W):
        for s in range(H):
            for x in range(W):
                M[t * H + s, x * H + (s + sigma * int(P[t, x])) % H] += 1
    return M


# ---------------------------------------------------------------------------
# The adjoint (back-projection).  The transform is linear: hough_lanes sends
# A to J with J[t][s] = sum_x A[x][(s + sigma pat_t(x)) mod H], so the pixel
# A[x][y] enters J[t][s] exactly for s = (y - sigma pat_t(x)) mod H.  The
# adjoint therefore sends a gradient G on the output back along the same
# patterns (Alg. 2).
# ---------------------------------------------------------------------------

def adjoint_lanes(G: np.ndarray, split: int, sigma: int = 1) -> np.ndarray:
    """``gA[x][y] = sum_t G[t][(y - sigma * pat_{W,t}(x)) mod H]`` in float64."""
    G = np.asarray(G, dtype=np.float64)
    W, H = G.shape
    P = patterns(W, split)
    y = np.arange(H)
    out = np.zeros((W, H), dtype=np.float64)
    for x in range(W):
        for t in range(W):
            out[x] += G[t][(y - sigma * int(P[t, x])) % H]
    return out


def adjoint4(Gs, split: int, shape) -> np.ndarray:
    """Image gradient of the quadrant images: ``Gs`` maps quadrant q to its
    output gradient (W_q x H_q); each view's adjoint is mapped back to the
    row-major R x C image (column-lane views transposed) and summed."""
    R, C = shape
    g = np.zeros((R, C), dtype=np.float64)
    sig = {0: 1, 1: -1, 2: 1, 3: -1}
    for q, G in Gs.items():
        gA = adjoint_lanes(G, split, sig[q])
        g += gA if q < 2 else gA.T
    return g


# ---------------------------------------------------------------------------
# Sec. 4: addition counts (Theorem 1) and orthotropic error (Theorem 2)
# ---------------------------------------------------------------------------

def nonleaf_width_sum(w: int, split: int) -> int:
    """Sum of the widths of the non-leaf nodes of the order tree G(w) (Sec. 4)."""
    if w <= 1:
        return 0
    w0, w1 = split_fn(split)(w)
    return w + nonleaf_width_sum(w0, split) + nonleaf_width_sum(w1, split)


def additions(n: int, split: int, h: int | None = None) -> int:
    """Number of summations of FHT2D on an n-wide image of height h (default n).

    A recursion step of width m costs m*h additions (proof of Theorem 1).
    """
    return (n if h is None else h) * nonleaf_width_sum(n, split)


def fs_closed_form(n: int) -> int:
    """Eq. (1) of Theorem 1: f_S(n) = (floor(log2 n) + 2) n^2 - 2^(floor(log2 n)+1) n."""
    k = n.bit_length() - 1
    return (k + 2) * n * n - (1 << (k + 1)) * n


def orthotropic_error(n: int, split: int) -> Fraction:
    """E(n) = max over t, x of |x t / (n - 1) - pat(n, t)(x)| (Sec. 4), exactly.

    For n = 1 the only pattern is <0> and the error is taken as 0.
    """
    if n == 1:
        return Fraction(0)
    P = patterns(n, split)
    x = np.arange(n, dtype=np.int64)
    worst = 0
    for t in range(n):
        worst = max(worst, int(np.abs(x * t - P[t] * (n - 1)).max()))
    return Fraction(worst, n - 1)


def theorem2_bound(n: int) -> Fraction:
    """Right-hand side of Theorem 2: floor(log2 n)/6 + 1 - 2^(-floor(log2 n))."""
    k = n.bit_length() - 1
    return Fraction(k, 6) + 1 - Fraction(1, 1 << k)
