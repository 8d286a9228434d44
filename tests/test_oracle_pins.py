"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them re-types the oracle's
own formula: they use closed forms and numbers printed in the paper, an
independently written Brady-Yong transform, the second formulation (Alg. 1
versus Alg. 2's pattern sums), hand-derived small cases and invariants.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import fht_oracle as O
from oracle import native

SPLITS = (O.SPLIT_S, O.SPLIT_T)


def _e(num, n):
    return Fraction(int(num[n]), n - 1) if n > 1 else Fraction(0)


# --------------------------------------------------------------------- rounding

def test_rhe_ties_to_even_and_exact():
    # [.] is nearest-integer; ties go to the even neighbour (reading of Alg. 2).
    assert [O.rhe(k, 2) for k in range(8)] == [0, 0, 1, 2, 2, 2, 3, 4]
    assert O.rhe(7, 3) == 2 and O.rhe(8, 3) == 3 and O.rhe(5, 4) == 1 and O.rhe(6, 4) == 2
    # exact on huge rationals where float rounding would not be
    big = 10**30
    assert O.rhe(2 * big + 1, 2) == big  # big is even
    assert O.rhe(2 * (big + 1) + 1, 2) == big + 2


def test_split_rules():
    # Sec. 3: Split_S bisects (floor left), Split_T cuts off the largest power of two.
    assert O.split_s(7) == (3, 4) and O.split_s(8) == (4, 4) and O.split_s(1021) == (510, 511)
    assert O.split_t(2) == (1, 1) and O.split_t(3) == (2, 1) and O.split_t(5) == (4, 1)
    assert O.split_t(17) == (16, 1) and O.split_t(1021) == (512, 509) and O.split_t(1024) == (512, 512)


# --------------------------------------------------------------------- patterns

def test_hand_derived_patterns_n5():
    """Alg. 2 by hand for n = 5 (the half-to-even tie rule decides slope 1).

    FHT2DS: Split_S(5) = (2, 3).  For t = 1: t0 = [1*1/4] = 0 and
    t1 = [1*2/4] = [1/2] = 0 (tie, even), so pat = pat(2,0) ++ (pat(3,0) + 1)
    = 00 ++ 111.  For t = 2: t0 = [2/4] = 0 (tie), t1 = [4/4] = 1;
    pat(3,1): Split_S(3) = (1, 2), t0 = 0, t1 = [1/2] = 0 (tie), so
    pat(3,1) = 0 ++ (00 + 1) = 011, lifted by 2 - 1 = 1 gives 122: 00122.
    FHT2DT: Split_T(5) = (4, 1).  t = 1: t0 = [3/4] = 1, t1 = 0;
    pat(4,1) = Brady-Yong slope 1 = 0011, right lane lifted by 1: 00111.
    t = 2: t0 = [6/4] = 2 (tie, even); pat(4,2) = 0112, right lifted by 2: 01122.
    """
    assert O.pattern(5, 1, O.SPLIT_S) == [0, 0, 1, 1, 1]
    assert O.pattern(5, 2, O.SPLIT_S) == [0, 0, 1, 2, 2]
    assert O.pattern(5, 1, O.SPLIT_T) == [0, 0, 1, 1, 1]
    assert O.pattern(5, 2, O.SPLIT_T) == [0, 1, 1, 2, 2]


@pytest.mark.parametrize("split", SPLITS)
def test_pattern_shape_invariants(split):
    # Every pattern starts at 0, ends at t, and rises by 0 or 1 per step
    # (Alg. 2: concatenation of child patterns, the right one lifted by t - t1).
    for n in range(1, 130):
        P = O.patterns(n, split)
        assert (P[:, 0] == 0).all()
        assert (P[:, -1] == np.arange(n)).all()
        if n > 1:
            d = np.diff(P, axis=1)
            assert ((d == 0) | (d == 1)).all()


@pytest.mark.parametrize("split", SPLITS)
def test_c_patterns_equal_python_patterns(split):
    for n in (1, 2, 3, 5, 17, 61, 100, 257):
        assert (native.patterns(n, split) == O.patterns(n, split)).all()


# --------------------------------------------------------------------- Theorem 1

def test_theorem1_eq1_closed_form():
    # Eq. (1): f_S(n) = (floor(log2 n) + 2) n^2 - 2^(floor(log2 n) + 1) n, for every n.
    for n in range(1, 4097):
        assert O.additions(n, O.SPLIT_S) == O.fs_closed_form(n), n
    for n in (1, 2, 3, 1021, 4096):
        assert native.nonleaf_width_sum(n, 0) * n == O.fs_closed_form(n)


def test_theorem1_sharp_constants(paper_stats):
    # Theorem 1 and Sec. 5: max of f/(n^2 log2 n) is 5 log3(2)/3 at n = 3 (S)
    # and 81 log17(2)/17 at n = 17 (T).
    def norm(n, split):
        return O.additions(n, split) / (n * n * math.log2(n))
    ns = range(2, 4097)
    ns_s = max(ns, key=lambda n: norm(n, O.SPLIT_S))
    ns_t = max(ns, key=lambda n: norm(n, O.SPLIT_T))
    assert ns_s == int(paper_stats["fs_max_n"])
    assert ns_t == int(paper_stats["ft_max_n"])
    assert norm(3, O.SPLIT_S) == pytest.approx(5 * math.log(2, 3) / 3, rel=1e-12)
    assert norm(17, O.SPLIT_T) == pytest.approx(81 * math.log(2, 17) / 17, rel=1e-12)
    assert norm(3, O.SPLIT_S) < 1.052 and norm(17, O.SPLIT_T) < 1.166


def test_theorem1_ft_at_two_power_plus_one():
    # Proof of Theorem 1: f_T(2^k + 1) = (2^k + 1)(2^k + 1 + k 2^k).
    for k in range(1, 12):
        n = (1 << k) + 1
        assert O.additions(n, O.SPLIT_T) == n * (n + k * (1 << k))


# ------------------------------------------------- Theorem 2 and Sec. 5 statistics

def test_theorem2_bound_holds(error_tables, paper_stats):
    nmax = int(paper_stats["n_max"])
    eT = error_tables[O.SPLIT_T]
    for n in range(1, nmax + 1):
        assert _e(eT, n) <= O.theorem2_bound(n), n


def test_error_tables_match_python_oracle(error_tables):
    for split in SPLITS:
        for n in (1, 2, 3, 5, 23, 64, 100, 181):
            assert _e(error_tables[split], n) == O.orthotropic_error(n, split)


def test_sec5_share_above_theorem2(error_tables, paper_stats):
    nmax = int(paper_stats["n_max"])
    eS = error_tables[O.SPLIT_S]
    above = sum(1 for n in range(1, nmax + 1) if _e(eS, n) > O.theorem2_bound(n))
    # The paper prints the share rounded to two decimals.
    assert round(100.0 * above / nmax, 2) == float(paper_stats["share_es_above_thm2_percent"])


def test_sec5_ratio_peak(error_tables, paper_stats):
    nmax = int(paper_stats["n_max"])
    eS, eT = error_tables[O.SPLIT_S], error_tables[O.SPLIT_T]
    ratios = {n: _e(eS, n) / _e(eT, n) for n in range(2, nmax + 1) if eT[n] > 0}
    n_best = max(ratios, key=ratios.get)
    assert n_best == int(paper_stats["es_over_et_n"])
    factor = float(paper_stats["es_over_et_factor"])
    assert factor < ratios[n_best] < factor + 0.01


def test_sec5_peak_sequence(error_tables, paper_stats):
    eS = error_tables[O.SPLIT_S]
    peaks = [int(v) for v in paper_stats["es_peaks"].split()]
    # n_{k+1} = 2 n_k + (-1)^(k+1), n_0 = 23
    for k in range(len(peaks) - 1):
        assert peaks[k + 1] == 2 * peaks[k] + (-1) ** (k + 1)
    # Reading: each listed n is the highest peak of E_S(n)/(log2 n / 6) in its octave.
    for n_peak in peaks:
        k = n_peak.bit_length() - 1
        octave = range(1 << k, 1 << (k + 1))
        best = max(octave, key=lambda n: float(_e(eS, n)) / (math.log2(n) / 6))
        assert best == n_peak


def test_karpenko_power_of_two_error(error_tables):
    # Sec. 2: at n = 2^q the maximal orthotropic error is log2(n)/6 for even q.
    # For odd q the paper quotes log2(n)/6 - 1/18; with its line y = x t/(n-1)
    # the computed error stays below that value by less than 1/(n-1).
    for split in SPLITS:
        for q in range(1, 13):
            n = 1 << q
            e = _e(error_tables[split], n)
            if q % 2 == 0:
                assert e == Fraction(q, 6)
            else:
                gap = Fraction(q, 6) - Fraction(1, 18) - e
                assert 0 < gap < Fraction(1, n - 1)


# ------------------------------------------------------------- sums (the transform)

@pytest.mark.parametrize("split", SPLITS)
def test_brady_yong_equals_both_variants_at_powers_of_two(split):
    # Sec. 3: at n = 2^q FHT2DS and FHT2DT coincide with Brady-Yong.
    rng = np.random.default_rng(11)
    for W in (1, 2, 4, 8, 16, 32, 64):
        for H in (1, 3, 16, 37):
            A = rng.integers(0, 256, size=(W, H))
            for sigma in (1, -1):
                assert (O.hough_lanes(A, split, sigma) == O.brady_yong(A, sigma)).all()


@pytest.mark.parametrize("split", SPLITS)
def test_alg1_recursion_equals_pattern_sums(split):
    # Alg. 1 (merge with Rotate) and Alg. 2 (sums along patterns) give the same numbers.
    rng = np.random.default_rng(12)
    for W in range(1, 26):
        for H in (1, 2, 5, 13):
            A = rng.integers(-50, 256, size=(W, H))
            for sigma in (1, -1):
                assert (O.fht2d(A, split, sigma) == O.hough_lanes(A, split, sigma)).all(), (W, H)


@pytest.mark.parametrize("split", SPLITS)
def test_single_pixel_gives_one_hit_per_slope(split):
    # A one-pixel image lies on exactly one line of each slope, in each quadrant.
    R, C = 9, 7
    for (r, c) in ((0, 0), (4, 3), (8, 6), (3, 0)):
        img = np.zeros((R, C), dtype=np.int64)
        img[r, c] = 5
        for J in O.hough4(img, split):
            assert ((J != 0).sum(axis=1) == 1).all()
            assert (J.sum(axis=1) == 5).all()


@pytest.mark.parametrize("split", SPLITS)
def test_line_sums_rows_and_diagonals(split):
    rng = np.random.default_rng(13)
    img = rng.integers(0, 256, size=(23, 17))
    for (A, sigma), J in zip(O.quadrant_views(img), O.hough4(img, split)):
        W, H = A.shape
        # every slope covers each pixel exactly once over its H shifts
        assert (J.sum(axis=1) == img.sum()).all()
        # slope 0 is the plain sum over the lanes
        assert (J[0] == A.sum(axis=0)).all()
        # slope W-1 steps by one position per lane: the wrapped diagonal
        s = np.arange(H)
        diag = sum(A[x][(s + sigma * x) % H] for x in range(W))
        assert (J[W - 1] == diag).all()


@pytest.mark.parametrize("split", SPLITS)
def test_linearity_and_quadrant_symmetry(split):
    rng = np.random.default_rng(14)
    a = rng.integers(0, 100, size=(12, 19))
    b = rng.integers(0, 100, size=(12, 19))
    for Ja, Jb, Jab in zip(O.hough4(a, split), O.hough4(b, split), O.hough4(3 * a - b, split)):
        assert (3 * Ja - Jb == Jab).all()
    # V- of an image equals V+ of its position-mirrored copy, mirrored back.
    J = O.hough4(a, split)
    mirror = (-np.arange(a.shape[1])) % a.shape[1]
    Jm = O.hough_lanes(a[:, mirror], split, 1)
    assert (J[1] == Jm[:, mirror]).all()


def test_explicit_matrix_matches_sums():
    rng = np.random.default_rng(15)
    for split in SPLITS:
        for W, H in ((5, 3), (7, 4), (3, 7)):
            for sigma in (1, -1):
                M = O.explicit_matrix(W, H, split, sigma)
                A = rng.integers(0, 256, size=(W, H))
                assert (M @ A.ravel() == O.hough_lanes(A, split, sigma).ravel()).all()
                # each row of the operator sums exactly W pixels, one per lane
                assert (M.sum(axis=1) == W).all()


@pytest.mark.parametrize("split", SPLITS)
def test_c_oracle_equals_python_oracle(split):
    rng = np.random.default_rng(16)
    for R, C in ((1, 1), (1, 9), (9, 1), (61, 47), (16, 33)):
        img = rng.integers(0, 256, size=(R, C), dtype=np.uint8)
        for x, y in zip(native.hough4_u8(img, split), O.hough4(img, split)):
            assert (x == y).all()
        f = rng.standard_normal((R, C))
        o, ab = native.hough4_f64(f, split)
        for x, y in zip(o, O.hough4(f, split)):
            assert np.allclose(x, y, rtol=0, atol=1e-9)
        for x, y in zip(ab, O.hough4(f, split, absolute=True)):
            assert np.allclose(x, y, rtol=0, atol=1e-9)
        # sampled outputs one by one
        qs = rng.integers(0, 4, size=50)
        ts = np.array([rng.integers(0, (R, R, C, C)[q]) for q in qs])
        ss = np.array([rng.integers(0, (C, C, R, R)[q]) for q in qs])
        full = native.hough4_u8(img, split)
        assert (native.sample_u8(img, split, qs, ts, ss) ==
                np.array([full[q][t, s] for q, t, s in zip(qs, ts, ss)])).all()


def test_direct_sum_against_brute_force_line_enumeration():
    """Tiny brute force: enumerate every lane's contribution by walking each line.

    For W = 3 (Split_S(3) = (1, 2), Split_T(3) = (2, 1)) the three generating
    patterns follow from Alg. 2 by hand: slope 0 -> 000, slope 2 -> 012, and
    slope 1 -> 011 under S (right pair lifted by 1 - [1/2] = 1) and 001 under T
    (left pair takes slope [1*1/2] = 0, the right lane is lifted by 1).
    """
    hand = {O.SPLIT_S: [[0, 0, 0], [0, 1, 1], [0, 1, 2]],
            O.SPLIT_T: [[0, 0, 0], [0, 0, 1], [0, 1, 2]]}
    rng = np.random.default_rng(17)
    A = rng.integers(0, 256, size=(3, 4))
    for split, pats in hand.items():
        for sigma in (1, -1):
            J = O.hough_lanes(A, split, sigma)
            for t in range(3):
                for s in range(4):
                    assert J[t, s] == sum(A[x, (s + sigma * pats[t][x]) % 4] for x in range(3))


def test_pins_reject_planted_mistakes(monkeypatch):
    """Plant plausible mistakes in the oracle (CPU only) and check a pin fails."""
    def half_up(num, den):
        q, r = divmod(num, den)
        return q + (1 if 2 * r >= den else 0)

    def floor_div(num, den):
        return num // den

    for wrong in (half_up, floor_div):
        monkeypatch.setattr(O, "rhe", wrong)
        O._patterns_cached.cache_clear()
        bad = (O.pattern(5, 1, O.SPLIT_S) != [0, 0, 1, 1, 1] or
               O.pattern(5, 2, O.SPLIT_S) != [0, 0, 1, 2, 2] or
               any(O.patterns(n, O.SPLIT_S)[n - 1, n - 1] != n - 1 for n in range(2, 20)))
        A = np.arange(8 * 5).reshape(8, 5)
        by_broken = not (O.hough_lanes(A, O.SPLIT_S) == O.brady_yong(A)).all()
        assert bad or by_broken
    monkeypatch.undo()
    O._patterns_cached.cache_clear()
    # a swapped split orientation changes the hand-derived patterns
    monkeypatch.setattr(O, "split_s", lambda w: (w - w // 2, w // 2))
    O._patterns_cached.cache_clear()
    assert O.pattern(5, 1, O.SPLIT_S) != [0, 0, 1, 1, 1]
    monkeypatch.undo()
    O._patterns_cached.cache_clear()


# --------------------------------------------------------------------- adjoint

ADJ_SHAPES = [(13, 11), (11, 13), (7, 5), (16, 3), (1, 5), (5, 1), (17, 9)]


@pytest.mark.parametrize("split", SPLITS)
@pytest.mark.parametrize("shape", ADJ_SHAPES)
def test_adjoint_dot_product_identity(split, shape):
    # <F A, G> = <A, F^T G> for the forward oracle F (integer data: exact)
    rng = np.random.default_rng(31 + shape[0] * 7 + shape[1])
    A = rng.integers(-9, 10, size=shape)
    G = rng.integers(-9, 10, size=shape)
    for sigma in (1, -1):
        lhs = int((O.hough_lanes(A, split, sigma) * G).sum())
        rhs = float((A * O.adjoint_lanes(G, split, sigma)).sum())
        assert rhs == lhs


@pytest.mark.parametrize("split", SPLITS)
@pytest.mark.parametrize("shape", [(13, 11), (11, 13), (7, 5), (16, 3)])
def test_adjoint_is_the_explicit_transpose(split, shape):
    rng = np.random.default_rng(5)
    W, H = shape
    G = rng.standard_normal(shape)
    for sigma in (1, -1):
        M = O.explicit_matrix(W, H, split, sigma)
        np.testing.assert_allclose(O.adjoint_lanes(G, split, sigma).ravel(), M.T @ G.ravel(),
                                   rtol=0, atol=1e-12)


@pytest.mark.parametrize("split", SPLITS)
def test_adjoint_of_one_line_is_its_pattern(split):
    # the gradient of a single output J[t][s] marks the pixels of that line:
    # one per lane, at (s + pat_t(x)) mod H (Alg. 2, Sec. 3)
    W, H = 9, 7
    for t in range(W):
        G = np.zeros((W, H))
        G[t, 3] = 1.0
        gA = O.adjoint_lanes(G, split)
        assert gA.sum() == W and (gA.sum(axis=1) == 1).all()
        pat = O.pattern(W, t, split)
        for x in range(W):
            assert gA[x, (3 + pat[x]) % H] == 1.0


@pytest.mark.parametrize("split", SPLITS)
def test_adjoint4_dot_product_identity(split):
    rng = np.random.default_rng(77)
    img = rng.integers(-5, 6, size=(9, 6))
    outs = O.hough4(img, split)
    Gs = {q: rng.integers(-5, 6, size=o.shape) for q, o in enumerate(outs)}
    lhs = sum(int((o * Gs[q]).sum()) for q, o in enumerate(outs))
    assert float((img * O.adjoint4(Gs, split, img.shape)).sum()) == lhs
    # a subset of quadrants contributes only its own terms
    sub = {0: Gs[0], 3: Gs[3]}
    lhs = int((outs[0] * Gs[0]).sum() + (outs[3] * Gs[3]).sum())
    assert float((img * O.adjoint4(sub, split, img.shape)).sum()) == lhs


def test_adjoint_pins_reject_a_sign_mistake():
    # the dot-product pin catches an adjoint that walks the pattern the wrong way
    rng = np.random.default_rng(3)
    A = rng.integers(-9, 10, size=(7, 5))
    G = rng.integers(-9, 10, size=(7, 5))
    P = O.patterns(7, O.SPLIT_S)
    wrong = np.zeros((7, 5))
    for x in range(7):
        for t in range(7):
            wrong[x] += G[t][(np.arange(5) + P[t, x]) % 5]
    assert float((A * wrong).sum()) != int((O.hough_lanes(A, O.SPLIT_S) * G).sum())


# ------------------------------------------------------------ sampled outputs

SAMPLE_SHAPES = [(7, 3), (3, 7), (13, 11), (5, 17), (23, 6), (1, 9), (9, 1)]


def _sample_f64_with(lib, img, split, q, t, s):
    """Call ``orc_hough_sample_f64`` of the C library ``lib`` (ctypes.CDLL)."""
    import ctypes
    img = np.ascontiguousarray(img, dtype=np.float64)
    q, t, s = (np.ascontiguousarray(v, dtype=np.int32) for v in (q, t, s))
    out = np.empty(q.shape[0])
    ab = np.empty_like(out)
    p = ctypes.c_void_p
    fn = lib.orc_hough_sample_f64
    fn.argtypes = [p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64, p, p, p, p, p]
    rc = fn(p(img.ctypes.data), img.shape[0], img.shape[1], split, q.shape[0],
            p(q.ctypes.data), p(t.ctypes.data), p(s.ctypes.data), p(out.ctypes.data),
            p(ab.ctypes.data))
    assert rc == 0
    return out, ab


def _every_output(R, C):
    """(q, t, s) of every output of the four quadrants of an R x C image."""
    qs, ts, ss = [], [], []
    for q, (W, H) in enumerate(((R, C), (R, C), (C, R), (C, R))):
        t, s = np.meshgrid(np.arange(W), np.arange(H), indexing="ij")
        qs.append(np.full(W * H, q))
        ts.append(t.ravel())
        ss.append(s.ravel())
    return np.concatenate(qs), np.concatenate(ts), np.concatenate(ss)


def _sampler_matches_full_transform(sample):
    """The sampled f64 outputs and absolute sums equal those of the whole
    transform, which the Python oracle pins (Sec. 3 definition), for all four
    quadrants, both splits, negative pixels, W > H (shifts that wrap more than
    once) and W < H."""
    rng = np.random.default_rng(41)
    for split in SPLITS:
        for R, C in SAMPLE_SHAPES:
            img = rng.standard_normal((R, C))
            q, t, s = _every_output(R, C)
            got, gab = sample(img, split, q, t, s)
            ref = O.hough4(img, split)
            rab = O.hough4(img, split, absolute=True)
            want = np.array([ref[a][b, c] for a, b, c in zip(q, t, s)])
            wab = np.array([rab[a][b, c] for a, b, c in zip(q, t, s)])
            if not (np.allclose(got, want, rtol=0, atol=1e-12) and
                    np.allclose(gab, wab, rtol=0, atol=1e-12)):
                return False
            # and the C whole-image oracle the f32 parity tests use beside it
            full, fab = native.hough4_f64(img, split)
            if not (np.allclose(got, [full[a][b, c] for a, b, c in zip(q, t, s)], atol=1e-12) and
                    np.allclose(gab, [fab[a][b, c] for a, b, c in zip(q, t, s)], atol=1e-12)):
                return False
    return True


def test_sample_f64_equals_full_transform():
    assert _sampler_matches_full_transform(lambda *a: native.sample_f64(*a))


def test_sample_u8_equals_full_transform_every_output():
    rng = np.random.default_rng(42)
    for split in SPLITS:
        for R, C in SAMPLE_SHAPES:
            img = rng.integers(0, 256, size=(R, C), dtype=np.uint8)
            q, t, s = _every_output(R, C)
            ref = O.hough4(img, split)
            want = np.array([ref[a][b, c] for a, b, c in zip(q, t, s)])
            assert (native.sample_u8(img, split, q, t, s) == want).all(), (split, R, C)


@pytest.mark.parametrize("mistake", ["sign_flip_columns", "abs_sum_signed"])
def test_sample_f64_pin_rejects_planted_mistakes(tmp_path, mistake):
    """Compile a copy of the C oracle with one mistake planted in its f64
    sampler (CPU only) and check that the pin above fails on it."""
    import ctypes
    import subprocess
    src = open(native._SRC).read()
    head, tail = src.split("int orc_hough_sample_f64", 1)
    if mistake == "sign_flip_columns":
        old = "(int64_t)sigma * pat[x]"
        new = "(int64_t)(q >= 2 ? -sigma : sigma) * pat[x]"
    else:
        old = "aacc += v < 0 ? -v : v;"
        new = "aacc += v;"
    assert old in tail
    (tmp_path / "bad.c").write_text(head + "int orc_hough_sample_f64" + tail.replace(old, new, 1))
    lib_path = tmp_path / "libbad.so"
    subprocess.run(["gcc", "-O1", "-std=c99", "-fopenmp", "-shared", "-fPIC", "-o",
                    str(lib_path), str(tmp_path / "bad.c")], check=True)
    bad = ctypes.CDLL(str(lib_path))
    assert not _sampler_matches_full_transform(lambda *a: _sample_f64_with(bad, *a))


# ------------------------------------------------- Alg. 1 recursion in C

@pytest.mark.parametrize("split", SPLITS)
def test_c_alg1_recursion_equals_direct_sums(split):
    """The C Alg. 1 recursion (the CPU timing baseline) gives the direct
    pattern sums (Sec. 3: the recursion sums exactly along Alg. 2's patterns)
    on every output, including W > H, W = 1, H = 1 and power-of-two sizes."""
    rng = np.random.default_rng(43)
    for R, C in ((1, 1), (1, 7), (7, 1), (2, 3), (13, 11), (5, 17), (61, 47), (32, 32),
                 (33, 100), (129, 6)):
        imgs = rng.integers(0, 256, size=(3, R, C), dtype=np.uint8)
        got = native.alg1_u8_batch(imgs, split)
        for i in range(3):
            ref = native.hough4_u8(imgs[i], split)
            assert (got[i] == np.concatenate([r.ravel() for r in ref])).all(), (R, C, i)
    # and the Python statement of Alg. 1 on a small case
    img = rng.integers(0, 256, size=(9, 6), dtype=np.uint8)
    got = native.alg1_u8_batch(img, split)[0]
    off = 0
    for A, sigma in O.quadrant_views(img):
        n = A.size
        assert (got[off:off + n].reshape(A.shape) == O.fht2d(A, split, sigma)).all()
        off += n
