#!/usr/bin/env python3
"""Writes paper_experiments.txt: the experiments of Sec. 5 (Fig. 1 and 2),
recomputed by the CPU oracle for every n <= 4096.

It calls only ``oracle/``.  Run from the repository root:
    python tests/golden/make_paper_experiments.py
"""
import math
import os
import sys
from fractions import Fraction

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import fht_oracle as O  # noqa: E402
from oracle import native  # noqa: E402

NMAX = 4096


def tables(nmax=NMAX):
    """Per n: f_S, f_T (Theorem 1 counts for n x n), E_S, E_T numerators
    (E = num / (n - 1), Theorem 2 and Sec. 5)."""
    fs = [0] * (nmax + 1)
    ft = [0] * (nmax + 1)
    for n in range(1, nmax + 1):
        fs[n] = O.additions(n, O.SPLIT_S)
        ft[n] = O.additions(n, O.SPLIT_T)
    es = native.error_numerators(nmax, O.SPLIT_S)
    et = native.error_numerators(nmax, O.SPLIT_T)
    return fs, ft, es, et


def report(fs, ft, es, et, nmax=NMAX):
    def E(num, n):
        return Fraction(int(num[n]), n - 1) if n > 1 else Fraction(0)

    def norm_adds(f, n):
        return f[n] / (n * n * math.log2(n)) if n > 1 else 0.0

    lines = [
        "# Sec. 5 experiments recomputed by the CPU oracle for n <= %d (FHT2DS = S, FHT2DT = T)." % nmax,
        "# Written by tests/golden/make_paper_experiments.py; checked by tests/test_paper_experiments.py.",
        "# adds: Theorem 1 count f(n) for an n x n image, one quadrant, normalised by n^2 log2 n (Fig. 1).",
        "# E: orthotropic error of the patterns, max over t, x of |x t/(n-1) - pat_t(x)| (Fig. 2);",
        "# bound: Theorem 2's estimate floor(log2 n)/6 + 1 - 2^-floor(log2 n).",
        "",
    ]
    above = sum(1 for n in range(1, nmax + 1) if E(es, n) > O.theorem2_bound(n))
    ratio_n = max(range(2, nmax + 1), key=lambda n: (E(es, n) / E(et, n)) if et[n] else 0)
    s_max_n = max(range(2, nmax + 1), key=lambda n: norm_adds(fs, n))
    t_max_n = max(range(2, nmax + 1), key=lambda n: norm_adds(ft, n))
    t_above = sum(1 for n in range(1, nmax + 1) if E(et, n) > O.theorem2_bound(n))
    lines += [
        "max_adds_S = %.6f  # at n = %d" % (norm_adds(fs, s_max_n), s_max_n),
        "max_adds_T = %.6f  # at n = %d" % (norm_adds(ft, t_max_n), t_max_n),
        "share_E_S_above_bound_percent = %.2f  # %d of %d" % (100.0 * above / nmax, above, nmax),
        "count_E_T_above_bound = %d" % t_above,
        "max_E_S_over_E_T = %.6f  # at n = %d" % (float(E(es, ratio_n) / E(et, ratio_n)), ratio_n),
        "",
        "# per octave [2^k, 2^(k+1)): largest normalised adds (S, T), largest E (S, T), where, and",
        "# the largest E_S / (log2 n / 6) (the peaks of Fig. 2)",
        "# k  adds_S@n  adds_T@n  E_S@n  E_T@n  E_S_norm@n",
    ]
    for k in range(0, int(math.log2(nmax)) + 1):
        ns = [n for n in range(max(2, 1 << k), min(nmax, (2 << k) - 1) + 1)]
        if not ns:
            continue
        a_s = max(ns, key=lambda n: norm_adds(fs, n))
        a_t = max(ns, key=lambda n: norm_adds(ft, n))
        e_s = max(ns, key=lambda n: E(es, n))
        e_t = max(ns, key=lambda n: E(et, n))
        p_s = max(ns, key=lambda n: float(E(es, n)) / (math.log2(n) / 6))
        lines.append("octave_%d = %.6f@%d %.6f@%d %.6f@%d %.6f@%d %.6f@%d" % (
            k, norm_adds(fs, a_s), a_s, norm_adds(ft, a_t), a_t, float(E(es, e_s)), e_s,
            float(E(et, e_t)), e_t, float(E(es, p_s)) / (math.log2(p_s) / 6), p_s))
    lines += ["", "# selected n: f_S f_T E_S E_T bound (E as exact fractions)"]
    sel = sorted({2, 3, 5, 7, 17, 23, 45, 61, 91, 181, 257, 363, 384, 725, 1021, 1024, 1451,
                  2048, 2049, 2897, 4095, 4096})
    for n in sel:
        if n > nmax:
            continue
        lines.append("n_%d = %d %d %s %s %s" % (n, fs[n], ft[n], E(es, n), E(et, n),
                                                  O.theorem2_bound(n)))
    return "\n".join(lines) + "\n"


def main():
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_experiments.txt")
    with open(out, "w") as fh:
        fh.write(report(*tables()))
    print(out)


if __name__ == "__main__":
    main()
