"""The stored report of the paper's Sec. 5 experiments (Fig. 1 and 2) is what
the oracle computes, and it shows the numbers the paper prints."""
import importlib.util
import os

from conftest import ROOT, read_golden
from oracle import fht_oracle as O


def _generator():
    path = os.path.join(ROOT, "tests", "golden", "make_paper_experiments.py")
    spec = importlib.util.spec_from_file_location("make_paper_experiments", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_report_is_reproduced(error_tables, paper_stats):
    gen = _generator()
    nmax = int(paper_stats["n_max"])
    fs = [O.additions(n, O.SPLIT_S) for n in range(nmax + 1)]
    ft = [O.additions(n, O.SPLIT_T) for n in range(nmax + 1)]
    text = gen.report(fs, ft, error_tables[0], error_tables[1], nmax)
    with open(os.path.join(ROOT, "tests", "golden", "paper_experiments.txt")) as fh:
        assert fh.read() == text


def test_report_shows_the_printed_numbers(paper_stats):
    rep = read_golden("paper_experiments.txt")
    assert float(rep["share_E_S_above_bound_percent"]) == float(paper_stats["share_es_above_thm2_percent"])
    assert int(rep["count_E_T_above_bound"]) == 0  # Theorem 2 holds for FHT2DT
    assert 1.69 < float(rep["max_E_S_over_E_T"]) < 1.70
    assert abs(float(rep["max_adds_S"]) - 5 * 0.6309297535714574 / 3) < 1e-6  # 5 log3(2)/3
    peaks = [int(rep[f"octave_{k}"].split()[4].split("@")[1]) for k in range(4, 11)]
    assert peaks == [int(v) for v in paper_stats["es_peaks"].split()]
