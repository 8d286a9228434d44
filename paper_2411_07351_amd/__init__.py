"""Dyadic-pattern fast Hough transform (FHT2DS / FHT2DT) for MI355X (gfx950).

The transform of arXiv 2411.07351 (Sec. 3, Alg. 1) runs in the hand-written
HIP kernels of ``libfht.so``; this package is its thin binding.  Build the
library with ``python paper_2411_07351_amd/build.py``.
"""
from ._binding import *  # noqa: F401,F403
from ._binding import Batch, FhtError, HoughFunction, Plan, hough, hough_autograd  # noqa: F401
