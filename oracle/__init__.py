"""CPU oracle package (test infrastructure only; see ``fht_oracle.py``).

``fht_oracle`` is the NumPy oracle; ``native`` wraps the same definitions in
plain C (``fht_oracle.c``) for the sizes NumPy is too slow for.  The product
library never imports this package.
"""
from . import fht_oracle  # noqa: F401
