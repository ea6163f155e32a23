"""MI355X-native flip Monte Carlo for rigid triangular A/B/C molecules.

The engine is the HIP library ``libflipmc.so`` behind the C ABI of
``include/flipmc.h``; :mod:`paper_2506_21290_amd.flipmc` is its Python binding.
"""
from . import flipmc  # noqa: F401

__all__ = ["flipmc"]
