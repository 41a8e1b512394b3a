"""MI355X-native twisted-mass Wilson Dslash, CG and fermion force (arXiv:1209.5942).

The compute path is the HIP library ``libtmqcd.so`` (C ABI declared in
``include/tmqcd.h``); :mod:`paper_1209_5942_amd.tmqcd` is its thin Python
binding.  Importing this package loads nothing; the binding loads the library on
first use and raises if it is missing.
"""
__all__ = ["synth", "tmqcd"]
