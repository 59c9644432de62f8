"""MI355X-native inexact policy iteration (iPI) for discounted finite MDPs.

The compute path is the HIP library ``libipi.so`` (C ABI declared in
``include/ipi.h``); ``paper_2507_22538_amd.ipi`` is its thin ctypes binding.
Importing this package loads nothing; the binding loads the library on first
use and raises if it is missing.
"""
__version__ = "0.1.0"
