"""Wall-corrected Rotne-Prager-Yamakawa blob mobility on MI355X (gfx950).

The compute path lives in the HIP library ``librpywall.so`` (C ABI declared in
``include/rpywall.h``); ``paper_1709_02410_amd.rpywall`` is the thin Python
binding over it.  Importing this package loads nothing; the binding loads the
library on first use and raises if it is missing.
"""
__all__ = ["rpywall", "workloads"]
