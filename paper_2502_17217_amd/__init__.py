"""MI355X (gfx950) Jacobian-free Newton-Krylov library for cell-centred
finite-volume solid mechanics.

The compute path is the HIP library ``libjfnk.so`` (C ABI in
``include/jfnk.h``); ``paper_2502_17217_amd.jfnk`` is its thin Python
binding.  Importing the binding fails loudly when the library is not built.
"""

__all__ = ["jfnk"]
