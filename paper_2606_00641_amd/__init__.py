"""MI355X (gfx950) implementation of the vectorial lattice Boltzmann method for MHD.

The hot path (collide + stream sweep, diagnostics) lives in the HIP library
``libvlbm.so`` behind the C ABI of ``include/vlbm.h``; ``vlbm`` is its Python
binding.  Import ``paper_2606_00641_amd.vlbm`` explicitly: it raises if the
library has not been built.
"""
__all__ = ["vlbm"]
