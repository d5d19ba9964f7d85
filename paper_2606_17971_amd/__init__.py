"""MI355X (gfx950) restricted-system A-DEF2 solver.

The solver lives in the HIP library ``libadef2.so`` (C ABI in include/adef2.h);
``paper_2606_17971_amd.binding`` is its Python binding.  Build the library with
``python -m paper_2606_17971_amd.build``.
"""
__all__ = ["binding", "build"]
