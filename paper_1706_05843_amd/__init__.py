"""MI355X (gfx950) EOFA Mobius domain-wall solver.

The compute path is the HIP library ``libeofa.so`` built from ``csrc/``;
``paper_1706_05843_amd.eofa`` is a thin ctypes binding over its C ABI
(``include/eofa.h``). The library is loaded on first use and a missing or
unloadable library raises: there is no CPU fallback.
"""
