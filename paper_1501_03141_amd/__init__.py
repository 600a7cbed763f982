"""MI355X-native PDEP chi0 hot path.

The compute path is a HIP shared library (``libpdep.so``) with a C ABI declared in
``include/pdep.h``; :mod:`paper_1501_03141_amd.pdep` is a thin ctypes binding over it.
:mod:`paper_1501_03141_amd.inputs` holds the seeded synthetic workload generators.

Nothing is imported eagerly so that the input generators can be used without the
shared library being built.
"""

__all__ = ["inputs", "pdep"]
