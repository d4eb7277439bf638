"""MI355X-native frontier-based belief propagation (LBP, frontier residual BP and
randomized BP) behind a C ABI (``include/bp.h``, library ``libbp.so``).

``paper_1909_11469_amd.bp`` is the ctypes binding; ``paper_1909_11469_amd.inputs``
holds the seeded problem generators.  Importing the package loads nothing; the
HIP library is loaded on first use of ``bp`` and its absence is an error.
"""
__all__ = ["bp", "inputs"]
