"""MI355X-native sparse Fast Chebyshev Transform.

The transform's hot path (alias plan, sampling, separable DCT-I, CGLS least
squares) lives in the HIP library ``libfct.so`` behind the C ABI declared in
``include/fct.h``; ``paper_2309_14584_amd.fct`` is its Python binding.
Build the library with ``python -m paper_2309_14584_amd.build``.
"""
__all__ = ["fct", "build"]
