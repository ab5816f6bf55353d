"""Fast discrete Walsh transforms on digital nets, native on AMD MI355X (gfx950).

The compute path is the C-ABI library ``libfdwt.so`` built from ``csrc/``
(hand-written HIP kernels); ``fdwt`` is its thin Python binding.  Importing
this package does not load the library; ``fdwt`` loads it on first use and
raises if it is missing.
"""
__all__ = ["fdwt", "inputs"]
