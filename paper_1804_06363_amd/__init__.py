"""MI355X (gfx950) reduced-basis iterative solvers: RBCG, RBI and the adaptive greedy.

The compute lives in librb.so (HIP kernels + C ABI, see include/rb.h); ``rb`` is its
ctypes binding.  Import ``paper_1804_06363_amd.rb`` explicitly: it fails loudly when
the library has not been built.
"""

__all__ = ["rb"]
