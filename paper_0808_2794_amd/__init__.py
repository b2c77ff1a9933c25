"""MI355X (gfx950) mixed-precision dense linear solver.

Low-precision LU (or Cholesky) on the GPU, refined to FP64 accuracy by FP64
residuals (Algorithm 1 of Baboulin et al., arXiv:0808.2794), exposed through
the C ABI in ``include/mixlu.h``; ``paper_0808_2794_amd.mixlu`` is the Python
binding.  Importing this package does not load the shared library; the
first call into ``mixlu`` does, and fails loudly if it has not been built.
"""
from . import mixlu  # noqa: F401
