"""MI355X (gfx950) implementation of the LAPW+LO real-time TDDFT hot path.

The compute path is the HIP library ``libltd.so`` (C ABI in include/ltd.h);
``ltd`` is its Python binding.  Importing this package does not load the
library; ``ltd.Ltd`` does, and raises if it has not been built.
"""

__all__ = ["ltd", "build"]
