"""MI355X (gfx950) online solver for the velocity-only reduced-basis Navier-Stokes method.

The product is the C-ABI shared library ``librbns.so`` (declared in ``include/rbns.h``),
built from the HIP sources in ``csrc/`` by ``paper_1807_11866_amd.build``. ``rbns`` is its
Python binding: argument marshalling only, with PyTorch supplying device memory and streams.
"""

from . import rbns  # noqa: F401
