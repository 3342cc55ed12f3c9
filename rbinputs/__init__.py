"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package stands in for the offline stage of the reduced-basis method (high-fidelity
snapshots, POD, supremizers and Galerkin projection, paper Sections 3.1-3.5): it builds a
solenoidal reduced velocity basis, a pressure basis with its supremizers, and the affine
operators that the online stage consumes. It also draws the parameter samples mu.

It holds none of the online method's arithmetic: no parameter functions theta(mu), no affine
sums, no Newton iteration and no linear solves. Both the oracle and the HIP library receive
its arrays as inputs.
"""

from .configs import CONFIGS, get_config  # noqa: F401
from .synth import TensorSet, make_tensor_set, draw_mu, draw_basis_sizes  # noqa: F401
