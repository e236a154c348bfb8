"""Plain FP64 CPU oracle for the voxel-wise 3D structure-tensor pipeline.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test-suite, the entry point's smoke check and
the benchmark's CPU-baseline leg use it.  It shares no code with the HIP
library (no kernels, headers, helpers, tap tables or pre/post-processing).

The paper (Figure 1 and the "orientation" module of its Architecture section)
names the steps of the method -- 3D structure tensor, eigen-decomposition with
the fibre as the smallest-eigenvalue eigenvector, rotation into a cylindrical
frame, helix angle (HA), intrusion angle (IA) and fractional anisotropy (FA) --
but prints no formula.  Each function here writes out the textbook definition
of its step, slowly and in float64, and states the reading taken where the
paper is silent.

Modules
-------
filters   Gaussian / derivative-of-Gaussian taps, reflect boundary, 1-D correlation
tensor    gradients at sigma, outer products, integration at rho
eigen     sorted eigen-pairs (LAPACK), cyclic Jacobi cross-check, FA, degeneracy
angles    cylindrical frame about the given axis, HA and IA
pipeline  the whole path on one volume (or one padded block) -> every output map
surrogate forward pass of the learned orientation surrogate (a dense 3-D CNN)

Parity pins: every function is pinned by the ``-m "not gpu"`` tests
(brute-force 3-D correlation, SciPy's ``gaussian_filter``, closed forms,
eigen invariants, exact special cases, hand-derived angle fixtures, an
analytic phantom, invariances and halo exactness).  No function is
"parity unpinned".
"""

from .filters import radius, taps, reflect_index, correlate_axis  # noqa: F401
from .tensor import gradients, outer_products, integrate, structure_tensor  # noqa: F401
from .eigen import (  # noqa: F401
    eigen_sorted, canonical_sign, jacobi_eigen, fractional_anisotropy, gap_ratio,
    degenerate, DEGENERATE_GAP,
)
from .angles import cylindrical_frame, helix_intrusion, ON_AXIS_RADIUS  # noqa: F401
from .pipeline import (  # noqa: F401
    compute, FLAG_DEGENERATE, FLAG_OUTSIDE_MASK, FLAG_ON_AXIS,
)
from . import surrogate  # noqa: F401
