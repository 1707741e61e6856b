"""FP64 CPU oracle for PURSE boundary sampling and the MEGB.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
HIP path is checked against.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does, and
it shares no code with the HIP kernels or their host library.

Every function follows a passage of the paper ("CLOSURE: Fast Quantification
of Pose Uncertainty Sets", arXiv 2403.09990) or, where the paper leaves a step
open, the reading listed in the design notes.  Arithmetic is float64 torch on
the CPU, vectorised only across independent trajectories; each trajectory's
steps are taken in the order the method states.

Parity unpinned: which boundary point a given trajectory lands on.  Outside
the zero-radius collapse there is no closed form for it; it is pinned only by
feasibility, equivariance and agreement with the GPU.
"""
from .params import OracleParams  # noqa: F401
