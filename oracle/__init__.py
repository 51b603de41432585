"""FP64 CPU oracle for the angle-averaged polyspectrum estimator.

TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path imports,
links or runs this package; only the tests, the smoke check and the benchmark's
CPU-baseline leg do.  It shares no code with the HIP path.
"""
from .polyspec import *  # noqa: F401,F403
from .bruteforce import bruteforce_polyspectrum, shell_vectors  # noqa: F401
from .analytic import n_tri_leading, n_quad_leading  # noqa: F401
