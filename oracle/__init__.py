"""CPU oracle for C = A x B on CSC matrices -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package. The GPU library never imports, links or calls it, and it imports
nothing from the GPU package.
"""
from .oracle import *  # noqa: F401,F403
