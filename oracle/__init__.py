"""CPU FP64 oracle for the Galerkin capacitance method (test infrastructure only).

Only tests/, the smoke check and the bench's CPU-baseline leg may import this
package.  It shares no code with the GPU library.
"""
from .oracle import *  # noqa: F401,F403
