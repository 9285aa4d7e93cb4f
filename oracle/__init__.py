"""CPU oracle for the Magnus time-evolution path and numerical NPAD (test
infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg may import this
package; the library never does.  `oracle.npad` holds the NPAD oracle.
"""
from .magnus import *  # noqa: F401,F403
from . import npad  # noqa: F401
