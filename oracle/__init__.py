"""CPU oracle for the Magnus time-evolution path (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg may import this
package; the library never does.
"""
from .magnus import *  # noqa: F401,F403
