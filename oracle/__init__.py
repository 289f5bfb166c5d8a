"""FP64 CPU oracle for CoNet-Rx. TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the bench's CPU-baseline leg may import this
package. The GPU product path never calls it and shares no code with it.

Parity status: every function here is pinned by a CPU test against something other
than itself (brute force, closed forms, special cases, finite differences).
"""
from . import conet64, classical
