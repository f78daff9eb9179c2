"""Plain FP64 CPU oracle for the w-product hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
Python binding, the timed part of the benchmark) may import or call this
package: only the tests, the smoke check and the benchmark's CPU-baseline leg
do.  It shares no code with the HIP implementation.
"""

from .wprod_oracle import *  # noqa: F401,F403
