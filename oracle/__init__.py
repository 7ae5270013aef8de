"""FP64 CPU oracle of the NEDNER reconstruction (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package. The GPU library never does.
"""
from .nedner_oracle import *  # noqa: F401,F403
from .nedner_oracle import __all__  # noqa: F401
