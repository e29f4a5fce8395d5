"""Plain FP64 CPU oracle for partitioned KRR.  Test infrastructure only: the
library never imports it; tests, the smoke check and the benchmark's CPU
baseline do."""
from .krr_oracle import *  # noqa: F401,F403
