"""Thread count of the oracle's FFTs (test infrastructure only).

Uses OMP_NUM_THREADS when set (the GPU hosts set it to their per-GPU CPU
share), else every CPU this process may run on, capped at 16.
"""

import os

try:
    WORKERS = int(os.environ.get("OMP_NUM_THREADS", "0"))
except ValueError:
    WORKERS = 0
if WORKERS <= 0:
    WORKERS = min(16, len(os.sched_getaffinity(0)))
