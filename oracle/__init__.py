"""Plain FP64 CPU oracle for the Ewald-summed RPY Brownian-dynamics step.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the HIP library and the HIP library never routes through it.
"""
from .oracle import *  # noqa: F401,F403
