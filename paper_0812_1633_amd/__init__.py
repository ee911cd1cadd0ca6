"""MI355X-native replica-exchange Lennard-Jones molecular dynamics.

The engine lives in the HIP library ``libre_hip.so`` (C ABI in
``include/re.h``); :mod:`paper_0812_1633_amd.re` is its ctypes binding and
:mod:`paper_0812_1633_amd.workloads` holds the seeded workload recipes.
"""
from .re import Engine, ReError, lib  # noqa: F401
