"""MI355X-native multigroup M1 radiation-moment step (FORNAX method, static medium).

The compute path is the HIP library ``libfornax_m1.so`` built from ``csrc/``; the Python
binding lives in :mod:`paper_1806_07390_amd.m1` and is imported explicitly (it raises if the
library has not been built).  :mod:`paper_1806_07390_amd.workloads` draws seeded inputs.
"""

__all__ = ["m1", "workloads"]
