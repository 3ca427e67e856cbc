"""MI355X-native CE-MPPI replan engine (clustering-embedded MPPI).

The compute path lives in the HIP library ``libcemppi.so`` (sources under
``csrc/``, C-ABI declared in ``include/cemppi.h``); ``binding`` marshals
arguments to it through ctypes.  ``workloads`` builds seeded synthetic
scenes.  Importing this package loads nothing; the library is opened on
first use of ``binding``.
"""
__all__ = ["binding", "workloads"]
