"""MI355X-native enriched-finite-element residual Chebyshev eigensolver.

The compute path lives in the HIP library ``libefe.so`` (sources under
``csrc/``, C-ABI in ``include/efe.h``); ``paper_2607_06848_amd.efe`` is the thin
ctypes binding.  Importing this package loads nothing: ``workloads`` holds the
seeded synthetic inputs.
"""
