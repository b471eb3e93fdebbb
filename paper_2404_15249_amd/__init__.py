"""MI355X-native kernel-free boundary integral (KFBI) solver.

The compute lives in the HIP library ``_lib/libkfbi.so`` (sources in
``csrc/``, C ABI in ``include/kfbi.h``); ``paper_2404_15249_amd.kfbi`` is its
Python binding.  Build with ``python -m paper_2404_15249_amd.build``.
"""

__all__ = ["kfbi", "build"]
