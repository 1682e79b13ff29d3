"""MI355X-native asynchronous discontinuous Galerkin (ADG) solver.

The compute path is the HIP library ``libadg.so`` (C ABI in ``include/adg.h``);
``paper_2501_01747_amd.adg`` is its ctypes binding.  Importing the binding
loads the library and raises if it has not been built.
"""
