"""MI355X-native KAZE nonlinear scale space and detector response.

The compute path is the HIP library ``libkaze.so`` (``include/kaze.h``);
``paper_1706_06750_amd.kaze`` is its ctypes binding.
"""
