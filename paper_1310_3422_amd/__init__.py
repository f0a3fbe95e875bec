"""MI355X-native group explicit (GE) sweep for the 1D diffusion equation.

The numerical work runs in the HIP library ``libge.so`` (built from
``csrc/``) behind the C ABI declared in ``include/ge.h``; ``ge`` is its thin
ctypes binding.  ``inputs`` holds the seeded synthetic workloads.
"""
__all__ = ["ge", "inputs"]
