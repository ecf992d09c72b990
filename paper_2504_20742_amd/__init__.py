"""MI355X-native explicit finite-volume step of the non-equilibrium contrail
solver of Tegethoff & Wheeler (arXiv 2504.20742).

The compute path is the HIP library ``libcontrail.so`` (C ABI declared in
``include/contrail.h``); ``binding`` marshals torch tensors / raw device
pointers into it.  ``inputs`` holds the seeded synthetic workloads.
Importing the package does not load the library; ``binding.load()`` does and
raises if it is missing.
"""
__all__ = ["inputs", "binding"]
