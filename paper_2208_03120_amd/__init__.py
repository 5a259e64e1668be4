"""MI355X (gfx950) multi-marginal Sinkhorn with NFFT fast summation.

The compute path is the HIP library ``libmot.so`` (C ABI in include/mot.h); the
Python binding is ``paper_2208_03120_amd.mot``.  Importing the package itself loads
nothing, so the seeded input generators in ``workloads`` are usable without a GPU.
"""
