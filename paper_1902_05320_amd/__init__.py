"""Batch SHA-3 (Keccak-f[1600] sponge) for AMD MI355X (gfx950).

The HIP library and its ctypes binding live in ``paper_1902_05320_amd.kbatch``
(imported on demand so that the seeded workload generators in
``paper_1902_05320_amd.workloads`` load without a GPU stack).
"""
