"""MI355X-native hot path of the mesh-constrained discrete point (MCD) method.

The compute path is the HIP library `libmcd.so` (C ABI, declared in
include/mcd.h); `paper_2404_17542_amd.mcd` is its thin ctypes binding.
Importing this package does not load the library; `inputs` and `configs`
hold seeded synthetic data and workload definitions only.
"""
