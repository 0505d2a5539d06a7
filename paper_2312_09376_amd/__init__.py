"""MI355X-native generalized random butterfly transform (RBT) solver.

The compute path lives in the HIP/C++ shared library built from csrc/ and is
reached through the C ABI declared in include/rbt.h; `rbt` is the thin ctypes
binding (argument marshalling only).  `workloads` draws seeded synthetic
inputs.
"""
