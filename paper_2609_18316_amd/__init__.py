"""MI355X-native k-d tree: GPU build, kNN and ball queries, friends-of-friends
grouping and adaptive SPH particle-to-mesh deposit (with adjoint).

The compute path is the HIP library ``libkdt.so`` (C ABI in include/kdt.h);
``paper_2609_18316_amd.kdt`` is its Python binding.
"""
__all__ = ["kdt", "workloads"]
