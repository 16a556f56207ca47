"""MI355X-native PLE decomposition over GF(2) (Albrecht, Bard, Pernet).

The compute path is the C-ABI library ``libgf2ple.so`` (HIP kernels for
gfx950); ``paper_1111_6549_amd.gf2ple`` is its thin Python binding and
``paper_1111_6549_amd.inputs`` synthesises seeded workloads.
"""
__all__ = ["gf2ple", "inputs"]
