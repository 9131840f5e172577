"""MI355X-native Lindhard / RPA susceptibility (arXiv:1208.3210) -- package root.

The compute path is the C ABI of ``liblindhard.so`` (see include/lindhard.h);
``paper_1208_3210_amd.lindhard`` is its Python binding and
``paper_1208_3210_amd.workloads`` holds the seeded synthetic inputs.
Importing the package loads nothing heavy.
"""
__all__ = ["lindhard", "workloads"]
