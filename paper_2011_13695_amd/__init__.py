"""MI355X-native exact-LLR Monte-Carlo GMI / MI (HIP kernels behind a C ABI).

The compute path is libmdgmi.so (paper_2011_13695_amd/csrc, built by
paper_2011_13695_amd.build); paper_2011_13695_amd.mdgmi is its ctypes
binding. Importing the package does not load the library.
"""
__all__ = ["mdgmi", "build"]
