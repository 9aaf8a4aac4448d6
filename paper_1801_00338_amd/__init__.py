"""Butterfly counting in bipartite graphs on AMD MI355X (gfx950).

The computation lives in ``libbfc.so`` (HIP kernels behind the C ABI of
``include/bfc.h``); ``api`` binds it for PyTorch device tensors and streams,
``gen`` makes seeded synthetic workloads.  Importing the package loads
nothing; ``api`` loads the library on first use and fails if it is missing.
"""
__all__ = ["api", "gen"]
