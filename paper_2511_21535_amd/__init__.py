"""MI355X (gfx950) near-field (P2P) operator of the multilevel fast multipole
algorithm, with the redundant data layout of arXiv 2511.21535.

The compute path is libp2p.so (hand-written HIP, C ABI in include/p2p.h);
``api`` is its torch-facing binding and ``autograd`` wraps the adjoints.
Importing this package does not load the library; ``api`` calls do, and they
fail loudly if it has not been built.
"""
__all__ = ["api", "autograd", "workloads"]
