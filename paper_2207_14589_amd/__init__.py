"""SPED on MI355X: eigengap dilation p(L) of graph Laplacians, hand-written HIP for gfx950.

The compute path is the C-ABI library ``libsped.so`` (built from ``csrc/``);
``paper_2207_14589_amd.sped`` is its argument-marshalling binding over torch
device tensors, and ``paper_2207_14589_amd.autograd`` holds ``PolyApply``.
``paper_2207_14589_amd.synth`` draws seeded synthetic graphs and blocks.
Nothing here loads the library at import time; the first call does, and it
raises if the library is missing.
"""
__all__ = ["synth", "sped", "autograd"]
