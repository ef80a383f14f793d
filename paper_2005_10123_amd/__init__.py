"""MI355X (gfx950) library for the exact O(N^2) spatiotemporal Hawkes log-likelihood of
arXiv 2005.10123 and its gradient.

The compute lives in ``libhawkes.so`` (HIP kernels behind a C ABI, ``include/hawkes.h``).  Import
``paper_2005_10123_amd.binding`` for the thin ctypes layer, ``paper_2005_10123_amd.autograd`` for
the ``torch.autograd.Function``, ``paper_2005_10123_amd.synth`` for seeded synthetic events and
``paper_2005_10123_amd.mcmc`` for the samplers that drive the serving API.
Importing this package loads nothing.
"""
__all__ = ["binding", "autograd", "synth", "mcmc"]
