"""MI355X (gfx950) Gaussian-mixture training: k-means seeding and EM for
diagonal and full covariances, after Sanderson & Curtin, arXiv:1707.09094.

The compute path is the HIP library ``libgmm.so`` behind the C ABI in
``include/gmm.h``; ``gmm`` is its Python binding, ``train`` a small host
driver (the learn() sequence of the paper's Sec. 4 API), ``synth`` the seeded
synthetic workloads.
"""
__all__ = ["gmm", "train", "synth"]
