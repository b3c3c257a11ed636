"""MI355X (gfx950) randomized block-Lanczos PCA: HIP kernels behind a C ABI (include/rpca.h).

Import ``paper_1007_5510_amd.rpca`` for the Python surface; the shared library
is built in-tree by ``paper_1007_5510_amd.build``.
"""
