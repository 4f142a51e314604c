"""GBEES hot path for MI355X: hashed sparse-grid CTU advection of a probability
density (arXiv 2508.13986) as hand-written HIP kernels behind a C-ABI library.

Import ``paper_2508_13986_amd.gbees`` for the binding (it loads libgbees.so and
fails loudly if the library has not been built) and
``paper_2508_13986_amd.scenarios`` for the seeded synthetic workloads.
"""
