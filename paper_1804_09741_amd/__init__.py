"""MI355X-native Motifs-k hot path (arXiv 1804.09741).

Importing the package loads nothing native; ``paper_1804_09741_amd.motifs``
is the binding to the HIP library and ``paper_1804_09741_amd.inputs`` the
seeded graph generators.
"""
