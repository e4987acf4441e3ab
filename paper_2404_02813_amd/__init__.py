"""MI355X-native RSF level-set evolution (arXiv 2404.02813), HIP for gfx950.

Importing the package loads nothing; ``paper_2404_02813_amd.rsf`` binds the
C-ABI library ``librsf.so`` on first use and fails loudly if it is missing.
"""
