"""MI355X-native entropic Gromov-Wasserstein on uniform grids (arXiv 2404.08970).

The compute path is the HIP library ``libgw.so`` built from ``csrc/``; the
Python binding in :mod:`paper_2404_08970_amd.gw` only marshals arguments.
Importing this package does not load the library; import ``.gw`` for that.
"""
