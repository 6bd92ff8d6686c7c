"""spkMC on MI355X (gfx950): the synchronous parallel kinetic Monte Carlo cycle
of Martinez, Monasterio and Marian (arXiv:1005.4713) for the 3D Ising lattice,
as hand-written HIP kernels behind the C ABI of include/spkmc.h.

``paper_1005_4713_amd.spkmc`` is the Python binding (ctypes); the shared
library is built in-tree by ``paper_1005_4713_amd.build``.
"""
