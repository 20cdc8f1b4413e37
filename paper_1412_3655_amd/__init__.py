"""paper_1412_3655_amd -- SU(3) lattice Landau gauge fixing by checkerboard
overrelaxation on AMD Instinct MI355X (gfx950).

The compute path is the HIP library ``libgf.so`` (sources in ``csrc/``, C ABI
in ``include/gf.h``).  ``paper_1412_3655_amd.gf`` is a thin ctypes binding
with the same entry-point names; it only marshals arguments.  Method:
H. Vogt and M. Schroeck, "cuLGT: Lattice Gauge Fixing on GPUs",
arXiv:1412.3655.
"""

__all__ = ["gf"]
