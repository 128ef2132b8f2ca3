"""MI355X (gfx950) implementation of the matrix-free Hermite Galerkin method on
hyperbolically reduced index sets (Brumm, arXiv 1403.3511).

The compute path is the C-ABI library libhs.so (include/hs.h) built from csrc/;
paper_1403_3511_amd.hs is its ctypes binding.
"""
__all__ = ["hs"]
