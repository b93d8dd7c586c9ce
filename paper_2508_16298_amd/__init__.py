"""MI355X-native HQMC hot path for lattice QED3 (compact U(1) gauge field
coupled to two fermion flavours).

The compute path lives in ``libqedhmc.so`` (HIP, gfx950) behind the C ABI
declared in ``include/qedhmc.h``; ``qedhmc`` is its thin ctypes binding.
Importing the package does not load the library; the first call does, and
fails loudly if it is missing.
"""
__all__ = ["inputs", "qedhmc"]
