"""MI355X-native wavelet tree and wavelet matrix construction.

Bottom-up construction of the level-wise wavelet tree and the wavelet matrix
(Fischer, Kurpicz, Loebel, arXiv 1702.07578) as hand-written HIP kernels for
gfx950 behind a small C ABI (``include/wt.h``), with a thin ctypes binding.

Submodules are imported lazily: ``inputs`` (seeded synthetic texts) needs no
GPU library; ``binding`` loads ``libwt.so`` and fails loudly if it is absent.
"""
__all__ = ["binding", "inputs"]
