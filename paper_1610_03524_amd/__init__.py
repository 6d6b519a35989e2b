"""MI355X-native wavelet tree / wavelet matrix construction.

Builds the structures of Shun, "Improved Parallel Construction of Wavelet
Trees and Rank/Select Structures" (balanced and shaped binary wavelet trees,
multiary wavelet trees, wavelet matrices, with rank/select directories) with
hand-written HIP kernels for gfx950, behind the C-ABI of include/wavelet.h.

``paper_1610_03524_amd.binding`` is the Python binding of that C-ABI;
``paper_1610_03524_amd.inputs`` holds the seeded input generators.  Importing
the package loads nothing; the library is loaded on first use.
"""
__all__ = ["binding", "inputs"]
