"""libwdirac: the even-odd Wilson-Dirac hot path of HiRep v2 (arXiv:2503.06721)
for fermions in higher representations of SU(N), on AMD MI355X (gfx950).

Submodules
----------
wdirac   ctypes binding of the C-ABI library libwdirac.so (HIP kernels)
synth    seeded synthetic inputs (links, sources)

Importing the package loads nothing; ``paper_2503_06721_amd.wdirac`` loads the
shared library and raises if it has not been built.
"""
