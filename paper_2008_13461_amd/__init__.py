"""MI355X (gfx950) implementation of the pixel-track hot path of Bocci et al.,
"Heterogeneous reconstruction of tracks and primary vertices with the CMS
pixel tracker": doublets, cellular-automaton links, n-tuplets with duplicate
removal, the broken-line fit and its adjoint, as HIP kernels behind the C
interface of include/pixeltrack.h.

    from paper_2008_13461_amd import api, build
    build.build()                      # compiles libpixeltrack.so for gfx950
    pipe = api.Pipeline(cfg, n_hits=..., ...)
"""
__all__ = ["api", "build", "autograd"]
