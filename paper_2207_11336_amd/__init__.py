"""MI355X-native hot path of plug-and-play forward-backward radio-interferometric
imaging (wide-field Phi = G F Z, its adjoint, the fused gradient, the Haar-l1 +
positivity prox and the learned residual CNN denoiser), as HIP kernels for
gfx950 behind the C ABI of include/ri.h.

``paper_2207_11336_amd.ri`` is the thin Python binding with the C ABI's names.
Importing this package does not load the library; the first call does, and
fails loudly if libri.so has not been built.
"""
