"""FP64 CPU oracle of the plug-and-play forward-backward hot path.

TEST INFRASTRUCTURE ONLY. This package is the plain, slow, obviously correct
reference that the GPU library is checked against. Only the test-suite, the
smoke check and the benchmark's CPU-baseline leg may import it; the product
path (``paper_2207_11336_amd``) never imports, links or runs anything here,
and this package never imports the product. The two share no code; the only
common inputs are the seeded draws of the ``synth`` module.

Modules:
  ``operator``  the measurement operator Phi = G F Z, its adjoint, Phi^dagger Phi,
                the brute-force direct model (paper eq. 1, appendix E);
  ``fb``        power method for L, the Haar-l1 + positivity prox, forward-backward
                iterations, parameter rules (appendices A, B, C, F);
  ``cnn``       the residual CNN denoiser forward/backward in FP64 (appendix C).

Parity status of each function is stated in its docstring.
"""
