"""MI355X (gfx950) implementation of the Morse-Smale-complex-preserving correction stage of
error-bounded lossy compression (DMTz, arXiv 2409.17346).

``paper_2409_17346_amd.dmt`` is the Python binding of the C ABI (``include/dmt.h``);
``paper_2409_17346_amd.synth`` draws seeded synthetic inputs; ``paper_2409_17346_amd.build``
compiles the HIP library.  Importing the package does not load the library.
"""
__all__ = ["dmt", "synth", "build"]
