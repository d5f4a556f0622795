"""MI355X (gfx950) robust-SOCP inner solver of nonlinear robust trajectory
optimisation (NRTO-DR and NRTO-FullADMM, cuNRTO arXiv 2603.02642).

The compute lives in libnrto.so (HIP, built by `paper_2603_02642_amd.build`);
`paper_2603_02642_amd.nrto` is its ctypes binding.  Importing this package
does not load the library; `nrto.load()` does and raises if it is missing.
"""
