"""MI355X (gfx950) implementation of the PMCHWT fill, CBF projection and
Calderon-preconditioned reduced solve of the CBFM (arXiv 2111.11058).

The computation lives in ``libcbfm.so`` (HIP, built by ``build.py``); the
``cbfm`` module is its ctypes binding.
"""
