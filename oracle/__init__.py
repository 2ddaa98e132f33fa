"""Plain, slow FP64 CPU oracle for the CBFM + Calderon-preconditioned PMCHWT
method of Tanaka, Niino and Nishimura (arXiv 2111.11058).

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) may import, call, link or execute anything in this package.
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it, as the independent reference the GPU path is checked
against.  It shares no code with the GPU path; both consume only the seeded
inputs of :mod:`synth`.

Each function cites the passage of the paper it follows.  Readings taken
where the paper is silent or garbled are stated where they are used:

* time convention e^{jwt}, G = e^{-jkR}/(4 pi R) (Sec. II-A);
* the gradient in the K operator acts on the source point (the reading that
  makes the printed block system consistent with Maxwell's equations; the
  solved currents are then the negatives of the physical ones and the RCS
  is unchanged);
* Galerkin testing with the RWG functions themselves (n x t) . (n x X) =
  t . X_tan;
* 7-point degree-5 triangle rule everywhere, singularity subtraction of the
  1/R and R (resp. 1/R^3 and 1/R) terms with closed-form inner integrals on
  near pairs (P == Q, sharing a vertex, or centroid distance < 1.5 times the
  longer of the two longest edges); K of a coplanar near pair is exactly 0.
"""
