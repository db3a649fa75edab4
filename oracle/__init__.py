"""CPU oracle for the non-standard-form operator apply (TEST INFRASTRUCTURE ONLY).

This package is a plain, slow, deliberately unoptimised restatement of the
method of Beylkin, Cheruvu and Perez, "Fast Adaptive Algorithms in the
Non-Standard Form for Multidimensional Problems".  It exists to check the
HIP implementation in ``paper_0706_0747_amd``; it is NOT part of the product.

Rules this package keeps:
  * It shares no code, tables or constants with the HIP library and never
    imports it.  The only common module is ``workloads`` (seeded synthetic
    inputs, which contains none of the method's arithmetic).
  * Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
    ``bench.py`` may import or execute anything here.
  * All floating point is IEEE binary64.

Modules
  mra          1-D multiresolution tables: Gauss-Legendre rule, Legendre
               scaling functions, two-scale filters, cross-correlations,
               operator blocks F^{j;m,l}                     (App. A.1-A.4, eq. KernelFactor)
  fit          Gaussian-sum fit of the kernels (-Delta+mu^2)^(-alpha)
                                                             (Sec. 3, eqs. IntegralRepr, KernelApproxByGaussians)
  plan         1-D block norms, 3-D norm estimates, per-(scale, L) term ranges
                                                             (Sec. 4, eqs. BlockNorms, NormEstimateUsing1DBlocks)
  tree         adaptive projection (Alg. 1), redundant tree (Sec. 2.2.1),
               keys, evaluation                              (Sec. 2.2, App. A.1)
  apply        modified ns-form apply (eq. apply_algo, Alg. 3), the
               difference form (eq. g_scales_band) as a self-check,
               assembly (eq. g_assemble), and the dense plain definition
  closed_forms analytic potentials of Gaussian sources used as references
"""
