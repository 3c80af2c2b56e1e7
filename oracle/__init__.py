"""FP64 CPU oracle for the Celeste ELBO / trust-region Newton hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package; only the tests, the smoke check and the
CPU-baseline leg of the benchmark do.  It shares no code with the HIP path:
its only common dependency is the seeded input generator (``synth``), which
holds no variational arithmetic.

It is a plain, slow, obviously-checkable implementation in NumPy FP64,
vectorised over the pixels of a patch, with plain loops elsewhere.

Modules
  model       brightness moments, PSF/galaxy mixtures with analytic first and
              second derivatives, the delta-method pixel term, KL terms, the
              ELBO with its gradient and dense Hessian (section III-A/B)
  transforms  the unconstrained coordinates the optimiser works in
  newton      trust-region Newton (section III-B) with the exact subproblem
  init        the plain initialisation heuristic
  cnn         FP64 reference of the surrogate network (forward/backward)

Parity status of each function is stated in its docstring; every function
here is pinned by a CPU test against a property the mathematics fixes.
"""
