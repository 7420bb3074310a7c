"""Plain FP64 CPU oracle for the NESA EFIE matrix-vector product and the GMRES
solve around it.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  The product library never calls
it, shares no code with it, and must fail loudly when its HIP extension is
missing instead of falling back to anything here.

Every function follows the paper (Zafari et al., "Task parallel implementation
of a solver for electromagnetic scattering problems") by section and equation:

* Sec. 2, Eq. (1)-(3): EFIE radiated field, Galerkin testing, the dense system
  Z j = b  (``efie``);
* Sec. 2, Eq. (4)-(7) and Sec. 3, Eq. (9)-(14): the near-field product and the
  five far-field stages of the nested equivalent source approximation
  (``tree``, ``nesa``);
* Sec. 2 (the iterative solver around the product): restarted GMRES and
  flexible GMRES (``krylov``);
* the Mie series for the PEC sphere (``mie``) and the per-leaf MLP (``mlp``)
  are outside the paper and pin the discretisation and the learned
  preconditioner respectively.

Where the paper is silent, each module states the reading it takes.
"""
