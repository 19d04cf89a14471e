"""CPU oracle for tent-pitched space-time Trefftz-DG (test infrastructure only).

This package is a plain, slow, FP64 re-statement of what the hot path
computes, written from the paper (Perugia, Schoeberl, Stocker, Wintersteiger,
"Tent pitching and Trefftz-DG method for the acoustic wave equation").  It is
the yardstick the GPU library is checked against and nothing else: only the
tests, the smoke check and the CPU-baseline leg of the benchmark may import it.
The product path never calls into it, and it shares no code with the library
(only the seeded mesh/data generators in ``workloads`` serve both).

Modules:
  quadrature  Gauss-Legendre / Gauss-Jacobi (Golub-Welsch) and collapsed
              simplex rules (Sec. 4.1: one n-simplex rule mapped to all faces)
  trefftz     exact-rational Trefftz basis of U^p via the recursion (eq. 3.1)
  topology    vertex patches, boundary and interface facets
  pitcher     advancing-front tent pitcher with layers (Sec. 2.2)
  tdg         per-tent local system (eq. 4.1, Sec. 4.2, Sec. 5), solve, front
              update, error and energy (Sec. 6, Sec. 6.5)
  global_tdg  the global Trefftz-DG system (eq. 2.5) assembled face by face
  mlp         FP64 reference of the degree-selection MLP (forward, backward)
"""
