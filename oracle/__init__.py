"""CPU FP64 oracle for the lattice Boltzmann particle-resolved method.

TEST INFRASTRUCTURE ONLY. Nothing on the product path may import this
package: only the test-suite, the smoke check and the CPU-baseline leg of
the benchmark call it. It shares no code, tables or constants with the HIP
library; both sides take their inputs from the ``synth`` package alone.

The method is the one compared in Peng, Ayala, Brandle de Motta & Wang,
"A comparative study of immersed boundary method and interpolated
bounce-back scheme for no-slip boundary treatment in the lattice Boltzmann
method: Part II, turbulent flows" (arXiv 1906.05448). The paper names each
scheme by citation and gives no formulas; every module here states the
standard published form it follows and the reading taken where the paper is
silent. Everything is plain numpy in float64, written for checking by eye,
not for speed.

Modules
  lattice     D3Q19 velocities, weights, d'Humieres moment basis (Sec. 3.1)
  collide     equilibrium, Guo forcing, MRT collision, pull streaming
  geometry    sphere / pipe classification, boundary links and q (Sec. 3.1)
  ibb         Bouzidi interpolated bounce-back, fallback chain, GIMEM (Sec. 3.1)
  ibm         Peskin 4-point delta, markers, multi-direct forcing, Kempe
              inner inertia (Sec. 2.1, Sec. 3.1)
  particles   rigid-body motion and soft-sphere normal contact (Sec. 3.1)
  refill      refilling of freshly uncovered nodes (Sec. 3.1)
  stats       kinetic energy, dissipation, particle energies, local
              profiles (Sec. 2.2, Sec. 3.2)
  sim         the time-stepping driver tying these together
  mlp         the near-surface gradient corrector network, forward/backward
"""
