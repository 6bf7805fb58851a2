"""Plain FP64 CPU oracle for one minSR iteration on GRU wave functions.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call
or execute anything in this directory; only the test suite, the smoke check
and the CPU-baseline leg of the benchmark do.  The oracle shares no code,
constants tables or helpers with the HIP path.

Every function follows the paper ("Quantum Geometric Tensor Preconditioning
for Stable Training of Recurrent Neural Quantum States") step by step, in
float64, with numpy primitives (matmul, Cholesky, eigh) as the only library
steps.  Each function cites the section / equation / algorithm it follows.

Modules
  philox       Philox4x64-10 counter RNG (Salmon et al., SC'11), uniforms.
  model        parameter layout, Glorot init, 1D/2D GRU forward (App. A),
               autoregressive sampling (Sec. 2, Eqs. 3-7), log-amplitudes.
  hamiltonian  connected configurations and local energies (Sec. 2.3 local
               energy; Sec. 3 TFIM, cluster, J1-J2 with Marshall sign).
  jacobian     per-sample log-derivative rows O (Sec. 2.3, Alg. 1) by a
               hand-written reverse pass through the GRU recurrence.
  minsr        centring, real form, T, regularised solve, update with
               momentum (Eqs. lstsq, real-valued, minsrR; Alg. 1; App. B).
  adaptive     trust-region rate, lambda = c ||T||^(2/3) schedule and
               Levenberg-Marquardt damping (Sec. 3.3; Apps. F, G).
  conditioning spectrum of T, kappa_2(T + lambda I) and the digit estimate
               of App. E.
  qgt          population and subsampled QGT, the bound of Prop. 3 (App. H).
  linear_rnn   the linear recurrent test model of App. C: forward, sampling,
               log-derivatives, gauge directions (Prop. 1), population S
               and the closed form of Prop. 2.

Pins (tests marked "not gpu") tie every function to something other than
itself: exact enumeration, dense exact diagonalisation, closed forms,
central finite differences, the push-through identity and numpy's own
Philox generator.
"""
