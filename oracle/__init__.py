"""Reference oracle for the Holstein DQMC sweep (Li, Dee, Khatami, Johnston,
"Accelerating lattice quantum Monte Carlo simulations using artificial neural
networks: an application to the Holstein model").

TEST INFRASTRUCTURE ONLY.  This package is a plain, serial, FP64 CPU
implementation of what the GPU library computes.  It exists so that tests, the
smoke check and the benchmark's CPU-baseline leg can check the HIP path against
something written directly from the paper.  Nothing in the product package
imports it, and it imports nothing from the product package; the two share
only the seeded input generators in ``workloads``.

Modules
  philox  -- Philox4x64-10 counter-based generator (Salmon et al., SC'11)
  model   -- Holstein model: hopping matrix, B_l, phonon action (paper: Model,
             Determinant quantum Monte Carlo)
  udt     -- stabilised G and log|det M| from scratch (UDT chain)
  dqmc    -- the conventional sweep: wraps, local moves with rank-1 updates,
             periodic recomputation, global (block) moves, observables
  nnmc    -- the fully connected local-move network and the cumulative update
             (paper: Local Updates, and the p_c equation)

Parity status of each function is stated in its module header.
"""
