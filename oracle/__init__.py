"""FP64 CPU oracle for one AERO-MPPI planning step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP library; the two
meet only at the seeded inputs built by `fixtures`.

Every routine is a plain, slow, literal transcription of the paper's
definitions (section / equation cited in each docstring), evaluated in
float64 on the float32 inputs the GPU sees.  Readings of passages the paper
leaves open are stated where they are used.

Modules
  partition  Sec. IV-A (multi-resolution partition) and IV-B-1/2 (anchors)
  guides     Sec. IV-B-3, eq. (polynomial): quintic guiding trajectories
  philox     counter-based normal noise (Philox4x32-10 + Box-Muller)
  dynamics   Sec. III-A, eq. (dynamics) and RK4, eq. (mppi_rollout)
  cost       Sec. IV-C, eq. (total cost) and its five terms
  mppi       Sec. III-B, eqs. (mppi_weights), (mppi_update); Stage II select
  adjoint    gradient of the summed Stage-I cost (PyTorch autograd, FP64)
"""
