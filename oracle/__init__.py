"""CPU oracle for Neural Bounding (arXiv 2310.06822) -- TEST INFRASTRUCTURE.

A plain, slow, obviously-correct numpy implementation of everything the GPU
hot path computes.  It exists only to check the GPU path: only the test suite,
the smoke check and the benchmark's CPU-baseline leg may import it.  The
product path never calls it and has no CPU fallback.

It shares no code with the HIP library or its Python binding; the only common
dependency is the seeded input generator module ``synth`` (random draws only).

Modules (each function cites the passage of the paper it follows):
  philox      counter-based generator Philox4x32-10 (Salmon et al., SC'11),
              written from its published definition.
  sampling    region sampling for training batches (Alg. 1, step "Uniform").
  indicators  indicator f and region query g (Sec. 3.1, Sec. 4.2 "Query
              types"): discs, metaball voxel grids, rays, boxes, planes,
              moving 4-D metaballs; float32 with a fixed operation order.
  mlp         the bound h_theta as an MLP (Sec. 3.4 "Architecture"), forward
              and backward in float64, optional bfloat16 quantisation points.
  loss        Eq. 1 (weighted BCE), its gradient, the decision threshold from
              the output epsilon (supplemental "Numerics"), TP/FP/TN/FN.
  adam        Adam (Kingma & Ba 2014), the optimiser of Sec. 3.4 "Training".
  train       Alg. 1 as a training loop with the FN-weight ramp.
  cascade     bound-then-exact cascade and the benefit inequality (Sec. 6).
  kdop        k-DOP bounds trained with the asymmetric loss (Sec. 4.1).
  hierarchy   neural bounding hierarchies: a user tree of bounds, descended
              from the root (Sec. 3.3).

Parity status: every function here is pinned by a test in tests/ against a
closed form, a brute-force enumeration, a library routine or a value printed
in the paper -- except where a module docstring says "parity unpinned".
"""
