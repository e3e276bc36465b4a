"""Plain FP64 CPU oracle for the AMR topology-optimisation hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package; only the tests, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the HIP library: it consumes the
same seeded inputs (``synth``) and re-derives everything from the paper.

Paper: S. Wang, E. de Sturler, G. H. Paulino, "Dynamic Adaptive Mesh
Refinement for Topology Optimization" (arXiv:1009.4975).

Modules
-------
element   Q1 hexahedral element stiffness K0 (Sec. 3 discretisation).
mesh      Leaves -> nodes, connectivity, hanging-node interpolation P
          (Sec. 6, Eq. (6)), supports and consistent loads.
system    Sparse assembly, the projected system (Eq. (7)-(9)), direct and
          Jacobi-PCG solves (Sec. 5 diagonal rescaling).
topopt    Compliance (Eq. (1)), sensitivities, the filters (Eq. (3)-(5)) and
          the Optimality Criteria update (Sec. 3).
amr       Octree marking, the two compatibility sweeps, the level-one
          closure and field transfer (Sec. 4, Sec. 6).
net       Reference 3-D convolution network (forward, backward, Adam) used to
          check the learned warm start's kernels.  Parity of the trained
          network's *outputs* is unpinned; see its header.
"""
