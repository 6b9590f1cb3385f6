"""Plain, slow FP64 CPU oracle for the H-matrix mobility product U = M(X) F.

TEST INFRASTRUCTURE ONLY. Nothing on the product path may import, call, link
or execute this package: only the tests, the smoke check of the graft entry
point and the CPU-baseline leg of the benchmark use it. It shares no code with
the HIP library (no kernels, headers, helpers, constants or pre/post
processing); the only common module is `workloads`, which draws the seeded
inputs and holds none of the method's arithmetic.

Contents, each following the paper (arXiv 2505.08174) directly:
  kernels    -- the 3x3 two-body kernels (closed-form RPY tensor; a seeded tanh
                MLP standing in for the learned h/|r| of Eq. (4)) and the
                self mobility alpha_1 of Eq. (2)
  dense      -- the exact dense sum U_i = alpha_1 F_i + sum_{j!=i} K(x_i-x_j) F_j
                (Eq. (2) restricted to alpha_1 and the two-body term, i.e. the
                first two matvecs of Eq. (6)), on all rows or on sampled rows
  tree       -- the cluster tree of Definition 1 by literal recursive bisection
                of a bounding cube along x, then y, then z (Sec. 3.1, Fig. 2)
  partition  -- BuildPartition, Algorithm 1, with the admissibility test Eq. (7)
                on bounding boxes (Fig. 3b)
  aca        -- block ACA with 3x3 entries, Algorithm 2 with Eqs. (8)-(10)
  hmatvec    -- the H-matrix product assembled from the above, and the error
                measure Eq. (11)
  grad       -- dense FP64 gradients of L = sum_i w_i . U_i with respect to F,
                X and the MLP parameters, and the adjoint of the H-matrix
                product with frozen structure
  short      -- the short-range many-body terms M^(s,2) F + M^(t,3) F +
                M^(s,3) F of Eq. (6) over neighbours and 3-cliques within R_cut
  stepping   -- gravity, filament tension and bending forces and the explicit
                Euler step of Sec. 4.3
  rotation   -- the 6N mobility of Eq. (1) with torques and rotational
                velocities (Rotne-Prager rotational blocks), dense and as the
                H-matrix over its grid of 3x3 entries
"""
from . import kernels, dense, tree, partition, aca, hmatvec, grad, short, stepping  # noqa: F401
from . import rotation  # noqa: F401
