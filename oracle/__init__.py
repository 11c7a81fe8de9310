"""CPU oracle for the convex clustering model (CCM) -- TEST INFRASTRUCTURE.

This package is the plain, slow, FP64 reference that the GPU library is
checked against.  Only the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import it; the library itself never does, and this
package imports nothing from the library (it shares no code, kernels,
headers, tables or helpers with it).

What it computes (the paper is arXiv 2501.15964, "PyClustrPath"):

* the model (CCM) of Section 1: for each gamma,
  min_X 1/2 sum_i ||x_i - a_i||_2^2 + gamma sum_{i<j} w_ij ||x_i - x_j||_q,
  over a sparse weight graph, for q in {1, 2, inf};
* the cluster rule of Section 1 (a_i, a_j share a cluster iff x_i* = x_j*),
  with the numeric fusion threshold stated in ``labels``;
* the relative duality gap eta of Section 4 (used as a reported stopping
  quantity) and a relative KKT residual (the stopping test);
* ADMM and SSNAL, the two path solvers of Section 1 / Table 3, written
  from the algorithms' definitions (the paper names them but prints no
  steps);
* the k-NN Gaussian weight graph that the Data Processor of Section 2.2
  builds;
* the implicit-differentiation adjoint of the solution map;
* brute-force solvers for tiny inputs, used only to pin the above.

Parity status per function is given in each module's header.
"""
from .operators import (  # noqa: F401
    incidence,
    dual_exponent,
    row_norms,
    project,
    prox,
    jacobian_apply,
    primal_objective,
    dual_objective,
    kkt_residuals,
    distance_bound,
)
from .solvers import ssnal, admm, ama, hpr, solve_path  # noqa: F401
from .labels import fusion_scale, cluster_labels, fusion_margins  # noqa: F401
from .graph import knn_brute, knn_graph, knn_brute_u8, knn_graph_u8, canonicalize_edges  # noqa: F401
from .adjoint import path_vjp  # noqa: F401
