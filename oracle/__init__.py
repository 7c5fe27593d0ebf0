"""FP64 CPU oracle of the accelerated spectral clustering hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls, links or
executes anything under ``oracle/``; only the tests, the smoke check and the
CPU-baseline leg of the bench do.  The oracle shares no code with the HIP
library (no kernels, headers, helpers or constant tables); both sides only
share the seeded input generators of ``workloads``.

Everything is float64, written plainly from the definitions of Tremblay, Puy,
Borgnat, Gribonval & Vandergheynst, "Accelerated spectral clustering using
graph filtering of random signals" (ICASSP 2016):

  graph.py     the combinatorial Laplacian L = S - W            (Sec. 2.1)
  spectrum.py  dense spectrum, Lanczos estimate of lambda_N      (Sec. 2.1; Sec. 4.1 step 1)
  cheb.py      ideal low-pass h_lc, its Chebyshev approximation,
               the polynomial filter of random signals           (Eq. ideal, Sec. 2.3-2.4, 3.1, 4.1 steps 3-5)
  eigcount.py  eigenvalue count below a cut-off, dichotomy       (Sec. 3.2; Sec. 4.1 step 2)
  cluster.py   row normalisation, k-means                         (Sec. 2.2 step 4, Sec. 4.1 step 6, footnote of Sec. 2.1)
  grad.py      Gaussian-kernel weights, loss, adjoint gradients  (extension beyond the paper)
  stability.py adjusted Rand index, stability measure gamma(k)    (Sec. 4.3, Eq. stab)
  order.py     least polynomial order for a tolerance, m*(rho; delta) (Sec. 2.4, note on m)
  knn.py       K-nearest-neighbour graph, union-symmetrised             (Sec. 5)
  cpu_baseline.c  the same FP64 recurrence over CSR in plain C/OpenMP, for timing

Parity status of each function is stated in its docstring ("pinned by ..."
or "parity unpinned").
"""
from .graph import strength, laplacian_sparse, laplacian_dense, laplacian_normalized, check_graph  # noqa: F401
from .spectrum import (dense_spectrum, lambda_max_exact, lanczos_tridiag,  # noqa: F401
                       lanczos_lmax, lmax_estimate)
from .cheb import (jackson, step_coeffs, cheb_coeffs, cheb_eval, cheb_filter,  # noqa: F401
                   cheb_states, dense_filter, ideal_filter, scaled_laplacian)
from .eigcount import (moments, eigcount_from_moments, eigcount_literal,  # noqa: F401
                       exact_count, dichotomy, dichotomy_moments, dichotomy_literal)
from .cluster import normalize_rows, kmeans_assign, kmeans_update, kmeans_lloyd  # noqa: F401
from .kmeanspp import kmeans_pp_rows  # noqa: F401
from .grad import (gauss_weights, rownorm_loss_grad, cheb_filter_adjoint,  # noqa: F401
                   daleckii_krein_M, dW_from_M, dsigma, loss_of_weights, cheb_filter_adjoint_sampled)
from .stability import (contingency, ari_terms, ari, ari_pairs, gamma, inertia,  # noqa: F401
                        kmeans_replicates, realisation_signals, features, cluster_once, stability)
from .order import grid_points, band_error, order_errors, m_star  # noqa: F401
from .knn import sqdist_to, knn_bruteforce, union_graph  # noqa: F401
from .knn import knn as knn_exact  # noqa: F401
