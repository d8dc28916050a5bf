"""FP64 CPU oracle for the Vecchia / VIF likelihood path.

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, obviously correct
NumPy/SciPy implementation of what the GPU library computes. Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import
it; the library's product path never does, and this package never imports the
library.

Sections of the paper followed (arXiv 2602.03609):
  * kernels      -- Eq. (Gneiting) with the closed-form Matern smoothness values
                    nu in {1/2, 3/2, 5/2} named in Sec. "GPU acceleration";
  * neighbors    -- the correlation metric d_c and index-ordered neighbor sets
                    of Sec. "Correlation-based Vecchia neighbor selection"
                    (Alg. 2 is an exact kNN among earlier points; the oracle
                    takes the plain definition, brute force);
  * likelihood   -- the negative log-marginal likelihood of Sec.
                    "Estimation and prediction", the Vecchia factor of Sec.
                    "Vecchia approximation" and the VIF residual factor of Sec.
                    "The Vecchia-inducing-point full-scale approximation";
  * dense        -- exact, FITC and dense-VIF likelihoods used only as pins.

Parity status: the kernels, neighbor sets and both likelihoods are pinned by
the tests under tests/ (closed forms, printed effective ranges, reductions
that hold exactly). No absolute likelihood value is printed in the paper, so
no likelihood number is pinned to the paper directly.
"""
from . import kernels, neighbors, likelihood, dense  # noqa: F401
