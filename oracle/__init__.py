"""CPU float64 oracle for the sBMDS embedding path.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline leg
of the benchmark import this package; the library (``paper_1705_10887_amd``)
never does, and the two share no code.  Inputs for both sides come from the
seeded generator package ``synth``.

Modules:
  eig       top-k eigenpairs of B = -1/2 J P W P^T J by three routes
            (dense, l x l reduction, ARPACK on the implicit operator)
  mds       textbook classical MDS, strain, approximation error
  refchain  brute-force dense reference of the input chain for tiny meshes
            (cotangent operator, biharmonic P, thresholding, geodesics, FPS)
  mlp       landmark features, the warm-start network, its alignment loss,
            gradients and the Adam update
"""
from . import eig, mds, mlp, refchain  # noqa: F401
from .eig import top_k, embed, b_matrix  # noqa: F401
