"""MI355X-native H-matrix mobility product U = M(X) F (arXiv 2505.08174, Sec. 3).

The work runs in the HIP library libhh.so (C ABI in include/hh.h); this package
only marshals arguments. Importing it does not load the library; the first
call does, and raises if the library has not been built.
"""
from ._lib import HHError, load  # noqa: F401
from .stepping import Suspension  # noqa: F401
from .api import (  # noqa: F401
    Context, Kernel, Tree, Partition, LowRank, HMatrix, Batch, ShortRange, build_tree,
    build_tree6, build_tree_batch, partition,
    aca_build, aca_build_pivots, tree_refit, matvec, matvec_noalloc,
    hmatvec, pack_mlp, PRECISION, matvec_backward, HMatvecFn, hmatvec_autograd,
)
