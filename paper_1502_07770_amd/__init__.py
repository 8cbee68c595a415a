"""MI355X-native exact TV-chain prox and 2D TV (ROF) solver.

Implements the data-parallel hot path of Kolmogorov, Pock, Rolinek, "Total
variation on a tree" (arXiv 1502.07770): the O(n) chain dynamic program of
Sec. 4.1, batched over the row and column chains of the Sec. 5.1 Lagrangian
decomposition of 2D ROF, as hand-written HIP kernels for gfx950 behind the C
ABI in ``include/tvchain.h``.  ``binding`` marshals torch tensors into that
ABI; ``synth`` draws the seeded synthetic workloads.
"""
from .binding import (Tv2dSolver, TvChainError, chain_dp, chain_prox, chain_prox_backward,  # noqa: F401
                      chain_prox_l1,
                      chain_nc, chain_nc_concave, chain_prox_multi, load, prox, tree_dp, tree_nc,
                      tree_nc_concave, tv2d, tv2d_batched,
                      tv2d_l1, tv2d_nc)

__all__ = ["Tv2dSolver", "TvChainError", "chain_dp", "chain_prox", "chain_prox_l1", "chain_prox_backward",
           "chain_nc", "chain_nc_concave", "chain_prox_multi", "load", "prox", "tree_dp", "tree_nc",
           "tree_nc_concave", "tv2d", "tv2d_batched", "tv2d_l1", "tv2d_nc"]
