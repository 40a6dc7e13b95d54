"""MI355X aggregation algebraic multigrid (Gandham, Esler & Zhang, arXiv 1403.1649).

Thin Python binding over the C ABI of ``libamg_hip.so`` (declared in
``include/amg.h``).  Every step of setup and solve runs in the library's HIP
kernels; this module only marshals arguments.  PyTorch provides device memory
(tensors) and the stream (its current stream).  Importing the package does not
load the library; the first call does, and raises if the library is missing.
"""
from .binding import (  # noqa: F401
    AmgError,
    Hierarchy,
    Options,
    default_options,
    galerkin,
    galerkin_noalloc,
    hessenberg_radius,
    lib,
    mlp_adam,
    mlp_coarse_corrected,
    mlp_features,
    mlp_loss_grad,
    mlp_num_params,
    mlp_omega,
    library_path,
    node_hash,
    release_cached_memory,
    setup,
    setup_batched,
    solve,
    solve_multi,
    spmv,
    status_string,
)
