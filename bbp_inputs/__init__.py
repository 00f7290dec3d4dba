"""Seeded synthetic inputs shared by the GPU library tests, the benchmark and the oracle.

This module holds no block-BP arithmetic: it only draws PEPS site tensors,
defines the one-site and two-site operator matrices, and names the lattice
configurations the tests and the benchmark use.

Tensor layout (one site): ``A[s, u, l, d, r]`` in C order, physical index ``s``
(dimension ``d``), virtual legs up/left/down/right, every virtual leg stored with
dimension ``D``.  Legs on an open lattice edge have true dimension 1 and are
zero-padded to ``D``.  Sites are stored row-major (``y`` outer, ``x`` inner).

The synthetic tensors are near-product states, ``A = e_0 + 0.1 * N(0, 1)``,
standing in for the imaginary-time-evolved ground states the paper measures on
(its Sections III-V); those tensors are not available.
"""

from .gen import (  # noqa: F401
    peps_finite,
    peps_infinite,
    ising_peps,
    ising_single_layer,
    peps_tiled,
    peps_rotate,
    peps_transpose,
    pauli,
    op_sz,
    op_sx,
    op_sy_real,
    op_szsz,
    op_heis,
    dense_matrices,
    CONFIGS,
)
