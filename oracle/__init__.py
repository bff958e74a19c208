"""Oracle for dynamic random walk with restart -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct CPU implementations of what the HIP path
computes.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import this package; the product package never does,
and the two share no code (only the seeded generators in ``synth`` feed both).

Contents
  * ``rwr_static``   static RWR of Eq. (1): CPI of Section 2.2 from c*e_s to
                      1e-14 in FP64, then Theorem 4's dead-end normalisation
                      (C, single-threaded; ``rwr_oracle.c``)
  * ``cpi``          cumulative power iteration for any seed vector
  * ``rwr_static_vector`` static scores for a general restart vector q
                      (global PageRank for q = 1/n), Theorem 4 as above
  * ``osp``          one OSP / OSP-T update, Section 3.1 / Algorithm 1
  * ``rwr_dense``    the same static RWR by a dense LU solve of
                      (I - (1-c) A~^T) r = c e_s (numpy / LAPACK), n <= ~2000
  * ``apply_batch``  the graph G + Delta G of a batch, by plain set
                      operations on edge keys (Section 3.4.1 for new nodes)
  * ``apply_stream`` the same for a sequence of batches, in one pass
  * ``delta_weight`` ||D r_old||_1 of the effects of Delta G (Section 3.3),
                      the bound of ||q_offset||_1 / (1-c) before propagation
"""

from .core import (  # noqa: F401
    OracleError,
    apply_batch,
    apply_stream,
    cpi,
    dead_end_reachable,
    delta_weight,
    lib,
    osp,
    rwr_dense,
    rwr_static,
    rwr_static_vector,
    reachable_from,
    row_normalised_dense,
)
