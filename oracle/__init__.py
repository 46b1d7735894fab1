"""Plain, sequential FP64 CPU oracle of the sparse hierarchical solver (LoRaSp and GC).

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this package. The GPU
library never calls it, and it shares no code with the GPU library: it reads plain CSR
arrays and coordinates and computes everything itself with NumPy/SciPy in float64.

What it follows (sections, equations and algorithms of arXiv:1611.03189):

* §2-§3.1: graph of A, block partition, red nodes from recursive bisection, pairwise
  merge into super nodes, adjacency by the original graph ("well separated" = not a
  neighbour).
* §3.2 Factorization: compression (eq. local_compression / compression_sw),
  extension (eq. extended), elimination (eq. extended_rearranged, the K = L K2 L^T
  factorisation), level recursion and exact root (Algorithm "Setup").
* §6 GC: compression that keeps phi_x and A_sw phi_y in span U (eq. compression_xy,
  eq. preserve, Lemma lm:compression), the parent-level vector U^T phi_x
  (Lemma lm:extension and the summary that follows it).
* §3.3 / Appendix A: solve phase (Algorithm "Solve"), with P_ss and M_ss as defined
  there.
* §7: stationary iteration and GMRES as outer loops; PCG added for SPD A.

Readings where the paper is silent or ambiguous are listed in ``hsolver.py`` next to
the code that takes them.
"""
from .tree import tree_depth, cluster_leaves, footprint_adjacency, GeometricNeighbours
from .hsolver import (Factorization, NotSPDError, compress, pivot, eliminate_node,
                      factor, apply, apply_matrix, level_eps, truncated_left_basis,
                      LORASP, GC, GC_PROJ1)
from .krylov import pcg, fpcg, gmres, stationary

__all__ = [
    "tree_depth", "cluster_leaves", "footprint_adjacency", "GeometricNeighbours",
    "Factorization", "NotSPDError", "compress", "pivot", "eliminate_node", "factor",
    "apply", "apply_matrix", "level_eps", "truncated_left_basis", "LORASP", "GC", "GC_PROJ1",
    "pcg", "gmres", "stationary",
]
