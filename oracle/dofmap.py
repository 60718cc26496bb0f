"""Entity numbering, the broken-to-conforming map pi and multiplicities d_i.

Section 2.2: every broken degree of freedom j has a unique conforming owner
pi(j); P copies u_{pi(j)} into slot j and D = P^T P = diag(d_i) with
d_i = #{j : pi(j) = i}.

Canonical numbering (cells must list their vertices in ascending order):
  * edges are the sorted vertex pairs of all cells, numbered in
    lexicographic order; faces (3D) the sorted triples, likewise; cells keep
    their index;
  * conforming DOFs come in blocks [vertex | edge | face | cell] (2D:
    [vertex | edge | cell]); inside a block entity e owns DOFs
    offset + e*k + (0..k-1) in the element's entity-local order;
  * pi[K, l] follows the element's local order (vertices, local edges in lex
    order of local vertex pairs, local faces likewise, interior).
Because local vertex order equals global order, an entity's DOFs are read in
the same order from every cell that shares it.
"""
import itertools

import numpy as np


def entities(cells, edim):
    """Sorted unique global entities of dimension edim and, per cell, the index
    of each local entity (local entities in lex order of local vertices)."""
    E, nv = cells.shape
    combos = list(itertools.combinations(range(nv), edim + 1))
    keys = np.stack([cells[:, list(c)] for c in combos], axis=1).reshape(-1, edim + 1)
    uniq, inv = np.unique(keys, axis=0, return_inverse=True)
    return uniq, inv.reshape(E, len(combos))


def build_dofmap(cells, nvert, dofs_per_entity):
    """Return (pi [E, n_loc] int64, n, per-block offsets).

    dofs_per_entity = (k_vertex, k_edge, ..., k_cell) for entity dims 0..d.
    """
    cells = np.asarray(cells, dtype=np.int64)
    E, nv = cells.shape
    d = nv - 1
    counts = list(dofs_per_entity)
    if len(counts) != d + 1:
        raise ValueError("need one count per entity dimension")
    ent_index = []
    ent_count = []
    for edim in range(d + 1):
        if edim == 0:
            ent_index.append(cells)
            ent_count.append(nvert)
        elif edim == d:
            ent_index.append(np.arange(E, dtype=np.int64)[:, None])
            ent_count.append(E)
        else:
            uniq, idx = entities(cells, edim)
            ent_index.append(idx)
            ent_count.append(len(uniq))
    offsets = [0]
    for edim in range(d + 1):
        offsets.append(offsets[-1] + ent_count[edim] * counts[edim])
    n = offsets[-1]
    cols = []
    for edim in range(d + 1):
        k = counts[edim]
        if k == 0:
            continue
        idx = ent_index[edim]
        for le in range(idx.shape[1]):
            for j in range(k):
                cols.append(offsets[edim] + idx[:, le] * k + j)
    pi = np.stack(cols, axis=1)
    return pi, n, offsets


def multiplicity(pi, n):
    """d_i = #{j : pi(j) = i} (Section 2.2)."""
    return np.bincount(np.asarray(pi).ravel(), minlength=n)
