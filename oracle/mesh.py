"""Structured simplicial meshes of the unit square / cube (oracle side).

The paper's experiments use simplicial meshes of the unit square and unit
cube (Section 3, setup paragraph before Table h1_mass_solve).  The diagonal
direction is not stated; the reading used here is the Kuhn (Freudenthal)
split: every square is cut into 2 triangles and every cube into the 6
tetrahedra that contain its main diagonal, one per monotone lattice path.

Vertex numbering: vertex (i, j[, k]) has id i + (N+1)*(j + (N+1)*k) and
coordinates (i*h, j*h[, k*h]) with h = 1.0/N.

Cells (vertex ids are ascending inside every cell by construction):
  2D  square c = i + N*j gives triangles 2c   = [v(i,j), v(i+1,j), v(i+1,j+1)]
                                   and 2c+1 = [v(i,j), v(i,j+1), v(i+1,j+1)].
  3D  cube c = i + N*(j + N*k) gives tetrahedra 6c+s, s = 0..5: start at the
      cube's corner (i,j,k) and step by one along the axes in the order of the
      s-th permutation of (0,1,2) in lexicographic order.

Jitter (optional): every interior vertex moves each coordinate by
(frac*h)*(2u-1), u in [0,1) drawn from a counter-based SplitMix64 stream:
  z = mix64(seed + (dim*vid + axis + 1) * GAMMA),  u = (z >> 11) * 2^-53,
where GAMMA = 0x9E3779B97F4A7C15 and mix64 is the SplitMix64 output function
of Steele, Lea and Flood (OOPSLA 2014) in the constants of Vigna's reference
implementation.  Each arithmetic operation is written out so that an
independent implementation reproduces the coordinates bit for bit:
  jit = (frac*h) * (2.0*u - 1.0);  x = i*h + jit.
"""
import itertools

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_mix(z):
    """SplitMix64 output function applied to uint64 array z (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def splitmix64_counter(seed, counter):
    """Counter-based SplitMix64: the counter-th output of a stream seeded with seed.

    A sequential SplitMix64 generator seeded with s returns mix64(s + t*GAMMA)
    as its t-th output (t = 1, 2, ...); this evaluates that directly.
    """
    counter = np.asarray(counter, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = np.uint64(seed) + counter * GAMMA
    return splitmix64_mix(state)


def uniform01(seed, counter):
    """u = (z >> 11) * 2^-53 in [0, 1)."""
    z = splitmix64_counter(seed, counter)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def _kuhn_perms(dim):
    return list(itertools.permutations(range(dim)))


def structured_mesh(dim, N, jitter=0.0, seed=0):
    """Return (coords [V, dim] float64, cells [E, dim+1] int32).

    jitter is the fraction of h by which interior vertices may move per
    coordinate (0.2 for the jittered workloads), seed the SplitMix64 seed.
    """
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    if N < 1:
        raise ValueError("N must be >= 1")
    n1 = N + 1
    h = 1.0 / N
    idx = np.arange(n1 ** dim, dtype=np.int64)
    lattice = np.stack([(idx // n1 ** a) % n1 for a in range(dim)], axis=1)
    coords = lattice.astype(np.float64) * h
    if jitter:
        interior = np.all((lattice > 0) & (lattice < N), axis=1)
        vid = idx[interior]
        amp = jitter * h
        for a in range(dim):
            u = uniform01(seed, dim * vid + a + 1)
            jit = amp * (2.0 * u - 1.0)
            coords[interior, a] = lattice[interior, a].astype(np.float64) * h + jit

    stride = np.array([n1 ** a for a in range(dim)], dtype=np.int64)
    cidx = np.arange(N ** dim, dtype=np.int64)
    corner = np.stack([(cidx // N ** a) % N for a in range(dim)], axis=1)
    base = corner @ stride
    if dim == 2:
        v00 = base
        v10 = base + stride[0]
        v01 = base + stride[1]
        v11 = base + stride[0] + stride[1]
        cells = np.empty((2 * N * N, 3), dtype=np.int64)
        cells[0::2] = np.stack([v00, v10, v11], axis=1)
        cells[1::2] = np.stack([v00, v01, v11], axis=1)
    else:
        perms = _kuhn_perms(3)
        cells = np.empty((6 * N ** 3, 4), dtype=np.int64)
        for s, perm in enumerate(perms):
            cur = base.copy()
            verts = [cur.copy()]
            for ax in perm:
                cur = cur + stride[ax]
                verts.append(cur.copy())
            cells[s::6] = np.stack(verts, axis=1)
    return coords, cells.astype(np.int32)


def mesh_counts(dim, N):
    """Closed-form entity counts of the Kuhn mesh: (V, edges, faces, cells).

    In 2D faces == cells (triangles).
    """
    if dim == 2:
        V = (N + 1) ** 2
        Ed = 2 * N * (N + 1) + N * N
        T = 2 * N * N
        return V, Ed, T, T
    V = (N + 1) ** 3
    Ed = 3 * N * (N + 1) ** 2 + 3 * N * N * (N + 1) + N ** 3
    F = 12 * N ** 3 + 6 * N ** 2
    T = 6 * N ** 3
    return V, Ed, F, T


def jacobians(coords, cells):
    """J[K] with columns v_i - v_0 (reference simplex conv{0, e_1, ..., e_d})."""
    X = coords[cells]                      # [E, d+1, d]
    return np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))
