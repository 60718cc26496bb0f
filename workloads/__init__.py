"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle.

This module holds only workload definitions and random inputs (right-hand
sides, densities, targets, sampled element sets).  It contains none of the
method's arithmetic and imports neither the oracle nor the HIP library.

Workloads mirror the paper's mass-solve experiments (Section 3): simplicial
meshes of the unit square / cube, a random right-hand side, u_0 = 0, and a
relative-residual stopping rule.  Meshes themselves are built on each side
from their definition (Kuhn split plus a counter-based SplitMix64 jitter of
interior vertices by at most `jitter` * h per coordinate) with `mesh_seed`.
"""
from dataclasses import dataclass

import numpy as np

SEED_BASE = 0x260712138


@dataclass(frozen=True)
class Workload:
    name: str
    family: str          # "P" (H1 Lagrange), "B" (H1 Bernstein), "N1curl", "RT"
    dim: int
    degree: int
    N: int               # squares / cubes per side
    jitter: float        # fraction of h
    nrhs: int
    prec: str            # BRAS apply precision: "f64", "f32", "bf16"
    tol: float
    index: int
    density: bool = False

    def seed(self, role):
        """role: 0 mesh, 1 rhs, 2 rho, 3 x*, 4 sampled elements / rows."""
        return SEED_BASE + 16 * self.index + role

    @property
    def mesh_seed(self):
        return self.seed(0)

    @property
    def n_cells(self):
        return (2 if self.dim == 2 else 6) * self.N ** self.dim


WORKLOADS = [
    Workload("h1p1_2d_32", "P", 2, 1, 32, 0.0, 1, "f64", 1e-10, 1),
    Workload("h1p3_3d_24_jit", "P", 3, 3, 24, 0.2, 1, "f64", 1e-10, 2),
    Workload("n1curl2_3d_48_jit", "N1curl", 3, 2, 48, 0.2, 1, "f32", 1e-8, 3),
    Workload("rt4_3d_32_jit_r32", "RT", 3, 4, 32, 0.2, 32, "bf16", 1e-8, 4),
    Workload("h1p4_3d_32_rho", "P", 3, 4, 32, 0.0, 1, "f64", 1e-10, 5, density=True),
    # the paper's largest H1 gap: Bernstein p = 4 in 3D at about 1e6 DOFs (Table h1_mass_solve)
    Workload("h1b4_3d_25", "B", 3, 4, 25, 0.0, 1, "f64", 1e-10, 6),
]

BY_NAME = {w.name: w for w in WORKLOADS}


def scaled(w, N):
    """The same workload on an N^dim mesh (small parity cases)."""
    return Workload(w.name + "@N%d" % N, w.family, w.dim, w.degree, N, w.jitter,
                    w.nrhs, w.prec, w.tol, w.index, w.density)


def rhs(n, nrhs, seed):
    """b ~ U[-1, 1] i.i.d.; shape [n] for one column, else [n, nrhs] (column fastest)."""
    g = np.random.default_rng(seed)
    b = g.uniform(-1.0, 1.0, size=(n, nrhs))
    return b[:, 0].copy() if nrhs == 1 else b


def density(E, seed):
    """rho_e ~ lognormal(0, 1)."""
    return np.random.default_rng(seed).lognormal(0.0, 1.0, size=E)


def target(n, seed):
    """x* ~ N(0, 1)."""
    return np.random.default_rng(seed).standard_normal(n)


def sample(count, k, seed):
    """k distinct indices in [0, count), sorted."""
    return np.sort(np.random.default_rng(seed).choice(count, size=min(k, count), replace=False))


def vector(n, seed, lo=-1.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, size=n)


def rotated_stretch(coords, r):
    """Coordinates under the affine map x -> c + R S R^T (x - c), c = (1/2, 1/2),
    R the rotation by pi/4, S = diag(r, 1/r) (the rotated-stretch meshes of
    eq. rot_stretch_map; 2D, det = 1)."""
    coords = np.asarray(coords, dtype=np.float64)
    c = np.array([0.5, 0.5])
    q = np.sqrt(0.5)
    R = np.array([[q, -q], [q, q]])
    A = R @ np.diag([r, 1.0 / r]) @ R.T
    return c + (coords - c) @ A.T
