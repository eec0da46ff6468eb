"""Seeded synthetic workloads: meshes, level sets, coefficients and input vectors.

This module only describes inputs (shapes, geometry, seeds, distributions).
It holds none of the ghost-penalty arithmetic and is shared by the tests,
the benchmark and the smoke check, so that the HIP path and the CPU oracle
see identical inputs.

Geometry follows the paper's test problems (§3: a Cartesian mesh of a box cut
by a ball); the coefficients are gamma_j = gamma_A h^{2j-1} / (j!)^2 with
gamma_A = 0.5 (§2.2, applied once).
"""

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    d: int
    k: int
    n: tuple
    lo: tuple
    centre: tuple
    radius: float
    note: str = ""
    balls: tuple = ()  # union of balls (c0, c1, c2, r) instead of the one ball (centre, radius)

    @property
    def h(self):
        return 2.0 / self.n[0]

    @property
    def lattice(self):
        return tuple(self.k * m + 1 for m in self.n)

    @property
    def n_lattice(self):
        return int(np.prod(self.lattice))

    @property
    def n_p(self):
        """Patch DoFs per face: (2k+1)(k+1)^(d-1)."""
        return (2 * self.k + 1) * (self.k + 1) ** (self.d - 1)

    def gamma(self):
        return gamma_paper(self.k, self.h)

    def gamma_macro(self):
        """gamma_M of the macro-patch stabilisation: the paper's gamma_A = 0.5 (its h-scaling is in the form)."""
        return GAMMA_MACRO


GAMMA_MACRO = 0.5


def gamma_paper(k, h, gamma_a=0.5):
    return [gamma_a * h ** (2 * j - 1) / math.factorial(j) ** 2 for j in range(1, k + 1)]


BALL3 = (0.011, 0.017, 0.023)

WORKLOADS = {
    w.name: w
    for w in [
        Workload("disk2d_q2_32", 2, 2, (32, 32), (-1.0, -1.0), (0.013, 0.021), 0.71,
                 "2D Q2, 32x32 cells on [-1,1]^2, disk r=0.71"),
        Workload("ball3d_q3_64", 3, 3, (64,) * 3, (-1.0,) * 3, BALL3, 0.73,
                 "3D Q3, 64^3 cells on [-1,1]^3, ball r=0.73"),
        Workload("ball3d_q5_128", 3, 5, (128,) * 3, (-1.0,) * 3, BALL3, 0.73,
                 "3D Q5, 128^3 cells on [-1,1]^3, ball r=0.73"),
        Workload("ball3d_q4_96", 3, 4, (96,) * 3, (-1.0,) * 3, BALL3, 0.73,
                 "3D Q4, 96^3 cells on [-1,1]^3, ball r=0.73"),
        Workload("ball3d_q7_96", 3, 7, (96,) * 3, (-1.0,) * 3, BALL3, 0.73,
                 "3D Q7, 96^3 cells on [-1,1]^3, ball r=0.73"),
    ]
}


def sweep_workload(k, n):
    """Same ball on an n^3 mesh of [-1,1]^3 with degree k (roofline sweeps)."""
    return Workload(f"ball3d_q{k}_{n}", 3, k, (n,) * 3, (-1.0,) * 3, BALL3, 0.73)


SEED_BALLS = 6
BALLS_R1 = 2.0


def multiball_workload(k, n, n_balls, seed=SEED_BALLS):
    """The multiple-ball problem (§3): the union of n_balls balls with centres drawn uniformly in
    [-1,1]^3 (seeded; the centres of a smaller count are the first ones of a larger count) and the
    common radius BALLS_R1 / n_balls, inversely proportional to the number of balls (one ball of
    radius 2 covers most of the box), on an n^3 mesh of [-1,1]^3 with degree k."""
    centres = np.random.default_rng(seed).uniform(-1.0, 1.0, size=(n_balls, 3))
    r = BALLS_R1 / n_balls
    balls = tuple((float(c[0]), float(c[1]), float(c[2]), r) for c in centres)
    return Workload(f"balls3d_q{k}_{n}_b{n_balls}", 3, k, (n,) * 3, (-1.0,) * 3, tuple(centres[0]), r,
                    f"3D Q{k}, {n}^3 cells on [-1,1]^3, union of {n_balls} balls of radius {r:g}", balls)


def submesh_q4_16():
    """16^3-cell block of the 96^3 Q4 mesh straddling the sphere: cells [76,92) x [40,56) x [40,56)."""
    h = 2.0 / 96
    lo = tuple(-1.0 + c * h for c in (76, 40, 40))
    return Workload("ball3d_q4_96_block16", 3, 4, (16, 16, 16), lo, BALL3, 0.73,
                    "16^3 block of the 96^3 Q4 mesh, cells [76,92)x[40,56)x[40,56)")


# seeds: u = 1, t = 2, b = 3, face subset = 4, finite-difference directions = 5
SEED_U, SEED_T, SEED_B, SEED_SUBSET, SEED_FD = 1, 2, 3, 4, 5


def uniform_vector(n, seed, dtype=np.float64):
    """n values ~ U[-1, 1] from numpy's default_rng(seed), drawn in index order in float64."""
    v = np.random.default_rng(seed).uniform(-1.0, 1.0, n)
    return v if dtype == np.float64 else v.astype(dtype)


def face_subset(n_faces, fraction=0.01, seed=SEED_SUBSET):
    """Sorted seeded sample of face indices (at least one face)."""
    m = max(1, int(round(fraction * n_faces)))
    return np.sort(np.random.default_rng(seed).choice(n_faces, size=m, replace=False))
