"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

This module holds no arithmetic of the method (no Hamiltonian, no MPO, no environment
contraction, no matvec).  It only draws random numbers and sizes:

* the charge sectors (N, k) and their dimensions on every bond of a finite cylinder
  MPS (a Gaussian in N around the mean filling, uniform in k, apportioned by largest
  remainder and clipped so that each site tensor can be an isometry);
* random isometric site tensors (complex Gaussian entries, QR per charge block with a
  positive diagonal of R);
* random two-site wavefunctions.

Blocks are plain numpy arrays in dicts keyed by charges: a charge is a tuple (N, k)
with 0 <= k < ly.  A site tensor A[a, s, b] is {(qa, s, qb): array (m_a, m_b)}.
"""
from .synthetic import (Workload, bond_sectors, left_isometry, right_isometry,
                        random_theta, site_charges, make_workload, preset,
                        centre_workload, PRESETS, random_env, random_site,
                        GrowthStart, growth_start)

__all__ = ["GrowthStart", "growth_start", "Workload", "bond_sectors", "left_isometry", "right_isometry", "random_theta",
           "site_charges", "make_workload", "preset",
           "centre_workload", "PRESETS", "random_env", "random_site"]
