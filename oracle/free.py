"""Free-fermion closed form.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

At V = 0, eq. H_kin is quadratic and block diagonal in the ring momentum k: for each
k it is the Lx x Lx tridiagonal matrix h_k with diagonal -2 t cos(k + x phi) and
off-diagonal -t (open ends in x).  The N-particle ground energy is the sum of the
lowest N single-particle levels of the direct sum of all h_k (the magnetic bands of
Sec. III A, Fig. 2, on a finite cylinder).
"""
from __future__ import annotations

import numpy as np

from .model import Cylinder


def levels(cyl: Cylinder) -> tuple[np.ndarray, np.ndarray]:
    """All single-particle levels (sorted) and their momentum labels m."""
    ev, ms = [], []
    for m in range(cyl.Ly):
        k = 2.0 * np.pi * m / cyl.Ly
        h = np.diag(-2.0 * cyl.t * np.cos(k + np.arange(cyl.Lx) * cyl.phi))
        h -= cyl.t * (np.eye(cyl.Lx, k=1) + np.eye(cyl.Lx, k=-1))
        e = np.linalg.eigvalsh(h)
        ev.append(e)
        ms.append(np.full(cyl.Lx, m))
    ev, ms = np.concatenate(ev), np.concatenate(ms)
    order = np.argsort(ev, kind="stable")
    return ev[order], ms[order]


def ground_energy(cyl: Cylinder, N: int) -> float:
    """E0(V=0, N) = sum of the lowest N levels."""
    return float(np.sum(levels(cyl)[0][:N]))


def fock_ground_energy(cyl: Cylinder) -> float:
    """Ground energy over all particle numbers: the sum of all negative levels."""
    e = levels(cyl)[0]
    return float(np.sum(e[e < 0]))
