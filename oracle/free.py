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


def bulk_energy_per_orbital(Ly: int, flux_p: int, flux_q: int, t: float = 1.0,
                            bands: int = 1, nk: int = 4096) -> float:
    """Ground energy per orbital of the infinite cylinder at V = 0 with the lowest
    ``bands`` magnetic bands of every ring momentum filled (density bands / flux_q).

    For ring momentum k = 2 pi m / Ly, eq. H_kin is a chain in x with on-site energy
    -2 t cos(k + x phi), phi = 2 pi p / q, which repeats every q rings; its Bloch matrix
    at quasi-momentum kappa is q x q with that diagonal, -t between neighbouring rings
    and -t e^{+-i q kappa} across the magnetic cell.  The filled bands contribute their
    average over the magnetic Brillouin zone; the average of a smooth periodic function
    over a uniform grid of ``nk`` points converges exponentially."""
    q = flux_q
    phi = 2.0 * np.pi * flux_p / flux_q
    kap = (np.arange(nk) + 0.5) * (2.0 * np.pi / q) / nk
    total = 0.0
    for m in range(Ly):
        k = 2.0 * np.pi * m / Ly
        diag = -2.0 * t * np.cos(k + np.arange(q) * phi)
        acc = 0.0
        for kp in kap:
            h = np.diag(diag).astype(np.complex128)
            if q == 1:
                h[0, 0] += -2.0 * t * np.cos(kp)
            else:
                for x in range(q - 1):
                    h[x, x + 1] += -t
                    h[x + 1, x] += -t
                h[q - 1, 0] += -t * np.exp(1j * q * kp)
                h[0, q - 1] += -t * np.exp(-1j * q * kp)
            acc += float(np.sum(np.linalg.eigvalsh(h)[:bands]))
        total += acc / nk
    return total / (q * Ly)
