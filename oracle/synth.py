"""Environments of a seeded synthetic MPS, contracted with the exact Hofstadter MPO.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The site tensors come from ``workloads`` (seeded left isometries left of the two-site
window, right isometries right of it).  The left environment at the window is the
left boundary (state R) updated site by site with ``env_left_update``; the right
environment is the right boundary (state F, total charge) updated with
``env_right_update`` from the right end.  Because the site tensors are isometries and
the MPO is the exact Hamiltonian of eqs. H_kin + H_int (or eq. H_real), H_eff is the
Hamiltonian projected on the span of the two-site window, so it is Hermitian.
"""
from __future__ import annotations

from fractions import Fraction

from . import blocksparse as bs
from . import mpo as mpo_mod
from .model import Cylinder


def cylinder_of(wl) -> Cylinder:
    return Cylinder(wl.Ly, wl.Lx, Fraction(wl.flux[0], wl.flux[1]), wl.t, wl.V)


def window_problem(wl, mpo=None):
    """(L, W1, W2, R, theta0, theta_keys, mpo) for the window (j, j+1) of a workload."""
    if mpo is None:
        mpo = mpo_mod.build(cylinder_of(wl), wl.basis, real=getattr(wl, "real", False))
    j = wl.j
    L = bs.left_boundary()
    for i in range(j):
        L = bs.env_left_update(L, wl.site_tensor(i), mpo.W[i])
    R = bs.right_boundary((wl.N_tot, wl.K_tot))
    for i in range(wl.n - 1, j + 1, -1):
        R = bs.env_right_update(R, wl.site_tensor(i), mpo.W[i])
    keys = bs.theta_keys(wl.bonds[j], wl.bonds[j + 2], wl.qsite[j], wl.qsite[j + 1], wl.ly)
    return L, mpo.W[j], mpo.W[j + 1], R, wl.theta(), keys, mpo
