"""Hofstadter cylinder term lists in both bases.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Follows Sec. III A (eq. H: Hofstadter model with nearest-neighbour repulsion, Landau
gauge A = (0, Bx) so only ring hoppings carry a phase) and Sec. IV C/D:

* real-space basis, eq. H_real: orbitals are lattice sites (x, y), the chain orders
  them with increasing x and then increasing y inside a ring;
* mixed basis, eqs. H_kin and H_int: each ring is Fourier transformed around the
  cylinder, orbitals are (x, k) with k = 2 pi m / Ly, and the chain orders them with
  increasing x and then sequentially in m (Sec. II, Fig. 1b).

Readings of the paper that this module fixes (the paper is silent or only treats the
infinite cylinder):

* geometry: finite cylinder, open ends in x (x = 0 .. Lx-1), periodic in y; Ly >= 3
  because at Ly = 2 eq. H_real counts the ring bond twice;
* flux phi = 2 pi p / q per plaquette, ring phase e^{i x phi} with x counted from 0;
* Fourier convention c_{x,y} = Ly^{-1/2} sum_m e^{i 2 pi m y / Ly} c_{x,m}, which gives
  the 2 cos(k + x phi) on-site term of eq. H_kin;
* the q = 0 terms of eq. H_int are kept (they are needed for the two bases to agree).

Every term is stored as a coefficient times an ordered product of single-orbital
operators.  Besides the plain coefficient each term carries the factorisation that
the finite-state-machine MPO construction of Sec. IV uses: a family key, a family
coefficient, one amplitude factor per operator ("role") and the conserved charge each
role transfers.  For the mixed basis the charge of an orbital (x, m) is (N=1, k=m);
for the real-space basis only N is conserved and the momentum modulus is 1.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from fractions import Fraction
from itertools import product

import numpy as np


@dataclass(frozen=True)
class Cylinder:
    """Model parameters of eq. H on an Ly x Lx cylinder with flux 2 pi * flux per plaquette."""

    Ly: int
    Lx: int
    flux: Fraction = Fraction(1, 4)
    t: float = 1.0
    V: float = 1.0

    def __post_init__(self):
        if self.Ly < 3:
            raise ValueError("Ly >= 3 required (eq. H_real double counts the ring bond at Ly = 2)")
        if self.Lx < 1:
            raise ValueError("Lx >= 1 required")

    @property
    def phi(self) -> float:
        return 2.0 * np.pi * float(self.flux)

    @property
    def n_orb(self) -> int:
        return self.Lx * self.Ly

    def orb(self, x: int, m: int) -> int:
        """Chain index of orbital (x, m): x-major, then m (Fig. 1)."""
        return x * self.Ly + m


# Operator kinds: '+' creation, '-' annihilation, 'n' number operator.
FERMIONIC = {"+": True, "-": True, "n": False}
DELTA_N = {"+": 1, "-": -1, "n": 0}


@dataclass(frozen=True)
class Term:
    """coef * ops[0] ops[1] ... (operators applied right to left, product order as written).

    ``fam`` identifies the term family (it, together with the set of roles already placed
    and the charge they carry, labels a state of the finite-state machine); the total
    coefficient equals fam_coef * prod(role_f).  ``charge[r]`` = (dN, dk) transferred by
    role r, with dk taken modulo ``ly``.
    """

    ops: tuple            # ((site, kind), ...)
    fam: tuple
    fam_coef: complex
    role_f: tuple
    charge: tuple         # ((dN, dk), ...)
    ly: int

    @property
    def coef(self) -> complex:
        c = complex(self.fam_coef)
        for f in self.role_f:
            c *= f
        return c


def _mk(ops, fam, fam_coef, role_f, charge, ly):
    return Term(tuple(ops), tuple(fam), complex(fam_coef), tuple(complex(f) for f in role_f),
                tuple(charge), ly)


def mixed_terms(cyl: Cylinder) -> list[Term]:
    """Eqs. H_kin and H_int in the mixed (x, k) basis.

    H_kin = -t sum_{x,k} [(c+_{x,k} c_{x+1,k} + h.c.) + 2 cos(k + x phi) n_{x,k}]
    H_int = V/L sum_{x,q} [cos q n_{x,q} n_{x,-q} + n_{x+1,q} n_{x,-q}],
    n_{x,q} = sum_k c+_{x,k+q} c_{x,k}.

    The intra-ring cos q is split as (e^{iq} + e^{-iq})/2 with the phase of branch s
    carried by the first bilinear's two operators (e^{is a alpha} on c+_a, e^{-is b alpha}
    on c_b, alpha = 2 pi / L), which is the factorisation Sec. IV D uses to build the
    momentum-labelled states A_mu(k), C_mu(k).
    """
    L, t, V = cyl.Ly, cyl.t, cyl.V
    al = 2.0 * np.pi / L
    o = cyl.orb
    terms: list[Term] = []
    for x in range(cyl.Lx):
        # on-site term of eq. H_kin
        for m in range(L):
            f = -2.0 * t * np.cos(al * m + x * cyl.phi)
            terms.append(_mk([(o(x, m), "n")], ("onsite", x), 1.0, [f], [(0, 0)], L))
        # hopping along the cylinder, eq. H_kin, and its Hermitian conjugate
        if x + 1 < cyl.Lx:
            for m in range(L):
                terms.append(_mk([(o(x, m), "+"), (o(x + 1, m), "-")], ("hop", x, 1), -t,
                                 [1, 1], [(1, m), (-1, -m % L)], L))
                terms.append(_mk([(o(x + 1, m), "+"), (o(x, m), "-")], ("hop", x, -1), -t,
                                 [1, 1], [(1, m), (-1, -m % L)], L))
        # intra-ring interaction (V/L) sum_q cos q n_{x,q} n_{x,-q}
        for s in (1, -1):
            for a, b, c in product(range(L), repeat=3):
                d = (a - b + c) % L
                terms.append(_mk([(o(x, a), "+"), (o(x, b), "-"), (o(x, c), "+"), (o(x, d), "-")],
                                 ("intra", x, s), V / (2.0 * L),
                                 [np.exp(1j * s * al * a), np.exp(-1j * s * al * b), 1, 1],
                                 [(1, a), (-1, -b % L), (1, c), (-1, -d % L)], L))
        # inter-ring interaction (V/L) sum_q n_{x+1,q} n_{x,-q}
        if x + 1 < cyl.Lx:
            for a, b, c in product(range(L), repeat=3):
                d = (a - b + c) % L
                terms.append(_mk([(o(x + 1, a), "+"), (o(x + 1, b), "-"), (o(x, c), "+"), (o(x, d), "-")],
                                 ("inter", x), V / L, [1, 1, 1, 1],
                                 [(1, a), (-1, -b % L), (1, c), (-1, -d % L)], L))
    return terms


def real_terms(cyl: Cylinder) -> list[Term]:
    """Eq. H_real in the real-space basis (orbital (x, y) at chain index x*Ly + y).

    Hopping -t c+_{x,y} c_{x+1,y}, ring hopping -t e^{i x phi} c+_{x,y} c_{x,y+1} (y+1 taken
    modulo Ly, which includes the c+_{x,L} c_{x,1} bond), their Hermitian conjugates, and
    V n n on the same bonds.  Only N is conserved: charges are (dN, 0) with modulus 1.
    """
    L, t, V = cyl.Ly, cyl.t, cyl.V
    o = cyl.orb
    terms: list[Term] = []
    for x in range(cyl.Lx):
        ph = np.exp(1j * x * cyl.phi)
        for y in range(L):
            yp = (y + 1) % L
            if x + 1 < cyl.Lx:
                terms.append(_mk([(o(x, y), "+"), (o(x + 1, y), "-")], ("rxhop", x, y, 1), -t,
                                 [1, 1], [(1, 0), (-1, 0)], 1))
                terms.append(_mk([(o(x + 1, y), "+"), (o(x, y), "-")], ("rxhop", x, y, -1), -t,
                                 [1, 1], [(1, 0), (-1, 0)], 1))
                terms.append(_mk([(o(x, y), "n"), (o(x + 1, y), "n")], ("rxint", x, y), V,
                                 [1, 1], [(0, 0), (0, 0)], 1))
            terms.append(_mk([(o(x, y), "+"), (o(x, yp), "-")], ("ryhop", x, y, 1), -t * ph,
                             [1, 1], [(1, 0), (-1, 0)], 1))
            terms.append(_mk([(o(x, yp), "+"), (o(x, y), "-")], ("ryhop", x, y, -1), -t * np.conj(ph),
                             [1, 1], [(1, 0), (-1, 0)], 1))
            terms.append(_mk([(o(x, y), "n"), (o(x, yp), "n")], ("ryint", x, y), V,
                             [1, 1], [(0, 0), (0, 0)], 1))
    return terms


def orbital_momenta(cyl: Cylinder, basis: str) -> np.ndarray:
    """Z_Ly charge of each orbital: m for (x, m) in the mixed basis, 0 in real space."""
    if basis == "mixed":
        return np.tile(np.arange(cyl.Ly), cyl.Lx)
    return np.zeros(cyl.n_orb, dtype=np.int64)


def terms_for(cyl: Cylinder, basis: str) -> list[Term]:
    if basis == "mixed":
        return mixed_terms(cyl)
    if basis == "real":
        return real_terms(cyl)
    raise ValueError(basis)
