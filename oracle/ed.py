"""Bitstring exact diagonalisation.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The many-body basis is the occupation basis of the chain orbitals, a basis state is
the integer sum_i n_i 2^i.  Fermion operators follow the Jordan-Wigner ordering of
eq. JW, written in occupation language: c_i = prod_{j<i} (-1)^{n_j} a_i, so applying
c_i or c+_i to a basis state multiplies it by (-1)^(number of occupied orbitals below
i).  The Hamiltonian is assembled term by term directly from the term lists of
``oracle.model`` (never from an MPO), which keeps it independent of the MPO builder.
"""
from __future__ import annotations

from itertools import combinations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .model import Term


def sector_basis(n_orb: int, N: int | None = None, momenta=None, K: int | None = None,
                 ly: int = 1) -> np.ndarray:
    """Sorted basis states with particle number N (all N if None) and total momentum
    sum_{occupied} momenta[i] = K mod ly (no momentum constraint if K is None)."""
    if n_orb > 62:
        raise ValueError("at most 62 orbitals")
    if N is None:
        states = np.arange(1 << n_orb, dtype=np.uint64)
    else:
        states = np.array([sum(1 << i for i in c) for c in combinations(range(n_orb), N)],
                          dtype=np.uint64)
    if K is not None:
        mom = np.asarray(momenta, dtype=np.int64)
        tot = np.zeros(len(states), dtype=np.int64)
        for i in range(n_orb):
            tot += ((states >> np.uint64(i)) & np.uint64(1)).astype(np.int64) * mom[i]
        states = states[(tot % ly) == (K % ly)]
    return np.sort(states)


def apply_op(states: np.ndarray, amp: np.ndarray, site: int, kind: str):
    """Apply one operator to a batch of basis states; returns (states, amp) with
    amp = 0 where the operator annihilates the state."""
    bit = np.uint64(1) << np.uint64(site)
    occ = (states & bit) != 0
    below = states & (bit - np.uint64(1))
    sign = np.where(np.bitwise_count(below) % 2 == 1, -1.0, 1.0)
    if kind == "+":
        amp = np.where(occ, 0.0, amp * sign)
        states = states | bit
    elif kind == "-":
        amp = np.where(occ, amp * sign, 0.0)
        states = states & ~bit
    elif kind == "n":
        amp = np.where(occ, amp, 0.0)
    else:
        raise ValueError(kind)
    return states, amp


def apply_term(states: np.ndarray, term: Term):
    """coef * ops[0] ... ops[-1] |state>, the rightmost operator acting first."""
    amp = np.full(len(states), term.coef, dtype=np.complex128)
    out = states.copy()
    for site, kind in reversed(term.ops):
        out, amp = apply_op(out, amp, site, kind)
    return out, amp


def hamiltonian(terms: list[Term], basis: np.ndarray) -> sp.csr_matrix:
    """Sparse H restricted to a charge sector given by a sorted basis array."""
    dim = len(basis)
    rows, cols, vals = [], [], []
    col_idx = np.arange(dim)
    for term in terms:
        out, amp = apply_term(basis, term)
        keep = amp != 0
        if not keep.any():
            continue
        out, amp, src = out[keep], amp[keep], col_idx[keep]
        pos = np.searchsorted(basis, out)
        pos = np.minimum(pos, dim - 1)
        inside = basis[pos] == out
        if not inside.all():
            raise ValueError(f"term {term.fam} leaves the charge sector")
        rows.append(pos)
        cols.append(src)
        vals.append(amp)
    if not rows:
        return sp.csr_matrix((dim, dim), dtype=np.complex128)
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(dim, dim)).tocsr()


def lowest(H: sp.csr_matrix, k: int = 1) -> np.ndarray:
    """Lowest k eigenvalues (dense eigh below 3000 states, ARPACK above)."""
    dim = H.shape[0]
    if dim <= 3000:
        return np.linalg.eigvalsh(H.toarray())[:k]
    vals = spla.eigsh(H, k=k, which="SA", tol=1e-13, maxiter=100000)[0]
    return np.sort(vals)


def ground_state(H: sp.csr_matrix):
    """(E0, psi0) of a sector Hamiltonian."""
    dim = H.shape[0]
    if dim <= 3000:
        w, v = np.linalg.eigh(H.toarray())
        return w[0], v[:, 0]
    w, v = spla.eigsh(H, k=1, which="SA", tol=1e-14, maxiter=100000)
    return w[0], v[:, 0]
