"""U(1) x Z_Ly block-sparse tensors, environment updates and the two-site matvec.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper relies on standard (i)DMRG (Sec. I, Sec. III A) and on the extra block
structure that the ring momentum gives every tensor (Sec. II: the onsite form of T_y
makes k a conserved Z_Ly charge; Sec. III B: this block structure is what cuts the
cost).  It does not restate the DMRG contractions, so this module writes out the
standard definitions, block by block, as plain sums of matrix products:

* bond charges: a bond carries the total (N, k mod Ly) of everything left of it;
* MPS tensor A[a, s, b]: q(b) = q(a) + q(s); blocks {(qa, s, qb): (m_a, m_b)};
* MPO tensor W[w, s', s, w'] (``oracle.mpo``): q(w') = q(w) + q(s') - q(s);
* left environment L[a', w, a], q(a') = q(a) + q(w); blocks {(qa', w, qa): (m_a', m_a)};
* right environment R[c', w, c], q(c') = q(c) + q(w); blocks {(qc', w, qc): (m_c', m_c)};
* two-site wavefunction theta[a, s1, s2, c]; blocks {(qa, s1, s2, qc): (m_a, m_c)};

  H_eff theta [a', s1', s2', c'] =
      sum L[a', w, a] W1[w, s1', s1, w'] W2[w', s2', s2, w''] R[c', w'', c] theta[a, s1, s2, c]
  L'[b', w', b] = sum conj(A[a', s', b']) L[a', w, a] W[w, s', s, w'] A[a, s, b]
  R'[b', w, b]  = sum conj(B[b', s', c']) W[w, s', s, w'] R[c', w', c] B[b, s, c]

Boundaries follow the boundary vectors of eq. MPO: the left end is the 1 x 1 block of
the "ready" state R, the right end the 1 x 1 block of the "final" state F.
"""
from __future__ import annotations

from collections import defaultdict

import numpy as np


def qadd(a, b, ly):
    return (int(a[0] + b[0]), int((a[1] + b[1]) % ly))


def mpo_entries(W: np.ndarray) -> dict:
    """{(w, s): [(s', w', value), ...]} for the nonzero entries of W[w, s', s, w']."""
    out = defaultdict(list)
    for w, sp, s, wp in zip(*np.nonzero(W)):
        out[(int(w), int(s))].append((int(sp), int(wp), W[w, sp, s, wp]))
    return out


def mpo_entries_right(W: np.ndarray) -> dict:
    """{(w', s): [(s', w, value), ...]} for the nonzero entries of W[w, s', s, w']."""
    out = defaultdict(list)
    for w, sp, s, wp in zip(*np.nonzero(W)):
        out[(int(wp), int(s))].append((int(sp), int(w), W[w, sp, s, wp]))
    return out


def left_boundary() -> dict:
    return {((0, 0), 0, (0, 0)): np.ones((1, 1), dtype=np.complex128)}


def right_boundary(qtot) -> dict:
    q = (int(qtot[0]), int(qtot[1]))
    return {(q, 0, q): np.ones((1, 1), dtype=np.complex128)}


def _acc(out: dict, key, val):
    if key in out:
        out[key] = out[key] + val
    else:
        out[key] = val


def env_left_update(L: dict, A: dict, W: np.ndarray) -> dict:
    """L'[b', w', b] = sum conj(A[a', s', b']) L[a', w, a] W[w, s', s, w'] A[a, s, b]."""
    by_left = defaultdict(list)
    for (qa, s, qb), blk in A.items():
        by_left[(qa, s)].append((qb, blk))
    wnz = mpo_entries(W)
    out: dict = {}
    for (qap, w, qa), lblk in L.items():
        for s in (0, 1):
            for qb, ablk in by_left.get((qa, s), []):
                t = lblk @ ablk
                for sp, wp, val in wnz.get((w, s), []):
                    for qbp, apblk in by_left.get((qap, sp), []):
                        _acc(out, (qbp, wp, qb), val * (apblk.conj().T @ t))
    return out


def env_right_update(R: dict, B: dict, W: np.ndarray) -> dict:
    """R'[b', w, b] = sum conj(B[b', s', c']) W[w, s', s, w'] R[c', w', c] B[b, s, c]."""
    by_right = defaultdict(list)
    for (qb, s, qc), blk in B.items():
        by_right[(qc, s)].append((qb, blk))
    wnz = mpo_entries_right(W)
    out: dict = {}
    for (qcp, wp, qc), rblk in R.items():
        for s in (0, 1):
            for qb, bblk in by_right.get((qc, s), []):
                t = rblk @ bblk.T
                for sp, w, val in wnz.get((wp, s), []):
                    for qbp, bpblk in by_right.get((qcp, sp), []):
                        _acc(out, (qbp, w, qb), val * (bpblk.conj() @ t))
    return out


def heff_apply(L: dict, W1: np.ndarray, W2: np.ndarray, R: dict, theta: dict) -> dict:
    """Two-site effective Hamiltonian applied to theta (definition in the module doc).

    The sum is evaluated left to right: X = L theta, Y = W1 X, Z = W2 Y, theta' = Z R."""
    by_left = defaultdict(list)
    for (qa, s1, s2, qc), blk in theta.items():
        by_left[qa].append((s1, s2, qc, blk))
    X: dict = {}
    for (qap, w, qa), lblk in L.items():
        for s1, s2, qc, tblk in by_left.get(qa, []):
            X[(qap, w, s1, s2, qc)] = lblk @ tblk
    w1 = mpo_entries(W1)
    Y: dict = {}
    for (qap, w, s1, s2, qc), xblk in X.items():
        for s1p, wp, val in w1.get((w, s1), []):
            _acc(Y, (qap, wp, s1p, s2, qc), val * xblk)
    w2 = mpo_entries(W2)
    Z: dict = {}
    for (qap, wp, s1p, s2, qc), yblk in Y.items():
        for s2p, wpp, val in w2.get((wp, s2), []):
            _acc(Z, (qap, wpp, s1p, s2p, qc), val * yblk)
    r_by = defaultdict(list)
    for (qcp, wpp, qc), rblk in R.items():
        r_by[(wpp, qc)].append((qcp, rblk))
    out: dict = {}
    for (qap, wpp, s1p, s2p, qc), zblk in Z.items():
        for qcp, rblk in r_by.get((wpp, qc), []):
            _acc(out, (qap, s1p, s2p, qcp), zblk @ rblk.T)
    return out


def theta_keys(ba: dict, bc: dict, qs1, qs2, ly: int) -> list:
    """Canonical (sorted) list of allowed theta blocks (qa, s1, s2, qc) with their shapes."""
    keys = []
    for qa in sorted(ba):
        for s1 in (0, 1):
            for s2 in (0, 1):
                qc = qadd(qadd(qa, qs1[s1], ly), qs2[s2], ly)
                if qc in bc:
                    keys.append(((qa, s1, s2, qc), (ba[qa], bc[qc])))
    return keys


def flatten(blocks: dict, keys: list) -> np.ndarray:
    parts = []
    for key, shape in keys:
        blk = blocks.get(key)
        parts.append(np.zeros(shape[0] * shape[1], dtype=np.complex128) if blk is None
                     else np.asarray(blk, dtype=np.complex128).reshape(-1))
    return np.concatenate(parts) if parts else np.zeros(0, dtype=np.complex128)


def unflatten(vec: np.ndarray, keys: list) -> dict:
    out, off = {}, 0
    for key, (m, n) in keys:
        out[key] = vec[off:off + m * n].reshape(m, n)
        off += m * n
    return out


def contract_two_site(A: dict, B: dict, ly: int) -> dict:
    """theta[a, s1, s2, c] = sum_b A[a, s1, b] B[b, s2, c]."""
    by_left = defaultdict(list)
    for (qb, s2, qc), blk in B.items():
        by_left[qb].append((s2, qc, blk))
    out: dict = {}
    for (qa, s1, qb), ablk in A.items():
        for s2, qc, bblk in by_left.get(qb, []):
            _acc(out, (qa, s1, s2, qc), ablk @ bblk)
    return out
