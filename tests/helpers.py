"""Test helpers: dense contraction of small block-sparse MPS (test code, not oracle)."""
import numpy as np


def _offsets(bond):
    off, c = {}, 0
    for q, m in bond.items():
        off[q] = (c, m)
        c += m
    return off, c


def dense_site(blocks, bl, br):
    ol, dl = _offsets(bl)
    orr, dr = _offsets(br)
    out = np.zeros((dl, 2, dr), dtype=np.complex128)
    for (qa, s, qb), blk in blocks.items():
        out[ol[qa][0]:ol[qa][0] + ol[qa][1], s, orr[qb][0]:orr[qb][0] + orr[qb][1]] = blk
    return out


def dense_theta(theta, ba, bc):
    ol, dl = _offsets(ba)
    oc, dc = _offsets(bc)
    out = np.zeros((dl, 2, 2, dc), dtype=np.complex128)
    for (qa, s1, s2, qc), blk in theta.items():
        out[ol[qa][0]:ol[qa][0] + ol[qa][1], s1, s2, oc[qc][0]:oc[qc][0] + oc[qc][1]] = blk
    return out


def mps_vector(wl, theta):
    """Full 2^n state vector (index sum_i s_i 2^i) of A_0..A_{j-1} theta B_{j+2}..B_{n-1}."""
    j = wl.j
    psi = np.ones((1, 1), dtype=np.complex128)
    for i in range(j):
        A = dense_site(wl.site_tensor(i), wl.bonds[i], wl.bonds[i + 1])
        psi = np.einsum("pa,asb->spb", psi, A).reshape(-1, A.shape[2])
    T = dense_theta(theta, wl.bonds[j], wl.bonds[j + 2])
    psi = np.einsum("pa,astc->tspc", psi, T).reshape(-1, T.shape[3])
    for i in range(j + 2, wl.n):
        B = dense_site(wl.site_tensor(i), wl.bonds[i], wl.bonds[i + 1])
        psi = np.einsum("pa,asb->spb", psi, B).reshape(-1, B.shape[2])
    return psi[:, 0]
