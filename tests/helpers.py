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


# ---------------------------------------------------------------------------------
# Algorithmic flop counts from charges and bond dimensions alone (8 real flops per
# complex multiply-add over every charge-allowed block pair), written independently
# of the library's planner so that the task-table counts it reports can be checked.
# ---------------------------------------------------------------------------------
def _qa(a, b, ly):
    return (int(a[0] + b[0]), int((a[1] + b[1]) % ly))


def _qs(a, b, ly):
    return (int(a[0] - b[0]), int((a[1] - b[1]) % ly))


def heff_flops(ba, bc, W1, W2, ql, qr, qs1, qs2, ly):
    """(L.theta GEMMs, MPO mixing, (.).R GEMMs) of one two-site matvec.  ba, bc: bond
    dicts {(N, k): dim}; W1, W2: MPO site tensors W[w, s', s, w']; ql / qr: charges of
    W1's left and W2's right MPO states; qs1 / qs2: local charges of the two orbitals."""
    ql = [tuple(map(int, q)) for q in ql]
    qr = [tuple(map(int, q)) for q in qr]
    s12 = [(s1, s2) for s1 in (0, 1) for s2 in (0, 1)]
    q12 = [_qa(qs1[s1], qs2[s2], ly) for s1, s2 in s12]
    f1 = 0.0
    for qa, ma in ba.items():
        M = sum(ba.get(_qa(qa, qw, ly), 0) for qw in ql)
        N = sum(bc.get(_qa(qa, q, ly), 0) for q in q12)
        f1 += 8.0 * M * N * ma
    f4 = 0.0
    for qcp, mcp in bc.items():
        M = sum(ba.get(_qs(qcp, q, ly), 0) for q in q12)
        if M == 0:
            continue
        K = sum(bc.get(_qs(qcp, qw, ly), 0) for qw in qr)
        f4 += 8.0 * M * mcp * K
    # two-site MPO W12[w, s12', s12, w''] and its nonzeros
    W12 = np.einsum("apsb,bqtc->apqstc", W1, W2).reshape(W1.shape[0], 4, 4, W2.shape[3])
    fm = 0.0
    for qcp in bc:
        for i12p, qp in enumerate(q12):
            qap = _qs(qcp, qp, ly)
            if qap not in ba:
                continue
            for wpp, qw in enumerate(qr):
                qc = _qs(qcp, qw, ly)
                if qc not in bc:
                    continue
                nsrc = 0
                for w, qwl in enumerate(ql):
                    qa = _qs(qap, qwl, ly)
                    if qa not in ba:
                        continue
                    for i12, q in enumerate(q12):
                        if W12[w, i12p, i12, wpp] != 0 and _qa(qa, q, ly) == qc:
                            nsrc += 1
                fm += 8.0 * nsrc * ba[qap] * bc[qc]
    return f1, fm, f4


def env_left_flops(ba, bb, W, ql, qr, qs, ly):
    """T1 = L.A, the MPO mixing and T3 = A^H.(.) of L'[b', w', b] =
    sum conj(A[a', s', b']) L[a', w, a] W[w, s', s, w'] A[a, s, b]."""
    ql = [tuple(map(int, q)) for q in ql]
    qr = [tuple(map(int, q)) for q in qr]
    f = 0.0
    for qa, ma in ba.items():  # T1 per ket sector a: rows (w, a'), columns (s, b)
        M = sum(ba.get(_qa(qa, qw, ly), 0) for qw in ql)
        N = sum(bb.get(_qa(qa, qs[s], ly), 0) for s in (0, 1))
        f += 8.0 * M * N * ma
    for qb, mb in bb.items():
        for wp, qwp in enumerate(qr):
            qbp = _qa(qb, qwp, ly)
            if qbp not in bb:
                continue
            K = 0
            for sp in (0, 1):
                qap = _qs(qbp, qs[sp], ly)
                if qap not in ba:
                    continue
                K += ba[qap]
                nsrc = 0
                for w, qw in enumerate(ql):
                    qa = _qs(qap, qw, ly)
                    if qa not in ba:
                        continue
                    for s in (0, 1):
                        if W[w, sp, s, wp] != 0 and _qa(qa, qs[s], ly) == qb:
                            nsrc += 1
                f += 8.0 * nsrc * ba[qap] * mb
            f += 8.0 * bb[qbp] * mb * K  # T3
    return f


def env_right_flops(bb, bc, W, ql, qr, qs, ly):
    """T1 = R.B^T, the MPO mixing and T3 = conj(B).(.) of R'[b', w, b] =
    sum conj(B[b', s', c']) W[w, s', s, w'] R[c', w', c] B[b, s, c]."""
    ql = [tuple(map(int, q)) for q in ql]
    qr = [tuple(map(int, q)) for q in qr]
    f = 0.0
    for qc, mc in bc.items():  # T1 per (c, s): rows (w', c'), columns b
        for s in (0, 1):
            qb = _qs(qc, qs[s], ly)
            if qb not in bb:
                continue
            M = sum(bc.get(_qa(qc, qw, ly), 0) for qw in qr)
            f += 8.0 * M * bb[qb] * mc
    for w, qw in enumerate(ql):
        for qb, mb in bb.items():
            qbp = _qa(qb, qw, ly)
            if qbp not in bb:
                continue
            K = 0
            for sp in (0, 1):
                qcp = _qa(qbp, qs[sp], ly)
                if qcp not in bc:
                    continue
                K += bc[qcp]
                nsrc = 0
                for wp, qwp in enumerate(qr):
                    qc = _qs(qcp, qwp, ly)
                    if qc not in bc:
                        continue
                    for s in (0, 1):
                        if W[w, sp, s, wp] != 0 and _qs(qc, qs[s], ly) == qb:
                            nsrc += 1
                f += 8.0 * nsrc * bc[qcp] * mb
            f += 8.0 * bb[qbp] * mb * K  # T3
    return f
