"""Marshalling between oracle block dictionaries and the library's device layouts."""
import numpy as np

import paper_1512_03318_amd as pk


def device():
    import torch
    return torch.device("cuda:0")


def to_dev(flat):
    import torch
    return torch.from_numpy(np.ascontiguousarray(flat)).to(device())


def mpo_site(mpo, i):
    return pk.MpoSite(mpo.W[i], mpo.qbond[i], mpo.qbond[i + 1], mpo.qsite[i])


class WindowGPU:
    """Packs an oracle window problem (L, W1, W2, R, theta) for the library."""

    def __init__(self, wl, L, R, mpo, j=None):
        j = wl.j if j is None else j
        self.ly = wl.ly
        self.a = pk.Bond(wl.bonds[j])
        self.c = pk.Bond(wl.bonds[j + 2])
        self.w1 = mpo_site(mpo, j)
        self.w2 = mpo_site(mpo, j + 1)
        self.qs1 = [tuple(q) for q in mpo.qsite[j]]
        self.qs2 = [tuple(q) for q in mpo.qsite[j + 1]]
        self.Lf = pk.pack(L, pk.LAYOUT_ENV_L, self.ly, self.a, qw=mpo.qbond[j])
        self.Rf = pk.pack(R, pk.LAYOUT_ENV_R, self.ly, self.c, qw=mpo.qbond[j + 2])

    def plan(self, prec=pk.DM_FP64):
        return pk.HeffPlan(self.ly, self.a, self.c, self.w1, self.w2, to_dev(self.Lf),
                           to_dev(self.Rf), prec)

    def pack_theta(self, theta):
        return pk.pack(theta, pk.LAYOUT_THETA, self.ly, self.a, self.c, qs1=self.qs1, qs2=self.qs2)

    def unpack_theta(self, flat):
        return pk.unpack(flat, pk.LAYOUT_THETA, self.ly, self.a, self.c, qs1=self.qs1, qs2=self.qs2)


def max_rel(got: dict, ref: dict, keys):
    num = max((np.abs(got[k] - ref.get(k, 0)).max() for k, _ in keys if got[k].size), default=0.0)
    den = max((np.abs(ref[k]).max() for k, _ in keys if k in ref and ref[k].size), default=1.0)
    return num / den


_problems = {}


def problem(name):
    """(wl, L, W1, W2, R, theta, keys, mpo) of a preset window, built once per process by
    the oracle from the seeded workload."""
    if name not in _problems:
        import workloads
        from oracle import synth
        wl = workloads.preset(name)
        L, W1, W2, R, th, keys, mpo = synth.window_problem(wl)
        _problems[name] = (wl, L, W1, W2, R, th, keys, mpo)
    return _problems[name]


def block_rel(got: dict, ref: dict, keys):
    """Largest relative error of one block, |got_b - ref_b|_F / |ref_b|_F, over the blocks
    whose reference is not zero (the per-block companion of max_rel)."""
    worst = 0.0
    for k, _ in keys:
        r = ref.get(k)
        if r is None or r.size == 0:
            continue
        nr = np.linalg.norm(r)
        if nr == 0.0:
            continue
        worst = max(worst, float(np.linalg.norm(got[k] - r) / nr))
    return worst
