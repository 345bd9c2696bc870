"""Distinct plans created and solved from several host threads at once, each on its own
stream (the library's calls release the interpreter lock, so they overlap): every solve
equals the same solve run alone, bit for bit, and matches the FP64 oracle's Lanczos."""
import sys
import threading

import numpy as np
import pytest

from oracle import blocksparse as bs
from oracle import lanczos as olz

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1512_03318_amd as pk  # noqa: E402
from gpu_helpers import WindowGPU, problem, to_dev  # noqa: E402

JOBS = [("ly4_chi64", pk.DM_FP64), ("ly6_chi200", pk.DM_FP64), ("ly4_chi64", pk.DM_BF16X3),
        ("ly6_chi200", pk.DM_BF16X3)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _inputs():
    out = []
    for name, prec in JOBS:
        wl, L, W1, W2, R, th, keys, mpo = problem(name)
        g = WindowGPU(wl, L, R, mpo)
        out.append(dict(name=name, prec=prec, g=g, keys=keys, L=to_dev(g.Lf), R=to_dev(g.Rf),
                        x0=to_dev(g.pack_theta(th))))
    torch.cuda.synchronize()
    return out


def _solve(job, stream, x):
    g = job["g"]
    plan = pk.HeffPlan(g.ly, g.a, g.c, g.w1, g.w2, job["L"], job["R"], job["prec"], stream)
    e, k = pk.lanczos_ground(plan, x, 30, 1e-14, stream)
    return e, k


def test_concurrent_plans_on_host_threads():
    jobs = _inputs()
    say("solves one at a time")
    alone = []
    for job in jobs:
        x = job["x0"].clone()
        torch.cuda.synchronize()
        e, k = _solve(job, None, x)
        torch.cuda.synchronize()
        alone.append((e, k, x.cpu().numpy()))
    say("the same solves from four host threads, one stream each")
    streams = [torch.cuda.Stream() for _ in jobs]
    xs = [job["x0"].clone() for job in jobs]
    torch.cuda.synchronize()
    res = [None] * len(jobs)
    errs = []

    def run(i):
        try:
            res[i] = _solve(jobs[i], streams[i], xs[i])
        except Exception as exc:  # reported below, on the test's thread
            errs.append((i, exc))

    threads = [threading.Thread(target=run, args=(i,)) for i in range(len(jobs))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=60)
    assert not any(t.is_alive() for t in threads), "a solve did not finish"
    assert not errs, errs
    torch.cuda.synchronize()
    for i, job in enumerate(jobs):
        e, k = res[i]
        ea, ka, xa = alone[i]
        assert (e, k) == (ea, ka), (job["name"], job["prec"], e, ea, k, ka)
        assert np.array_equal(xs[i].cpu().numpy(), xa), (job["name"], job["prec"])
        if job["prec"] == pk.DM_FP64:
            wl, L, W1, W2, R, th, keys, mpo = problem(job["name"])
            mv = lambda v: bs.flatten(bs.heff_apply(L, W1, W2, R, bs.unflatten(v, keys)), keys)
            eo = olz.lanczos(mv, bs.flatten(th, keys), max_iter=30)[0]
            assert abs(e - eo) <= 1e-10 * abs(eo), (job["name"], e, eo)
