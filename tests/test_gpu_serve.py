"""Serving on the GPU: requests of different datasets, image sizes, profile
lengths, with and without gradients, submitted together; every result equals
the same evaluation made alone (chi^2 to 1e-12, gradients to 1e-10 relative:
the gradient scatter uses atomics)."""
import numpy as np
import pytest

import workloads as wl
from gpu_util import device, t

pytestmark = pytest.mark.gpu


def test_each_result_alone_equals_in_the_mix():
    dev = device()
    import torch

    import paper_1709_06999_amd as gal
    from paper_1709_06999_amd.serve import GpuExecutor, Request, Server

    ex = GpuExecutor(dev, torch.float64, max_batch=8, max_inflight=3)
    cases = {}
    for d in range(3):
        c = wl.random_case(256 * (1 + d % 2), 20000 + 7000 * d, seed=3000 + d, kind="profile",
                           fill=0.6)
        re, im = c.noise_re + 0.01, c.noise_im
        ex.add_dataset(f"d{d}", c.u, c.v, re, im, c.w)
        cases[f"d{d}"] = c
    rng = np.random.default_rng(3100)
    reqs = []
    for i in range(40):
        name = f"d{rng.integers(0, 3)}"
        c = cases[name]
        Nr = int(rng.choice([c.I.size, c.I.size // 2]))
        dR = c.dR * c.I.size / Nr
        I = c.I[:Nr] * rng.uniform(0.5, 1.5)
        reqs.append(Request(name, I, c.Rmin, dR, c.N, c.dxy, inc=rng.uniform(0, 1), PA=rng.uniform(0, 3),
                            dRA=rng.normal(0, 2 * c.dxy), dDec=rng.normal(0, 2 * c.dxy),
                            grad=bool(i % 3 == 0)))
    srv = Server(ex, max_batch=8, max_inflight=3).start()
    futs = [srv.submit(r) for r in reqs]
    res = [f.result(timeout=120) for f in futs]
    srv.stop()
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["batches"] < len(reqs)
    for r, (c2, g) in zip(reqs, res):
        ds = ex.datasets[r.dataset]
        I = torch.as_tensor(r.I, dtype=torch.float64, device=dev)
        if r.grad:
            c2a, ga = ds.chi2Profile_grad(I, r.Rmin, r.dR, r.Nxy, r.dxy, r.inc, r.PA, r.dRA, r.dDec)
            ga = ga.cpu().numpy()
            assert np.linalg.norm(g - ga) <= 1e-10 * np.linalg.norm(ga)
        else:
            c2a = ds.chi2Profile(I, r.Rmin, r.dR, r.Nxy, r.dxy, r.inc, r.PA, r.dRA, r.dDec)
        assert abs(c2 - float(c2a)) <= 1e-12 * abs(float(c2a))
