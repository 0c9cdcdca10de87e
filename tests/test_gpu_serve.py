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


def test_served_results_match_oracle_and_central_differences():
    # Config-4 datasets (8 resident, M log-uniform in [1e5, 2e6], uv radius
    # in [2e4, 1e6] lambda), observations = the oracle's model of one "true"
    # profile plus noise.  Requests are served all together (one stream of
    # mixed micro-batches): per dataset one chi^2 + gradient request checked
    # against the oracle, and central differences on 32 random profile bins of
    # that request (h = 0.1 max|I|; chi^2 is quadratic in I, so they are
    # exact up to rounding) against its served gradient, rel. l2 < 1e-6.
    # Requests use Nxy in {512, 1024} so that the oracle finishes in seconds.
    dev = device()
    import torch

    import oracle
    from gpu_util import chi2_bound
    from paper_1709_06999_amd.serve import GpuExecutor, Request, Server

    ex = GpuExecutor(dev, torch.float64, max_batch=16, max_inflight=4)
    truth = wl.serve_requests(1, seed=1549, sizes=(1024,))[0]
    obs = {}
    for dset in wl.serve_datasets(8):
        print(f"served oracle: dataset {dset['name']} M={dset['u'].size}", flush=True)
        Vt = oracle.sampleProfile(truth["I"], truth["Rmin"], truth["dR"], truth["Nxy"],
                                  truth["dxy"], dset["u"], dset["v"], truth["inc"], truth["PA"],
                                  truth["dRA"], truth["dDec"])
        re, im = Vt.real + dset["noise_re"], Vt.imag + dset["noise_im"]
        ex.add_dataset(dset["name"], dset["u"], dset["v"], re, im, dset["w"])
        obs[dset["name"]] = (dset, re, im)
    prm = wl.serve_requests(64, seed=1570, sizes=(512, 1024))
    checked = {}
    for p in prm:  # the first request of each dataset
        checked.setdefault(p["dataset"], p)
    assert len(checked) == 8
    rng = np.random.default_rng(1571)
    reqs, fd_plan = [], {}
    for name, p in checked.items():
        reqs.append((name, "grad", Request(grad=True, **p)))
        I = np.asarray(p["I"], dtype=np.float64)
        h = 0.1 * np.max(np.abs(I))
        idx = rng.choice(I.size, 32, replace=False)
        fd_plan[name] = (idx, h)
        for j in idx:
            for sgn in (+1.0, -1.0):
                Ij = I.copy()
                Ij[j] += sgn * h
                q = dict(p)
                q["I"] = Ij
                reqs.append((name, (int(j), sgn), Request(grad=False, **q)))
    order = rng.permutation(len(reqs))  # interleave datasets, sizes and kinds
    srv = Server(ex, max_batch=16, max_inflight=4).start()
    futs = {int(k): srv.submit(reqs[k][2]) for k in order}
    res = {k: f.result(timeout=300) for k, f in futs.items()}
    srv.stop()
    assert srv.stats()["completed"] == len(reqs)
    served_grad, fd_val = {}, {}
    for k, (name, tag, r) in enumerate(reqs):
        c2, g = res[k]
        if tag == "grad":
            served_grad[name] = (c2, g, r)
        else:
            fd_val[(name,) + tag] = c2
    for name, (c2, g, r) in served_grad.items():
        dset, re, im = obs[name]
        args = (r.I, r.Rmin, r.dR, r.Nxy, r.dxy, dset["u"], dset["v"], re, im, dset["w"], r.inc,
                r.PA, r.dRA, r.dDec)
        c2o, go = oracle.grad_profile(*args)
        Vo = oracle.sampleProfile(r.I, r.Rmin, r.dR, r.Nxy, r.dxy, dset["u"], dset["v"], r.inc,
                                  r.PA, r.dRA, r.dDec)
        dV = np.full(Vo.size, 1e-10 * np.max(np.abs(Vo)))
        rel = np.linalg.norm(g - go) / np.linalg.norm(go)
        el = np.max(np.abs(g - go)) / np.max(np.abs(go))
        idx, h = fd_plan[name]
        fd = np.array([(fd_val[(name, int(j), 1.0)] - fd_val[(name, int(j), -1.0)]) / (2 * h)
                       for j in idx])
        rel_fd = np.linalg.norm(g[idx] - fd) / np.linalg.norm(fd)
        print(f"served {name} N={r.Nxy} Nr={np.size(r.I)}: chi2 {c2:.15g} oracle {c2o:.15g}; "
              f"grad rel l2 {rel:.2e} max el {el:.2e}; FD rel l2 {rel_fd:.2e}", flush=True)
        assert abs(c2 - c2o) <= chi2_bound(c2o, dV, dset["w"]), (c2, c2o)
        assert rel <= 1e-8 and el <= 1e-8, (rel, el)
        assert rel_fd < 1e-6, rel_fd


def test_footprint_is_the_device_memory_a_micro_batch_holds():
    # the executor's footprint is the planner's workspace for the batch_exec
    # call plus the staging it carves; gradient requests and long profiles
    # included; every launch allocates exactly that
    dev = device()
    import torch

    import paper_1709_06999_amd as gal
    from paper_1709_06999_amd.serve import GpuExecutor, Request

    ex = GpuExecutor(dev, torch.float64, max_batch=16, max_inflight=2)
    for d, M in enumerate((30_000, 70_001)):
        c = wl.random_case(512, M, seed=3200 + d, kind="profile", fill=0.7)
        ex.add_dataset(f"d{d}", c.u, c.v, c.noise_re, c.noise_im, c.w)
    rho = max(ds.rho_max for ds in ex.datasets.values())
    rng = np.random.default_rng(3210)
    mixes = []
    for trial in range(6):
        reqs = []
        for k in range(int(rng.integers(1, 9))):
            Nr = int(rng.choice([64, 1500, 8000]))           # up to the gradient limit
            N = int(rng.choice([128, 256, 512]))
            dxy = 0.8 * (N / 2 - 1) / (N * rho)              # both datasets inside the grid
            reqs.append(Request(f"d{k % 2}", rng.uniform(0.5, 1.5, Nr), 1e-9, 1e-8 * 512 / Nr,
                                N, dxy, grad=bool(rng.random() < 0.5)))
        mixes.append(reqs)
    for reqs in mixes:
        specs = [(ex.datasets[r.dataset], gal.JOB_PROFILE, r.Nxy, r.dxy, np.size(r.I), r.grad)
                 for r in reqs]
        need_ws = gal.exec_workspace_bytes(specs)
        el = 8
        staging = sum(el * np.size(r.I) for r in reqs) + 56 * len(reqs) + \
            sum(el * np.size(r.I) for r in reqs if r.grad)
        fp = ex.footprint(reqs)
        assert fp >= need_ws + staging, (fp, need_ws, staging)
        assert fp <= need_ws + staging + 5 * 256
        h = ex.launch(reqs, 0)
        assert h[3].numel() == fp        # the launch holds exactly the footprint
        out = ex.collect(h)
        assert len(out) == len(reqs) and all(np.isfinite(c) for c, _ in out)
