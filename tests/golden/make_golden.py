"""Writes golden values of the FP64 oracle (and nothing else) under tests/golden/.

sc_sphere_32.json:
The 32^3 periodic box with one solid sphere of radius 8 voxels (simple-cubic
array), g = (1e-6, 0, 0), tau = 1, Set E with Lambda = 3/16: the per-step
mean velocity is recorded and the run stops when the per-step relative change
of <u_x> falls below 1e-9 or after 5000 steps.
grf_crop128.json: the 128^3 corner crop (re-filtered for x-spanning fluid) of
the 512^3 Gaussian-random-field rock of porosity 0.2, tau = 1, Set E,
Lambda = 3/16, g = (1e-6, 0, 0); <u_x> after 500, 1000 and 2000 steps.
sc_sphere_32_steady.json: the same problem stepped until the paper's
per-step test holds (relative change of k below 1e-6, Eq. convergence) or
5000 steps: the stopping step and k there (oracle.run_to_steady).
pack_crop32_adjoint.json: the 32^3 corner crop of the 128^3 sphere pack at the
adjoint's full-size settings (tau = 1, Set E, Lambda = 3/16, g = (1e-6, 0, 0),
k after 4000 steps, segments of 200): the oracle's FP64 gradient (dk/dtau,
dk/dLambda, sum and 512 seeded nodes of dk/dg_x, raster order among fluid
voxels) with the FP64 central differences (h = 1e-4) of the oracle's k in
tau and Lambda and, at 4 of those nodes, in g_x (relative step 1e-2: one
voxel's force moves k by ~1e-10 of itself per 1e-4, below what a difference
of two FP64 runs resolves to 1e-4; k is linear in g up to O(g^2) terms).
Run: python tests/golden/make_golden.py [sc_sphere_32|grf_crop128|sc_sphere_32_steady|pack_crop32_adjoint]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from lbm_inputs import crop, workload  # noqa: E402


def grf_crop128():
    m = crop(workload("grf_512"), 128)
    p = O.Problem(m, 1.0, 3 / 16, "E", (1e-6, 0.0, 0.0))
    fh = p.initial()
    marks = (500, 1000, 2000)
    out = {}
    t0 = time.time()
    for n in range(1, marks[-1] + 1):
        fh, u = p.step(fh)
        if n in marks:
            out[str(n)] = float(p.mean_velocity(u)[0])
            print(n, out[str(n)], time.time() - t0, flush=True)
    res = dict(
        about="FP64 oracle, 128^3 corner crop of the grf_512 workload (x-spanning fluid kept), tau=1, "
              "Set E Lambda=3/16, g=(1e-6,0,0); written by tests/golden/make_golden.py",
        n_fluid=int((m == 0).sum()),
        umean_x=out,
    )
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "grf_crop128.json")
    with open(path, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res, indent=1))


def sc_sphere_32_steady():
    m = workload("sc_sphere_32")
    p = O.Problem(m, 1.0, 3 / 16, "E", (1e-6, 0.0, 0.0))
    t0 = time.time()
    r = O.run_to_steady(p, 1e-6, 5000)
    res = dict(
        about="FP64 oracle, sc_sphere_32 workload, tau=1, Set E Lambda=3/16, g=(1e-6,0,0), stepped until the "
              "per-step relative change of k_x falls below 1e-6 (oracle.run_to_steady); written by "
              "tests/golden/make_golden.py",
        eps=1e-6,
        max_steps=5000,
        steps=int(r["steps"]),
        converged=bool(r["converged"]),
        k_x=float(r["k"][0]),
    )
    print(f"{time.time() - t0:.1f} s")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sc_sphere_32_steady.json")
    with open(path, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res, indent=1))


def pack_crop32_adjoint():
    import numpy as np

    m = crop(workload("pack_128"), 32)
    N, K, tau, lam, g0 = 4000, 200, 1.0, 3 / 16, 1e-6
    p = O.Problem(m, tau, lam, "E", (g0, 0.0, 0.0))
    t0 = time.time()
    r = O.gradients(p, N, segment=K)
    print(f"gradients {time.time() - t0:.0f} s", flush=True)
    dg = r["dk_dg"][0].numpy()
    rng = np.random.default_rng(1907)
    sample = np.sort(rng.choice(p.nf, 512, replace=False))

    def k_of(tau_=tau, lam_=lam, field=None):
        q = O.Problem(m, tau_, lam_, "E", (g0, 0.0, 0.0), g_field=field)
        return float(O.run(q, N, keep_state=False)["k"][0])

    h = 1e-4
    fd_tau = (k_of(tau_=tau + h) - k_of(tau_=tau - h)) / (2 * h)
    fd_lam = (k_of(lam_=lam + h) - k_of(lam_=lam - h)) / (2 * h)
    print(f"fd tau/Lambda {time.time() - t0:.0f} s", flush=True)
    fluid = np.flatnonzero(m.reshape(-1) == 0)
    fd_g = {}
    hg = 1e-2
    for k in sample[:4]:
        fd = []
        for sgn in (1, -1):
            field = np.zeros((3,) + m.shape)
            field[0].reshape(-1)[fluid] = g0
            field[0].reshape(-1)[fluid[k]] += sgn * hg * g0
            fd.append(k_of(field=field))
        fd_g[str(int(k))] = (fd[0] - fd[1]) / (2 * hg * g0)
    print(f"fd g {time.time() - t0:.0f} s", flush=True)
    res = dict(
        about="FP64 oracle, 32^3 corner crop of the pack_128 workload, tau=1, Set E Lambda=3/16, g=(1e-6,0,0), "
              "k after 4000 steps, gradient segments of 200 (oracle.gradients); FP64 central differences of the "
              "oracle's k (h=1e-4 in tau and Lambda, 1e-2 relative in g_x at single voxels); written by "
              "tests/golden/make_golden.py",
        n_steps=N, segment=K, n_fluid=int(p.nf),
        k=r["k"], dk_dtau=r["dk_dtau"], dk_dLambda=r["dk_dLambda"],
        dk_dgx_sum=float(dg.sum()), dk_dgx_max=float(np.abs(dg).max()),
        sample=[int(v) for v in sample], dk_dgx_sample=[float(dg[v]) for v in sample],
        fd_dk_dtau=fd_tau, fd_dk_dLambda=fd_lam, fd_dk_dgx=fd_g,
    )
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "pack_crop32_adjoint.json")
    with open(path, "w") as f:
        json.dump(res, f, indent=1)
    print({k: v for k, v in res.items() if k not in ("sample", "dk_dgx_sample")})


def main():
    m = workload("sc_sphere_32")
    p = O.Problem(m, 1.0, 3 / 16, "E", (1e-6, 0.0, 0.0))
    fh = p.initial()
    hist = []
    prev = None
    t0 = time.time()
    steps = 0
    for n in range(1, 5001):
        fh, u = p.step(fh)
        ux = float(p.mean_velocity(u)[0])
        hist.append(ux)
        steps = n
        if n % 500 == 0:
            print(n, ux, time.time() - t0, flush=True)
        if prev is not None and abs(ux - prev) < 1e-9 * abs(ux):
            break
        prev = ux
    nu = (1.0 - 0.5) / 3
    out = dict(
        about="FP64 oracle, sc_sphere_32 workload (32^3, one sphere R=8 centred at 15.5), tau=1, "
              "Set E Lambda=3/16, g=(1e-6,0,0); written by tests/golden/make_golden.py",
        steps=steps,
        converged=steps < 5000,
        n_solid=int(m.sum()),
        k_final=nu * hist[-1] / 1e-6,
        umean_x={str(n): hist[n - 1] for n in (1, 2, 10, 100, 500, 1000, 2000, steps) if n <= steps},
    )
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sc_sphere_32.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "sc_sphere_32"
    {"sc_sphere_32": main, "grf_crop128": grf_crop128, "sc_sphere_32_steady": sc_sphere_32_steady,
     "pack_crop32_adjoint": pack_crop32_adjoint}[which]()
