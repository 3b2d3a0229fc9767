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
Run: python tests/golden/make_golden.py [sc_sphere_32|grf_crop128|sc_sphere_32_steady]
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
    {"sc_sphere_32": main, "grf_crop128": grf_crop128, "sc_sphere_32_steady": sc_sphere_32_steady}[which]()
