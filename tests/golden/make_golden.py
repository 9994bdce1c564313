"""Write the stored oracle values used by the full-length GPU parity test.

Runs ONLY the FP64 oracle (oracle/) on the seeded 256 x 256 lid-driven
cavity (lid 0.1, Re 1000, tau = 0.5768, rho0 = 1 with 1e-6 noise, seed 1802)
for 20000 steps, and stores rho, u_x, u_y at a fixed set of fluid nodes --
both centre lines plus 512 nodes drawn with SplitMix64 (seed 7) -- as hex
floats, together with whole-field sums.

Usage: python tests/golden/make_golden.py   (about 15-25 minutes, one core)
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import oracle as O  # noqa: E402
from paper_1801_03863_amd import inputs as I  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "cavity256_re1000_20000.json")


def sample_nodes(n):
    mid = n // 2
    pts = set()
    for k in range(1, n - 1):
        pts.add((mid, k))   # vertical centre line x = n/2
        pts.add((k, mid))   # horizontal centre line y = n/2
    idx = np.arange(512, dtype=np.uint64)
    xs = 1 + np.floor(I.splitmix_uniform(7, 2 * idx) * (n - 2)).astype(int)
    ys = 1 + np.floor(I.splitmix_uniform(7, 2 * idx + np.uint64(1)) * (n - 2)).astype(int)
    pts.update(zip(xs.tolist(), ys.tolist()))
    return sorted(pts)


def main():
    c = I.cavity_256()
    n, steps = c["nx"], c["steps"]
    t0 = time.time()
    r = O.run(O.D2Q9, O.MINXENT4, O.BC_CAVITY, n, n, c["tau"], c["rho"], c["ux"], c["uy"], steps=steps,
              u_lid=c["u_lid"], rho0=c["rho0"])
    secs = time.time() - t0
    pts = sample_nodes(n)
    fl = (slice(1, n - 1), slice(1, n - 1))
    data = {
        "_what": "FP64 oracle (oracle/lbm_oracle.c) after %d steps of the seeded 256x256 MinxEnt4 cavity; "
                 "written by tests/golden/make_golden.py" % steps,
        "n": n, "steps": steps, "tau": c["tau"], "u_lid": c["u_lid"], "re": c["re"], "seed": c["seed"],
        "oracle_seconds": round(secs, 1),
        "unstable": r["unstable"], "guarded": int(r["guarded"]),
        "fluid_sum_rho": float(r["rho"][fl].sum()).hex(),
        "fluid_sum_jx": float((r["rho"] * r["ux"])[fl].sum()).hex(),
        "fluid_max_abs": {k: float(np.abs(r[k][fl]).max()).hex() for k in ("rho", "ux", "uy")},
        "fluid_l2": {k: float(np.sqrt((r[k][fl] ** 2).sum())).hex() for k in ("rho", "ux", "uy")},
        "nodes": [[x, y] for x, y in pts],
        "rho": [float(r["rho"][y, x]).hex() for x, y in pts],
        "ux": [float(r["ux"][y, x]).hex() for x, y in pts],
        "uy": [float(r["uy"][y, x]).hex() for x, y in pts],
    }
    with open(OUT, "w") as fh:
        json.dump(data, fh, indent=0)
    print("wrote", OUT, "in %.0f s" % secs)


if __name__ == "__main__":
    main()
