"""Write the oracle's full-size reference results used by the GPU parity tests.

Calls only the FP64 CPU oracle (oracle/) on the seeded synthetic inputs of a
named workload and stores, after every timestep, the values of u and w at a
fixed seeded sample of nodes, their global norms and sums, the Newton and
FGMRES iteration counts and the residual history, and the 2-norm of each
field over every grid plane normal to each axis (N+1 values per axis, field
and step), so that an error confined to a few nodes anywhere in the grid
shows up in three of them.  Output: an .npz (no pickles) plus a small JSON
summary beside this script.

    python tests/golden/make_golden.py 3d128 5     # 3D 128^3, 5 timesteps
    python tests/golden/make_golden.py 3d256 5     # 3D 256^3, 5 timesteps
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.okref import Oracle  # noqa: E402
from paper_1603_04570_amd.inputs import CONFIGS, noise_state, sample_nodes  # noqa: E402

NSAMPLE = 2048


def plane_norms(v, dim, n):
    """[axis][plane]: 2-norm of v over each grid plane normal to each axis
    (axis 0 = x, the fastest index)."""
    g = v.reshape((n + 1,) * dim)  # indices [z][y][x] in 3D, [y][x] in 2D
    out = []
    for ax in range(dim):
        other = tuple(a for a in range(dim) if a != dim - 1 - ax)
        out.append(np.sqrt(np.sum(g * g, axis=other)))
    return np.array(out)


def main(name, steps):
    cfg = CONFIGS[name]
    dim, n = cfg["dim"], cfg["n"]
    t0 = time.time()
    o = Oracle(dim, n, cfg["eps"], cfg["sigma"], cfg["m"], cfg["dt"], cfg["theta"])
    print(f"assembled in {time.time() - t0:.1f} s", flush=True)
    u, w = noise_state(dim, n, cfg["m"], cfg["seed"])
    idx = sample_nodes(o.nodes, NSAMPLE, seed=77)
    rec = {"u": [], "w": [], "unorm": [], "wnorm": [], "usum": [], "wsum": [], "uplanes": [],
           "wplanes": []}
    meta = {"workload": name, "config": cfg, "steps": steps, "newton_its": [], "fgmres_its": [],
            "fnorms": [], "seconds": []}
    for s in range(steps):
        t1 = time.time()
        u, w, info, st = o.timestep(u, w, 1)
        if st != 0:
            raise SystemExit(f"oracle failed at step {s}: {st}")
        meta["seconds"].append(time.time() - t1)
        meta["newton_its"].append(info.newton_its)
        meta["fgmres_its"].append(info.its())
        meta["fnorms"].append(info.fnorms())
        rec["u"].append(u[idx])
        rec["w"].append(w[idx])
        rec["unorm"].append(np.linalg.norm(u))
        rec["wnorm"].append(np.linalg.norm(w))
        rec["usum"].append(u.sum())
        rec["wsum"].append(w.sum())
        rec["uplanes"].append(plane_norms(u, dim, n))
        rec["wplanes"].append(plane_norms(w, dim, n))
        print(f"step {s}: newton {info.newton_its} fgmres {info.its()} "
              f"{meta['seconds'][-1]:.1f} s", flush=True)
    np.savez(os.path.join(HERE, f"oracle_{name}.npz"), idx=idx,
             **{k: np.array(v) for k, v in rec.items()})
    with open(os.path.join(HERE, f"oracle_{name}.json"), "w") as f:
        json.dump(meta, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 1)
