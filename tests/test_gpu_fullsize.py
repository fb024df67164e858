"""Full-size GPU parity in the launch configuration the benchmark times
(autotuned stencil shapes, the default solver parameters).

The oracle's results at 3D 128^3 and 3D 256^3 (5 timesteps each) were
written by tests/golden/make_golden.py, which calls only the oracle: sampled
node values of u and w after every step, global norms and sums, the 2-norm
of each field over every grid plane normal to each axis, and the
Newton/FGMRES iteration counts.  Bars: identical iteration counts; sampled
values within 1e-10 relative (2-norm over the sample) per field and step;
every plane norm within 1e-10 relative (an error confined to a few nodes
anywhere moves the norms of the three planes through them); global norms
within 1e-12.  Properties that hold at any size are checked with
the oracle's matrix-free local rows: J x at sampled nodes (1e-13) and the
residual of the final state at sampled nodes (below the Newton tolerance).
"""
import json
import os

import numpy as np
import pytest

from oracle.okref import local_jacobian, local_residual, make_params
from paper_1603_04570_amd.inputs import CONFIGS, noise_state, sample_nodes, uniform01

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name):
    path = os.path.join(GOLDEN, f"oracle_{name}.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    z = np.load(path)
    meta = json.load(open(os.path.join(GOLDEN, f"oracle_{name}.json")))
    return z, meta


def plane_norms(v, dim, n):
    """[axis][plane]: 2-norm over each grid plane normal to each axis (axis 0
    = x, the fastest index), as the golden writer computes them."""
    g = v.reshape((n + 1,) * dim)
    out = []
    for ax in range(dim):
        other = tuple(a for a in range(dim) if a != dim - 1 - ax)
        out.append(torch.sqrt(torch.sum(g * g, dim=other)))
    return torch.stack(out).cpu().numpy()


def problem(cfg, **kw):
    from paper_1603_04570_amd import ok
    p = ok.default_params(dim=cfg["dim"], n=cfg["n"], eps=cfg["eps"], sigma=cfg["sigma"],
                          m=cfg["m"], dt=cfg["dt"], theta=cfg["theta"], **kw)
    P = ok.Problem(p)
    P.autotune()
    return P


@pytest.mark.parametrize("name", ["3d128", "3d256"])
def test_timesteps_match_oracle(name):
    z, meta = load_golden(name)
    cfg = CONFIGS[name]
    print("full-size timesteps", name, flush=True)
    P = problem(cfg)
    u0, w0 = noise_state(cfg["dim"], cfg["n"], cfg["m"], cfg["seed"])
    u = torch.from_numpy(u0).cuda()
    w = torch.from_numpy(w0).cuda()
    idx = torch.from_numpy(z["idx"]).cuda()
    del u0, w0
    for s in range(meta["steps"]):
        st = P.timestep(u, w, 1)
        assert st.its() == meta["fgmres_its"][s], (s, st.its(), meta["fgmres_its"][s])
        us = u[idx].cpu().numpy()
        ws = w[idx].cpu().numpy()
        eu = np.linalg.norm(us - z["u"][s]) / np.linalg.norm(z["u"][s])
        ew = np.linalg.norm(ws - z["w"][s]) / np.linalg.norm(z["w"][s])
        print(f"step {s}: its {st.its()} rel err u {eu:.2e} w {ew:.2e}", flush=True)
        assert eu < 1e-10 and ew < 1e-10
        assert abs(torch.linalg.norm(u).item() - z["unorm"][s]) <= 1e-12 * z["unorm"][s]
        assert abs(torch.linalg.norm(w).item() - z["wnorm"][s]) <= 1e-12 * z["wnorm"][s]
        if "uplanes" in z.files:
            for v, key in ((u, "uplanes"), (w, "wplanes")):
                got = plane_norms(v, cfg["dim"], cfg["n"])
                ref = z[key][s]
                err = np.abs(got - ref) / ref
                print(f"step {s}: {key} worst plane rel err {err.max():.2e}", flush=True)
                assert err.max() <= 1e-10, (s, key, np.unravel_index(err.argmax(), err.shape))


@pytest.mark.parametrize("name", ["3d128", "3d256"])
def test_jacobian_rows_at_full_size(name):
    cfg = CONFIGS[name]
    print("full-size J rows", name, flush=True)
    P = problem(cfg)
    dim, n = cfg["dim"], cfg["n"]
    u0, _ = noise_state(dim, n, cfg["m"], cfg["seed"])
    nodes = (n + 1) ** dim
    x0 = uniform01(91, 2 * nodes) - 0.5
    y = P.jacobian_apply(torch.from_numpy(u0).cuda(), torch.from_numpy(x0).cuda())
    idx = sample_nodes(nodes, 4096, seed=78)
    # the boundary and corner nodes too
    idx = np.unique(np.concatenate([idx, [0, n, nodes - 1, (n + 1) ** 2 - 1]]))
    ys = y.cpu().numpy()
    prm = make_params(dim, n, cfg["eps"], cfg["sigma"], cfg["m"], cfg["dt"], cfg["theta"])
    r1, r2 = local_jacobian(prm, u0, x0, idx)
    ref = np.concatenate([r1, r2])
    got = np.concatenate([ys[idx], ys[nodes + idx]])
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_final_state_satisfies_discrete_equations():
    """After a 256^3 timestep the oracle's residual rows at sampled nodes are
    below the Newton tolerance, and the mean of u follows its exact law."""
    name = "3d256"
    cfg = CONFIGS[name]
    print("full-size residual property", flush=True)
    P = problem(cfg)
    dim, n = cfg["dim"], cfg["n"]
    u0, w0 = noise_state(dim, n, cfg["m"], cfg["seed"])
    u = torch.from_numpy(u0).cuda()
    w = torch.from_numpy(w0).cuda()
    st = P.timestep(u, w, 1)
    assert st.status == 0
    un = u0
    uh, wh = u.cpu().numpy(), w.cpu().numpy()
    idx = sample_nodes(uh.size, 4096, seed=79)
    prm = make_params(dim, n, cfg["eps"], cfg["sigma"], cfg["m"], cfg["dt"], cfg["theta"])
    f1, f2 = local_residual(prm, uh, wh, un, None, idx)
    assert max(np.abs(f1).max(), np.abs(f2).max()) <= 1e-10
    # mean law (theta = 1): (int u1 - m)(1 + dt sigma) = int u0 - m, int by the trapezoid rule
    t = np.full(n + 1, 1.0 / n)
    t[0] = t[-1] = 0.5 / n

    def integral(v):
        g = v.reshape((n + 1,) * dim)
        for _ in range(dim):
            g = g @ t
        return float(g)
    e0 = integral(u0) - cfg["m"]
    e1 = integral(uh) - cfg["m"]
    assert abs(e1 * (1 + cfg["dt"] * cfg["sigma"]) - e0) <= 1e-12
