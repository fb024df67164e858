"""Robustness of the preconditioner (Sec. 4, Tables 1-2 analogues): average
FGMRES iterations per Newton step under mesh refinement at fixed parameters
and under eps -> 0 with h = eps/2 and dt = eps^2, for the default solver and
the paper's preset (two Richardson iterations of S~^-1, five V-cycles per
S^^-1).  The paper reports counts that stay at about 8 in both experiments
(robustness: no growth as the mesh is refined or eps -> 0); here no later
case may need more than 1.5x the iterations per Newton step of the first,
and one case of each experiment is checked against the oracle (identical
counts, 1e-10 states).
The workload is the paper's: m = 0.4, sigma = 100, theta = 1/2, cosine
initial condition; w0 = 0."""
import numpy as np
import pytest

from oracle.okref import Oracle
from paper_1603_04570_amd.inputs import cosine_state, table1_cases, table2_cases

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

PRESETS = {"default": {}, "paper": dict(schur_richardson=2, mg_cycles=5)}


def run_gpu(case, preset, steps):
    from paper_1603_04570_amd import ok
    p = ok.default_params(dim=case["dim"], n=case["n"], eps=case["eps"], sigma=case["sigma"],
                          m=case["m"], dt=case["dt"], theta=case["theta"], **preset)
    u0, w0 = cosine_state(case["dim"], case["n"], case["m"])
    u = torch.from_numpy(u0).cuda()
    w = torch.from_numpy(w0).cuda()
    st = ok.Problem(p).timestep(u, w, steps)
    assert st.status == 0
    return st.its(), u.cpu().numpy(), w.cpu().numpy()


def flat(avgs):
    """No growth along the sequence of cases (decreasing counts are fine)."""
    return max(avgs[1:]) <= 1.5 * avgs[0]


@pytest.mark.parametrize("preset", list(PRESETS))
def test_eps_sweep_counts_flat(preset):
    avgs = []
    for case in table2_cases():
        its, _, _ = run_gpu(case, PRESETS[preset], 3)
        avgs.append(float(np.mean(its)))
        print("eps", case["eps"], "N", case["n"], preset, "its", its, flush=True)
    assert flat(avgs), avgs


@pytest.mark.parametrize("preset", list(PRESETS))
def test_refinement_counts_flat(preset):
    avgs = []
    for case in table1_cases(3, (16, 32, 64)):
        its, _, _ = run_gpu(case, PRESETS[preset], 2)
        avgs.append(float(np.mean(its)))
        print("N", case["n"], preset, "its", its, flush=True)
    assert flat(avgs), avgs


@pytest.mark.parametrize("case", [table2_cases()[0], table1_cases(3, (16,))[0]])
@pytest.mark.parametrize("preset", list(PRESETS))
def test_robustness_case_matches_oracle(case, preset):
    its, u, w = run_gpu(case, PRESETS[preset], 1)
    o = Oracle(case["dim"], case["n"], case["eps"], case["sigma"], case["m"], case["dt"],
               case["theta"], **PRESETS[preset])
    u0, w0 = cosine_state(case["dim"], case["n"], case["m"])
    uo, wo, info, st = o.timestep(u0, w0, 1)
    assert st == 0 and info.its() == its
    assert np.linalg.norm(u - uo) / np.linalg.norm(uo) < 1e-10
    assert np.linalg.norm(w - wo) / np.linalg.norm(wo) < 1e-10
