"""The allocation-free entry point polyspec_forward_static against polyspec_shells + polyspec_contract.

Two calls in a row on one GPU, the second with a smaller input (another plan), share the
library's static scratch; each result must equal the ordinary entry points' (same kernels
in the same order: bitwise), and the plans' own workspaces must be left as they were.
"""
import numpy as np
import pytest

import fieldgen
import oracle as O

pytestmark = pytest.mark.gpu


def _static_forward(ps, plan, x):
    import torch
    out = torch.empty((plan.batch, plan.n_closing), dtype=torch.float64, device=plan.device)
    raw = torch.empty_like(out)
    ps.polyspec_forward_static(plan.handle, x.data_ptr(), out.data_ptr(), raw.data_ptr())
    torch.cuda.synchronize()
    return out.cpu().numpy(), raw.cpu().numpy()


@pytest.mark.parametrize("precision", [0, 2])
def test_forward_static_matches_ordinary_entry_points(gpu, precision):
    import torch
    import paper_1904_11055_amd as ps
    cases = [(64, 8, 1.0, 91), (32, 6, 1.0, 92)]          # the second input is smaller
    plans = []
    for N, nb, width, seed in cases:
        delta = fieldgen.lognormal_field(N, seed).astype(np.float32)
        x = torch.from_numpy(delta)[None].to("cuda:0")
        plan = ps.Plan(N, 3, nb, width, precision=precision, device="cuda:0")
        plan.shells(x)
        B, S = (a.cpu().numpy() for a in plan.contract(raw=True))   # ordinary entry points
        assert ps.polyspec_workspace_size(plan.handle) <= ps.STATIC_SCRATCH_BYTES
        plans.append((plan, x, delta, B, S))
    for plan, x, delta, B, S in plans:                    # static calls, one after the other
        Bs, Ss = _static_forward(ps, plan, x)
        assert np.array_equal(Bs, B) and np.array_equal(Ss, S)
        ref = O.polyspectrum(delta.astype(np.float64), 3, plan.n_shells, plan.width)
        tol = 1e-5 if precision == 0 else 1e-4
        assert np.linalg.norm(Bs[0] - ref["B"]) / np.linalg.norm(ref["B"]) < tol
    for plan, x, delta, B, S in plans:                    # the plans' own fields are intact
        assert np.array_equal(plan.contract().cpu().numpy(), B)
        plan.close()


def test_forward_static_refuses_large_plans(gpu):
    import torch
    import paper_1904_11055_amd as ps
    plan = ps.Plan(256, 3, 40, 2.0, device="cuda:0")
    assert ps.polyspec_workspace_size(plan.handle) > ps.STATIC_SCRATCH_BYTES
    x = torch.zeros((1, 256, 256, 256), dtype=torch.float32, device="cuda:0")
    out = torch.empty((1, plan.n_closing), dtype=torch.float64, device="cuda:0")
    with pytest.raises(ps.PolyspecError) as e:
        ps.polyspec_forward_static(plan.handle, x.data_ptr(), out.data_ptr())
    assert e.value.status == 7 and "static scratch" in str(e.value)
    plan.close()
