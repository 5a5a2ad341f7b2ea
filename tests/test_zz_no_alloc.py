"""The allocation-free load operator (stls_load_apply_noalloc) against the
allocating one (stls_load_apply): same result bit for bit on two calls in a
row, the second on a smaller problem, and a clear refusal of a problem whose
chain temporaries exceed the static device workspace.  F = B_kappa f is the
least-squares load of §3.2 for a forcing spline over the full space."""
import numpy as np
import pytest

from stls_inputs import problem_knots, uniform_pm1

pytestmark = pytest.mark.gpu


def _load_pair(S, seed):
    import torch
    import paper_1809_10026_amd as stls
    nfull = S.forcing_shape[1]
    f = torch.as_tensor(uniform_pm1(nfull, seed)).cuda()
    F_ref = torch.full((S.ndof,), np.nan, dtype=torch.float64, device="cuda")
    F_new = torch.full((S.ndof,), np.nan, dtype=torch.float64, device="cuda")
    stls.stls_load_apply(S.handle, nfull, S.ndof, f, F_ref)
    stls.stls_load_apply_noalloc(S.handle, nfull, S.ndof, f, F_new)
    torch.cuda.synchronize()
    return F_ref.cpu().numpy(), F_new.cpu().numpy()


def test_noalloc_load_matches_allocating_entry_point_on_two_calls():
    import paper_1809_10026_amd as stls
    print("noalloc: d=3 p=3 nel=20 kappa=0.7, then d=2 p=2 nel=9 kappa=3", flush=True)
    big = stls.Solver(*problem_knots(3, 20, 3), kappa=0.7)
    small = stls.Solver(*problem_knots(2, 9, 2), kappa=3.0)
    for S, seed in ((big, 41), (small, 42), (big, 43)):
        ref, new = _load_pair(S, seed)
        assert np.all(np.isfinite(ref)) and np.linalg.norm(ref) > 0
        assert np.array_equal(ref, new), float(np.max(np.abs(ref - new)))
    big.close()
    small.close()


def test_noalloc_load_refuses_problems_beyond_its_workspace():
    import paper_1809_10026_amd as stls
    print("noalloc: oversized d=3 p=3 nel=60 (host-side refusal)", flush=True)
    S = stls.Solver(*problem_knots(3, 60, 3))
    import torch
    nfull = S.forcing_shape[1]
    f = torch.zeros(nfull, dtype=torch.float64, device="cuda")
    F = torch.zeros(S.ndof, dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError, match="static workspace"):
        stls.stls_load_apply_noalloc(S.handle, nfull, S.ndof, f, F)
    S.close()
