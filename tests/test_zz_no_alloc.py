"""dse_lu_solve_noalloc (the LU solve with static scratch, for callers that
cannot allocate) against dse_lu_solve on the same matrices: two calls in a row,
the second smaller, both transposes, then the pivot status and the size limit."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dse():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1206_1779_amd import dse as m
    m.load()
    return m


def _system(n):
    rng = np.random.default_rng(1000 + n)
    A = rng.standard_normal((n, n)) + np.diag(rng.uniform(-3, 3, n))
    return A, rng.standard_normal(n)


def _solver(dse, n):
    return dse.Solver(**workloads.config("cfg1", n_z=n // 2, n_g=n - n // 2))


@pytest.mark.parametrize("trans", [False, True])
def test_noalloc_matches_lu_solve_two_calls(ref, dse, trans):
    import torch
    # first call: n = 200 (factors in the static scratch, not LDS);
    # second call: n = 40 (LDS), reusing the array the first call left behind
    for n in (200, 40):
        print("noalloc lu n=%d trans=%d" % (n, trans), flush=True)
        A, b = _system(n)
        s = _solver(dse, n)
        x_ref = s.lu_solve(A, b, trans=trans)
        J = torch.as_tensor(A, device="cuda:0").contiguous()
        bd = torch.as_tensor(b, device="cuda:0")
        x = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda:0")
        info = torch.full((1,), -1, dtype=torch.int32, device="cuda:0")
        dse.lu_solve_noalloc(J, bd, x, trans=trans, info=info)
        torch.cuda.synchronize()
        assert int(info.item()) == 0
        # the same kernel on the same input: identical to the context's solve
        assert torch.equal(x, x_ref), float((x - x_ref).abs().max())
        xr = ref.lu_solve(A, b, trans=trans)
        assert np.linalg.norm(x.cpu().numpy() - xr) <= 1e-12 * np.linalg.cond(A) * np.linalg.norm(xr)
        # the status word in the static array (info omitted) and an in-place solve
        x2 = bd.clone()
        dse.lu_solve_noalloc(J, x2, x2, trans=trans)
        torch.cuda.synchronize()
        assert torch.equal(x2, x_ref)


def test_noalloc_largest_size(ref, dse):
    import torch
    n = 256
    print("noalloc lu n=%d" % n, flush=True)
    A, b = _system(n)
    x = torch.empty(n, dtype=torch.float64, device="cuda:0")
    info = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    dse.lu_solve_noalloc(torch.as_tensor(A, device="cuda:0"), torch.as_tensor(b, device="cuda:0"), x, info=info)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    xr = ref.lu_solve(A, b)
    assert np.linalg.norm(x.cpu().numpy() - xr) <= 1e-12 * np.linalg.cond(A) * np.linalg.norm(xr)


def test_noalloc_singular_and_limits(dse):
    import torch
    info = torch.full((1,), -1, dtype=torch.int32, device="cuda:0")
    x = torch.empty(4, dtype=torch.float64, device="cuda:0")
    dse.lu_solve_noalloc(torch.ones(4, 4, dtype=torch.float64, device="cuda:0"),
                         torch.ones(4, dtype=torch.float64, device="cuda:0"), x, info=info)
    torch.cuda.synchronize()
    assert int(info.item()) == 4
    big = torch.zeros(257, dtype=torch.float64, device="cuda:0")
    with pytest.raises(dse.DSEError) as e:
        dse.lu_solve_noalloc(torch.eye(257, dtype=torch.float64, device="cuda:0"), big, big.clone())
    assert e.value.status == 1 and "257" in str(e.value)


@pytest.mark.parametrize("case", workloads.near_singular_matrices(), ids=lambda c: c[0])
def test_noalloc_relative_singularity(ref, dse, case):
    """Same verdict and solution as the oracle on matrices on both sides of
    the relative pivot test."""
    import torch
    name, A, b, singular = case
    info = torch.full((1,), -1, dtype=torch.int32, device="cuda:0")
    Ad = torch.tensor(A, dtype=torch.float64, device="cuda:0")
    bd = torch.tensor(b, dtype=torch.float64, device="cuda:0")
    x = torch.empty_like(bd)
    dse.lu_solve_noalloc(Ad, bd, x, info=info)
    torch.cuda.synchronize()
    if singular:
        assert int(info.item()) == 4
        return
    assert int(info.item()) == 0
    xr = ref.lu_solve(A, b)
    assert np.max(np.abs(x.cpu().numpy() - xr)) <= 1e-13 * np.max(np.abs(xr))

