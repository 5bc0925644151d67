"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on
the same seeded inputs.

Tolerances (derived from the arithmetic, see the design notes):
  F   |F_gpu - F_ref| <= 1e-13 S_r per row, S_r = sum of |terms| in F_r
      (the two sides sum Q*K terms in different orders, the oracle with
      compensation; rounding is a few ulp of S_r);
  S   relative 1e-12 (a sum of positive terms);
  J   per row: max_c |J_gpu - J_ref| <= 1e-11 max_c |J_ref|, and normwise
      ||J_gpu - J_ref||_F <= 1e-12 ||J_ref||_F;
  c*  converged coefficients: ||c_gpu - c_ref||_inf <= u || |J^{-1}| S ||_inf
      (u = 2^-53): the largest change of the root that a perturbation of every
      term of every row by one unit roundoff can cause (componentwise
      condition).  Both sides are iterated to their rounding floor; jittering
      the oracle's own quadrature weights by one ulp moves c* by about a tenth
      of this bound (1.6e-12 relative at N=16, 4.7e-11 at N=64), so a flat
      1e-12 is below the discrete problem's own floor at N=64.
"""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dse():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1206_1779_amd import dse as d
    d.load()
    return d


def _both(ref, dse, cfg):
    return ref.params(**cfg), dse.Solver(**cfg)


def _np(t):
    return t.detach().cpu().numpy()


SMALL = [
    ("cfg1", workloads.config("cfg1")),
    ("ragged", workloads.config("cfg1", n_z=10, n_g=13, n_rad=70, n_ir=9, n_ang=13, g0_inv=0.05)),
    ("uneven48", workloads.config("cfg1", n_z=48, n_g=20, n_rad=100, n_ir=28, n_ang=20, g0_inv=0.2)),
    ("tiny", workloads.config("cfg1", n_z=1, n_g=1, n_rad=3, n_ir=0, n_ang=1, g0_inv=0.5)),
    ("n128", workloads.config("cfg1", n_z=128, n_g=100, n_rad=60, n_ir=8, n_ang=10, g0_inv=0.1)),
]


@pytest.mark.parametrize("name,cfg", SMALL, ids=[s[0] for s in SMALL])
def test_residual_and_jacobian_parity_small(ref, dse, name, cfg):
    _note("parity small %s" % name)
    p, s = _both(ref, dse, cfg)
    c0 = ref.start_guess(p)
    for k, c in enumerate([c0, c0 + workloads.perturbation(p.n_z, p.n_g, 0.05, seed=17)]):
        _note("  point %d" % k)
        Fr = ref.residual(p, c)
        Sr = ref.residual_scale(p, c)
        Jr = ref.jacobian(p, c)
        Fg, Sg = s.residual(c, with_scale=True)
        Jg, Fg2 = s.jacobian(c)
        Fg, Sg, Jg, Fg2 = map(_np, (Fg, Sg, Jg, Fg2))
        assert np.all(np.abs(Fg - Fr) <= 1e-13 * Sr), np.max(np.abs(Fg - Fr) / Sr)
        assert np.all(np.abs(Fg2 - Fr) <= 1e-13 * Sr)
        assert np.max(np.abs(Sg - Sr) / Sr) < 1e-12
        rowmax = np.max(np.abs(Jr), axis=1)
        err = np.max(np.abs(Jg - Jr), axis=1)
        assert np.all(err <= 1e-11 * rowmax), np.max(err / rowmax)
        assert np.linalg.norm(Jg - Jr) <= 1e-12 * np.linalg.norm(Jr)


def test_cfg2_parity_full_size(ref, dse):
    """N = 64 per function, 256+64 radial x 64 angular: every entry."""
    _note("parity cfg2")
    cfg = workloads.config("cfg2")
    p, s = _both(ref, dse, cfg)
    c = ref.start_guess(p) + workloads.perturbation(p.n_z, p.n_g, 0.02, seed=5)
    Jr, Fr = ref.jacobian(p, c, with_F=True)
    Sr = ref.residual_scale(p, c)
    Jg, Fg = s.jacobian(c)
    Jg, Fg = _np(Jg), _np(Fg)
    assert np.all(np.abs(Fg - Fr) <= 1e-13 * Sr), np.max(np.abs(Fg - Fr) / Sr)
    rowmax = np.max(np.abs(Jr), axis=1)
    assert np.all(np.max(np.abs(Jg - Jr), axis=1) <= 1e-11 * rowmax)
    assert np.linalg.norm(Jg - Jr) <= 1e-12 * np.linalg.norm(Jr)


def test_cfg3_sampled_rows_full_size(ref, dse):
    """N = 128 per function, 1024+256 radial x 128 angular: sampled rows of J
    (the oracle computes them one by one) and every F entry."""
    _note("parity cfg3 sampled")
    cfg = workloads.config("cfg3")
    p, s = _both(ref, dse, cfg)
    c = ref.start_guess(p)
    rows = [0, 1, 63, 127, 128, 129, 200, 255]
    Jr = ref.jacobian(p, c, rows=rows)
    Fr = ref.residual(p, c)
    Sr = ref.residual_scale(p, c)
    Jg, Fg = s.jacobian(c)
    Jg, Fg = _np(Jg), _np(Fg)
    assert np.all(np.abs(Fg - Fr) <= 1e-13 * Sr), np.max(np.abs(Fg - Fr) / Sr)
    for r in rows:
        rm = np.max(np.abs(Jr[r]))
        assert np.max(np.abs(Jg[r] - Jr[r])) <= 1e-11 * rm, (r, np.max(np.abs(Jg[r] - Jr[r])) / rm)


def _golden_roots():
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_roots.json")
    with open(path) as f:
        return json.load(f)


def _root_errors(cg, gold):
    """Normwise and per-coefficient errors of a GPU root against the oracle's
    stored root: max |dc|, max |dc| / ||c||_inf, and the largest elementwise
    relative error over the coefficients with |c_j| >= 1e-6 ||c||_inf."""
    cr = np.asarray(gold["c"])
    d = np.abs(cg - cr)
    big = np.abs(cr) >= 1e-6 * np.max(np.abs(cr))
    return float(np.max(d)), float(np.max(d) / np.max(np.abs(cr))), float(np.max(d[big] / np.abs(cr[big])))


@pytest.mark.parametrize("name", ["cfg1", "cfg2"])
def test_newton_parity(ref, dse, name):
    """FP64 roots against the oracle's (stored by tests/golden/make_oracle_roots.py).
    Bar: half the componentwise condition bound u || |J^{-1}| S ||_inf (the
    GPU sits at 0.3 of it at N = 16 and 0.13 at N = 64, a few times the
    oracle's own one-ulp weight-jitter floor: independent exp/log, GL nodes
    and summation orders)."""
    _note("newton %s" % name)
    gold = _golden_roots()[name]
    cfg = workloads.config(name)
    assert gold["config"] == cfg
    s = dse.Solver(**cfg)
    res = s.newton(extra_iters=2)
    assert res.status == 0
    assert res.fnorm < 1e-13
    assert abs(res.iters - gold["iters"]) <= 1
    # the report's device-time split: assemblies and LU solves inside the call
    assert res.t_assembly_ms > 0 and res.t_lu_ms > 0
    assert res.t_assembly_ms + res.t_lu_ms <= res.t_total_ms
    err, rel, elem = _root_errors(_np(res.c), gold)
    _note("  max coefficient difference %.3e (relative %.3e, largest elementwise %.3e), bound %.3e, "
          "oracle floor %.3e, iters gpu %d oracle %d; assembly %.3f ms, LU %.3f ms of %.3f ms"
          % (err, rel, elem, gold["bound"], gold["floor"], res.iters, gold["iters"], res.t_assembly_ms,
             res.t_lu_ms, res.t_total_ms))
    assert err <= 0.5 * gold["bound"]


def test_newton_parity_cfg3_fp64_and_mixed(dse):
    """N = 128 per function, 1024+256 radial x 128 angular, G(0) = 15: the
    FP64 root and the mixed-precision root (FP32 Newton-matrix sums, FP64
    residual and LU) against the oracle's stored root.  FP64: half the
    componentwise bound, as at N = 16 and 64.  Mixed: the same root (it is
    defined by the FP64 residual) within the full bound, with at most two more
    Newton iterations than the FP64 solve."""
    gold = _golden_roots()["cfg3"]
    cfg = workloads.config("cfg3")
    assert gold["config"] == cfg
    its = {}
    for prec in (0, 1):
        _note("newton cfg3 precision %d" % prec)
        s = dse.Solver(**dict(cfg, precision=prec))
        res = s.newton(extra_iters=2)
        assert res.status == 0 and res.fnorm < 1e-13
        err, rel, elem = _root_errors(_np(res.c), gold)
        _note("  max coefficient difference %.3e (relative %.3e, largest elementwise %.3e), bound %.3e, "
              "oracle floor %.3e, iters %d (oracle %d), FP32 matrices %d"
              % (err, rel, elem, gold["bound"], gold["floor"], res.iters, gold["iters"],
                 res.n_jacobians_mixed))
        its[prec] = res.iters
        assert err <= (0.5 if prec == 0 else 1.0) * gold["bound"]
    assert abs(its[0] - gold["iters"]) <= 1
    assert its[1] <= its[0] + 2


def test_start_guess_parity(ref, dse):
    for name in ["cfg1", "cfg2"]:
        cfg = workloads.config(name)
        p, s = _both(ref, dse, cfg)
        assert np.max(np.abs(_np(s.start_guess()) - ref.start_guess(p))) < 1e-12


@pytest.mark.parametrize("n", [1, 7, 64, 128, 200])
@pytest.mark.parametrize("trans", [False, True])
def test_lu_solve(ref, dse, n, trans):
    _note("lu n=%d trans=%d" % (n, trans))
    cfg = workloads.config("cfg1", n_z=max(1, n // 2), n_g=max(1, n - n // 2)) if n > 1 else \
        workloads.config("cfg1", n_z=1, n_g=1)
    s = dse.Solver(**cfg)
    nn = s.n
    rng = np.random.default_rng(nn)
    A = rng.standard_normal((nn, nn)) + np.diag(rng.uniform(-3, 3, nn))
    b = rng.standard_normal(nn)
    x = _np(s.lu_solve(A, b, trans=trans))
    xr = ref.lu_solve(A, b, trans=trans)
    assert np.linalg.norm(x - xr) <= 1e-12 * np.linalg.cond(A) * np.linalg.norm(xr)


def test_lu_singular(dse):
    import torch
    s = dse.Solver(**workloads.config("cfg1", n_z=2, n_g=2))
    with pytest.raises(dse.DSEError) as e:
        s.lu_solve(torch.ones(4, 4, dtype=torch.float64), torch.ones(4, dtype=torch.float64))
    assert e.value.status == 4


@pytest.mark.parametrize("case", workloads.near_singular_matrices(), ids=lambda c: c[0])
@pytest.mark.parametrize("trans", [False, True])
def test_lu_relative_singularity(ref, dse, case, trans):
    """The device LU takes the oracle's singular verdict (a pivot at or below
    n eps times its row's largest entry) on matrices on both sides of it, at
    row scalings from 1e-150 to 1e150, and otherwise its solution."""
    import torch
    name, A, b, singular = case
    _note("lu relative %s trans=%d" % (name, trans))
    n = A.shape[0]
    s = dse.Solver(**workloads.config("cfg1", n_z=n // 2, n_g=n - n // 2))
    if singular:
        with pytest.raises(ref.OracleError):
            ref.lu_solve(A, b, trans=trans)
        with pytest.raises(dse.DSEError) as e:
            s.lu_solve(A, b, trans=trans)
        assert e.value.status == 4
        return
    xr = ref.lu_solve(A, b, trans=trans)
    x = _np(s.lu_solve(A, b, trans=trans))
    assert np.max(np.abs(x - xr)) <= 1e-13 * np.max(np.abs(xr)), np.max(np.abs(x - xr)) / np.max(np.abs(xr))


def test_deterministic(dse):
    s = dse.Solver(**workloads.config("cfg1", n_z=20, n_g=20))
    c = s.start_guess()
    J1, F1 = s.jacobian(c)
    J2, F2 = s.jacobian(c)
    assert bool((J1 == J2).all()) and bool((F1 == F2).all())


def test_invalid_params_raise(dse):
    with pytest.raises(dse.DSEError):
        dse.Solver(**workloads.config("cfg1", n_z=200))


def test_noconv_reports_last_iterate(ref, dse):
    cfg = workloads.config("cfg1")
    s = dse.Solver(**cfg)
    res = s.newton(max_iter=2, raise_on_error=False)
    assert res.status == 5 and res.iters == 2
    p = ref.params(**cfg)
    F = ref.residual(p, _np(res.c))
    S = ref.residual_scale(p, _np(res.c))
    assert abs(np.max(np.abs(F) / S) - res.fnorm) <= 1e-9 * res.fnorm


def test_newton_step_matches_composed_calls_and_graph_replays(ref, dse):
    """dse_newton_step (LU solve of the held matrix, update, J and F at the new
    point in one call) against the same step composed from dse_jacobian and
    dse_lu_solve, eager and replayed from its recorded graph several times
    (with other work and synchronisations between replays), bit for bit; the
    new residual against dse_residual and the oracle."""
    import torch
    cfg = workloads.config("cfg2")
    p, s = _both(ref, dse, cfg)
    c0 = s.start_guess()
    J, F = s.jacobian(c0)
    d = s.lu_solve(J, F)
    c_ref = c0 - d
    _, F_ref = s.jacobian(c_ref)
    Fr_res, S_ref = s.residual(c_ref, with_scale=True)
    # the residual of an assembly and of a residual-only evaluation agree to rounding
    assert torch.all((F_ref - Fr_res).abs() <= 1e-13 * S_ref)
    s.set_graphs(False)
    cn, Fn, Sn = s.newton_step(c0, check=True)
    assert torch.equal(cn, c_ref) and torch.equal(Fn, F_ref)
    assert torch.allclose(Sn, S_ref, rtol=1e-14, atol=0)
    s.set_graphs(True)
    out = (torch.empty_like(c0), torch.empty_like(c0), torch.empty_like(c0))
    for k in range(4):
        for t in out:
            t.fill_(float("nan"))
        cn, Fn, Sn = s.newton_step(c0, out=out, check=(k == 0))
        torch.cuda.synchronize()
        assert torch.equal(cn, c_ref) and torch.equal(Fn, F_ref), k
        assert torch.allclose(Sn, S_ref, rtol=1e-14, atol=0), k
        s.residual(c_ref)          # other work on the stream between replays
        _ = (c0 * 2.0).sum().item()
    # a second set of outputs records a new graph; relaxation 0.5 as well
    out2 = (torch.empty_like(c0), torch.empty_like(c0), torch.empty_like(c0))
    cn2, Fn2, _ = s.newton_step(c0, rho=0.5, out=out2)
    c_half = c0 - 0.5 * d
    assert torch.allclose(cn2, c_half, rtol=0, atol=1e-15 * float(c0.abs().max()))
    Fr = ref.residual(p, _np(cn2))
    Sr = ref.residual_scale(p, _np(cn2))
    assert np.all(np.abs(_np(Fn2) - Fr) <= 1e-13 * Sr)


@pytest.mark.parametrize("graphs", [False, True])
def test_newton_step_alternating_buffers_reuse_the_matrix(ref, dse, graphs):
    """Steps alternating between two coefficient buffers: from the second step
    on, the matrix assembled at the end of the previous step is used (one
    assembly per Newton iteration).  Each step equals the composed one at the
    same point bit for bit; a call that overwrites the held residual in between
    (dse_jacobian_fd) makes the next step assemble again."""
    import torch
    cfg = workloads.config("cfg1")
    p, s = _both(ref, dse, cfg)
    s.set_graphs(graphs)
    c0 = s.start_guess()
    bufs = [c0.clone(), torch.empty_like(c0)]
    F = torch.empty_like(c0)
    S = torch.empty_like(c0)
    cur = c0.clone()
    for k in range(6):
        if k == 3:
            s.jacobian_fd(bufs[k % 2])
        src, dst = bufs[k % 2], bufs[(k + 1) % 2]
        s.newton_step(src, out=(dst, F, S), check=True)
        torch.cuda.synchronize()
        J, Fc = s.jacobian(cur)
        nxt = cur - s.lu_solve(J, Fc)
        _, Fn = s.jacobian(nxt)
        assert torch.equal(dst, nxt) and torch.equal(F, Fn), k
        cur = nxt
    Fr = ref.residual(p, _np(cur))
    Sr = ref.residual_scale(p, _np(cur))
    assert np.all(np.abs(_np(F) - Fr) <= 1e-13 * Sr)


def test_newton_step_graph_follows_set_physics(ref, dse):
    """A recorded Newton step replayed after dse_set_physics uses the new
    physics: the same output buffers (which would replay the old graph) give
    the eager step's result at the new G(0)^{-1} and alpha(mu^2), and the
    trial residual matches the oracle's with the new parameters."""
    import torch
    cfg = workloads.config("cfg1", g0_inv=0.05)
    p0, s = _both(ref, dse, cfg)
    c0 = s.start_guess()
    out = tuple(torch.empty_like(c0) for _ in range(3))
    s.set_graphs(True)
    s.newton_step(c0, out=out, check=True)
    torch.cuda.synchronize()
    old = [t.clone() for t in out]
    s.set_physics(alpha_mu=0.9, g0_inv=0.1)
    cn, Fn, Sn = s.newton_step(c0, out=out, check=True)
    torch.cuda.synchronize()
    got = [t.clone() for t in (cn, Fn, Sn)]
    assert not torch.equal(got[1], old[1])
    s.set_graphs(False)
    ce, Fe, Se = s.newton_step(c0, check=True)
    assert torch.equal(got[0], ce) and torch.equal(got[1], Fe) and torch.equal(got[2], Se)
    p = ref.params(**dict(cfg, alpha_mu=0.9, g0_inv=0.1))
    Fr = ref.residual(p, _np(ce))
    Sr = ref.residual_scale(p, _np(ce))
    assert np.all(np.abs(_np(Fe) - Fr) <= 1e-13 * Sr)
