"""Adjoint: vector-Jacobian products against J^T u and the oracle, and the
implicit-function gradient of the loss sum_m ln Z(p_m)^2 against central
finite differences of full re-solves and against the oracle's gradient."""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _note(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def dse():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1206_1779_amd import dse as d
    d.load()
    return d


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("name,cfg", [
    ("cfg1", workloads.config("cfg1", g0_inv=0.05)),
    ("ragged", workloads.config("cfg1", n_z=10, n_g=13, n_rad=70, n_ir=9, n_ang=13, g0_inv=0.05)),
    ("cfg2", workloads.config("cfg2")),
])
def test_vjp_matches_transposed_jacobian_and_oracle(ref, dse, name, cfg):
    _note("vjp %s" % name)
    p = ref.params(**cfg)
    s = dse.Solver(**cfg)
    c = ref.start_guess(p) + workloads.perturbation(p.n_z, p.n_g, 0.02, seed=3)
    u = np.random.default_rng(11).standard_normal(p.n_z + p.n_g)
    uJ, ut = s.vjp(c, u)
    uJ, ut = _np(uJ), _np(ut)
    Jg = _np(s.jacobian(c, with_F=False))
    Jr = ref.jacobian(p, c)
    Dr = ref.dF_dtheta(p, c)
    # u^T J summed two ways on the GPU and against the oracle
    scale = np.abs(u) @ np.abs(Jr)
    assert np.all(np.abs(uJ - u @ Jg) <= 1e-11 * scale + 1e-300)
    assert np.all(np.abs(uJ - u @ Jr) <= 1e-11 * scale + 1e-300)
    scale_t = np.abs(u) @ np.abs(Dr)
    assert np.all(np.abs(ut - u @ Dr) <= 1e-11 * scale_t + 1e-300), (ut, u @ Dr)
    # parameter-only mode gives the same numbers
    _, ut2 = s.vjp(c, u, with_c=False)
    assert np.array_equal(_np(ut2), ut)


def _loss_and_grad_gpu(dse, s, theta):
    import torch
    from paper_1206_1779_amd.adjoint import DressingsAt, ImplicitSolve
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    c = ImplicitSolve.apply(th, s, None, {"extra_iters": 2})
    lnz, _ = DressingsAt.apply(c, s, workloads.adjoint_loss_points())
    L = (lnz ** 2).sum()
    L.backward()
    return float(L), th.grad.numpy().copy()


def _loss_gpu(dse, s, theta):
    s.set_physics(*theta)
    r = s.newton(extra_iters=2)
    _, lnz, _ = s.running_coupling(r.c, workloads.adjoint_loss_points())
    return float((lnz ** 2).sum())


@pytest.mark.parametrize("name,cfg", [
    ("cfg1", workloads.config("cfg1", g0_inv=0.05)),
    ("uneven", workloads.config("cfg1", n_z=48, n_g=20, n_rad=40, n_ir=8, n_ang=8, g0_inv=0.2)),
    ("n128", workloads.config("cfg1", n_z=128, n_g=100, n_rad=40, n_ir=8, n_ang=8, g0_inv=0.1)),
])
def test_dressing_vjp_against_oracle_basis(ref, dse, name, cfg):
    """dse_dressing_vjp: sum_i w_i d ln Z(u_i)/d a_j (and the ln G half) at
    momenta inside, below and above [eps2, lambda2], against the oracle's
    mapping and Chebyshev rows (each pinned on the CPU); the empty case gives
    zeros.  Bar: the rounding growth of the two recurrences,
    N^2 u sum_i |w_i| per entry."""
    _note("dressing vjp %s" % name)
    p = ref.params(**cfg)
    s = dse.Solver(**cfg)
    rng = np.random.default_rng(23)
    u = np.concatenate([10.0 ** rng.uniform(-9, 7, 500), [p.eps2, p.lambda2, 1e-12, 1e9, 1.0]])
    wz = rng.standard_normal(len(u))
    wg = rng.standard_normal(len(u))
    g = _np(s.dressing_vjp(u, wz, wg))
    Tz = np.array([ref.cheb(ref.mapping(p, x), p.n_z) for x in u])
    Tg = np.array([ref.cheb(ref.mapping(p, x), p.n_g) for x in u])
    ref_g = np.concatenate([wz @ Tz, wg @ Tg])
    nmax = max(p.n_z, p.n_g)
    tol = nmax ** 2 * 2.0 ** -53 * np.concatenate([np.full(p.n_z, np.abs(wz).sum()),
                                                   np.full(p.n_g, np.abs(wg).sum())])
    assert np.all(np.abs(g - ref_g) <= tol), np.max(np.abs(g - ref_g) / tol)
    gz = _np(s.dressing_vjp(u, wz, None))
    assert np.array_equal(gz[: p.n_z], g[: p.n_z]) and not gz[p.n_z:].any()
    assert not _np(s.dressing_vjp(u[:0])).any()


def test_ift_gradient_cfg5(ref, dse):
    """Gradient of L = sum_m ln Z(p_m)^2 with respect to alpha(mu^2) and G(0)
    at N = 64 (256+64 x 64), by the implicit-function VJP, against the oracle's
    gradient (same formula in plain FP64, to ten times the gradient's own
    one-ulp rounding floor) and against central
    differences of full re-solves with h = 1e-6.  The differences carry the
    rounding noise of each re-solved root divided by h: with
    dc ~ u || |J^{-1}| S || per coefficient, |dL| <= u sum_j |dL/dc_j| (|J^{-1}| S)_j,
    so the difference quotient is trusted to that noise / h."""
    _note("ift cfg5")
    cfg = workloads.config("cfg5")
    s = dse.Solver(**cfg)
    theta = [cfg["alpha_mu"], cfg["g0_inv"], cfg["z_lambda_inv"]]
    L, g = _loss_and_grad_gpu(dse, s, theta)
    G0 = 1.0 / theta[1]
    dG0 = -g[1] / G0 ** 2          # chain rule, g0_inv = 1/G(0)

    # oracle gradient: lambda = J^{-T} dL/dc, dL/dtheta = -lambda^T dF/dtheta
    p = ref.params(**cfg)
    pts = workloads.adjoint_loss_points()
    Bz = np.array([ref.cheb(ref.mapping(p, x), p.n_z) for x in pts])

    def oracle_grad(jitter):
        ref.set_jitter(jitter)
        try:
            cr, rr = ref.newton(p, extra_iters=2)
            assert rr["status"] == 0
            gc = np.zeros(p.n_z + p.n_g)
            gc[: p.n_z] = 2 * (Bz @ cr[: p.n_z]) @ Bz
            J = ref.jacobian(p, cr)
            lam = ref.lu_solve(J, gc, trans=True)
            return cr, gc, J, -lam @ ref.dF_dtheta(p, cr)
        finally:
            ref.set_jitter(0.0)

    cr, gc, J, gr = oracle_grad(0.0)
    # rounding floor of the gradient itself: the oracle re-run with every
    # quadrature weight moved by one ulp (both signs).  That moves the root by
    # about a tenth of its componentwise bound u || |J^{-1}| S ||, so the
    # tolerance is ten times the larger of the two moves, per component.
    floor = np.maximum(np.abs(oracle_grad(2.0 ** -52)[3] - gr), np.abs(oracle_grad(-2.0 ** -52)[3] - gr))
    _note("  gpu dL/dalpha %.12e dL/dg0_inv %.12e" % (g[0], g[1]))
    _note("  oracle        %.12e            %.12e" % (gr[0], gr[1]))
    _note("  difference %.3e %.3e, 1-ulp floor %.3e %.3e"
          % (abs(g[0] - gr[0]), abs(g[1] - gr[1]), floor[0], floor[1]))
    assert abs(g[0] - gr[0]) <= 10 * floor[0]
    assert abs(g[1] - gr[1]) <= 10 * floor[1]

    # finite differences of full re-solves
    h = 1e-6
    tp, tm = list(theta), list(theta)
    tp[0] += h; tm[0] -= h
    fd_a = (_loss_gpu(dse, s, tp) - _loss_gpu(dse, s, tm)) / (2 * h)
    tp, tm = list(theta), list(theta)
    tp[1] = 1.0 / (G0 + h); tm[1] = 1.0 / (G0 - h)
    fd_g = (_loss_gpu(dse, s, tp) - _loss_gpu(dse, s, tm)) / (2 * h)
    S = ref.residual_scale(p, cr)
    noise_c = 2.0 ** -53 * (np.abs(np.linalg.inv(J)) @ S)
    noise_L = np.abs(gc) @ noise_c
    _note("  fd dL/dalpha %.10e dL/dG0 %.10e (ift %.10e), FD noise bound %.3e"
          % (fd_a, fd_g, dG0, noise_L / h))
    assert abs(g[0] - fd_a) <= noise_L / h + 1e-7 * abs(fd_a)
    assert abs(dG0 - fd_g) <= noise_L / h + 1e-7 * abs(fd_g)
