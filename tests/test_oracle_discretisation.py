"""Pins of the oracle's paper discretisation (quad bits): the tanh-sinh rule
in xi = cos(theta) for the angle (Sec. 2) and the radial integral split at the
external momentum x into [0, eps2] + [eps2, x] + [x, Lambda^2] with n Gauss-
Legendre nodes in each (Sec. 3 and the Table 1 caption), against closed forms,
moments and central differences."""
import math

import numpy as np
import pytest

import workloads

TS, SPLIT = 1, 2


def _unit(ref, quad, n_rad=32, n_ir=32, n_ang=65, n=8, eps2=1e-2, L2=1e4):
    """kappa = delta = gamma = 0 and c = 0: G = Z = 1 at every momentum."""
    return ref.params(kappa=0.0, delta=0.0, gamma=0.0, eps2=eps2, lambda2=L2, n_z=n, n_g=n, n_rad=n_rad,
                      n_ir=n_ir, n_ang=n_ang, quad=quad, g0_inv=0.1, z_lambda_inv=1.3, alpha_mu=1.0)


@pytest.mark.parametrize("n_ang", [33, 65])
def test_tanh_sinh_rule_moments_and_symmetry(ref, n_ang):
    g = ref.grid(ref.params(n_ang=n_ang, quad=TS))
    th, v = g.theta, g.v
    s2 = np.sin(th) ** 2
    assert abs(np.dot(v, s2) - math.pi / 2) < 1e-13            # int sqrt(1 - xi^2)
    assert abs(np.dot(v, s2 * s2) - 3 * math.pi / 8) < 1e-13   # int (1 - xi^2)^{3/2}
    assert abs(np.dot(v, s2 * np.cos(th) ** 2) - math.pi / 8) < 1e-13
    # nodes symmetric about theta = pi/2, reaching to 1 - |xi| = 4e-14 (theta = 3e-7)
    assert np.max(np.abs(th + th[::-1] - math.pi)) < 1e-15
    assert th.min() < 3e-7 and th.max() > math.pi - 3e-7 and np.all(v > 0)


def test_tanh_sinh_needs_an_odd_count(ref):
    with pytest.raises(ValueError):
        ref.grid(ref.params(n_ang=32, quad=TS))
    with pytest.raises(ValueError):
        ref.grid(ref.params(n_ang=1, quad=TS))


@pytest.mark.parametrize("x,y", [(1.0, 1.05), (1.0, 3.7), (2.0, 0.3)])
def test_tanh_sinh_angular_closed_forms(ref, x, y):
    """<M>, <Q> (normalised by pi/2) and the ghost average of sin^4/z^2
    (closed forms of the angular integrals at unit dressings); the tanh-sinh
    rule handles the near-singular y ~ x case at 65 nodes."""
    g = ref.grid(ref.params(n_ang=65, quad=TS))
    r = min(x, y) / max(x, y)
    s2 = np.sin(g.theta) ** 2
    M = sum(vk * s * ref.kernel_M(x, y, t) for t, vk, s in zip(g.theta, g.v, s2)) / (math.pi / 2)
    Q = sum(vk * s * ref.kernel_Q(x, y, t) for t, vk, s in zip(g.theta, g.v, s2)) / (math.pi / 2)
    Gh = sum(vk * s * s / ref.momentum_z(x, y, t) ** 2 for t, vk, s in zip(g.theta, g.v, s2))
    assert abs(M - (0.75 - 0.25 * r if y > x else 0.75 * r - 0.25 * r * r)) < 1e-9
    assert abs(Q - (-0.75 - 6.25 * r + 0.875 * r * r)) < 3e-9
    assert abs(Gh * max(x, y) ** 2 / (3 * math.pi / 8) - 1.0) < 1e-9


@pytest.mark.parametrize("x", [3e-2, 1.0, 7e3])
def test_row_grid_split_at_x(ref, x):
    p = ref.params(eps2=1e-2, lambda2=1e4, n_rad=32, n_ir=20, quad=SPLIT)
    y, W = ref.row_grid(p, x)
    assert len(y) == 20 + 64
    ymin = 1e-2 * math.exp(-40)
    assert np.all(y[:20] < 1e-2) and np.all((y[20:52] > 1e-2) & (y[20:52] < x)) and np.all(y[52:] > x)
    # GL in ln y on each interval: int dy/y and int dy exact to rounding
    assert abs(np.sum(W / y) - math.log(1e4 / ymin)) < 1e-12 * math.log(1e4 / ymin)
    assert abs(np.sum(W) - (1e4 - ymin)) < 1e-12 * 1e4
    assert abs(np.sum(W[20:52]) - (x - 1e-2)) < 1e-12 * x


def test_row_grid_subtraction_rows(ref):
    """x = Lambda^2 and x = 0 (the subtraction points) have one interval above
    eps2: the IR panel and n nodes on [eps2, Lambda^2]."""
    p = ref.params(eps2=1e-2, lambda2=1e4, n_rad=32, n_ir=20, quad=SPLIT)
    for x in (1e4, 0.0):
        y, W = ref.row_grid(p, x)
        assert len(y) == 52 and np.all(np.diff(y) > 0) and y[-1] < 1e4


def _closed_form_F(ref, p):
    """F at c = 0 and G = Z = 1 from the closed-form self-energies over
    y in [0, Lambda^2] (Sec. 2 kernels; the IR panel starts at
    y_min = eps2 e^{-40}, where the ghost subtraction at x = 0 is cut):
      F^Z_i = 1 - Z^{-1} + (alpha N_c/12 pi)[(7/8)(x_i/L2 - 1) + (13/2) ln(L2/x_i)]
      F^G_i = 1 - G(0)^{-1} + C (3 pi/8)[1/2 + ln(y_min/x_i)]."""
    g = ref.grid(p)
    L2 = p.lambda2
    C = p.alpha_mu * p.n_c / (2 * math.pi ** 2)
    ymin = p.eps2 * math.exp(-p.ir_efolds)
    a = p.alpha_mu * p.n_c / (12 * math.pi)
    Fz = [1 - p.z_lambda_inv + a * ((7 / 8) * (x / L2 - 1) + 6.5 * math.log(L2 / x)) for x in g.x_z]
    Fg = [1 - p.g0_inv + C * 3 * math.pi / 8 * (0.5 + math.log(ymin / x)) for x in g.x_g]
    return np.array(Fz + Fg)


def test_split_tanh_sinh_reproduces_unit_dressing_self_energies(ref):
    """The paper's discretisation (split at x, tanh-sinh, 32 nodes per radial
    interval, 65 angles) gives the closed-form residual at unit dressings to
    1e-9 relative; the shared grid at the same radial density misses it by
    more than 1e-4 (the kink of the angular integral at y = x lies inside its
    panels): the reason for the split (Sec. 3)."""
    c = np.zeros(16)
    p = _unit(ref, TS | SPLIT)
    F = ref.residual(p, c)
    Fc = _closed_form_F(ref, p)
    assert np.max(np.abs(F / Fc - 1.0)) < 1e-9, np.max(np.abs(F / Fc - 1.0))
    ps = _unit(ref, 0, n_rad=64, n_ang=64)
    Fs = ref.residual(ps, c)
    assert np.max(np.abs(Fs / _closed_form_F(ref, ps) - 1.0)) > 1e-4


def test_split_jacobian_matches_central_differences(ref):
    cfg = workloads.config("cfg1", n_z=6, n_g=5, n_rad=16, n_ir=16, n_ang=17, quad=TS | SPLIT)
    p = ref.params(**cfg)
    c = ref.start_guess(p) + workloads.perturbation(6, 5, 0.05, seed=3)
    J = ref.jacobian(p, c)
    Jfd = ref.jacobian_fd(p, c, 1e-5)
    assert np.linalg.norm(J - Jfd) <= 1e-7 * np.linalg.norm(J)


def test_split_tanh_sinh_scaling_solution(ref):
    """The scaling solution on the paper's discretisation: Newton converges,
    and alpha below eps2 is the IR fixed point N_c alpha(0) = 8.915 (Sec. 2.1)
    to the accuracy of N = 16 (2.6e-3 on the shared grid)."""
    cfg = workloads.config("cfg1", n_rad=32, n_ir=32, n_ang=33, quad=TS | SPLIT)
    p = ref.params(**cfg)
    c, r = ref.newton(p, extra_iters=2)
    assert r["status"] == 0
    a0 = ref.running_coupling(p, c, p.eps2 * 1e-6)
    assert abs(p.n_c * a0 / 8.91512 - 1.0) < 5e-3
