"""Newton matrix by central differences on the GPU (the paper's own method,
dse_jacobian_fd) against the oracle's central differences and against the
analytic matrix.

Tolerances.  Against the oracle: both sides take the same steps
h_j = h_rel max(1, |c_j|), and each residual agrees with the oracle's to
1e-13 S_r (the residual parity bound), so entry (r, j) agrees to about
(1e-13 S_r(c + h_j e_j) + 1e-13 S_r(c - h_j e_j)) / (2 h_j) = 1e-13 S_r / h_j;
the test allows twice that, with S_r taken at c.  Against the analytic
matrix: the central-difference truncation and rounding, pinned for the oracle
at normwise 1e-7 (test_analytic_jacobian_matches_central_differences); the
same bound holds here.
"""
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


@pytest.mark.parametrize("name", ["small", "ragged"])
def test_fd_jacobian_against_oracle(ref, dse, name):
    cfg = workloads.config("cfg1", n_z=10, n_g=12) if name == "small" else \
        workloads.config("cfg1", n_z=9, n_g=13, n_rad=70, n_ir=9, n_ang=13, g0_inv=0.05)
    p = ref.params(**cfg)
    s = dse.Solver(**cfg)
    c = ref.start_guess(p) + workloads.perturbation(p.n_z, p.n_g, 0.05, seed=3)
    h_rel = 1e-5
    Jg = _np(s.jacobian_fd(c, h_rel))
    Jr = ref.jacobian_fd(p, c, h_rel)
    S = ref.residual_scale(p, c)
    h = h_rel * np.maximum(1.0, np.abs(c))
    bound = 2e-13 * S[:, None] / h[None, :]
    ratio = np.max(np.abs(Jg - Jr) / bound)
    _note("%s: worst |J_gpu - J_oracle| / bound = %.3f" % (name, ratio))
    assert ratio <= 1.0


def test_fd_jacobian_against_analytic(ref, dse):
    cfg = workloads.config("cfg1")
    p = ref.params(**cfg)
    s = dse.Solver(**cfg)
    c = ref.start_guess(p) + workloads.perturbation(p.n_z, p.n_g, 0.05, seed=4)
    Jfd = _np(s.jacobian_fd(c, 1e-5))
    J, _ = s.jacobian(c)
    J = _np(J)
    nw = np.linalg.norm(J - Jfd) / np.linalg.norm(J)
    _note("cfg1: FD vs analytic, normwise %.2e" % nw)
    assert nw <= 1e-7
    for j in range(J.shape[1]):
        assert np.linalg.norm(J[:, j] - Jfd[:, j]) <= 1e-6 * np.linalg.norm(J[:, j]) + 1e-12 * np.linalg.norm(J)


def test_fd_jacobian_full_size_sampled(dse):
    """N = 64, 256+64 x 64: FD and analytic matrices of the GPU agree to the
    truncation bound; the step is rejected outside (0, 1)."""
    cfg = workloads.config("cfg2")
    s = dse.Solver(**cfg)
    c = s.start_guess()
    Jfd = _np(s.jacobian_fd(c, 1e-5))
    J, _ = s.jacobian(c)
    J = _np(J)
    nw = np.linalg.norm(J - Jfd) / np.linalg.norm(J)
    _note("cfg2: FD vs analytic, normwise %.2e" % nw)
    assert nw <= 1e-7
    with pytest.raises(dse.DSEError):
        s.jacobian_fd(c, 0.0)
