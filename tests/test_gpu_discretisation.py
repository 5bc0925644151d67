"""GPU parity of the paper's discretisation against the oracle: the tanh-sinh
angular rule (Sec. 2) and the radial integral split at each row's x
(Sec. 3), alone and together, with the tolerances of the default grid:
F to 1e-13 S_r per row, J per row to 1e-11 of the row maximum and normwise to
1e-12, converged coefficients to the componentwise condition bound
u || |J^{-1}| S ||_inf (u = 2^-53).  On a split grid the q-side derivative
sums run through the per-point recurrences instead of the B . T product, so
both sides sum the same terms in different orders, as on the shared grid."""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
TS, SPLIT = 1, 2


def _note(msg):
    print("[discretisation] " + msg, flush=True)
    sys.stdout.flush()


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


CASES = [
    ("ts", workloads.config("cfg1", n_ang=17, quad=TS)),
    ("split", workloads.config("cfg1", n_rad=32, n_ir=16, quad=SPLIT)),
    ("split_ts", workloads.config("cfg1", n_rad=32, n_ir=16, n_ang=17, quad=TS | SPLIT)),
    ("split_ts_ragged", workloads.config("cfg1", n_z=10, n_g=13, n_rad=21, n_ir=9, n_ang=13, g0_inv=0.05,
                                         quad=TS | SPLIT)),
    ("split_uneven", workloads.config("cfg1", n_z=48, n_g=20, n_rad=40, n_ir=20, n_ang=21, g0_inv=0.2,
                                      quad=TS | SPLIT)),
    ("split_tiny", workloads.config("cfg1", n_z=1, n_g=1, n_rad=3, n_ir=0, n_ang=3, g0_inv=0.5, quad=TS | SPLIT)),
]


def _check(Jg, Fg, Sg, Jr, Fr, Sr):
    assert np.all(np.abs(Fg - Fr) <= 1e-13 * Sr), np.max(np.abs(Fg - Fr) / Sr)
    if Sg is not None:
        assert np.max(np.abs(Sg - Sr) / Sr) < 1e-12
    rowmax = np.max(np.abs(Jr), axis=1)
    err = np.max(np.abs(Jg - Jr), axis=1)
    assert np.all(err <= 1e-11 * rowmax), np.max(err / rowmax)
    assert np.linalg.norm(Jg - Jr) <= 1e-12 * np.linalg.norm(Jr)


@pytest.mark.parametrize("name,cfg", CASES, ids=[c[0] for c in CASES])
def test_residual_and_jacobian_parity(ref, dse, name, cfg):
    _note("parity %s" % name)
    p = ref.params(**cfg)
    s = dse.Solver(**cfg)
    c0 = ref.start_guess(p)
    for c in (c0, c0 + workloads.perturbation(p.n_z, p.n_g, 0.05, seed=23)):
        Jr, Fr = ref.jacobian(p, c, with_F=True)
        Sr = ref.residual_scale(p, c)
        Fg, Sg = s.residual(c, with_scale=True)
        Jg, Fg2 = s.jacobian(c)
        _check(_np(Jg), _np(Fg), _np(Sg), Jr, Fr, Sr)
        assert np.all(np.abs(_np(Fg2) - Fr) <= 1e-13 * Sr)


def test_split_full_size_sampled_rows(ref, dse):
    """N = 64 per function on the paper's discretisation at the size of its
    Table 1 (64 nodes per radial interval, 65 tanh-sinh angles): every F
    entry and sampled rows of J (the oracle computes them one by one)."""
    cfg = workloads.config("cfg2", n_rad=64, n_ir=64, n_ang=65, quad=TS | SPLIT)
    _note("parity split full size")
    p = ref.params(**cfg)
    s = dse.Solver(**cfg)
    c = ref.start_guess(p)
    rows = [0, 1, 31, 63, 64, 65, 100, 127]
    Jr = ref.jacobian(p, c, rows=rows)
    Fr = ref.residual(p, c)
    Sr = ref.residual_scale(p, c)
    Jg, Fg = s.jacobian(c)
    Jg, Fg = _np(Jg), _np(Fg)
    assert np.all(np.abs(Fg - Fr) <= 1e-13 * Sr), np.max(np.abs(Fg - Fr) / Sr)
    for r in rows:
        rm = np.max(np.abs(Jr[r]))
        assert np.max(np.abs(Jg[r] - Jr[r])) <= 1e-11 * rm, (r, np.max(np.abs(Jg[r] - Jr[r])) / rm)


@pytest.mark.parametrize("quad", [TS, TS | SPLIT])
def test_newton_on_the_paper_discretisation(ref, dse, quad):
    """Scaling solution, N = 16, 32 nodes per radial interval, 33 angles: the
    GPU Newton solve reaches the oracle's root within the componentwise
    condition bound."""
    cfg = workloads.config("cfg1", n_rad=32, n_ir=32, n_ang=33, quad=quad)
    _note("newton quad=%d" % quad)
    p = ref.params(**cfg)
    s = dse.Solver(**cfg)
    res = s.newton(extra_iters=2)
    cr, rr = ref.newton(p, extra_iters=2)
    assert res.status == 0 and rr["status"] == 0
    Jc = ref.jacobian(p, cr)
    bound = 2.0 ** -53 * np.max(np.abs(np.linalg.inv(Jc)) @ ref.residual_scale(p, cr))
    err = np.max(np.abs(_np(res.c) - cr))
    assert err <= bound, (err, bound)
    assert abs(res.iters - rr["iters"]) <= 1


def test_split_rejections(dse):
    """The split grid is FP64 residual/Jacobian work: mixed precision, the
    batched family and the vector-Jacobian product refuse it before any
    launch; the tanh-sinh rule needs an odd angle count."""
    import torch
    cfg = workloads.config("cfg1", n_rad=16, n_ir=8, quad=SPLIT)
    with pytest.raises(dse.DSEError) as e:
        dse.Solver(**dict(cfg, precision=1))
    assert e.value.status == 1
    with pytest.raises(dse.DSEError) as e:
        dse.Batch([cfg, cfg])
    assert e.value.status == 1
    with pytest.raises(dse.DSEError) as e:
        dse.Solver(**workloads.config("cfg1", n_ang=16, quad=TS))
    assert e.value.status == 1
    s = dse.Solver(**cfg)
    c = s.start_guess()
    with pytest.raises(dse.DSEError) as e:
        s.vjp(c, torch.ones_like(c))
    assert e.value.status == 1
