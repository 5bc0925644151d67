"""Batched family: every problem of a batch against the oracle and against the
single-problem GPU path, for every launch form (angular slices, one workgroup
per item or persistent workgroups, queue order), and the 256-problem family
solved in one batched Newton iteration.

Tolerances are those of the single-problem parity tests (same arithmetic per
point; the angular split only changes the order of the partial sums):
F to 1e-13 S_r, J per row to 1e-11 of the row maximum and normwise 1e-12, c*
to u || |J^{-1}| S ||_inf.  Launch forms with the same angular split must give
bit-identical results: every queue item writes its own partial sums, so the
order in which items run cannot change them.
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


SMALL_FAMILY = [
    dict(),
    dict(n_z=10, n_g=13, g0_inv=0.05),
    dict(n_z=20, n_g=12, g0_inv=0.1),
    dict(n_z=8, n_g=8, g0_inv=0.2),
    dict(n_z=16, n_g=24, g0_inv=0.02),
    dict(n_z=12, n_g=9, n_rad=70, n_ir=9, n_ang=13, g0_inv=0.07),
    dict(n_z=24, n_g=24, n_rad=96, n_ir=24, n_ang=24, g0_inv=1 / 15.0),
]


def _small():
    return [workloads.config("cfg1", **d) for d in SMALL_FAMILY]


def _check_JF(ref, cfg, c, J, F):
    p = ref.params(**cfg)
    Jr, Fr = ref.jacobian(p, c, with_F=True)
    Sr = ref.residual_scale(p, c)
    assert np.all(np.abs(F - Fr) <= 1e-13 * Sr), np.max(np.abs(F - Fr) / Sr)
    rowmax = np.max(np.abs(Jr), axis=1)
    assert np.all(np.max(np.abs(J - Jr), axis=1) <= 1e-11 * rowmax)
    assert np.linalg.norm(J - Jr) <= 1e-12 * np.linalg.norm(Jr)


def test_batch_jacobian_every_launch_form(ref, dse):
    cfgs = _small()
    b = dse.Batch(cfgs)
    c0 = b.start_guess()
    pert = np.concatenate([workloads.perturbation(d["n_z"], d["n_g"], 0.03, seed=40 + i)
                           for i, d in enumerate(cfgs)])
    c = _np(c0) + pert
    cs = [c[b.off_c[i]: b.off_c[i + 1]] for i in range(b.count)]
    results = {}
    for slices in (1, 2, 4):
        for blocks in (0, 37):
            for order in (1, 0):
                _note("launch slices=%d blocks=%d order=%d" % (slices, blocks, order))
                b.set_launch(slices, blocks, order)
                assert b.get_launch() == dict(slices=slices, persistent_blocks=blocks, order=order)
                J, F = b.jacobian(c)
                J, F = _np(J), _np(F)
                key = slices
                if key in results:
                    assert np.array_equal(results[key][0], J) and np.array_equal(results[key][1], F)
                    continue
                results[key] = (J, F)
                for i, cfg in enumerate(cfgs):
                    n = cfg["n_z"] + cfg["n_g"]
                    Ji = J[b.off_J[i]: b.off_J[i + 1]].reshape(n, n)
                    Fi = F[b.off_c[i]: b.off_c[i + 1]]
                    _check_JF(ref, cfg, cs[i], Ji, Fi)


def test_batch_matches_single_problem_path(dse):
    cfgs = _small()
    b = dse.Batch(cfgs)
    c = b.start_guess()
    J, F = b.jacobian(c)
    for i, cfg in enumerate(cfgs):
        s = dse.Solver(**cfg)
        # the single path picks its own angular split: equal to the J tolerance
        n = s.n
        Js, Fs = s.jacobian(c[b.off_c[i]: b.off_c[i + 1]])
        Jb = _np(J[b.off_J[i]: b.off_J[i + 1]]).reshape(n, n)
        rowmax = np.max(np.abs(_np(Js)), axis=1)
        assert np.all(np.max(np.abs(Jb - _np(Js)), axis=1) <= 1e-11 * rowmax)


def test_batch_newton_small_family(ref, dse):
    cfgs = _small()
    b = dse.Batch(cfgs)
    _note("batched Newton, %d problems" % b.count)
    c, res = b.newton(extra_iters=2)
    for i, cfg in enumerate(cfgs):
        p = ref.params(**cfg)
        cr, rr = ref.newton(p, extra_iters=2)
        r = res[i]
        assert r.status == 0 and rr["status"] == 0
        assert abs(r.iters - rr["iters"]) <= 1, (i, r.iters, rr["iters"])
        J = ref.jacobian(p, cr)
        S = ref.residual_scale(p, cr)
        bound = 2.0 ** -53 * np.max(np.abs(np.linalg.inv(J)) @ S)
        err = np.max(np.abs(_np(r.c) - cr))
        _note("  problem %d: iters %d (oracle %d), diff %.2e, bound %.2e" % (i, r.iters, rr["iters"], err, bound))
        assert err <= bound


def test_batch_family_256(ref, dse):
    """The 256-problem family (N in {32, 48, 64}, G(0) in [5, 50], 256+64 x 64):
    autotuned launch, every problem converged, three of them against the
    single-problem path within the componentwise rounding bound."""
    fam = workloads.family(256)
    b = dse.Batch(fam)
    c0 = b.start_guess()
    tune = b.autotune(c0)
    _note("autotune: %s" % {k: v for k, v in tune.items() if k != "candidates"})
    for cd in tune["candidates"]:
        _note("  %s" % cd)
    c, res = b.newton(c0, extra_iters=2)
    bad = [i for i, r in enumerate(res) if r.status != 0 or not r.fnorm < 1e-10]
    assert not bad, bad
    _note("iterations: min %d max %d" % (min(r.iters for r in res), max(r.iters for r in res)))
    for i in (0, 101, 255):
        cfg = fam[i]
        s = dse.Solver(**cfg)
        rs = s.newton(extra_iters=2)
        assert rs.status == 0
        p = ref.params(**cfg)
        cs = _np(rs.c)
        J = ref.jacobian(p, cs)
        S = ref.residual_scale(p, cs)
        bound = 2.0 ** -53 * np.max(np.abs(np.linalg.inv(J)) @ S)
        err = np.max(np.abs(_np(res[i].c) - cs))
        _note("  problem %d (n_z %d n_g %d G0 %.2f): diff to single %.2e, bound %.2e"
              % (i, cfg["n_z"], cfg["n_g"], 1 / cfg["g0_inv"], err, bound))
        assert err <= 2 * bound  # both sides at their rounding floor
