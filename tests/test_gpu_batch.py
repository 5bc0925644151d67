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


def test_batch_fused_launch_and_tile_groups(ref, dse):
    """The fused cooperative assembly (dressings, points, contraction, rows in
    one launch with grid-wide barriers) and items of 2 or 4 partial tiles give
    the same J and F bit for bit as the staged launches with one tile per
    item, for every angular split; the fused form solves the family like the
    staged one."""
    cfgs = _small()
    b = dse.Batch(cfgs)
    c0 = b.start_guess()
    pert = np.concatenate([workloads.perturbation(d["n_z"], d["n_g"], 0.03, seed=50 + i)
                           for i, d in enumerate(cfgs)])
    c = _np(c0) + pert
    for slices in (1, 2, 4):
        b.set_launch(slices, 0, 1)
        J0, F0 = (_np(t) for t in b.jacobian(c))
        for blocks, tpi, fused in ((0, 2, 0), (0, 4, 0), (29, 2, 0), (16, 1, 1), (16, 4, 1), (3, 2, 1)):
            _note("launch slices=%d blocks=%d tiles=%d fused=%d" % (slices, blocks, tpi, fused))
            b.set_launch(slices, blocks, 1, tiles_per_item=tpi, fused=fused)
            assert b.get_launch(full=True) == dict(slices=slices, persistent_blocks=blocks, order=1,
                                                   tiles_per_item=tpi, fused=fused)
            J, F = (_np(t) for t in b.jacobian(c))
            assert np.array_equal(J, J0) and np.array_equal(F, F0)
    b.set_launch(2, 0, 1)
    cs, rs = b.newton(c0)
    b.set_launch(2, 16, 1, tiles_per_item=2, fused=1)
    cf, rf = b.newton(c0)
    assert all(r.status == 0 for r in rf)
    assert [r.iters for r in rf] == [r.iters for r in rs]
    assert np.array_equal(_np(cf), _np(cs))


def test_batch_launch_rejections(dse):
    b = dse.Batch(_small())
    for kw in (dict(tiles_per_item=0), dict(tiles_per_item=65), dict(fused=2)):
        with pytest.raises(dse.DSEError) as e:
            b.set_launch(1, 0, 1, **kw)
        assert e.value.status == 1
    with pytest.raises(dse.DSEError) as e:
        b.set_launch(1, 0, 1, fused=1)  # the fused form needs its resident grid
    assert e.value.status == 1
    with pytest.raises(dse.DSEError) as e:
        b.set_launch(1, 1 << 30, 1, fused=1)
    assert e.value.status == 1 and "persistent_blocks" in str(e.value)


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


# Members whose padded orders are 48 and 64: the order-48 and order-64 bodies
# of the batch point kernel (the ones the 256-problem family runs), on a grid
# small enough for the oracle to check every entry.
WIDE_FAMILY = [
    dict(n_z=48, n_g=64, g0_inv=0.1),
    dict(n_z=64, n_g=40, g0_inv=0.03),
    dict(n_z=40, n_g=48, g0_inv=0.2),
    dict(n_z=33, n_g=20, g0_inv=1 / 15.0),
    dict(n_z=20, n_g=30, g0_inv=0.05),
]


def _wide():
    return [workloads.config("cfg1", n_rad=60, n_ir=8, n_ang=10, **d) for d in WIDE_FAMILY]


def test_batch_orders_48_64_small_grid(ref, dse):
    """Every Newton-matrix and residual entry of members with padded orders 48
    and 64 against the oracle, for the per-item and the persistent launch at
    one and two angular slices; one member's root against the oracle's."""
    cfgs = _wide()
    b = dse.Batch(cfgs)
    c0 = b.start_guess()
    pert = np.concatenate([workloads.perturbation(d["n_z"], d["n_g"], 0.03, seed=70 + i)
                           for i, d in enumerate(cfgs)])
    c = _np(c0) + pert
    for slices, blocks in ((1, 0), (2, 48), (1, 300)):
        _note("orders 48/64 small grid: slices=%d blocks=%d" % (slices, blocks))
        b.set_launch(slices, blocks, 1)
        J, F = b.jacobian(c)
        J, F = _np(J), _np(F)
        for i, cfg in enumerate(cfgs):
            n = cfg["n_z"] + cfg["n_g"]
            _check_JF(ref, cfg, c[b.off_c[i]: b.off_c[i + 1]],
                      J[b.off_J[i]: b.off_J[i + 1]].reshape(n, n), F[b.off_c[i]: b.off_c[i + 1]])
    b.set_launch(1, 0, 1)
    _, res = b.newton(extra_iters=2)
    for i in (0, 1):
        p = ref.params(**cfgs[i])
        cr, rr = ref.newton(p, extra_iters=2)
        assert res[i].status == 0 and rr["status"] == 0
        Jr = ref.jacobian(p, cr)
        bound = 2.0 ** -53 * np.max(np.abs(np.linalg.inv(Jr)) @ ref.residual_scale(p, cr))
        err = np.max(np.abs(_np(res[i].c) - cr))
        _note("  member %d: iters %d (oracle %d), diff %.2e, bound %.2e"
              % (i, res[i].iters, rr["iters"], err, bound))
        assert abs(res[i].iters - rr["iters"]) <= 1
        assert err <= bound


def _cfg4_members():
    """Members of the 256-problem family (grid 256+64 x 64) covering the
    padded orders 48 and 64: the first member of each (N_Z, N_G) pair below."""
    fam = workloads.family(256)
    want = [(48, 64), (64, 48), (48, 48), (64, 64), (32, 48)]
    out = []
    for pair in want:
        i = next(k for k, f in enumerate(fam) if (f["n_z"], f["n_g"]) == pair)
        out.append((i, fam[i]))
    return out


def test_batch_family_members_full_grid_vs_oracle(ref, dse):
    """Family members with N_Z, N_G in {48, 64} on the family's own grid
    (256+64 radial x 64 angular), batched with the family's launch forms:
    every F entry and every J entry against the oracle, and three converged
    roots against the oracle's roots within the componentwise bound."""
    members = _cfg4_members()
    cfgs = [f for _, f in members]
    b = dse.Batch(cfgs)
    c = _np(b.start_guess())
    for slices, blocks in ((1, 512), (2, 0)):
        _note("family members full grid: slices=%d blocks=%d" % (slices, blocks))
        b.set_launch(slices, blocks, 1)
        J, F = b.jacobian(c)
        J, F = _np(J), _np(F)
        for i, cfg in enumerate(cfgs):
            n = cfg["n_z"] + cfg["n_g"]
            _note("  member %d (n_z %d n_g %d)" % (members[i][0], cfg["n_z"], cfg["n_g"]))
            _check_JF(ref, cfg, c[b.off_c[i]: b.off_c[i + 1]],
                      J[b.off_J[i]: b.off_J[i + 1]].reshape(n, n), F[b.off_c[i]: b.off_c[i + 1]])
    b.set_launch(1, 512, 1)
    _, res = b.newton(extra_iters=2)
    for i in (0, 1, 3):
        p = ref.params(**cfgs[i])
        cr, rr = ref.newton(p, extra_iters=2)
        assert res[i].status == 0 and rr["status"] == 0
        Jr = ref.jacobian(p, cr)
        bound = 2.0 ** -53 * np.max(np.abs(np.linalg.inv(Jr)) @ ref.residual_scale(p, cr))
        err = np.max(np.abs(_np(res[i].c) - cr))
        _note("  member %d root: iters %d (oracle %d), diff %.2e, bound %.2e"
              % (members[i][0], res[i].iters, rr["iters"], err, bound))
        assert abs(res[i].iters - rr["iters"]) <= 1
        assert err <= bound
