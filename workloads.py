"""Seeded synthetic workloads for the ghost-gluon Dyson-Schwinger solver.

This module only *describes inputs*: problem sizes, physical parameters, the
seeded family of boundary conditions and seeded coefficient perturbations.  It
holds none of the method's arithmetic, so the oracle tests, the GPU tests and
the benchmark can all draw their inputs from it.

The paper's workloads are parameter and grid sizes, not a dataset (Sec. 5,
Table 1: 36/60/96 Chebyshev polynomials and 32/64/128 radial nodes per
interval; Sec. 2: eps^2, Lambda^2, Z(x_Z), alpha(mu^2)).  The configurations
below use the same physics on the grids of the five benchmark shapes.

z_lambda_inv values.  The paper pairs alpha(mu^2) = 1 with Z(5e4 GeV^2) = 0.256
(Sec. 2.1).  That pair matches one-loop running, alpha(x) = alpha(mu^2) /
(1 + omega ln(x/mu^2)) with omega = 11 N_c alpha(mu^2) / (12 pi), with
Z = (alpha(x)/alpha(mu^2))^{13/22} at mu^2 = 1.64915 GeV^2.  The same scale
gives the Z(Lambda^2) used for the cutoffs below: 0.223179 at 1e6 and 0.189535
at 1e8.  A CPU test recomputes both numbers.
"""
from __future__ import annotations

import numpy as np

#: Z(Lambda^2) at the two cutoffs (see the module docstring)
Z_LAMBDA_1E6 = 0.223179
Z_LAMBDA_1E8 = 0.189535

CONFIGS = {
    # 1: small correctness configuration, scaling solution (G(0)^{-1} = 0)
    "cfg1": dict(n_z=16, n_g=16, n_rad=64, n_ir=16, n_ang=16, eps2=1e-6, lambda2=1e6,
                 ir_efolds=40.0, alpha_mu=1.0, n_c=3.0, g0_inv=0.0,
                 z_lambda_inv=1.0 / Z_LAMBDA_1E6),
    # 2: paper-scale plain solve: 64 coefficients per function, decoupling G(0) = 15
    "cfg2": dict(n_z=64, n_g=64, n_rad=256, n_ir=64, n_ang=64, eps2=1e-8, lambda2=1e8,
                 ir_efolds=40.0, alpha_mu=1.0, n_c=3.0, g0_inv=1.0 / 15.0,
                 z_lambda_inv=1.0 / Z_LAMBDA_1E8),
    # 3: large assembly: 128 coefficients per function, 1024 (+256 IR) x 128 quadrature
    "cfg3": dict(n_z=128, n_g=128, n_rad=1024, n_ir=256, n_ang=128, eps2=1e-8, lambda2=1e8,
                 ir_efolds=40.0, alpha_mu=1.0, n_c=3.0, g0_inv=1.0 / 15.0,
                 z_lambda_inv=1.0 / Z_LAMBDA_1E8),
    # the paper's own physics (Sec. 2.1): Lambda^2 = 5e4 GeV^2, eps^2 = 1e-6 GeV^2,
    # Z(Lambda^2) = 0.256, alpha(mu^2) = 1, scaling solution; 24 coefficients per
    # function on a 96+24 x 24 grid (the renormalisation scale, alpha(M_Z^2) and
    # the Schwinger function are evaluated on its solution)
    "paper": dict(n_z=24, n_g=24, n_rad=96, n_ir=24, n_ang=24, eps2=1e-6, lambda2=5e4,
                  ir_efolds=40.0, alpha_mu=1.0, n_c=3.0, g0_inv=0.0, z_lambda_inv=1.0 / 0.256),
    # 5: adjoint configuration (same physics and grid as 2)
    "cfg5": dict(n_z=64, n_g=64, n_rad=256, n_ir=64, n_ang=64, eps2=1e-8, lambda2=1e8,
                 ir_efolds=40.0, alpha_mu=1.0, n_c=3.0, g0_inv=1.0 / 15.0,
                 z_lambda_inv=1.0 / Z_LAMBDA_1E8),
}

WORKLOAD_NAMES = {
    "cfg1": "ghost-gluon DSE, N=16 per function, 64+16 radial x 16 angular, scaling",
    "cfg2": "ghost-gluon DSE, N=64 per function, 256+64 radial x 64 angular, G(0)=15",
    "cfg3": "ghost-gluon DSE, N=128 per function, 1024+256 radial x 128 angular, G(0)=15",
    "cfg4": "ghost-gluon DSE family, 256 solves, N in {32,48,64}, 256+64 x 64, G(0) in [5,50]",
    "cfg5": "ghost-gluon DSE adjoint, N=64, 256+64 x 64, G(0)=15",
    "paper": "ghost-gluon DSE at the paper's parameters, N=24, 96+24 x 24, Lambda^2=5e4, scaling",
}

#: Schwinger function workload (Sec. 2.2, Table 2): 2^17 mapped Gauss-Legendre
#: nodes over p in [0, P], Euclidean times t = 0.02 k GeV^-1, k < 1024
SCHWINGER = dict(n_nodes=1 << 17, p_max=1.0e3, n_t=1024, dt=0.02)


def schwinger_times(n_t: int = SCHWINGER["n_t"], dt: float = SCHWINGER["dt"]) -> np.ndarray:
    """Euclidean times t_k = k dt (GeV^-1), k < n_t."""
    return dt * np.arange(n_t)


def config(name: str, **overrides) -> dict:
    """A copy of a named configuration with optional overrides."""
    d = dict(CONFIGS[name])
    d.update(overrides)
    return d


def family(count: int = 256, seed: int = 1206) -> list[dict]:
    """Batched family: decoupling boundary values G(0) log-uniform in [5, 50] and
    Chebyshev orders drawn from {32, 48, 64} per function, on the grid of cfg2.
    Draw order: G(0) for all members, then N_Z, then N_G."""
    rng = np.random.default_rng(seed)
    g0 = np.exp(rng.uniform(np.log(5.0), np.log(50.0), count))
    nz = rng.choice([32, 48, 64], count)
    ng = rng.choice([32, 48, 64], count)
    base = CONFIGS["cfg2"]
    out = []
    for i in range(count):
        d = dict(base)
        d.update(n_z=int(nz[i]), n_g=int(ng[i]), g0_inv=1.0 / float(g0[i]))
        out.append(d)
    return out


def adjoint_loss_points(m: int = 64) -> np.ndarray:
    """Momenta p_m^2 = 10^{-4 + 8 m/63}, m < 64, log-spaced on [1e-4, 1e4]."""
    return 10.0 ** (-4.0 + 8.0 * np.arange(m) / (m - 1))


def perturbation(n_z: int, n_g: int, scale: float, seed: int) -> np.ndarray:
    """Seeded Gaussian perturbation of c = [a; b], each half decaying with the
    Chebyshev index j like 1/(1+j) (the coefficients of a smooth function)."""
    rng = np.random.default_rng(seed)
    da = rng.standard_normal(n_z) / (1.0 + np.arange(n_z))
    db = rng.standard_normal(n_g) / (1.0 + np.arange(n_g))
    return scale * np.concatenate([da, db])


def near_singular_matrices() -> list:
    """Dense systems on both sides of the LU's singularity test (a pivot at or
    below n eps times the largest |entry| of its row): (name, A, b, singular).
    The right-hand sides are 1, 2, ..., n scaled like the rows of A."""
    u = 2.0 ** -52
    rng = np.random.default_rng(5)
    G = rng.standard_normal((6, 6)) + 4 * np.eye(6)
    R = rng.integers(-4, 5, size=(5, 5)).astype(float)
    R[2] = R[0] + R[1]  # rank deficient in real arithmetic
    cases = [("one_ulp", np.array([[1.0, 1.0], [1.0, 1.0 + u]]), True),
             ("one_ulp_row_scaled", np.array([[1e12, 1e12], [1.0, 1.0 + u]]), True),
             ("eight_ulp", np.array([[1.0, 1.0], [1.0, 1.0 + 8 * u]]), False),
             ("row_scaled_well_conditioned", np.diag([1e-150, 1e-75, 1.0, 1e75, 1e150, 1.0]) @ G, False),
             ("rank_deficient_integers", R, True)]
    return [(name, A, np.arange(1.0, A.shape[0] + 1) * np.max(np.abs(A), axis=1), sing)
            for name, A, sing in cases]

