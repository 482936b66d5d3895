"""Pins of the oracle's compressible Neo-Hookean law (the paper's material in
its inverse-analysis example, Sec. 4.5): tau = mu (b - 1) + lambda ln J 1.
Checked against closed forms (uniaxial strain, the self-weight column),
its small-strain limit (linear elasticity), objectivity and the symmetry of
a hyperelastic stiffness.  None compares the oracle with itself."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import oracle as O
from paper_2507_09435_amd import workloads as W


def _homogeneous_stress(G, E=1e6, nu=0.3):
    """Kirchhoff stress of a 3-D particle under the homogeneous increment
    du_i = (G - 1) x_i (reproduced exactly by the B-splines, so dF = G)."""
    P = W.Problem(dim=3, n=(4, 4, 4), h=0.25, E=E, nu=nu, elastic=1, g=(0.0, 0.0, 0.0))
    st = W.identity_state(3, np.array([[0.41], [0.52], [0.47]]), P.h, 8)
    idx = P.node_grid_index()
    X = np.stack([P.x0[k] + idx[k] * P.h for k in range(3)], axis=1)
    dof = X @ (np.asarray(G) - np.eye(3)).T
    tau, reg = O.stress(P, st, dof)
    return tau[0]


def _lame(E, nu):
    return E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))


@pytest.mark.parametrize("stretch", [0.6, 0.9, 1.2])
def test_uniaxial_strain_closed_form(stretch):
    E, nu = 1e6, 0.3
    lam, mu = _lame(E, nu)
    tau = _homogeneous_stress(np.diag([1.0, stretch, 1.0]), E, nu)
    assert abs(tau[1, 1] - (mu * (stretch ** 2 - 1) + lam * math.log(stretch))) < 1e-9 * E
    assert abs(tau[0, 0] - lam * math.log(stretch)) < 1e-9 * E
    assert abs(tau[2, 2] - tau[0, 0]) < 1e-9 * E
    assert np.abs(tau - np.diag(np.diag(tau))).max() < 1e-9 * E


def test_small_strain_limit_is_linear_elasticity():
    E, nu = 1e6, 0.3
    lam, mu = _lame(E, nu)
    rng = np.random.default_rng(3)
    for _ in range(5):
        A = rng.normal(size=(3, 3)) * 1e-5
        eps = 0.5 * (A + A.T)
        tau = _homogeneous_stress(np.eye(3) + eps, E, nu)
        lin = lam * np.trace(eps) * np.eye(3) + 2 * mu * eps
        assert np.abs(tau - lin).max() < 1e-4 * np.abs(lin).max()


def test_objectivity_under_rotation():
    E, nu = 1e6, 0.3
    rng = np.random.default_rng(4)
    G = np.eye(3) + rng.normal(size=(3, 3)) * 0.1
    t = 0.7
    R = np.array([[math.cos(t), -math.sin(t), 0], [math.sin(t), math.cos(t), 0], [0, 0, 1]])
    a = _homogeneous_stress(G, E, nu)
    b = _homogeneous_stress(R @ G, E, nu)
    np.testing.assert_allclose(b, R @ a @ R.T, atol=1e-8 * E)


def test_hyperelastic_stiffness_is_symmetric():
    """J = d f_int / d du is the Hessian of sum V0 psi(dF F^n): symmetric at
    any state, here a deformed plane-strain block (dense dual Jacobian)."""
    P = W.Problem(dim=2, n=(4, 4, 0), h=0.25, E=1e6, nu=0.3, elastic=1)
    x = W.gauss_particles(2, P.h, (0.0, 0.0), (1, 1), (3, 3))
    st = W.identity_state(2, x, P.h, 4)
    rng = np.random.default_rng(5)
    dof = rng.normal(size=(P.n_nodes, 2)) * 0.02 * P.h
    Jd = O.dense_jacobian(P, st, dof)
    assert np.linalg.norm(Jd - Jd.T) <= 1e-13 * np.linalg.norm(Jd)


def test_neohookean_bar_height_closed_form():
    """The self-weight column of Sec. 4.2's geometry with the Neo-Hookean law
    (nu = 0, so lambda = 0) and E = 50 kPa (the paper's 10 kPa compresses the
    base of a Neo-Hookean column below a tenth of its height, finer than
    these cells resolve): tau_yy = mu (s^2 - 1) = -s rho0 g (l0 - Y0) for the
    vertical stretch s, so s = (-q + sqrt(q^2 + 4 mu^2)) / (2 mu) with
    q = rho0 g (l0 - Y0); the final height is the integral of s."""
    w = W.bar_column(n_cells=32, n_steps=20, E=5e4)
    w.prob.elastic = 1
    mu = w.prob.E / 2
    st = w.particles
    for k in range(1, 21):
        Pk = W.with_gravity(w.prob, k / 20)
        bc = w.bc(k)
        dof, rep, _ = O.newton(Pk, st, bc.mask, bc.value, tol=1e-11)
        assert rep.converged and rep.iters <= 6
        st = O.update(Pk, st, dof)
    s = lambda y: (lambda q: (-q + math.sqrt(q * q + 4 * mu * mu)) / (2 * mu))(80.0 * 9.81 * (50.0 - y))
    Y0 = w.particles.x[1]
    ref = np.array([quad(s, 0.0, y, epsabs=1e-12)[0] for y in Y0])
    H = quad(s, 0.0, 50.0, epsabs=1e-12)[0]
    assert 30.0 < H < 40.0
    assert np.abs(st.x[1] - ref).max() < 0.01 * 50.0   # discretization error, as the Hencky column pin
