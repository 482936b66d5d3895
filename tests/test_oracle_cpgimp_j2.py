"""Pins of the oracle's cpGIMP weights, its J2 return and the paper's
elastoplastic bar (Sec. 4.2) against what mathematics fixes: quadrature of
the defining integral, partition of unity and linear reproduction, the von
Mises surface, and the closed-form uniaxial-strain solution of a Hencky-J2
column under its own weight.  None compares the oracle with itself."""
import ctypes as C
import json
import math
import os

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.optimize import brentq

from oracle import oracle as O
from paper_2507_09435_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def gimp(u, o, l):
    w, dw = np.zeros(3), np.zeros(3)
    O.lib().orc_gimp(float(u), int(o), float(l), w.ctypes.data, dw.ctypes.data)
    return w, dw


def _cases(n=200, seed=5):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        u = rng.uniform(-0.5, 20.0)
        l = rng.uniform(0.02, 0.5)
        yield u, int(math.floor(u - 0.5)), l


# -------------------------------------------------------------- cpGIMP -----
def test_gimp_weight_is_the_hat_averaged_over_the_particle_domain():
    """Definition: w_a = (1/2l) * integral over [u-l, u+l] of the linear hat
    of node o+a (in cell units), evaluated by adaptive quadrature."""
    hat = lambda y, node: max(0.0, 1.0 - abs(y - node))
    for u, o, l in _cases(60):
        w, _ = gimp(u, o, l)
        for a in range(3):
            node = o + a
            ref = quad(lambda y: hat(y, node), u - l, u + l, points=[node - 1, node, node + 1], epsabs=1e-14)[0]
            assert abs(w[a] - ref / (2 * l)) < 1e-12, (u, l, a, w[a], ref / (2 * l))


def test_gimp_partition_of_unity_and_linear_reproduction():
    for u, o, l in _cases():
        w, dw = gimp(u, o, l)
        assert abs(w.sum() - 1.0) < 1e-14
        assert abs((w * (o + np.arange(3))).sum() - u) < 1e-12
        assert abs(dw.sum()) < 1e-13
        assert abs((dw * (o + np.arange(3))).sum() - 1.0) < 1e-12


def test_gimp_derivative_matches_central_differences():
    for u, o, l in _cases(80, seed=6):
        _, dw = gimp(u, o, l)
        h = 1e-6
        wp, _ = gimp(u + h, o, l)
        wm, _ = gimp(u - h, o, l)
        np.testing.assert_allclose(dw, (wp - wm) / (2 * h), atol=1e-7)


def test_gimp_reduces_to_the_linear_hat_for_a_point_domain():
    for u, o, _ in _cases(40, seed=7):
        w, _ = gimp(u, o, 1e-9)
        ref = np.maximum(0.0, 1.0 - np.abs(u - (o + np.arange(3))))
        np.testing.assert_allclose(w, ref, atol=1e-8)


def test_gimp_domain_follows_the_axis_stretch():
    """cpGIMP convects the domain: with F_yy = 1/2 the half-width along y is
    lp0 / 2, along x it stays lp0."""
    P = W.Problem(dim=2, n=(4, 4, 0), h=0.25, shape=1, lp0=(0.0625, 0.0625, 0.0))
    st = W.identity_state(2, np.array([[0.41], [0.63]]), P.h, 4)
    st.F[3] = 0.5
    dof = np.zeros((P.n_nodes, 2))
    # the weights enter f_ext = sum_a w_a m g: compare with the 1-D products
    _, fext = O.forces(P, st, dof)
    o = O.origins(P, st)
    wx, _ = gimp(0.41 / 0.25, o[0, 0], 0.25)
    wy, _ = gimp(0.63 / 0.25, o[1, 0], 0.125)
    ny = P.n[0] + 3
    m = P.rho0 * st.vol0[0]
    for a in range(3):
        for b in range(3):
            node = (o[0, 0] + a + 1) + ny * (o[1, 0] + b + 1)
            assert abs(fext[node, 1] - wx[a] * wy[b] * m * P.g[1]) < 1e-12 * m * 9.81


# ------------------------------------------------------------------ J2 -----
def _j2_cfg(E=1e4, kappa=5e3):
    return O.cfg(W.Problem(dim=2, n=(4, 4, 0), h=0.25, dp=1, dp_match=3, E=E, nu=0.0, c=kappa))


def _return(cfg, E, eps):
    tau, ee = np.zeros(9), np.zeros(9)
    reg = O.lib().orc_return_map(C.byref(cfg), E, 0.0, np.ascontiguousarray(eps.reshape(9)).ctypes.data,
                                 tau.ctypes.data, ee.ctypes.data)
    return reg, tau.reshape(3, 3), ee.reshape(3, 3)


def test_j2_return_lands_on_the_von_mises_surface():
    """sqrt(2 J2) = kappa after a plastic return, the mean stress and the
    deviator's direction are those of the trial state (radial return), and
    the elastic strain follows from the returned stress by Hooke's law."""
    E, nu, kappa = 1e4, 0.0, 5e3
    G, K = E / (2 * (1 + nu)), E / (3 * (1 - 2 * nu))
    cfg = _j2_cfg(E, kappa)
    rng = np.random.default_rng(11)
    n_pl = 0
    for _ in range(200):
        A = rng.normal(size=(3, 3)) * 0.5
        eps = 0.5 * (A + A.T)
        lam = K - 2 * G / 3
        tr = lam * np.trace(eps) * np.eye(3) + 2 * G * eps
        s_tr = tr - np.trace(tr) / 3 * np.eye(3)
        q_tr = math.sqrt((s_tr * s_tr).sum())
        reg, tau, ee = _return(cfg, E, eps)
        p = np.trace(tau) / 3
        s = tau - p * np.eye(3)
        if q_tr <= kappa:
            assert reg == 0
            np.testing.assert_allclose(tau, tr, atol=1e-9 * kappa)
            continue
        n_pl += 1
        assert reg == 1
        assert abs(math.sqrt((s * s).sum()) - kappa) < 1e-10 * kappa
        assert abs(p - np.trace(tr) / 3) < 1e-10 * kappa
        np.testing.assert_allclose(s, s_tr * (kappa / q_tr), atol=1e-10 * kappa)
        np.testing.assert_allclose(ee, s / (2 * G) + p / (3 * K) * np.eye(3), atol=1e-12)
    assert n_pl > 50


def test_j2_uniaxial_strain_yield_point():
    """Uniaxial strain eps = diag(0, e, 0) with nu = 0: elastic while
    (4G/3)|e| < sqrt(2/3) kappa; beyond it the axial stress is
    tau_yy = (E/3) e - sqrt(2/3) kappa (the plastic branch of the bar's
    closed form, G = E/2)."""
    E, kappa = 1e4, 5e3
    cfg = _j2_cfg(E, kappa)
    G = E / 2
    e_y = -math.sqrt(2 / 3) * kappa * 3 / (4 * G)
    for e in (0.5 * e_y, 0.99 * e_y):
        reg, tau, _ = _return(cfg, E, np.diag([0.0, e, 0.0]))
        assert reg == 0 and abs(tau[1, 1] - E * e) < 1e-9 * kappa and abs(tau[0, 0]) < 1e-9 * kappa
    for e in (1.01 * e_y, 2.0 * e_y, 4.0 * e_y):
        reg, tau, _ = _return(cfg, E, np.diag([0.0, e, 0.0]))
        assert reg == 1
        assert abs(tau[1, 1] - (E / 3 * e - math.sqrt(2 / 3) * kappa)) < 1e-9 * kappa
        assert abs(tau[0, 0] - tau[2, 2]) < 1e-9 * kappa


# --------------------------------------------------- elastoplastic bar -----
def bar_stretch(Y0, E, kappa, rho0, l0, g=9.81):
    """Closed form of the confined Hencky (nu = 0) column under its own
    weight: the vertical Cauchy stress is exactly -rho0 g (l0 - Y0) (the
    weight above a material point), Kirchhoff tau_yy = lambda sigma_yy with
    the vertical stretch lambda; elastic tau_yy = E ln(lambda); on the J2
    branch tau_yy = (E/3) ln(lambda) - sqrt(2/3) kappa (uniaxial strain,
    plastic flow isochoric and deviatoric)."""
    q = rho0 * g * (l0 - Y0)
    if q <= 0.0:
        return 1.0
    lam_e = brentq(lambda L: E * math.log(L) + L * q, 1e-12, 1.0, xtol=1e-15)
    if kappa is None or (2 * E / 3) * abs(math.log(lam_e)) <= math.sqrt(2 / 3) * kappa:
        return lam_e
    return brentq(lambda L: (E / 3) * math.log(L) - math.sqrt(2 / 3) * kappa + L * q, 1e-300, 1.0, xtol=1e-15)


def bar_height(Y0, E, kappa, rho0, l0):
    return quad(lambda y: bar_stretch(y, E, kappa, rho0, l0), 0.0, Y0, limit=200, epsabs=1e-12)[0]


def run_bar(n_cells, kappa, cpgimp=True, steps=40):
    w = W.bar_column(n_cells=n_cells, j2_yield=kappa, cpgimp=cpgimp, n_steps=steps)
    st = w.particles
    its = []
    for k in range(1, steps + 1):
        Pk = W.with_gravity(w.prob, k / steps)
        bc = w.bc(k)
        dof, rep, _ = O.newton(Pk, st, bc.mask, bc.value, tol=1e-11, maxit=25)
        assert rep.converged, (k, rep)
        its.append(rep.iters)
        last = (Pk, st, dof)
        st = O.update(Pk, st, dof)
    return w, st, its, last


@pytest.mark.parametrize("kappa", [None, 5e3])
def test_bar_compaction_matches_the_closed_form(kappa):
    """Sec. 4.2 setup with the paper's shape functions: l0 = 50 m,
    rho0 = 80, E = 10 kPa, nu = 0, 64 cells, 256 particles, 40 load steps,
    and for the elastoplastic case J2 with kappa = 5 kPa.  The final height
    (24.23 m elastic, 22.14 m elastoplastic, both below 25 m as the paper
    reports) and every particle's height follow the closed form to within
    the discretization error, with at most four Newton iterations to 1e-11
    per step (the paper's figure; one more is allowed for where the
    plastic zone moves)."""
    g = json.load(open(GOLDEN))["bar_compaction"]
    l0, rho0, E = g["l0_m"], g["rho0_kg_m3"], g["E_Pa"]
    if kappa is not None:
        assert kappa == g["elastoplastic_yield_kappa_Pa"]
    w, st, its, _ = run_bar(64, kappa)
    H = bar_height(l0, E, kappa, rho0, l0)
    assert H < g["final_height_below_m"]
    assert abs(H - (24.233 if kappa is None else 22.139)) < 2e-3
    Y0 = w.particles.x[1]
    ref = np.array([bar_height(y, E, kappa, rho0, l0) for y in Y0])
    assert np.abs(st.x[1] - ref).max() < 0.005 * l0
    top = st.x[1].max() + 0.25 * l0 / 64 * np.mean(st.F[3][st.x[1] > st.x[1].max() - 1e-9])
    assert abs(top - H) < 0.01 * H
    assert max(its) <= g["newton_iterations_at_most"] + 1, its


def _stress_error(n_cells, kappa):
    """The paper's error measure: sum_p |sigma_yy,p - sigma_a,yy| V0 /
    (g rho0 l0 sum_p V0) with sigma_a,yy = -rho0 g (l0 - Y0)."""
    w, _, _, (Pk, st, dof) = run_bar(n_cells, kappa, steps=10)
    tau, _ = O.stress(Pk, st, dof)
    new = O.update(Pk, st, dof)
    J = np.linalg.det(new.F.T.reshape(-1, 2, 2))
    sig = tau[:, 1, 1] / J
    Y0 = w.particles.x[1]
    sa = -Pk.rho0 * 9.81 * (50.0 - Y0)
    v = w.particles.vol0
    return (np.abs(sig - sa) * v).sum() / (9.81 * Pk.rho0 * 50.0 * v.sum())


def test_elastoplastic_bar_stress_converges_at_rate_one_to_two():
    """Sec. 4.2 reports convergence rates between 1 and 2 under refinement
    (cells from 2^2 to 2^9) for both cases; here the J2 case on 8 to 64 cells,
    the rate being the least-squares slope of log(error) over log(1/h)
    (about 1.1; the plastic zone's edge makes single halvings vary)."""
    ns = np.array([8, 16, 32, 64])
    errs = np.array([_stress_error(int(n), 5e3) for n in ns])
    rate = np.polyfit(np.log(1.0 / ns), np.log(errs), 1)[0]   # error ~ h^rate
    assert 1.0 <= rate <= 2.0, (errs, rate)
