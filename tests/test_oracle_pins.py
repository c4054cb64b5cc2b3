"""Pins of the CPU oracle to facts other than itself (no GPU).

Each test checks the oracle against something the paper or the mathematics
fixes: closed forms (simple and planar double pendulum), conservation laws
(power balance), the Lagrangian form of the bias, the paper's global matrix
formulas (built densely and independently), library routines (LAPACK
Cholesky) and brute force. A dropped term, a wrong sign, index or transposed
operand anywhere in the oracle fails at least one of them.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import dense
from paper_1609_06779_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _single(axis, com, inertia6, mass, home=None, offset=(0, 0, 0), gravity=(0, 0, -9.81)):
    return synth.Robots(
        n_links=np.array([1], np.int32), axis=np.array([axis], float),
        home_rot=np.array([np.eye(3).reshape(9) if home is None else np.asarray(home).reshape(9)]),
        offset=np.array([offset], float), mass=np.array([mass], float), com=np.array([com], float),
        inertia=np.array([inertia6], float), gravity=np.array(gravity, float))


# ---------------- P1: Lie-group primitives ----------------

def test_rodrigues_rotation_sense_and_orthonormality():
    # +q about z takes x to (cos q, sin q, 0) (right-hand rule)
    for q in (0.0, 0.3, -1.2, 2.9):
        r = oracle.link_rotation([0, 0, 1], np.eye(3).reshape(9), q)
        np.testing.assert_allclose(r @ [1, 0, 0], [np.cos(q), np.sin(q), 0], atol=1e-15)
    rng = np.random.default_rng(0)
    for _ in range(10):
        w = rng.standard_normal(3)
        w /= np.linalg.norm(w)
        q = rng.uniform(-np.pi, np.pi)
        r = oracle.link_rotation(w, np.eye(3).reshape(9), q)
        np.testing.assert_allclose(r @ r.T, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(r) - 1) < 1e-14
        np.testing.assert_allclose(r @ w, w, atol=1e-15)          # axis is fixed
        # angle: for v perpendicular to w, v . Rv = cos q |v|^2
        v = np.cross(w, [1.0, 0.0, 0.0])
        assert abs(v @ r @ v - np.cos(q) * (v @ v)) < 1e-14
    np.testing.assert_allclose(oracle.link_rotation([0.6, 0.8, 0], np.eye(3).reshape(9), 0.0), np.eye(3), atol=0)


def _rand_pose(rng):
    w = rng.standard_normal(3)
    w /= np.linalg.norm(w)
    return oracle.link_rotation(w, np.eye(3).reshape(9), rng.uniform(-3, 3)), rng.standard_normal(3)


def test_adjoint_is_a_homomorphism():
    rng = np.random.default_rng(1)
    for _ in range(10):
        r1, p1 = _rand_pose(rng)
        r2, p2 = _rand_pose(rng)
        r12, p12 = r1 @ r2, r1 @ p2 + p1
        np.testing.assert_allclose(oracle.adjoint(r12, p12),
                                   oracle.adjoint(r1, p1) @ oracle.adjoint(r2, p2), atol=1e-13)
        np.testing.assert_allclose(oracle.adjoint(r1, p1, inverse=True) @ oracle.adjoint(r1, p1),
                                   np.eye(6), atol=1e-13)


def test_adjoint_maps_point_velocities():
    # a twist V = (w; v) moves the point x with velocity v + w x x; Ad_T expresses
    # the same motion in the parent frame: check through one point.
    rng = np.random.default_rng(2)
    r, p = _rand_pose(rng)
    v6 = rng.standard_normal(6)
    x = rng.standard_normal(3)                       # point in child coordinates
    vel_child = v6[3:] + np.cross(v6[:3], x)
    vp = oracle.adjoint(r, p) @ v6
    xp = r @ x + p
    np.testing.assert_allclose(vp[3:] + np.cross(vp[:3], xp), r @ vel_child, atol=1e-13)


def test_spatial_inertia_matches_kinetic_energy():
    rng = np.random.default_rng(3)
    for _ in range(5):
        m = rng.uniform(0.5, 2)
        c = rng.uniform(-0.1, 0.1, 3)
        a = rng.standard_normal((3, 3))
        ic = a @ a.T + np.eye(3) * 0.1
        i6 = [ic[0, 0], ic[1, 1], ic[2, 2], ic[0, 1], ic[0, 2], ic[1, 2]]
        j = oracle.spatial_inertia(m, c, i6)
        v6 = rng.standard_normal(6)
        w, v = v6[:3], v6[3:]
        vc = v + np.cross(w, c)                      # velocity of the centre of mass
        ke = 0.5 * m * vc @ vc + 0.5 * w @ ic @ w
        assert abs(0.5 * v6 @ j @ v6 - ke) < 1e-13 * max(1, ke)
        assert np.all(np.linalg.eigvalsh(j) > 0)


# ---------------- P2: single pendulum ----------------

def test_simple_pendulum_golden():
    data = json.load(open(os.path.join(GOLDEN, "pendulum.json")))
    g = data["g"]
    for c in data["cases"]:
        rb = _single([0, 1, 0], [0, 0, -c["l"]], [1e-12] * 3 + [0] * 3, c["m"], gravity=(0, 0, -g))
        qdd = oracle.fd(rb, [c["q"]], [c["qd"]], [c["tau"]])
        assert abs(qdd[0] - c["qdd"]) <= 1e-10 * max(1.0, abs(c["qdd"]))


def test_single_link_closed_form_random():
    # (w^T (Ic - m[c]^2) w) qdd = tau + m w . ((Rot(w, q) c) x g); no velocity term
    rng = np.random.default_rng(4)
    rb = synth.make_robots([1] * 20, seed=11)
    for k in range(20):
        w, c, m = rb.axis[k], rb.com[k], rb.mass[k]
        i6 = rb.inertia[k]
        ic = np.array([[i6[0], i6[3], i6[4]], [i6[3], i6[1], i6[5]], [i6[4], i6[5], i6[2]]])
        one = _single(w, c, i6, m)
        q, qd, tau = rng.uniform(-3, 3), rng.uniform(-2, 2), rng.standard_normal()
        r = dense.rot(w, q)
        sc = dense.skew(c)
        expected = (tau + m * w @ np.cross(r @ c, [0, 0, -9.81])) / (w @ (ic - m * sc @ sc) @ w)
        got = oracle.fd(one, [q], [qd], [tau])[0]
        assert abs(got - expected) <= 1e-12 * max(1, abs(expected))


# ---------------- P3: planar double pendulum (Euler-Lagrange closed form) ----------------

def test_planar_double_pendulum_closed_form():
    g = 9.81
    m1, m2, l1, lc1, lc2, i1, i2 = 1.3, 0.7, 0.9, 0.4, 0.35, 0.05, 0.02
    rb = synth.Robots(
        n_links=np.array([2], np.int32), axis=np.array([[0, 0, 1.0], [0, 0, 1.0]]),
        home_rot=np.tile(np.eye(3).reshape(9), (2, 1)), offset=np.array([[0, 0, 0.0], [l1, 0, 0]]),
        mass=np.array([m1, m2]), com=np.array([[lc1, 0, 0.0], [lc2, 0, 0]]),
        inertia=np.array([[0.03, 0.04, i1, 0, 0, 0], [0.01, 0.02, i2, 0, 0, 0]]),
        gravity=np.array([0, -g, 0.0]))
    rng = np.random.default_rng(5)
    for _ in range(10):
        q1, q2 = rng.uniform(-3, 3, 2)
        d1, d2 = rng.uniform(-2, 2, 2)
        tau = rng.standard_normal(2)
        c2 = np.cos(q2)
        m = np.array([[m1 * lc1 ** 2 + m2 * (l1 ** 2 + lc2 ** 2 + 2 * l1 * lc2 * c2) + i1 + i2,
                       m2 * (lc2 ** 2 + l1 * lc2 * c2) + i2],
                      [m2 * (lc2 ** 2 + l1 * lc2 * c2) + i2, m2 * lc2 ** 2 + i2]])
        h = m2 * l1 * lc2 * np.sin(q2)
        bias = np.array([
            -h * (2 * d1 * d2 + d2 ** 2) + (m1 * lc1 + m2 * l1) * g * np.cos(q1) + m2 * lc2 * g * np.cos(q1 + q2),
            h * d1 ** 2 + m2 * lc2 * g * np.cos(q1 + q2)])
        np.testing.assert_allclose(oracle.crba(rb, [q1, q2])[0], m, rtol=1e-13, atol=1e-14)
        np.testing.assert_allclose(oracle.rnea(rb, [q1, q2], [d1, d2]), bias, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(oracle.fd(rb, [q1, q2], [d1, d2], tau), np.linalg.solve(m, tau - bias),
                                   rtol=1e-11, atol=1e-11)


# ---------------- P4: power balance ----------------

@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_power_balance(n):
    """dE/dt = qd . tau along the motion qdd = FD(q, qd, tau) (no dissipation)."""
    rb = synth.make_robots([n] * 6, seed=21, random_home=True)
    q, qd, tau = synth.make_state([n] * 6, seed=21)
    off = rb.offsets
    qdd = oracle.fd(rb, q, qd, tau)
    h = 1e-6
    kp, pp = oracle.energy(rb, q + h * qd, qd + h * qdd)
    km, pm = oracle.energy(rb, q - h * qd, qd - h * qdd)
    edot = (kp + pp - km - pm) / (2 * h)
    power = np.add.reduceat(qd * tau, off[:-1])
    scale = np.add.reduceat(np.abs(qd * tau) + np.abs(qd * (tau - qdd)), off[:-1]) + 1.0
    assert np.all(np.abs(edot - power) <= 2e-7 * scale), (edot, power)


def test_free_motion_conserves_energy_rk4():
    rb = synth.make_robots([4], seed=22)
    q, qd, _ = synth.make_state([4], seed=22)
    zero = np.zeros(4)

    def f(x):
        return np.concatenate([x[4:], oracle.fd(rb, x[:4], x[4:], zero)])

    x = np.concatenate([q, qd])
    e0 = sum(oracle.energy(rb, x[:4], x[4:]))
    dt = 1e-3
    for _ in range(200):
        k1 = f(x)
        k2 = f(x + dt / 2 * k1)
        k3 = f(x + dt / 2 * k2)
        k4 = f(x + dt * k3)
        x = x + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    e1 = sum(oracle.energy(rb, x[:4], x[4:]))
    assert abs(e1 - e0) < 1e-9 * max(1, abs(e0))


# ---------------- P5: Lagrangian form of the bias ----------------

@pytest.mark.parametrize("n", [2, 4, 6])
def test_bias_matches_lagrangian(n):
    """tau_bias = Mdot qd - 1/2 d/dq (qd^T M qd) + dP/dq, with M and P differentiated numerically."""
    rb = synth.make_robots([n], seed=31 + n, random_home=True)
    q, qd, _ = synth.make_state([n], seed=31 + n)
    h = 1e-6
    dm = []
    dp = np.zeros(n)
    for k in range(n):
        e = np.zeros(n)
        e[k] = h
        dm.append((oracle.crba(rb, q + e)[0] - oracle.crba(rb, q - e)[0]) / (2 * h))
        dp[k] = (oracle.energy(rb, q + e, qd)[1][0] - oracle.energy(rb, q - e, qd)[1][0]) / (2 * h)
    mdot = sum(dm[k] * qd[k] for k in range(n))
    grad_ke = np.array([0.5 * qd @ dm[k] @ qd for k in range(n)])
    expected = mdot @ qd - grad_ke + dp
    got = oracle.rnea(rb, q, qd)
    np.testing.assert_allclose(got, expected, rtol=0, atol=1e-7 * (1 + np.abs(expected).max()))


# ---------------- P6: the joint-space inertia ----------------

@pytest.mark.parametrize("n", [1, 2, 3, 6])
def test_joint_inertia_equals_global_formula(n):
    rb = synth.make_robots([n] * 4, seed=41, random_home=True)
    q, qd, _ = synth.make_state([n] * 4, seed=41)
    off = rb.offsets
    ms = oracle.crba(rb, q)
    ke, _ = oracle.energy(rb, q, qd)
    for b in range(4):
        sl = slice(off[b], off[b + 1])
        ch = dense.Chain(rb, off[b], n)
        md = dense.joint_inertia(ch, q[sl])
        np.testing.assert_allclose(ms[b], md, rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(ms[b], ms[b].T, atol=0)
        assert np.all(np.linalg.eigvalsh(ms[b]) > 0)
        assert abs(0.5 * qd[sl] @ ms[b] @ qd[sl] - ke[b]) <= 1e-13 * max(1, ke[b])


def test_joint_inertia_columns_are_unit_acceleration_inverse_dynamics():
    n = 7
    rb = synth.make_robots([n], seed=42)
    q, _, _ = synth.make_state([n], seed=42)
    m = oracle.crba(rb, q)[0]
    zero = np.zeros(n)
    for k in range(n):
        col = oracle.rnea(rb, q, zero, np.eye(n)[k], gravity=False)
        np.testing.assert_allclose(col, m[:, k], rtol=1e-12, atol=1e-13)


# ---------------- P7 and the bias in global matrix form ----------------

@pytest.mark.parametrize("n", [1, 3, 6])
def test_bias_equals_global_formula(n):
    rb = synth.make_robots([n] * 3, seed=51, random_home=True)
    q, qd, _ = synth.make_state([n] * 3, seed=51)
    off = rb.offsets
    bias = oracle.rnea(rb, q, qd)
    for b in range(3):
        sl = slice(off[b], off[b + 1])
        bd = dense.bias_torque(dense.Chain(rb, off[b], n), q[sl], qd[sl])
        np.testing.assert_allclose(bias[sl], bd, rtol=1e-12, atol=1e-12)


def test_round_trip_inverse_of_forward():
    lengths = np.array([1, 2, 8, 16, 33])
    rb = synth.make_robots(lengths, seed=61)
    q, qd, tau = synth.make_state(lengths, seed=61)
    qdd = oracle.fd(rb, q, qd, tau)
    back = oracle.rnea(rb, q, qd, qdd)
    np.testing.assert_allclose(back, tau, rtol=0, atol=1e-10 * (1 + np.abs(tau).max()))


def test_gravity_has_no_effect_when_axes_are_vertical():
    n = 6
    rb = synth.make_robots([n], seed=71)
    rb.axis[:] = [0, 0, 1.0]
    q, qd, tau = synth.make_state([n], seed=71)
    a = oracle.fd(rb, q, qd, tau)
    rb.gravity = np.array([0, 0, 0.0])
    b = oracle.fd(rb, q, qd, tau)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12)


# ---------------- the three factorisations (brute force on tiny chains) ----------------

@pytest.mark.parametrize("n", [1, 2, 3, 4, 6])
def test_three_factorisations_agree_with_oracle(n):
    rb = synth.make_robots([n] * 3, seed=81, random_home=True)
    q, qd, tau = synth.make_state([n] * 3, seed=81)
    off = rb.offsets
    qdd = oracle.fd(rb, q, qd, tau)
    bias = oracle.rnea(rb, q, qd)
    for b in range(3):
        sl = slice(off[b], off[b + 1])
        ch = dense.Chain(rb, off[b], n)
        td = tau[sl] - bias[sl]
        scale = 1e-11 * (1 + np.abs(qdd[sl]).max())
        np.testing.assert_allclose(dense.jsiia_qdd(ch, q[sl], td)[0], qdd[sl], atol=scale, rtol=0)
        np.testing.assert_allclose(dense.abia_qdd(ch, q[sl], td), qdd[sl], atol=scale, rtol=0)
        np.testing.assert_allclose(dense.cfa_qdd(ch, q[sl], td), qdd[sl], atol=scale, rtol=0)


@pytest.mark.parametrize("n", [1, 2, 5])
def test_cfa_schur_complement_and_force_consistency(n):
    rb = synth.make_robots([n], seed=91, random_home=True)
    q, qd, tau = synth.make_state([n], seed=91)
    ch = dense.Chain(rb, 0, n)
    phi, w, s, a, b, c = dense.cfa_matrices(ch, q)
    m = oracle.crba(rb, q)[0]
    minv = c - b.T @ np.linalg.solve(a, b)
    np.testing.assert_allclose(minv, np.linalg.inv(m), rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(w.T @ s, 0, atol=1e-15)
    # F = S tau_delta + W F_c satisfies Phi F = S qdd (eq. (cfa-eq0))
    td = tau - oracle.rnea(rb, q, qd)
    fc = -np.linalg.solve(a, b @ td)
    f = s @ td + w @ fc
    qdd = oracle.fd(rb, q, qd, tau)
    np.testing.assert_allclose(phi @ f, s @ qdd, rtol=0, atol=1e-10 * (1 + np.abs(qdd).max()))
    if n == 1:
        j = dense.inertia6(ch.mass[0], ch.com[0], ch.inertia[0])
        sv = ch.screw(0)
        assert abs(minv[0, 0] - 1.0 / (sv @ j @ sv)) < 1e-12 / (sv @ j @ sv)


@pytest.mark.parametrize("n", [2, 5])
def test_cfa_result_does_not_depend_on_the_constraint_basis(n):
    """Sec. III: W only has to span the complement of S at every joint (W^T S = 0,
    full column rank); the paper leaves other choices open. Any such W_i' = W_i Q_i
    (Q_i invertible, 5 x 5, not orthogonal here) turns A into Q^T A Q and B into
    Q^T B, so M^-1 = C - B^T A^-1 B and qdd are unchanged. The kernels take the
    canonical W_i = [e1 e2 e4 e5 e6] of their joint frames; the oracle's dense
    form takes an SVD basis; this is the statement that both are the same CFA."""
    rb = synth.make_robots([n], seed=93, random_home=True)
    q, qd, tau = synth.make_state([n], seed=93)
    ch = dense.Chain(rb, 0, n)
    phi, w, s, a, b, c = dense.cfa_matrices(ch, q)
    rng = np.random.default_rng(n)
    qb = np.zeros((5 * n, 5 * n))
    for i in range(n):
        qb[5 * i:5 * i + 5, 5 * i:5 * i + 5] = rng.standard_normal((5, 5)) + 3.0 * np.eye(5)
    w2 = w @ qb
    np.testing.assert_allclose(w2.T @ s, 0, atol=1e-13)
    a2, b2 = w2.T @ phi @ w2, w2.T @ phi @ s
    minv1 = c - b.T @ np.linalg.solve(a, b)
    minv2 = c - b2.T @ np.linalg.solve(a2, b2)
    np.testing.assert_allclose(minv2, minv1, rtol=1e-9, atol=1e-10)
    td = tau - oracle.rnea(rb, q, qd)
    np.testing.assert_allclose(minv2 @ td, oracle.fd(rb, q, qd, tau), rtol=1e-9, atol=1e-9)
    # and a W that is not a complement (it has a component along S) changes the result
    w3 = w.copy()
    w3[:, 0] += s[:, 0]
    a3, b3 = w3.T @ phi @ w3, w3.T @ phi @ s
    assert np.abs(c - b3.T @ np.linalg.solve(a3, b3) - minv1).max() > 1e-6


@pytest.mark.parametrize("n", [1, 2, 3, 6])
def test_cfa_projector_form_equals_the_definition(n):
    """The basis-free constraint system A^ = P Phi P + S S^T (projectors in place of
    W) gives the oracle's qdd, its solution X has no component along any S_i, and
    X = W F_c with F_c = -A^-1 B tau_delta of the W-form (x^T A^ x = a^T A a + |b|^2
    for x = W a + S b)."""
    rb = synth.make_robots([n], seed=95, random_home=True)
    q, qd, tau = synth.make_state([n], seed=95)
    ch = dense.Chain(rb, 0, n)
    td = tau - oracle.rnea(rb, q, qd)
    qdd, x = dense.cfa_proj_qdd(ch, q, td)
    np.testing.assert_allclose(qdd, oracle.fd(rb, q, qd, tau), rtol=1e-9, atol=1e-9)
    _, w, s, a, b, _ = dense.cfa_matrices(ch, q)
    np.testing.assert_allclose(s.T @ x, 0, atol=1e-12 * max(1.0, np.abs(x).max()))
    fc = -np.linalg.solve(a, b @ td)
    np.testing.assert_allclose(x, w @ fc, rtol=1e-9, atol=1e-10 * max(1.0, np.abs(x).max()))


def test_cfa_projector_form_needs_the_s_block():
    """Without the S S^T term the projected system P Phi P is singular (its null
    space holds every S_i): the term is what makes it solvable, not a regulariser
    that changes the answer."""
    n = 3
    rb = synth.make_robots([n], seed=96)
    q, _, _ = synth.make_state([n], seed=96)
    ch = dense.Chain(rb, 0, n)
    phi, _, s, _, _, _ = dense.cfa_matrices(ch, q)
    proj = np.eye(6 * n)
    for i in range(n):
        si = s[6 * i:6 * i + 6, i]
        proj[6 * i:6 * i + 6, 6 * i:6 * i + 6] -= np.outer(si, si) / (si @ si)
    ev = np.linalg.eigvalsh(proj @ phi @ proj)
    assert np.sum(np.abs(ev) < 1e-12 * ev.max()) == n
    assert np.linalg.eigvalsh(proj @ phi @ proj + s @ s.T).min() > 0


@pytest.mark.parametrize("n", [1, 2, 7, 16])
def test_abia_by_scans_equals_the_definition(n):
    """The ABIA's two bi-diagonal systems solved by the scan (Sec. II-B, II-C):
    the backward elements (Ad^T (I - h S^T / D), Ad^T h tau_delta / D) and the
    forward ones ((I - S h^T / D) Ad, S u / D) give the oracle's q-ddot."""
    rb = synth.make_robots([n], seed=97, random_home=True)
    q, qd, tau = synth.make_state([n], seed=97)
    ch = dense.Chain(rb, 0, n)
    td = tau - oracle.rnea(rb, q, qd)
    ref = oracle.fd(rb, q, qd, tau)
    np.testing.assert_allclose(dense.abia_scan_qdd(ch, q, td), ref, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(dense.abia_scan_qdd(ch, q, td), dense.abia_qdd(ch, q, td), rtol=1e-10, atol=1e-10)


def test_abia_single_link_is_axis_inertia():
    rb = synth.make_robots([1], seed=92)
    ch = dense.Chain(rb, 0, 1)
    j = dense.inertia6(ch.mass[0], ch.com[0], ch.inertia[0])
    sv = ch.screw(0)
    assert abs(dense.abia_qdd(ch, [0.4], [1.7])[0] - 1.7 / (sv @ j @ sv)) < 1e-13


# ---------------- P9: odd-even elimination ----------------

@pytest.mark.parametrize("k", [5, 6])
def test_oee_matches_dense_cholesky(k):
    lengths = list(range(1, 18))
    d, u, r = synth.make_btd(lengths, k=k, seed=100 + k)
    off = synth.offsets_of(lengths)
    for b, n in enumerate(lengths):
        sl = slice(off[b], off[b + 1])
        rec = []
        x = dense.oee_solve(d[sl], u[sl], r[sl], record=rec)
        ref = dense.btd_solve_dense(d[sl], u[sl], r[sl])
        np.testing.assert_allclose(x, ref, rtol=1e-11, atol=1e-11)
        assert len(rec) == (int(np.ceil(np.log2(n))) if n > 1 else 0)
        for level in rec:                      # every level's diagonal blocks stay SPD
            for blk in level:
                np.testing.assert_allclose(blk, blk.T, atol=1e-12)
                assert np.linalg.eigvalsh(blk).min() > 0


# ---------------- P10: the scan ----------------

@pytest.mark.parametrize("reverse", [False, True])
def test_scan_tree_equals_serial_recurrence(reverse):
    for n in (1, 2, 3, 7, 16, 33):
        b, c = synth.make_scan_elements([n], seed=200 + n)
        np.testing.assert_allclose(dense.scan_homogeneous(b, c, reverse), dense.scan_serial(b, c, reverse),
                                   rtol=1e-12, atol=1e-12)


def test_scan_serial_is_the_bidiagonal_solve():
    n, dd = 9, 6
    b, c = synth.make_scan_elements([n], seed=300)
    big = np.eye(n * dd)
    for i in range(1, n):
        big[dd * i:dd * i + dd, dd * (i - 1):dd * i] = -b[i]
    x = np.linalg.solve(big, c.reshape(-1)).reshape(n, dd)
    np.testing.assert_allclose(dense.scan_serial(b, c), x, rtol=1e-12, atol=1e-12)


# ---------------- derivatives (complex step) ----------------

def test_fd_jvp_matches_central_differences():
    lengths = [1, 4, 9]
    rb = synth.make_robots(lengths, seed=401, random_home=True)
    q, qd, tau = synth.make_state(lengths, seed=401)
    rng = np.random.default_rng(401)
    v = [rng.standard_normal(len(q)) for _ in range(3)]
    qdd, dqdd = oracle.fd_jvp(rb, q, qd, tau, *v)
    np.testing.assert_allclose(qdd, oracle.fd(rb, q, qd, tau), rtol=0, atol=1e-13 * (1 + np.abs(qdd).max()))
    h = 1e-6
    fp = oracle.fd(rb, q + h * v[0], qd + h * v[1], tau + h * v[2])
    fm = oracle.fd(rb, q - h * v[0], qd - h * v[1], tau - h * v[2])
    np.testing.assert_allclose(dqdd, (fp - fm) / (2 * h), rtol=0, atol=1e-7 * np.abs(dqdd).max())


def test_rnea_jvp_along_acceleration_is_the_joint_inertia():
    lengths = [2, 7]
    rb = synth.make_robots(lengths, seed=402, random_home=True)
    q, qd, tau = synth.make_state(lengths, seed=402)
    qdd = oracle.fd(rb, q, qd, tau)
    a = np.random.default_rng(402).standard_normal(len(q))
    z = np.zeros(len(q))
    dt = oracle.rnea_jvp(rb, q, qd, qdd, z, z, a)
    off = rb.offsets
    for b, m in enumerate(oracle.crba(rb, q)):
        np.testing.assert_allclose(dt[off[b]:off[b + 1]], m @ a[off[b]:off[b + 1]], rtol=1e-12, atol=1e-12)


def test_fd_jvp_along_torque_is_the_inverse_inertia():
    lengths = [5]
    rb = synth.make_robots(lengths, seed=403)
    q, qd, tau = synth.make_state(lengths, seed=403)
    v = np.random.default_rng(403).standard_normal(5)
    z = np.zeros(5)
    _, dqdd = oracle.fd_jvp(rb, q, qd, tau, z, z, v)
    np.testing.assert_allclose(dqdd, np.linalg.solve(oracle.crba(rb, q)[0], v), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 6])
def test_cfa_c_matrix_equals_the_global_form(n):
    """C = S^T Phi S assembled from Phi's blocks (dense.cfa_c_matrix, and the
    batched copy the GPU tests use for their diagnostics) equals the C of the
    global matrices, Phi = (I - Gamma) J^-1 (I - Gamma)^T built as 6n x 6n
    (Sec. III, eq. (fijany-final)). A slip in a block (a sign, an index, a
    transposed Ad) changes C."""
    import _errmodel

    lengths = [n] * 4
    rb = synth.make_robots(lengths, seed=93, random_home=True)
    q, _, _ = synth.make_state(lengths, seed=93)
    batched = _errmodel.cfa_c_batched(rb, q, n, np.arange(4))
    for b in range(4):
        ch = dense.Chain(rb, b * n, n)
        ref = dense.cfa_matrices(ch, q[b * n:(b + 1) * n])[5]
        scale = np.abs(ref).max()
        np.testing.assert_allclose(dense.cfa_c_matrix(ch, q[b * n:(b + 1) * n]), ref, rtol=0, atol=1e-12 * scale)
        np.testing.assert_allclose(batched[b], ref, rtol=0, atol=1e-12 * scale)
        assert np.count_nonzero(np.abs(ref) > 1e-14 * scale) <= 3 * n - 2     # tri-diagonal


def test_cfa_c_matrix_catches_a_planted_sign_error():
    """The pin above is sharp: flipping the sign of the coupling block
    Phi_{i,i+1} changes C by far more than the pin's bar."""
    n = 4
    rb = synth.make_robots([n], seed=94, random_home=True)
    q, _, _ = synth.make_state([n], seed=94)
    ch = dense.Chain(rb, 0, n)
    ref = dense.cfa_matrices(ch, q)[5]
    bad = dense.cfa_c_matrix(ch, q).copy()
    bad[np.arange(n - 1), np.arange(1, n)] *= -1
    bad[np.arange(1, n), np.arange(n - 1)] *= -1
    assert np.abs(bad - ref).max() > 1e-3 * np.abs(ref).max()
