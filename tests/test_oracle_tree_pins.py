"""Pins of the oracle on branched robots (trees).

The paper treats serial chains. A tree hangs link i from a parent p(i) < i,
and Gamma of eq. (EOM-full) carries its block at (i, p(i)). These tests pin
the oracle's tree recursions:
- against serial chains: branches hung from the base are independent chains,
  and a link's pose is the pose at the tip of its root path;
- against the global matrix formulas with the tree's Gamma (``oracle.dense``,
  written separately);
- against mechanics: power balance, the Lagrangian form of the bias, and
  energy conservation in free motion.
"""
import numpy as np
import pytest

import oracle
from oracle import dense
from paper_1609_06779_amd import synth


def _tree(n, count=1, seed=0, p_extend=0.6, random_home=True):
    rb = synth.make_tree_robots([n] * count, p_extend=p_extend, seed=seed, random_home=random_home)
    q, qd, tau = synth.make_state([n] * count, seed=seed)
    return rb, q, qd, tau


def _related(par, i, k):
    """True when link i is link k or one of its ancestors."""
    while k >= 0:
        if k == i:
            return True
        k = par[k]
    return False


def test_generator_numbers_links_in_depth_first_preorder():
    par = synth.make_tree_parents([40] * 50, seed=3)
    for b in range(50):
        p = par[40 * b:40 * b + 40]
        assert p[0] == -1 and np.all(p < np.arange(40))
        for i in range(40):   # the subtree of i is a contiguous run starting at i
            sub = [k for k in range(40) if _related(p, i, k)]
            assert sub == list(range(i, i + len(sub)))
    assert np.any(par[1:] != np.arange(1, len(par)) - 1)     # really branched


def test_branches_hung_from_the_base_are_independent_chains():
    """Two chains merged into one tree in an interleaved order give the same
    qdd, tau and M (permuted) as the chains on their own."""
    chains = synth.make_robots([3, 4], seed=5, random_home=True)
    q, qd, tau = synth.make_state([3, 4], seed=5)
    order = [(0, 0), (1, 0), (1, 1), (0, 1), (1, 2), (0, 2), (1, 3)]   # (chain, link) in tree order
    off = chains.offsets
    src = np.array([off[c] + i for c, i in order])
    pos = {ci: t for t, ci in enumerate(order)}
    parent = np.array([-1 if i == 0 else pos[(c, i - 1)] for c, i in order], np.int32)
    tree = synth.Robots(n_links=np.array([7], np.int32), axis=chains.axis[src], home_rot=chains.home_rot[src],
                        offset=chains.offset[src], mass=chains.mass[src], com=chains.com[src],
                        inertia=chains.inertia[src], gravity=chains.gravity, parent=parent)
    qt, qdt, taut = q[src], qd[src], tau[src]
    np.testing.assert_allclose(oracle.fd(tree, qt, qdt, taut), oracle.fd(chains, q, qd, tau)[src],
                               rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(oracle.rnea(tree, qt, qdt), oracle.rnea(chains, q, qd)[src], rtol=1e-13, atol=1e-13)
    mt = oracle.crba(tree, qt)[0]
    mc = oracle.crba(chains, q)
    full = np.zeros((7, 7))
    full[:3, :3] = mc[0]
    full[3:, 3:] = mc[1]
    np.testing.assert_allclose(mt, full[np.ix_(src, src)], rtol=1e-13, atol=1e-14)


def test_link_pose_is_the_tip_of_its_root_path():
    rb, q, _, _ = _tree(12, seed=7)
    rot, pos = oracle.fk(rb, q)
    par = rb.parent
    for i in range(12):
        path = []
        k = i
        while k >= 0:
            path.append(k)
            k = par[k]
        path = path[::-1]
        sub = rb.take([0])
        sub = synth.Robots(n_links=np.array([len(path)], np.int32), axis=sub.axis[path],
                           home_rot=sub.home_rot[path], offset=sub.offset[path], mass=sub.mass[path],
                           com=sub.com[path], inertia=sub.inertia[path], gravity=sub.gravity)
        r2, p2 = oracle.fk(sub, q[path])
        np.testing.assert_allclose(rot[i], r2[-1], rtol=0, atol=1e-14)
        np.testing.assert_allclose(pos[i], p2[-1], rtol=0, atol=1e-14)


@pytest.mark.parametrize("n", [2, 5, 9])
def test_joint_inertia_equals_global_formula_on_trees(n):
    rb, q, qd, _ = _tree(n, count=4, seed=11 + n)
    off = rb.offsets
    ms = oracle.crba(rb, q)
    ke, _ = oracle.energy(rb, q, qd)
    for b in range(4):
        sl = slice(off[b], off[b + 1])
        md = dense.joint_inertia(dense.Chain(rb, off[b], n), q[sl])
        np.testing.assert_allclose(ms[b], md, rtol=1e-12, atol=1e-13)
        np.testing.assert_array_equal(ms[b], ms[b].T)
        assert np.all(np.linalg.eigvalsh(ms[b]) > 0)
        assert abs(0.5 * qd[sl] @ ms[b] @ qd[sl] - ke[b]) <= 1e-13 * max(1, ke[b])
        par = rb.parent[sl]
        for i in range(n):             # links on different branches do not couple
            for k in range(n):
                if not (_related(par, i, k) or _related(par, k, i)):
                    assert ms[b][i, k] == 0.0


@pytest.mark.parametrize("n", [3, 7])
def test_bias_equals_global_formula_on_trees(n):
    rb, q, qd, _ = _tree(n, count=3, seed=21 + n)
    off = rb.offsets
    bias = oracle.rnea(rb, q, qd)
    qdd = synth.make_state([n] * 3, seed=99)[2]
    tau = oracle.rnea(rb, q, qd, qdd)
    for b in range(3):
        sl = slice(off[b], off[b + 1])
        ch = dense.Chain(rb, off[b], n)
        np.testing.assert_allclose(bias[sl], dense.bias_torque(ch, q[sl], qd[sl]), rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(tau[sl], dense.bias_torque(ch, q[sl], qd[sl], qdd[sl]), rtol=1e-12, atol=1e-12)


def test_joint_inertia_columns_are_unit_acceleration_inverse_dynamics_on_trees():
    n = 8
    rb, q, _, _ = _tree(n, seed=31)
    m = oracle.crba(rb, q)[0]
    zero = np.zeros(n)
    for k in range(n):
        col = oracle.rnea(rb, q, zero, np.eye(n)[k], gravity=False)
        np.testing.assert_allclose(col, m[:, k], rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("n", [2, 6, 10])
def test_power_balance_on_trees(n):
    """dE/dt = qd . tau along qdd = FD(q, qd, tau)."""
    rb, q, qd, tau = _tree(n, count=6, seed=41 + n)
    off = rb.offsets
    qdd = oracle.fd(rb, q, qd, tau)
    h = 1e-6
    kp, pp = oracle.energy(rb, q + h * qd, qd + h * qdd)
    km, pm = oracle.energy(rb, q - h * qd, qd - h * qdd)
    edot = (kp + pp - km - pm) / (2 * h)
    power = np.add.reduceat(qd * tau, off[:-1])
    scale = np.add.reduceat(np.abs(qd * tau) + np.abs(qd * (tau - qdd)), off[:-1]) + 1.0
    assert np.all(np.abs(edot - power) <= 2e-7 * scale), (edot, power)


@pytest.mark.parametrize("n", [3, 6])
def test_bias_matches_lagrangian_on_trees(n):
    """tau_bias = Mdot qd - 1/2 d/dq (qd^T M qd) + dP/dq, M and P differentiated numerically."""
    rb, q, qd, _ = _tree(n, seed=51 + n)
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
    np.testing.assert_allclose(oracle.rnea(rb, q, qd), expected, rtol=0, atol=1e-7 * (1 + np.abs(expected).max()))


def test_free_motion_conserves_energy_on_a_tree():
    n = 5
    rb, q, qd, _ = _tree(n, seed=61)
    zero = np.zeros(n)

    def f(x):
        return np.concatenate([x[n:], oracle.fd(rb, x[:n], x[n:], zero)])

    x = np.concatenate([q, qd])
    e0 = sum(oracle.energy(rb, x[:n], x[n:]))
    dt = 1e-3
    for _ in range(200):
        k1 = f(x)
        k2 = f(x + dt / 2 * k1)
        k3 = f(x + dt / 2 * k2)
        k4 = f(x + dt * k3)
        x = x + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    assert abs(sum(oracle.energy(rb, x[:n], x[n:])) - e0) < 1e-9 * max(1, abs(e0))


@pytest.mark.parametrize("n", [4, 9])
def test_factorisations_agree_with_the_oracle_on_trees(n):
    """The articulated-body factorisation and the constraint-force formula of
    Sec. III, written with the tree's Gamma, give the oracle's qdd."""
    rb, q, qd, tau = _tree(n, count=3, seed=71 + n)
    off = rb.offsets
    ref = oracle.fd(rb, q, qd, tau)
    td = tau - oracle.rnea(rb, q, qd)
    for b in range(3):
        sl = slice(off[b], off[b + 1])
        ch = dense.Chain(rb, off[b], n)
        np.testing.assert_allclose(dense.abia_qdd(ch, q[sl], td[sl]), ref[sl], rtol=1e-10, atol=1e-10)
        np.testing.assert_allclose(dense.cfa_qdd(ch, q[sl], td[sl]), ref[sl], rtol=1e-9, atol=1e-9)
        np.testing.assert_allclose(dense.jsiia_qdd(ch, q[sl], td[sl])[0], ref[sl], rtol=1e-10, atol=1e-10)


def test_fd_jvp_on_trees_matches_central_differences():
    n = 7
    rb, q, qd, tau = _tree(n, count=2, seed=81)
    rng = np.random.default_rng(3)
    dq, dqd, dtau = (rng.standard_normal(2 * n) for _ in range(3))
    qdd, d = oracle.fd_jvp(rb, q, qd, tau, dq, dqd, dtau)
    np.testing.assert_array_equal(qdd, oracle.fd(rb, q, qd, tau))
    h = 1e-6
    fd = (oracle.fd(rb, q + h * dq, qd + h * dqd, tau + h * dtau)
          - oracle.fd(rb, q - h * dq, qd - h * dqd, tau - h * dtau)) / (2 * h)
    np.testing.assert_allclose(d, fd, rtol=1e-6, atol=1e-6 * (1 + np.abs(fd).max()))


def test_a_tree_of_one_branch_is_the_serial_chain():
    rb = synth.make_robots([9], seed=91, random_home=True)
    q, qd, tau = synth.make_state([9], seed=91)
    tree = rb.take([0])
    tree.parent = np.arange(9, dtype=np.int32) - 1
    np.testing.assert_array_equal(oracle.fd(tree, q, qd, tau), oracle.fd(rb, q, qd, tau))


def test_cfa_system_couples_siblings_on_trees():
    """On a tree, A = W^T (I - Gamma) J^-1 (I - Gamma)^T W has a nonzero block exactly
    where two joints share a link: joint and parent joint, and any two siblings
    (through their common parent's J^-1; the base has none). So the CFA's system
    is not block tri-diagonal on a tree, nor tree-structured."""
    n = 7
    # 0 - 1 - 2, and 3, 4 hang from 1 (siblings of 2); 5 hangs from the base; 6 from 5
    parent = np.array([-1, 0, 1, 1, 1, -1, 5], np.int32)
    rb = synth.make_robots([n], seed=8, random_home=True)
    rb.parent = parent
    q = synth.make_state([n], seed=8)[0]
    _, _, _, a, _, _ = dense.cfa_matrices(dense.Chain(rb, 0, n), q)
    for i in range(n):
        for k in range(n):
            block = a[5 * i:5 * i + 5, 5 * k:5 * k + 5]
            share = i == k or parent[i] == k or parent[k] == i or (parent[i] == parent[k] >= 0)
            if share:
                assert np.abs(block).max() > 1e-6, (i, k)
            else:
                assert np.abs(block).max() < 1e-12, (i, k)
