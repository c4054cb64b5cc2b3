"""Dense numpy renderings of the paper's global formulas and building blocks.

TEST INFRASTRUCTURE ONLY (see the package docstring). Small chains only: every
quantity is built as an explicit 6n x 6n (or n x n) matrix so that each formula
can be compared with the paper by eye. Written independently of the C oracle
(its own Lie-group helpers), so agreement between the two pins both.

Conventions are those stated in ``fd_oracle.c``.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


# ---------- Lie-group helpers (Sec. II-A) ----------

def skew(v):
    return np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])


def rot(axis, q):
    k = skew(axis)
    return np.eye(3) + np.sin(q) * k + (1.0 - np.cos(q)) * (k @ k)


def ad_pose(r, p):
    """Ad_T = [[R, 0], [[p]R, R]]."""
    m = np.zeros((6, 6))
    m[:3, :3] = r
    m[3:, 3:] = r
    m[3:, :3] = skew(p) @ r
    return m


def ad_twist(v):
    """ad_V = [[[w], 0], [[v], [w]]]."""
    m = np.zeros((6, 6))
    m[:3, :3] = skew(v[:3])
    m[3:, 3:] = skew(v[:3])
    m[3:, :3] = skew(v[3:])
    return m


def inertia6(mass, com, inertia):
    ic = np.array([[inertia[0], inertia[3], inertia[4]],
                   [inertia[3], inertia[1], inertia[5]],
                   [inertia[4], inertia[5], inertia[2]]])
    c = skew(com)
    j = np.zeros((6, 6))
    j[:3, :3] = ic - mass * c @ c
    j[:3, 3:] = mass * c
    j[3:, :3] = -mass * c
    j[3:, 3:] = mass * np.eye(3)
    return j


class Chain:
    """One chain's parameters (slices of a robot set) and a joint configuration."""

    def __init__(self, robots, start, n):
        sl = slice(start, start + n)
        self.n = n
        self.axis = robots.axis[sl]
        self.home = robots.home_rot[sl].reshape(n, 3, 3)
        self.offset = robots.offset[sl]
        self.mass = robots.mass[sl]
        self.com = robots.com[sl]
        self.inertia = robots.inertia[sl]
        self.gravity = np.asarray(robots.gravity, dtype=np.float64)
        par = getattr(robots, "parent", None)
        self.parent = np.arange(n) - 1 if par is None else np.asarray(par[sl], dtype=np.int64)

    def pose(self, i, q):
        """T_{p(i),i} = (Rhome_i Rot(axis_i, q_i), offset_i), p(i) = i - 1 on a serial chain."""
        return self.home[i] @ rot(self.axis[i], q), self.offset[i]

    def ad_link(self, i, q):
        """Ad_i = Ad(T_{p(i),i}^-1): the (i, p(i)) block of Gamma."""
        r, p = self.pose(i, q)
        return ad_pose(r.T, -r.T @ p)

    def screw(self, i):
        return np.concatenate([self.axis[i], np.zeros(3)])


def global_matrices(ch: Chain, q):
    """Gamma (6n x 6n, block lower), S (6n x n), J (6n x 6n) of eq. (EOM-full).

    On a serial chain Gamma's blocks sit at (i, i - 1); on a tree at (i, p(i)),
    the parent of link i (the paper treats chains only; this is the tree reading).
    """
    n = ch.n
    gam = np.zeros((6 * n, 6 * n))
    s = np.zeros((6 * n, n))
    j = np.zeros((6 * n, 6 * n))
    for i in range(n):
        p = ch.parent[i]
        if p >= 0:
            gam[6 * i:6 * i + 6, 6 * p:6 * p + 6] = ch.ad_link(i, q[i])
        s[6 * i:6 * i + 6, i] = ch.screw(i)
        j[6 * i:6 * i + 6, 6 * i:6 * i + 6] = inertia6(ch.mass[i], ch.com[i], ch.inertia[i])
    return gam, s, j


def joint_inertia(ch: Chain, q):
    """M = S^T (I - Gamma)^-T J (I - Gamma)^-1 S (Sec. II-C)."""
    gam, s, j = global_matrices(ch, q)
    x = np.linalg.solve(np.eye(6 * ch.n) - gam, s)
    return x.T @ j @ x


def bias_torque(ch: Chain, q, qd, qdd=None, gravity=True):
    """tau of eq. (EOM-full) in global matrix form (qdd = 0 gives tau_bias).

    V = (I-Gamma)^-1 S qd; Vdot = (I-Gamma)^-1 (S qdd + [ad_{V_i}(S_i qd_i)] + base term);
    F = (I-Gamma)^-T (J Vdot - [ad_{V_i}^T J_i V_i]); tau = S^T F.
    """
    n = ch.n
    gam, s, j = global_matrices(ch, q)
    ig = np.eye(6 * n) - gam
    v = np.linalg.solve(ig, s @ qd)
    rhs = s @ (np.zeros(n) if qdd is None else qdd)
    for i in range(n):
        vi = v[6 * i:6 * i + 6]
        rhs[6 * i:6 * i + 6] += ad_twist(vi) @ (ch.screw(i) * qd[i])
    if gravity:                        # the base acceleration enters every link hung from the base
        a0 = np.concatenate([np.zeros(3), -ch.gravity])
        for i in np.flatnonzero(ch.parent < 0):
            rhs[6 * i:6 * i + 6] += ch.ad_link(i, q[i]) @ a0
    a = np.linalg.solve(ig, rhs)
    f = j @ a
    for i in range(n):
        vi = v[6 * i:6 * i + 6]
        f[6 * i:6 * i + 6] -= ad_twist(vi).T @ (j[6 * i:6 * i + 6, 6 * i:6 * i + 6] @ vi)
    force = np.linalg.solve(ig.T, f)
    return s.T @ force


# ---------- block bi-diagonal systems: the scan (Sec. II-B) ----------

def scan_serial(b, c, reverse=False):
    """x_i = B_i x_{i-1} + c_i (x_{-1} = 0); reverse: x_i = B_i x_{i+1} + c_i (x_n = 0).

    b: [n, d, d], c: [n, d]. This is the recurrence itself, one step at a time.
    """
    n = len(c)
    x = np.zeros_like(c)
    prev = np.zeros(c.shape[1:])
    order = range(n - 1, -1, -1) if reverse else range(n)
    for i in order:
        prev = b[i] @ prev + c[i]
        x[i] = prev
    return x


def scan_homogeneous(b, c, reverse=False):
    """Inclusive prefix of homogeneous elements a_i = [[B_i, c_i], [0, 1]] under
    a_{i-1} (+) a_i = a_i a_{i-1} (Sec. II-B); x_i is the last column of the prefix.
    Evaluated with a balanced tree (Hillis-Steele doubling)."""
    n, d = c.shape
    a = np.zeros((n, d + 1, d + 1))
    a[:, :d, :d] = b
    a[:, :d, d] = c
    a[:, d, d] = 1.0
    if reverse:
        a = a[::-1].copy()
    a[0, :d, :d] = np.eye(d)          # x_{-1} = 0 makes B_0 irrelevant
    step = 1
    while step < n:
        nxt = a.copy()
        for i in range(step, n):
            nxt[i] = a[i] @ a[i - step]
        a = nxt
        step *= 2
    x = a[:, :d, d]
    return x[::-1].copy() if reverse else x


# ---------- block tri-diagonal systems: odd-even elimination (Sec. IV) ----------

def btd_assemble(d, u):
    """Dense symmetric block tri-diagonal matrix with diagonal D_i and upper U_i (eq. (A_mat))."""
    n, k = d.shape[0], d.shape[1]
    a = np.zeros((n * k, n * k))
    for i in range(n):
        a[k * i:k * i + k, k * i:k * i + k] = d[i]
        if i + 1 < n:
            a[k * i:k * i + k, k * (i + 1):k * (i + 2)] = u[i]
            a[k * (i + 1):k * (i + 2), k * i:k * i + k] = u[i].T
    return a


def btd_solve_dense(d, u, r):
    """The definition: x = A^-1 r with A assembled densely (Cholesky, LAPACK)."""
    a = btd_assemble(d, u)
    x = sla.cho_solve(sla.cho_factor(a, lower=True), r.reshape(-1))
    return x.reshape(r.shape)


def oee_solve(d, u, r, record=None):
    """Odd-even elimination (Sec. IV, Algorithm 2), every row reading level j-1 values.

    At level j (stride s = 2^(j-1)), row i uses E_i = U_i D_{i+s}^-1 and
    K_i = U_{i-s}^T D_{i-s}^-1 (both by SPD solves) to remove its couplings:
      D_i <- D_i - E_i U_i^T - K_i U_{i-s};  R_i <- R_i - E_i R_{i+s} - K_i R_{i-s};
      U_i <- -E_i U_{i+s}.
    After ceil(log2 n) levels the matrix is block diagonal: x_i = D_i^-1 R_i.
    ``record`` (a list) receives the diagonal blocks of every level.
    """
    d = np.array(d, dtype=np.float64)
    u = np.array(u, dtype=np.float64)
    r = np.array(r, dtype=np.float64)
    n = d.shape[0]
    levels = int(np.ceil(np.log2(n))) if n > 1 else 0
    s = 1
    for _ in range(levels):
        nd, nu, nr = d.copy(), np.zeros_like(u), r.copy()
        for i in range(n):
            if i + s < n:
                e = sla.cho_solve(sla.cho_factor(d[i + s], lower=True), u[i].T).T
                nd[i] -= e @ u[i].T
                nr[i] -= e @ r[i + s]
                if i + 2 * s < n:
                    nu[i] = -e @ u[i + s]
            if i - s >= 0:
                kk = sla.cho_solve(sla.cho_factor(d[i - s], lower=True), u[i - s]).T
                nd[i] -= kk @ u[i - s]
                nr[i] -= kk @ r[i - s]
        d, u, r = nd, nu, nr
        if record is not None:
            record.append(d.copy())
        s *= 2
    return np.stack([sla.cho_solve(sla.cho_factor(d[i], lower=True), r[i]) for i in range(n)])


# ---------- the three factorisations of M^-1 ----------

def jsiia_qdd(ch: Chain, q, tau_delta):
    """JSIIA (Sec. II-C): column k of M is the inverse dynamics with qdd = e_k,
    qd = 0 and no gravity; then qdd = M^-1 tau_delta by a Cholesky solve."""
    n = ch.n
    zero = np.zeros(n)
    m = np.stack([bias_torque(ch, q, zero, np.eye(n)[k], gravity=False) for k in range(n)], axis=1)
    return sla.cho_solve(sla.cho_factor(m, lower=True), tau_delta), m


def abia_qdd(ch: Chain, q, tau_delta):
    """ABIA (Sec. II-C): articulated-body inertias by the nonlinear backward
    recursion, then the two linear (bi-diagonal) recursions, applied to
    tau_delta with zero velocity and no gravity. Returns qdd = M^-1 tau_delta.
    On a tree every link passes its terms to its parent p(i), where the
    children's terms add up (p(i) = i - 1 on a serial chain)."""
    n = ch.n
    par = ch.parent
    ad = [ch.ad_link(i, q[i]) for i in range(n)]
    s = [ch.screw(i) for i in range(n)]
    jhat = [inertia6(ch.mass[i], ch.com[i], ch.inertia[i]) for i in range(n)]
    p = [np.zeros(6) for _ in range(n)]  # bias wrench from the children of link i
    h = [None] * n
    dd = np.zeros(n)
    u = np.zeros(n)
    for i in range(n - 1, -1, -1):
        h[i] = jhat[i] @ s[i]
        dd[i] = s[i] @ h[i]
        pi = jhat[i] - np.outer(h[i], h[i]) / dd[i]
        u[i] = tau_delta[i] - s[i] @ p[i]
        if par[i] >= 0:
            jhat[par[i]] = jhat[par[i]] + ad[i].T @ pi @ ad[i]
            p[par[i]] = p[par[i]] + ad[i].T @ (p[i] + h[i] * u[i] / dd[i])
    qdd = np.zeros(n)
    acc = [None] * n
    for i in range(n):
        a = ad[i] @ acc[par[i]] if par[i] >= 0 else np.zeros(6)
        qdd[i] = (u[i] - h[i] @ a) / dd[i]
        acc[i] = a + s[i] * qdd[i]
    return qdd


def abia_scan_qdd(ch: Chain, q, tau_delta):
    """ABIA with its two linear recursions written as the bi-diagonal systems of
    Sec. II-C and solved by the scan of Sec. II-B (serial chains). After the
    articulated-inertia recursion (h_i, D_i), with Ad_i the (i, i-1) block of
    Gamma:
      backward  p_{i-1} = B_i p_i + c_i,  B_i = Ad_i^T (I - h_i S_i^T / D_i),
                c_i = Ad_i^T h_i tau_delta_i / D_i,  p_{n-1} = 0;
      forward   a_i = B'_i a_{i-1} + c'_i,  B'_i = (I - S_i h_i^T / D_i) Ad_i,
                c'_i = S_i u_i / D_i,  u_i = tau_delta_i - S_i^T p_i,  a_{-1} = 0;
      qdd_i = (u_i - h_i^T Ad_i a_{i-1}) / D_i.
    Each system is solved by scan_homogeneous (the all-prefix product of the
    homogeneous elements)."""
    n = ch.n
    assert all(ch.parent[i] == i - 1 for i in range(n)), "serial chains only"
    ad = [ch.ad_link(i, q[i]) for i in range(n)]
    s = [ch.screw(i) for i in range(n)]
    jhat = [inertia6(ch.mass[i], ch.com[i], ch.inertia[i]) for i in range(n)]
    h, dd = [None] * n, np.zeros(n)
    for i in range(n - 1, -1, -1):
        h[i] = jhat[i] @ s[i]
        dd[i] = s[i] @ h[i]
        if i > 0:
            jhat[i - 1] = jhat[i - 1] + ad[i].T @ (jhat[i] - np.outer(h[i], h[i]) / dd[i]) @ ad[i]
    # backward system: element k of the reversed sequence carries link n-1-k's map into p_{n-2-k}
    bb = np.stack([ad[i].T @ (np.eye(6) - np.outer(h[i], s[i]) / dd[i]) for i in range(n)])
    cc = np.stack([ad[i].T @ h[i] * tau_delta[i] / dd[i] for i in range(n)])
    incl = scan_homogeneous(bb, cc, reverse=True)       # incl[i] = E_i(E_{i+1}(... E_{n-1}(0)))
    p = [incl[i + 1] if i + 1 < n else np.zeros(6) for i in range(n)]
    u = np.array([tau_delta[i] - s[i] @ p[i] for i in range(n)])
    bf = np.stack([(np.eye(6) - np.outer(s[i], h[i]) / dd[i]) @ ad[i] for i in range(n)])
    cf = np.stack([s[i] * u[i] / dd[i] for i in range(n)])
    acc = scan_homogeneous(bf, cf)                      # acc[i] = a_i
    qdd = np.zeros(n)
    for i in range(n):
        a_prev = acc[i - 1] if i > 0 else np.zeros(6)
        qdd[i] = (u[i] - h[i] @ (ad[i] @ a_prev)) / dd[i]
    return qdd


def constraint_basis(s):
    """W_i: an orthonormal basis (6 x 5) of the complement of S_i (W_i^T S_i = 0)."""
    _, _, vt = np.linalg.svd(s.reshape(1, 6))
    return vt[1:].T


def cfa_matrices(ch: Chain, q):
    """Phi = (I-Gamma) J^-1 (I-Gamma)^T, W, and A = W^T Phi W, B = W^T Phi S,
    C = S^T Phi S of eq. (cfa-eq2) and (fijany-final)."""
    n = ch.n
    gam, s, j = global_matrices(ch, q)
    ig = np.eye(6 * n) - gam
    phi = ig @ np.linalg.inv(j) @ ig.T
    w = np.zeros((6 * n, 5 * n))
    for i in range(n):
        w[6 * i:6 * i + 6, 5 * i:5 * i + 5] = constraint_basis(ch.screw(i))
    return phi, w, s, w.T @ phi @ w, w.T @ phi @ s, s.T @ phi @ s


def cfa_qdd(ch: Chain, q, tau_delta):
    """CFA (Sec. III): F_c = -A^-1 B tau_delta, qdd = C tau_delta + B^T F_c."""
    _, _, _, a, b, c = cfa_matrices(ch, q)
    fc = -np.linalg.solve(a, b @ tau_delta)
    return c @ tau_delta + b.T @ fc


def cfa_proj_qdd(ch: Chain, q, tau_delta):
    """The CFA without a basis W (Sec. III, with the choice of W that Sec. VI
    leaves open replaced by projectors): P = diag(I - S_i S_i^T / |S_i|^2) and
    A^ = P Phi P + S S^T (6n x 6n), X = A^-1 (-P Phi S tau_delta), F = S tau_delta + X,
    qdd = S^T Phi F. Returns (qdd, X)."""
    phi, _, s, _, _, _ = cfa_matrices(ch, q)
    n = ch.n
    proj = np.eye(6 * n)
    for i in range(n):
        si = s[6 * i:6 * i + 6, i]
        proj[6 * i:6 * i + 6, 6 * i:6 * i + 6] -= np.outer(si, si) / (si @ si)
    ahat = proj @ phi @ proj + s @ s.T
    x = np.linalg.solve(ahat, -proj @ phi @ s @ tau_delta)
    f = s @ tau_delta + x
    return s.T @ phi @ f, x


def cfa_c_matrix(ch: Chain, q):
    """C = S^T Phi S (n x n, tri-diagonal) from the blocks of Phi:
    Phi_ii = J_i^-1 + Ad_i J_{i-1}^-1 Ad_i^T, Phi_{i,i+1} = -J_i^-1 Ad_{i+1}^T.
    ||C|| ||M|| bounds the cancellation in qdd = (C - B^T A^-1 B) tau_delta."""
    n = ch.n
    jinv = [np.linalg.inv(inertia6(ch.mass[i], ch.com[i], ch.inertia[i])) for i in range(n)]
    ad = [ch.ad_link(i, q[i]) for i in range(n)]
    s = [ch.screw(i) for i in range(n)]
    c = np.zeros((n, n))
    for i in range(n):
        phi = jinv[i] + (ad[i] @ jinv[i - 1] @ ad[i].T if i > 0 else 0.0)
        c[i, i] = s[i] @ phi @ s[i]
        if i + 1 < n:
            c[i, i + 1] = c[i + 1, i] = s[i] @ (-jinv[i] @ ad[i + 1].T) @ s[i + 1]
    return c
