"""Error-model diagnostics for the parity tests (test infrastructure, numpy only).

The parity bars themselves are fixed numbers (``CAP``); these helpers only
explain a chain's error when a test reports one: cond_2(M) for every
factorisation, and for the CFA the size of C = S^T Phi S, since its
M^-1 = C - B^T A^-1 B (eq. (fijany-final)) is a difference of terms of size
||C|| (Sec. III).
"""
from __future__ import annotations

import numpy as np

import oracle

# One cap per precision on every forward and reverse-mode parity bar: the
# tolerance of the forward-dynamics target (1e-10 FP64, 1e-4 FP32), times 10.
# A chain between the target and the cap passes the test but is counted, and
# every test reports how many of its chains meet the target itself.
TARGET = {"f64": 1e-10, "f32": 1e-4}
CAP = {"f64": 1e-9, "f32": 1e-3}
U = {"f64": 2.0 ** -53, "f32": 2.0 ** -24}


def skew_rows(v):
    """Cross-product matrices of the rows of v: (k, 3) -> (k, 3, 3)."""
    z = np.zeros(len(v))
    return np.stack([np.stack([z, -v[:, 2], v[:, 1]], -1), np.stack([v[:, 2], z, -v[:, 0]], -1),
                     np.stack([-v[:, 1], v[:, 0], z], -1)], 1)


def cfa_c_batched(rb, q, n, chains):
    """C = S^T Phi S (tri-diagonal n x n) of the chains `chains` of a uniform
    batch of n-link robots, all at once: Phi_ii = J_i^-1 + Ad_i J_{i-1}^-1 Ad_i^T,
    Phi_{i,i+1} = -J_i^-1 Ad_{i+1}^T with Ad_i = Ad(T_{i-1,i}^-1). [len(chains), n, n]."""
    b = len(chains)
    jinv, ad, s = [], [], []
    for i in range(n):
        li = chains * n + i
        m = rb.mass[li][:, None, None]
        it = rb.inertia[li]
        ic = np.stack([np.stack([it[:, 0], it[:, 3], it[:, 4]], -1), np.stack([it[:, 3], it[:, 1], it[:, 5]], -1),
                       np.stack([it[:, 4], it[:, 5], it[:, 2]], -1)], 1)
        c = skew_rows(rb.com[li])
        j = np.zeros((b, 6, 6))
        j[:, :3, :3] = ic - m * (c @ c)
        j[:, :3, 3:] = m * c
        j[:, 3:, :3] = -m * c
        j[:, 3:, 3:] = m * np.eye(3)
        jinv.append(np.linalg.inv(j))
        kx = skew_rows(rb.axis[li])
        qq = q[li][:, None, None]
        r = rb.home_rot[li].reshape(b, 3, 3) @ (np.eye(3) + np.sin(qq) * kx + (1.0 - np.cos(qq)) * (kx @ kx))
        rt = r.transpose(0, 2, 1)
        pt = -(rt @ rb.offset[li][:, :, None])[:, :, 0]
        x = np.zeros((b, 6, 6))                  # Ad(T^-1) = ad_pose(R^T, -R^T p)
        x[:, :3, :3] = rt
        x[:, 3:, 3:] = rt
        x[:, 3:, :3] = skew_rows(pt) @ rt
        ad.append(x)
        s.append(np.concatenate([rb.axis[li], np.zeros((b, 3))], 1))
    cm = np.zeros((b, n, n))
    for i in range(n):
        phi = jinv[i] + (ad[i] @ jinv[i - 1] @ ad[i].transpose(0, 2, 1) if i > 0 else 0.0)
        cm[:, i, i] = np.einsum("bi,bij,bj->b", s[i], phi, s[i])
        if i + 1 < n:
            cm[:, i, i + 1] = cm[:, i + 1, i] = np.einsum("bi,bij,bj->b", s[i],
                                                           -jinv[i] @ ad[i + 1].transpose(0, 2, 1), s[i + 1])
    return cm


def kappa(algo, rb, q, n, chains, chunk=1024):
    """The error-model factor of each listed chain of a uniform batch: cond_2(M),
    or for the CFA ||C||_2 ||M||_2. Diagnostics only; no bar is derived from it."""
    out = []
    for k0 in range(0, len(chains), chunk):
        ch = np.asarray(chains[k0:k0 + chunk])
        idx = (ch[:, None] * n + np.arange(n)).reshape(-1)
        ms = np.stack(oracle.crba(rb.take(ch), q[idx]))
        ev = np.linalg.eigvalsh(ms)
        if algo != "cfa":
            out.append(ev[:, -1] / ev[:, 0])
        else:
            out.append(np.abs(np.linalg.eigvalsh(cfa_c_batched(rb, q, n, ch))).max(axis=1) * ev[:, -1])
    return np.concatenate(out) if out else np.zeros(0)
