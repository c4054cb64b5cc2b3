"""Seeded synthetic robots and joint states for batched forward dynamics.

This module only draws random numbers and packs them into arrays. It holds
none of the dynamics arithmetic, so both the HIP path and the CPU oracle can
take their inputs from it.

The paper initialises robot parameters (twists) and joint inputs at random
(Sec. V, experiment setup). The distributions below make that concrete:

* joint axis ``axis``: a normalised N(0, I3) draw, expressed in link frame i;
* link offset ``offset`` (origin of frame i in frame i-1): a normalised
  N(0, I3) direction times a length drawn from U[0.1, 0.5] m;
* home rotation ``home_rot`` of frame i relative to frame i-1: the identity
  (a Haar-random rotation when ``random_home=True``, used by tests);
* mass ``mass`` ~ U[0.5, 2] kg; centre of mass ``com`` ~ U[-0.1, 0.1]^3 m in
  frame i;
* rotational inertia about the centre of mass ``inertia`` = R diag(d) R^T,
  d ~ U[0.01, 0.1]^3, R Haar-random; stored as (xx, yy, zz, xy, xz, yz);
* gravity (0, 0, -9.81) in the base frame;
* state: q ~ U[-pi, pi], qd ~ U[-1, 1], tau ~ N(0, 1).

Branched robots (trees) add a parent index per link (``make_tree_parents``):
links are numbered in depth-first preorder, so every parent precedes its
children and every subtree is a contiguous run of links. Link i extends the
previous link with probability ``p_extend``, else it hangs from a uniformly
drawn link of the current root-to-link path (or from the base). The per-link
parameters are drawn as above, with frame i-1 read as the parent's frame.

All per-link arrays are packed chain after chain (``offsets`` gives each
chain's first link), the layout the library and the oracle both take.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

ROOT_SEED = 1609
GRAVITY = (0.0, 0.0, -9.81)

# stream tags inside one config seed
_STREAM_MODEL = 0
_STREAM_STATE = 1
_STREAM_LENGTHS = 2
_STREAM_TOPOLOGY = 3


def _rng(seed: int, cfg: int, stream: int, extra: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, cfg, stream, extra])))


def offsets_of(n_links: np.ndarray) -> np.ndarray:
    """Start index of every chain in the packed per-link arrays, plus the end."""
    off = np.zeros(len(n_links) + 1, dtype=np.int64)
    np.cumsum(np.asarray(n_links, dtype=np.int64), out=off[1:])
    return off


def _unit(v: np.ndarray) -> np.ndarray:
    nrm = np.linalg.norm(v, axis=-1, keepdims=True)
    return v / nrm


def _haar_rotations(rng: np.random.Generator, count: int) -> np.ndarray:
    """Uniform random rotations from normalised Gaussian quaternions, [count, 3, 3]."""
    qt = _unit(rng.standard_normal((count, 4)))
    w, x, y, z = qt[:, 0], qt[:, 1], qt[:, 2], qt[:, 3]
    r = np.empty((count, 3, 3))
    r[:, 0, 0] = 1 - 2 * (y * y + z * z)
    r[:, 0, 1] = 2 * (x * y - w * z)
    r[:, 0, 2] = 2 * (x * z + w * y)
    r[:, 1, 0] = 2 * (x * y + w * z)
    r[:, 1, 1] = 1 - 2 * (x * x + z * z)
    r[:, 1, 2] = 2 * (y * z - w * x)
    r[:, 2, 0] = 2 * (x * z - w * y)
    r[:, 2, 1] = 2 * (y * z + w * x)
    r[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return r


@dataclass
class Robots:
    """Per-link robot parameters, packed chain after chain (float64)."""

    n_links: np.ndarray          # [R] int32
    axis: np.ndarray             # [N, 3] unit joint axis in frame i
    home_rot: np.ndarray         # [N, 9] row-major rotation of frame i in frame i-1 at q = 0
    offset: np.ndarray           # [N, 3] origin of frame i in frame i-1
    mass: np.ndarray             # [N]
    com: np.ndarray              # [N, 3] centre of mass in frame i
    inertia: np.ndarray          # [N, 6] about the COM: xx yy zz xy xz yz
    gravity: np.ndarray = field(default_factory=lambda: np.array(GRAVITY))
    parent: np.ndarray | None = None  # [N] int32 parent of link i within its robot, -1 = base; None = serial

    @property
    def offsets(self) -> np.ndarray:
        return offsets_of(self.n_links)

    @property
    def total_links(self) -> int:
        return int(np.sum(self.n_links, dtype=np.int64))

    def take(self, robot_ids: np.ndarray) -> "Robots":
        """Per-chain copy: chain b gets the links of robot robot_ids[b]."""
        off = self.offsets
        idx = np.concatenate([np.arange(off[r], off[r + 1]) for r in robot_ids]) if len(robot_ids) else np.zeros(0, np.int64)
        return Robots(
            n_links=self.n_links[robot_ids].astype(np.int32),
            axis=self.axis[idx], home_rot=self.home_rot[idx], offset=self.offset[idx],
            mass=self.mass[idx], com=self.com[idx], inertia=self.inertia[idx],
            gravity=self.gravity.copy(), parent=None if self.parent is None else self.parent[idx])

    def parents(self) -> np.ndarray:
        """Parent of every link within its robot (-1 = base), also for serial robots."""
        if self.parent is not None:
            return np.asarray(self.parent, dtype=np.int32)
        off = self.offsets
        return (np.arange(self.total_links, dtype=np.int64) - np.repeat(off[:-1], self.n_links) - 1).astype(np.int32)

    def astype_rounded(self, dtype) -> "Robots":
        """The same robots with every parameter rounded through ``dtype`` (kept as float64)."""
        def r(a):
            return np.asarray(a, dtype=dtype).astype(np.float64)
        return Robots(n_links=self.n_links.copy(), axis=r(self.axis), home_rot=r(self.home_rot),
                      offset=r(self.offset), mass=r(self.mass), com=r(self.com),
                      inertia=r(self.inertia), gravity=r(self.gravity),
                      parent=None if self.parent is None else self.parent.copy())


def make_robots(n_links, seed: int = ROOT_SEED, cfg: int = 0, random_home: bool = False) -> Robots:
    """Draw one robot per entry of ``n_links`` (all links of all robots in one pass)."""
    n_links = np.asarray(n_links, dtype=np.int32)
    total = int(np.sum(n_links, dtype=np.int64))
    rng = _rng(seed, cfg, _STREAM_MODEL)
    axis = _unit(rng.standard_normal((total, 3)))
    direction = _unit(rng.standard_normal((total, 3)))
    length = rng.uniform(0.1, 0.5, size=(total, 1))
    offset = direction * length
    mass = rng.uniform(0.5, 2.0, size=total)
    com = rng.uniform(-0.1, 0.1, size=(total, 3))
    rot = _haar_rotations(rng, total)
    d = rng.uniform(0.01, 0.1, size=(total, 3))
    full = np.einsum("nij,nj,nkj->nik", rot, d, rot)
    inertia = np.stack([full[:, 0, 0], full[:, 1, 1], full[:, 2, 2],
                        full[:, 0, 1], full[:, 0, 2], full[:, 1, 2]], axis=1)
    if random_home:
        home = _haar_rotations(rng, total).reshape(total, 9)
    else:
        home = np.tile(np.eye(3).reshape(1, 9), (total, 1))
    return Robots(n_links=n_links, axis=axis, home_rot=home, offset=offset, mass=mass,
                  com=com, inertia=inertia)


def make_tree_parents(n_links, p_extend: float = 0.85, seed: int = ROOT_SEED, cfg: int = 0) -> np.ndarray:
    """Parent of every link (-1 = base) of one random tree per entry of ``n_links``,
    numbered in depth-first preorder (see the module docstring)."""
    n_links = np.asarray(n_links, dtype=np.int32)
    rng = _rng(seed, cfg, _STREAM_TOPOLOGY)
    total = int(np.sum(n_links, dtype=np.int64))
    u = rng.random(total)
    pick = rng.random(total)
    out = np.empty(total, np.int32)
    k = 0
    for n in n_links:
        path = [-1]                               # the base, then the current root-to-link path
        for i in range(int(n)):
            if i > 0 and u[k] < p_extend:
                p = i - 1
            else:
                p = path[int(pick[k] * len(path))]
            del path[path.index(p) + 1:]
            path.append(i)
            out[k] = p
            k += 1
    return out


def make_tree_robots(n_links, p_extend: float = 0.85, seed: int = ROOT_SEED, cfg: int = 0,
                     random_home: bool = False, shared_topology: bool = False) -> Robots:
    """Random branched robots: ``make_robots`` parameters plus ``make_tree_parents``
    topology (one topology drawn once and given to every robot when
    ``shared_topology``; the robots must then have equal lengths)."""
    rb = make_robots(n_links, seed=seed, cfg=cfg, random_home=random_home)
    n_links = np.asarray(n_links, dtype=np.int32)
    if shared_topology:
        if len(n_links) and np.any(n_links != n_links[0]):
            raise ValueError("a shared topology needs robots of equal length")
        one = make_tree_parents(n_links[:1], p_extend=p_extend, seed=seed, cfg=cfg)
        rb.parent = np.tile(one, len(n_links))
    else:
        rb.parent = make_tree_parents(n_links, p_extend=p_extend, seed=seed, cfg=cfg)
    return rb


def make_state(n_links, seed: int = ROOT_SEED, cfg: int = 0, rep: int = 0):
    """Joint positions, velocities and torques for every link, packed like the robots."""
    total = int(np.sum(np.asarray(n_links, dtype=np.int64)))
    rng = _rng(seed, cfg, _STREAM_STATE, rep)
    q = rng.uniform(-np.pi, np.pi, size=total)
    qd = rng.uniform(-1.0, 1.0, size=total)
    tau = rng.standard_normal(total)
    return q, qd, tau


def uniform_lengths(batch: int, n: int) -> np.ndarray:
    return np.full(batch, n, dtype=np.int32)


def ragged_lengths(batch: int, lo: int, hi: int, seed: int = ROOT_SEED, cfg: int = 3) -> np.ndarray:
    """Chain lengths drawn i.i.d. from U{lo..hi}."""
    rng = _rng(seed, cfg, _STREAM_LENGTHS)
    return rng.integers(lo, hi + 1, size=batch).astype(np.int32)


# Workload presets: the shapes the library is exercised and timed on.
WORKLOADS = {
    "uniform-n8-b1024": dict(batch=1024, n=8, cfg=1),
    "uniform-n16-b65536": dict(batch=65536, n=16, cfg=2),
    "uniform-n32-b65536": dict(batch=65536, n=32, cfg=2),
    "uniform-n64-b65536": dict(batch=65536, n=64, cfg=2),
    "uniform-n128-b65536": dict(batch=65536, n=128, cfg=2),
    "tree-n64-b65536": dict(batch=65536, n=64, cfg=5, p_extend=0.85),
    "tree-shared-n64-b65536": dict(batch=65536, n=64, cfg=5, p_extend=0.85, shared_topology=True),
}


def make_btd(n_blocks, k: int = 6, seed: int = ROOT_SEED, cfg: int = 7):
    """Random SPD block tri-diagonal systems, packed like chains.

    A = L L^T with L block lower bi-diagonal (random diagonal blocks with a
    positive diagonal shift, random sub-diagonal blocks), so A is block
    tri-diagonal and SPD. Returns (D [N, k, k], U [N, k, k] with U of the last
    block of every system zero, R [N, k]).
    """
    n_blocks = np.asarray(n_blocks, dtype=np.int64)
    total = int(n_blocks.sum())
    rng = _rng(seed, cfg, _STREAM_MODEL)
    diag = rng.standard_normal((total, k, k)) * 0.3 + np.eye(k) * 1.5
    sub = rng.standard_normal((total, k, k)) * 0.5
    rhs = rng.standard_normal((total, k))
    d = np.empty((total, k, k))
    u = np.zeros((total, k, k))
    off = offsets_of(n_blocks)
    for b in range(len(n_blocks)):
        s, e = off[b], off[b + 1]
        for i in range(s, e):
            li = diag[i]
            d[i] = li @ li.T
            if i > s:
                lp = sub[i]                       # L block (i, i-1)
                d[i] += lp @ lp.T
                u[i - 1] = diag[i - 1] @ lp.T     # A block (i-1, i) = L_{i-1,i-1} L_{i,i-1}^T
    return d, u, rhs


def make_scan_elements(lengths, d: int = 6, seed: int = ROOT_SEED, cfg: int = 8):
    """Random affine elements (B [N, d, d], c [N, d]) with ||B||_2 <= 1 so long
    recurrences stay bounded."""
    lengths = np.asarray(lengths, dtype=np.int64)
    total = int(lengths.sum())
    rng = _rng(seed, cfg, _STREAM_MODEL)
    g = rng.standard_normal((total, d, d))
    qm, _ = np.linalg.qr(g)
    scale = rng.uniform(0.5, 1.0, size=(total, 1, d))
    return qm * scale, rng.standard_normal((total, d))
