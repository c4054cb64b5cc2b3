"""The LDS state stage of the lane-per-chain kernels (StateStage / OutTile in
lanes.h), emulated on the CPU index by index: for random ragged wavefronts of
64 chains, every global entry a tile loads or stores lies inside its own chain,
every LDS index inside the stage, every value a lane reads at sweep position
k + ahead (after the tile steps the kernels take) is its own chain's entry at
that position, forward and backward, and every output entry is stored exactly
once. The tile size and LDS row stride are read from lanes.h."""
import os
import random
import re

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
LANES_H = os.path.join(HERE, "..", "paper_1609_06779_amd", "csrc", "lanes.h")


def _constants():
    src = open(LANES_H).read()
    st_l = int(re.search(r"constexpr int ST_L = (\d+);", src).group(1))
    st_w = eval(re.search(r"constexpr int ST_W = ([0-9 +]+);", src).group(1))
    return st_l, st_w


def _run(lens, bases, total, na, fwd, ahead, st_l, st_w, stage, out=False):
    lds = {}
    nw = max(lens)

    def load(t):
        regs = []
        for lane in range(64):
            r = [[None] * st_l for _ in range(na)]
            for k in range(st_l):
                c, j = (k * 64 + lane) // st_l, lane % st_l
                pos, n = t * st_l + j, lens[c]
                e = bases[c] + pos if fwd else bases[c] + (n - 1 - pos)
                for v in range(na):
                    if pos < n:
                        assert bases[c] <= e < bases[c] + n and 0 <= e < total
                        r[v][k] = (v, e)
                    else:
                        r[v][k] = "zero"
            regs.append(r)
        return regs

    def commit(t, regs):
        d = (t & 1) * na * st_l * st_w
        for lane in range(64):
            for k in range(st_l):
                c, j = (k * 64 + lane) // st_l, lane % st_l
                for v in range(na):
                    idx = d + (v * st_l + j) * st_w + c
                    assert 0 <= idx < stage
                    lds[idx] = regs[lane][v][k]

    def get(lane, v, pos):
        idx = (((pos // st_l) & 1) * na + v) * st_l * st_w + (pos % st_l) * st_w + lane
        assert 0 <= idx < stage
        return lds[idx]

    def expect(lane, v, pos):
        n = lens[lane]
        return (v, bases[lane] + pos if fwd else bases[lane] + n - 1 - pos)

    r0, r1, pend = load(0), load(1), load(2)          # start: three tiles in flight, two committed
    commit(0, r0)
    commit(1, r1)
    for lane in range(64):
        for p in range(min(ahead + 1, lens[lane])):
            for v in range(na):
                assert get(lane, v, p) == expect(lane, v, p)
    otile, written = {}, set()
    for k in range(nw):
        if k > 0 and k % st_l == 0:                   # step: commit tile t + 1, load tile t + 2
            t = k // st_l
            commit(t + 1, pend)
            pend = load(t + 2)
        for lane in range(64):
            if k >= lens[lane]:
                continue
            for p in (k, k + ahead):
                if p < lens[lane]:
                    for v in range(na):
                        assert get(lane, v, p) == expect(lane, v, p), (lane, v, k, p)
            if out:
                otile[(k % st_l) * st_w + lane] = (lane, k)
        if out and (k % st_l == st_l - 1 or k == nw - 1):  # flush after a tile's last position
            t = k // st_l
            for lane in range(64):
                for kk in range(st_l):
                    c, j = (kk * 64 + lane) // st_l, lane % st_l
                    pos = t * st_l + j
                    if pos < lens[c]:
                        e = bases[c] + pos if fwd else bases[c] + lens[c] - 1 - pos
                        assert bases[c] <= e < bases[c] + lens[c]
                        assert otile[j * st_w + c] == (c, pos)
                        assert e not in written
                        written.add(e)
            otile = {}
    if out:
        assert len(written) == sum(lens)


@pytest.mark.parametrize("seed", range(40))
def test_stage_schedule(seed):
    st_l, st_w = _constants()
    assert st_w >= 64
    stage = 2 * 3 * st_l * st_w                       # the ABIA stage; the reverse mode's is larger
    rng = random.Random(seed)
    kind = seed % 4
    if kind == 0:
        lens = [64] * 64
    elif kind == 1:
        lens = [rng.randint(0, 256) for _ in range(64)]
    elif kind == 2:
        lens = [rng.choice([0, 1, 2, 3, 7, 8, 9, 15, 16, 17]) for _ in range(64)]
    else:
        lens = [0] * rng.randint(0, 63)
        lens += [rng.randint(1, 40) for _ in range(64 - len(lens))]
    if max(lens) == 0:
        lens[5] = 1
    order = list(range(64))
    rng.shuffle(order)
    bases, off = [0] * 64, 0
    for c in order:
        bases[c] = off
        off += lens[c] + rng.randint(0, 3)
    _run(lens, bases, off, 2, True, 2, st_l, st_w, stage)              # forward, two ahead (ABIA sweep 1)
    _run(lens, bases, off, 3, False, 1, st_l, st_w, stage)             # backward, one ahead (sweep 2)
    _run(lens, bases, off, 1, True, 2, st_l, st_w, stage, out=True)    # forward with outputs (sweep 3)
    _run(lens, bases, off, 2, False, 1, st_l, st_w, stage, out=True)   # backward with outputs (reverse mode)
