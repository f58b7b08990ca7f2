"""CPU emulation of the backward's transposing wave reduction: two permlane swap steps (wave
halves, then row pairs) and a four-step DPP butterfly inside each 16-lane row. Checks that
every lane ends with the wave total of the value index the lane-to-slot rule assigns it, and
that each of the K totals has exactly one owner, for K = 1..16 and either direction of the
hardware swap (the kernel reads the direction from the swap itself). The device code is
checked end to end by the GPU gradient parity tests."""
import numpy as np
import pytest


def swap_step(v, group, upper_gets_vdst):
    """Pairs (a, b) = (v[2i], v[2i+1]) swapped between lane l and l ^ group (group = 32: the
    halves; 16: neighbouring rows), then r0 + r1. Returns the new values and, per lane,
    whether it ended with the second value of each pair."""
    n, KI = v.shape
    KO = (KI + 1) // 2
    out = np.zeros((n, KO))
    side = np.zeros(n, bool)
    for l in range(n):
        p = l ^ group
        low = (l & group) == 0
        for i in range(KO):
            a_own = v[l, 2 * i]
            b_own = v[l, 2 * i + 1] if 2 * i + 1 < KI else v[l, 2 * i]
            a_p = v[p, 2 * i]
            b_p = v[p, 2 * i + 1] if 2 * i + 1 < KI else v[p, 2 * i]
            # r0 = new vdst (a before the swap), r1 = new vsrc (b before). Either the upper
            # side's vdst is exchanged with the lower side's vsrc, or the reverse.
            gets_b = (not low) if upper_gets_vdst else low
            r0, r1 = (b_p, b_own) if gets_b else (a_own, a_p)
            side[l] = gets_b
            out[l, i] = r0 + r1
    return out, side


def partner(step, l):
    r = l & 15
    base = l - r
    if step == 0:
        return base + 15 - r                       # row_mirror
    if step == 1:
        return base + ((r & 8) | (7 - (r & 7)))      # row_half_mirror
    if step == 2:
        return base + ((r & ~3) | (3 - (r & 3)))     # quad_perm [3, 2, 1, 0]
    return base + ((r & ~3) | [1, 0, 3, 2][r & 3])   # quad_perm [1, 0, 3, 2]


def row_step(v, step):
    n, KI = v.shape
    KO = (KI + 1) // 2
    out = np.zeros((n, KO))
    bit = 3 - step
    for l in range(n):
        p = partner(step, l)
        hi = ((l & 15) >> bit) & 1
        phi = ((p & 15) >> bit) & 1
        assert hi != phi
        for i in range(KI // 2):
            keep = v[l, 2 * i + 1] if hi else v[l, 2 * i]
            send = v[p, 2 * i] if phi else v[p, 2 * i + 1]
            out[l, i] = keep + send
        if KI & 1:
            out[l, KI // 2] = v[l, KI - 1] + v[p, KI - 1]
    return out


def slot(K, l, side_half, side_rows):
    """The lane-to-total rule of the kernel: which value a lane ends with, and ownership."""
    r = l & 15
    hi = [side_half, side_rows, r & 8, r & 4, r & 2, r & 1]
    ids, dup, n = list(range(16)), [False] * 16, K
    for s in range(6):
        h = bool(hi[s])
        for i in range(n // 2):
            ids[i] = ids[2 * i + 1] if h else ids[2 * i]
            dup[i] = dup[2 * i + 1] if h else dup[2 * i]
        if n & 1:
            i = n // 2
            ids[i], dup[i] = ids[n - 1], dup[n - 1] or h
        n = (n + 1) // 2
    return ids[0], not dup[0]


@pytest.mark.parametrize("upper_gets_vdst", [False, True])
@pytest.mark.parametrize("K", range(1, 17))
def test_each_total_lands_in_exactly_one_owner(K, upper_gets_vdst):
    rng = np.random.default_rng(K)
    v = rng.standard_normal((64, K))
    a, side_half = swap_step(v, 32, upper_gets_vdst)
    b, side_rows = swap_step(a, 16, upper_gets_vdst)
    # the kernel reads the sides by swapping (0, 1): the side that gets b = 1 is "high"
    probe = np.tile([0.0, 1.0], (64, 1))
    assert np.array_equal(swap_step(probe, 32, upper_gets_vdst)[0][:, 0] != 0, side_half)
    assert np.array_equal(swap_step(probe, 16, upper_gets_vdst)[0][:, 0] != 0, side_rows)
    c = b
    for step in range(4):
        c = row_step(c, step)
    tot = v.sum(0)
    owners = {}
    for l in range(64):
        idx, own = slot(K, l, side_half[l], side_rows[l])
        assert abs(c[l, 0] - tot[idx]) < 1e-12, (K, l, idx)
        if own:
            assert idx not in owners, (K, idx)
            owners[idx] = l
    assert sorted(owners) == list(range(K))
