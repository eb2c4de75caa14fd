"""The balanced block map of batched launches (locate_in in csrc/eqs_kernels.hip), restated on the
host: the hardware hands block b to XCD b % 8, and XCD x runs the x-th share of every set.  Checked
here for the properties the kernels rely on (no GPU needed): it is a bijection from blocks to
(set, tile); each XCD's blocks of one set cover a contiguous run of that set's tiles, in block order;
every share is within one tile of an eighth of its set; and each XCD gets exactly the blocks the
hardware hands it (those are the blocks b < n with b % 8 == x, so no block maps outside the sets).
"""
import random


def balanced(b, begin, nsets):
    x, slot = b % 8, b // 8
    c = o = 0
    for q in range(8):
        T = begin[q + 1] - begin[q]
        k, r = T >> 3, T & 7
        a = k + (1 if ((x - o) & 7) < r else 0)
        if q < nsets and (slot < c + a or q == nsets - 1):
            before = x * k + sum(1 for y in range(x) if ((y - o) & 7) < r)
            return q, before + slot - c
        c += a
        o = (o + r) & 7
    raise AssertionError("no set")


def check(counts):
    nsets = len(counts)
    begin = [0]
    for t in counts:
        begin.append(begin[-1] + t)
    begin += [begin[-1]] * (9 - len(begin))
    seen, runs = set(), {}
    for b in range(begin[nsets]):
        q, t = balanced(b, begin, nsets)
        assert 0 <= q < nsets and 0 <= t < counts[q]
        seen.add((q, t))
        runs.setdefault((q, b % 8), []).append(t)
    assert len(seen) == begin[nsets]
    for (q, x), ts in runs.items():
        assert ts == list(range(ts[0], ts[0] + len(ts)))
        assert counts[q] // 8 <= len(ts) <= counts[q] // 8 + 1


def test_balanced_map_small_and_ragged_counts():
    for counts in ([1], [7], [8], [9], [1, 1, 1], [7, 7, 7, 7, 7, 7, 7, 7], [432, 432, 432, 432],
                   [288, 292, 292, 360], [3, 864, 5, 1]):
        check(counts)


def test_balanced_map_random_counts():
    rng = random.Random(5)
    for _ in range(300):
        check([rng.choice([rng.randint(1, 20), rng.randint(1, 3000)]) for _ in range(rng.randint(1, 8))])


def test_balanced_map_of_one_set_is_the_contiguous_map():
    # one set: XCD x takes tiles [x q + min(x, r), ...), the contiguous map of the same launch
    for T in (1, 5, 8, 13, 432, 1001):
        q, r = T // 8, T % 8
        begin = [0, T] + [T] * 7
        for b in range(T):
            x, slot = b % 8, b // 8
            assert balanced(b, begin, 1) == (0, x * q + min(x, r) + slot)
