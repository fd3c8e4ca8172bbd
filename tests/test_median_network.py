"""The comparator network the GPU median filter sorts its 5x5 window with:
Batcher's odd-even merge sort for 32 slots, restricted to the comparators
whose both slots lie among the first 25 (the window; the 7 slots above it
would hold +inf and never move). The kernel unrolls the same four loops;
this checks the restriction still sorts, by the zero-one principle: a
comparator network sorts every input iff it sorts every 0/1 input, here all
2^25 of them, evaluated bit-parallel (one bit per input)."""
import numpy as np

N, SLOTS = 32, 25


def network():
    pairs = []
    p = 1
    while p < N:
        kk = p
        while kk >= 1:
            j = kk % p
            while j + kk < N:
                for i in range(kk):
                    a, b = i + j, i + j + kk
                    if b < SLOTS and a // (2 * p) == b // (2 * p):
                        pairs.append((a, b))
                j += 2 * kk
            kk //= 2
        p *= 2
    return pairs


def test_network_size():
    assert len(network()) == 140


def test_full_network_sorts_32_by_zero_one_sample():
    # the unrestricted network (b < 32) on random permutations: a check
    # that the loop structure is Batcher's
    pairs = []
    p = 1
    while p < N:
        kk = p
        while kk >= 1:
            j = kk % p
            while j + kk < N:
                for i in range(kk):
                    a, b = i + j, i + j + kk
                    if a // (2 * p) == b // (2 * p):
                        pairs.append((a, b))
                j += 2 * kk
            kk //= 2
        p *= 2
    assert len(pairs) == 191
    rng = np.random.default_rng(0)
    x = rng.permuted(np.tile(np.arange(N), (2000, 1)), axis=1)
    for a, b in pairs:
        lo, hi = np.minimum(x[:, a], x[:, b]), np.maximum(x[:, a], x[:, b])
        x[:, a], x[:, b] = lo, hi
    assert (x == np.arange(N)).all()


def test_restricted_network_sorts_every_zero_one_input():
    # input index t in [0, 2^25): slot s holds bit s of t; bit t of the
    # packed arrays below is that input's value in the slot
    total = 1 << SLOTS
    t = np.arange(total, dtype=np.uint32)
    slots = [np.packbits(((t >> s) & 1).astype(np.uint8)) for s in range(SLOTS)]
    del t
    for a, b in network():
        lo, hi = slots[a] & slots[b], slots[a] | slots[b]
        slots[a], slots[b] = lo, hi
    # sorted ascending: slot s <= slot s+1 for every input
    for s in range(SLOTS - 1):
        assert not (slots[s] & ~slots[s + 1]).any(), s
