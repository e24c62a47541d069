"""Philox4x32-10 and the draw conventions of the memetic operators (oracle side).

Test infrastructure only (see the package docstring).

The generator is the counter-based Philox4x32 with 10 rounds, as defined by
Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3"
(SC'11): each round multiplies counter words 0 and 2 by the constants
0xD2511F53 and 0xCD9E8D57, takes the 64-bit products apart into high and low
halves, and permutes/xors them with counter words 1 and 3 and the key; the key
is advanced by the Weyl increments 0x9E3779B9 and 0xBB67AE85 between rounds.

The paper names no generator; the memetic operators only need "random"
choices (Crossover appendix: RandomChoice, CrossoverMap).  The conventions
below make every random decision a pure function of (seed, purpose,
generation, member, draw) so that the GPU and this oracle take the same
decisions without sharing code:

* key      = (seed mod 2^32, seed >> 32)
* counter  = (block, member, generation, purpose); output word ``w`` of block
             ``b`` is draw number ``4*b + w``.
* uniform integer in [0, n):  (u32 * n) >> 32  (high word of a 64-bit product)
* Bernoulli(c):               u32 < floor(c * 2^32)   (compared in 64 bits)
"""

MASK32 = 0xFFFFFFFF
M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85

# purposes (counter word 3)
PURPOSE_CHOICE = 1    # RandomChoice: draws 0..2
PURPOSE_MAPPARAM = 2  # CrossoverMap tile size, grid shift, rotation: draws 0..4
PURPOSE_TILE = 3      # CrossoverMap tile election: block = tile key, word 0
PURPOSE_INIT = 4      # random-phase start: draw = FFT-order pixel index, generation 0
PURPOSE_SPHERES = 5   # sphere start: draws 4k..4k+3 = diameter, row and column centre, phase of sphere k


def _round(c, k):
    p0 = M0 * c[0]
    p1 = M1 * c[2]
    hi0, lo0 = p0 >> 32, p0 & MASK32
    hi1, lo1 = p1 >> 32, p1 & MASK32
    return [(hi1 ^ c[1] ^ k[0]) & MASK32, lo1, (hi0 ^ c[3] ^ k[1]) & MASK32, lo0]


def philox4x32_10(counter, key):
    """Return the four 32-bit output words for a 4-word counter and 2-word key."""
    c = [int(v) & MASK32 for v in counter]
    k = [int(v) & MASK32 for v in key]
    c = _round(c, k)
    for _ in range(9):
        k = [(k[0] + W0) & MASK32, (k[1] + W1) & MASK32]
        c = _round(c, k)
    return c


def seed_key(seed):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return (seed & MASK32, seed >> 32)


def draw(seed, purpose, generation, member, index):
    """Draw number ``index`` of the stream (seed, purpose, generation, member)."""
    block, word = divmod(int(index), 4)
    out = philox4x32_10((block, int(member) & MASK32, int(generation) & MASK32, purpose),
                        seed_key(seed))
    return out[word]


def uniform_int(u32, n):
    """Map a 32-bit draw to [0, n) by the high word of u32*n."""
    return (int(u32) * int(n)) >> 32


def bernoulli_threshold(prob):
    """Integer threshold t with Bernoulli(prob) <=> u32 < t (t may equal 2^32)."""
    t = int(prob * 4294967296.0)
    return max(0, min(t, 1 << 32))


def philox4x32_10_array(c0, c1, c2, c3, key):
    """Element-wise Philox4x32-10 over arrays of counter words (NumPy uint64
    arithmetic, the same rounds as ``philox4x32_10``).  Returns four uint32
    arrays."""
    import numpy as np

    m = np.uint64(MASK32)
    c = [np.asarray(v, dtype=np.uint64) & m for v in (c0, c1, c2, c3)]
    c = np.broadcast_arrays(*c)
    c = [np.array(v, dtype=np.uint64) for v in c]
    k0, k1 = np.uint64(int(key[0]) & MASK32), np.uint64(int(key[1]) & MASK32)
    for r in range(10):
        if r:
            k0 = np.uint64((int(k0) + W0) & MASK32)
            k1 = np.uint64((int(k1) + W1) & MASK32)
        p0 = np.uint64(M0) * c[0]
        p1 = np.uint64(M1) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & m
        hi1, lo1 = p1 >> np.uint64(32), p1 & m
        c = [(hi1 ^ c[1] ^ k0) & m, lo1, (hi0 ^ c[3] ^ k1) & m, lo0]
    return [v.astype(np.uint32) for v in c]


def draws_array(seed, purpose, generation, member, count):
    """Draws 0..count-1 of the stream (seed, purpose, generation, member)."""
    import numpy as np

    idx = np.arange(count, dtype=np.uint64)
    blocks = idx >> np.uint64(2)
    words = philox4x32_10_array(blocks, int(member), int(generation), purpose, seed_key(seed))
    out = np.stack(words, axis=-1)  # [draw][word of the draw's block]
    return out[np.arange(count), (idx & np.uint64(3)).astype(np.int64)]
