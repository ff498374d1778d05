"""Width-generic Philox-4xW-R written from Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11), section 4.

Test infrastructure only.  The 4x64 instance is checked against numpy's
``numpy.random.Philox`` (an independent implementation of the same published
generator); the 4x32 instance then serves as the known-answer source for the
oracle's and the GPU library's own Philox4x32-10 implementations.
"""

# Multipliers and Weyl key increments from the paper (table 2 and section 4.1).
_PARAMS = {
    32: dict(M0=0xD2511F53, M1=0xCD9E8D57, W0=0x9E3779B9, W1=0xBB67AE85),
    64: dict(M0=0xD2E7470EE14C6C93, M1=0xCA5A826395121157,
             W0=0x9E3779B97F4A7C15, W1=0xBB67AE8584CAA73B),
}


def philox4(counter, key, width=32, rounds=10):
    """One Philox-4xW block: returns 4 W-bit words for a 4-word counter and
    2-word key.  Each round multiplies words 0 and 2 by the two constants,
    splits the double-width products into hi/lo halves, and mixes the highs
    with words 1 and 3 and the key (the S-box/P-box of the paper); the key is
    bumped by the Weyl constants between rounds."""
    p = _PARAMS[width]
    mask = (1 << width) - 1
    c = [int(w) & mask for w in counter]
    k0, k1 = int(key[0]) & mask, int(key[1]) & mask
    for r in range(rounds):
        if r:
            k0 = (k0 + p["W0"]) & mask
            k1 = (k1 + p["W1"]) & mask
        prod0 = p["M0"] * c[0]
        prod1 = p["M1"] * c[2]
        hi0, lo0 = prod0 >> width, prod0 & mask
        hi1, lo1 = prod1 >> width, prod1 & mask
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return c


def u01(a, b):
    """Uniform double in (0,1) from two 32-bit words: 52 random bits k,
    u = (k + 1/2) 2^-52, exact in binary64, never 0 or 1."""
    k = ((int(a) >> 6) << 26) | (int(b) >> 6)
    return (float(k) + 0.5) * 2.0 ** -52


def counter_for(subject, step, purpose, block):
    """The library-wide counter layout: (subject, step, purpose<<24 | block
    low 24 bits, block >> 24)."""
    return [subject & 0xFFFFFFFF, step & 0xFFFFFFFF,
            ((purpose & 0xFF) << 24) | (block & 0xFFFFFF), (block >> 24) & 0xFFFFFFFF]
