"""Block sampler of the oracle: b distinct coordinates per iteration, drawn
uniformly without replacement, keyed by (seed, h) only.

The paper fixes only the distribution (uniform, without replacement within a
block; Section 1 footnote, Alg. 1-4 "choose ... uniformly at random without
replacement") and that every processor draws the same blocks from a shared seed
(Section 3.1, discussion after eq. (recur)).  The generator itself is our
specification, built from three published pieces:

* SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
  generators", OOPSLA 2014): state advances by the golden gamma
  0x9E3779B97F4A7C15 and each output is the state passed through the mix64
  finaliser with multipliers 0xBF58476D1CE4E5B9 and 0x94D049BB133111EB.
* Lemire's multiply-shift bounded integer with rejection ("Fast random integer
  generation in an interval", ACM TOMACS 2019) on 32-bit words.
* Floyd's sampling without replacement (Bentley & Floyd, "Programming pearls:
  a sample of brilliance", CACM 1987).

Composition:
  key(seed, h)    = output number h (0-based) of SplitMix64 seeded with `seed`
  word(key, t)    = upper 32 bits of output number t of SplitMix64 seeded with key
  bounded(m)      = Lemire on successive words t = 0, 1, 2, ... of the block
  block(seed,h,b,m): for j = m-b .. m-1: v = bounded(j+1); append (j if v already
                     drawn else v).  Output order = insertion order.

Keying by the global iteration h makes the block sequence independent of s,
which is what lets CA-BCD(s) and BCD(s=1) be compared on identical blocks.

Pure Python integer arithmetic; test infrastructure only.
"""

MASK32 = (1 << 32) - 1
MASK64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15


def mix64(z):
    """SplitMix64 output finaliser."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def splitmix64_output(seed, t):
    """Output number t (0-based) of the SplitMix64 stream seeded with `seed`."""
    return mix64((seed + GOLDEN_GAMMA * (t + 1)) & MASK64)


def iteration_key(seed, h):
    return splitmix64_output(seed & MASK64, h)


class _WordStream:
    def __init__(self, key):
        self.key = key
        self.t = 0

    def next32(self):
        x = splitmix64_output(self.key, self.t) >> 32
        self.t += 1
        return x


def bounded(stream, m):
    """Uniform integer in [0, m) for 1 <= m <= 2**32 (Lemire 2019)."""
    if not (1 <= m <= (1 << 32)):
        raise ValueError("range out of bounds")
    x = stream.next32()
    prod = x * m
    low = prod & MASK32
    if low < m:
        threshold = ((1 << 32) - m) % m
        while low < threshold:
            x = stream.next32()
            prod = x * m
            low = prod & MASK32
    return prod >> 32


def sample_block(seed, h, b, m):
    """b distinct integers from [0, m) for global iteration h (Floyd)."""
    if not (1 <= b <= m):
        raise ValueError("need 1 <= b <= m")
    stream = _WordStream(iteration_key(seed, h))
    out = []
    for j in range(m - b, m):
        v = bounded(stream, j + 1)
        out.append(j if v in out else v)
    return out


def sample_blocks(seed, h0, count, b, m):
    """Blocks for global iterations h0 .. h0+count-1, as a list of lists."""
    return [sample_block(seed, h0 + i, b, m) for i in range(count)]
