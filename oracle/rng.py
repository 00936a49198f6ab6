"""Counter-based random draws for the cross algorithm (oracle side).

The paper asks for random samples without replacement and random bits in the
update cross step (Algorithm 5) and for random starting multi-indices in the
index initialisation (Algorithm 7), but names no generator.  Both the oracle
and the GPU library therefore use splitmix64 (Steele, Lea & Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014), written here from
its published definition:

    state <- state + 0x9E3779B97F4A7C15            (mod 2^64)
    z <- state
    z <- (z xor (z >> 30)) * 0xBF58476D1CE4E5B9   (mod 2^64)
    z <- (z xor (z >> 27)) * 0x94D049BB133111EB   (mod 2^64)
    output z xor (z >> 31)

Keyed streams: a stream for key (seed, p_1, ..., p_m) starts from the state
s_0 = seed and s_{i} = mix((s_{i-1} xor p_i) + GOLDEN), where mix is the
three-line finaliser above.

Derived draws
  below(m)   integer in [0, m):  (x * m) >> 64 with a 128-bit product
  bit()      top bit of the next output
  floyd(M,k) k distinct integers of [0, M) by Floyd's algorithm (Bentley &
             Floyd, CACM 1987): for j = M-k .. M-1 draw t = below(j+1) and
             insert t, or j if t is already present; returned sorted.
"""

MASK = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15

# stream tags
TAG_INIT = 1      # Algorithm 7 random multi-indices
TAG_UPDATE = 2    # Algorithm 5 samples and bit, keyed by (sweep, k)
TAG_TEST = 3      # multi-indices of the sampled stopping test


def _mix(z):
    z &= MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


class SplitMix64:
    def __init__(self, state):
        self.state = state & MASK

    def next(self):
        self.state = (self.state + GOLDEN) & MASK
        return _mix(self.state)

    def below(self, m):
        return (self.next() * int(m)) >> 64

    def bit(self):
        return self.next() >> 63

    def floyd(self, M, k):
        chosen = set()
        for j in range(M - k, M):
            t = self.below(j + 1)
            chosen.add(j if t in chosen else t)
        return sorted(chosen)


def keyed(seed, *parts):
    s = int(seed) & MASK
    for p in parts:
        s = _mix(((s ^ (int(p) & MASK)) + GOLDEN) & MASK)
    return SplitMix64(s)
