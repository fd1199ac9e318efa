"""The random index set I of Eq. (2) / Algorithm 1 (draw I subset of [n]).

The paper asks for index sets drawn uniformly at random (Sec. III, which is
what makes Eq. (2) unbiased) but fixes no generator.  Reading used here:
I is a uniform k-subset drawn without replacement, realised as the first k
images of a keyed pseudo-random permutation of [0, n), key = (seed, step).

Specification (the HIP sampler implements the same text independently):

  mix64(z): the SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014):
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
      z = (z ^ (z >> 27)) * 0x94D049BB133111EB
      return z ^ (z >> 31)                       (all arithmetic mod 2^64)
  b  = smallest integer >= 2 with 2^b >= n;  hb = ceil(b / 2)
  round keys, r = 0..5:
      K_r = mix64(seed ^ mix64(step ^ (0x9E3779B97F4A7C15 * (r + 1))))
  round function:  F_r(x) = mix64(K_r ^ x) >> (64 - hb)
  E(x): L = x >> hb, R = x & (2^hb - 1);
        six times: (L, R) <- (R, L ^ F_r(R)), r = 0..5;  return (L << hb) | R
  pi(j): the first of E(j), E(E(j)), ... that is below n (cycle walking)
  I: the ranks pi(0..k-1), sorted ascending, mapped to grid indices through
     the FOV rank order.

E is a Feistel network on 2hb bits, hence a bijection of [0, 2^(2hb));
cycle walking restricts it to a bijection of [0, n).
"""
import numpy as np

M64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
ROUNDS = 6


def mix64(z):
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def half_bits(n):
    b = 2
    while (1 << b) < n:
        b += 1
    return (b + 1) // 2


def round_keys(seed, step):
    return [mix64((seed & M64) ^ mix64((step & M64) ^ ((GOLDEN * (r + 1)) & M64)))
            for r in range(ROUNDS)]


def feistel(x, keys, hb):
    mask = (1 << hb) - 1
    L, R = x >> hb, x & mask
    for K in keys:
        L, R = R, L ^ (mix64(K ^ R) >> (64 - hb))
    return (L << hb) | R


def permute(j, n, seed, step):
    """pi(j) for one j (pure Python integers)."""
    hb = half_bits(n)
    keys = round_keys(seed, step)
    y = feistel(j, keys, hb)
    while y >= n:
        y = feistel(y, keys, hb)
    return y


def sample_ranks(n, k, seed, step):
    """Sorted ranks pi(0..k-1).  Pure Python: keep k small (tests)."""
    if not 0 < k <= n:
        raise ValueError("need 0 < k <= n")
    hb = half_bits(n)
    keys = round_keys(seed, step)
    out = []
    for j in range(k):
        y = feistel(j, keys, hb)
        while y >= n:
            y = feistel(y, keys, hb)
        out.append(y)
    return np.array(sorted(out), dtype=np.int64)


def sample_indices(fov_idx, k, seed, step):
    """The index set I as grid linear indices (ascending)."""
    fov_idx = np.asarray(fov_idx)
    return fov_idx[sample_ranks(fov_idx.size, k, seed, step)]


def _mix64_np(z):
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def sample_ranks_np(n, k, seed, step):
    """sample_ranks with the Feistel rounds vectorised over j (uint64
    arithmetic wraps modulo 2^64 as the specification requires)."""
    if not 0 < k <= n:
        raise ValueError("need 0 < k <= n")
    hb = half_bits(n)
    keys = [np.uint64(kk) for kk in round_keys(seed, step)]
    mask = np.uint64((1 << hb) - 1)
    sh = np.uint64(hb)
    top = np.uint64(64 - hb)

    def E(x):
        L, R = x >> sh, x & mask
        for K in keys:
            L, R = R, L ^ (_mix64_np(K ^ R) >> top)
        return (L << sh) | R

    with np.errstate(over="ignore"):
        y = E(np.arange(k, dtype=np.uint64))
        bad = y >= np.uint64(n)
        while bad.any():
            y[bad] = E(y[bad])
            bad = y >= np.uint64(n)
    return np.sort(y.astype(np.int64))
