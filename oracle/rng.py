"""Counter-based random numbers for the seeded initial conditions.

The paper draws its initial conditions from seeded random fields (App. C.1,
"10 seeds with Gaussian random field") without naming a generator.  Both the
oracle and the HIP library therefore implement, independently, one published
generator:

* SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
  generators", OOPSLA 2014): state += 0x9E3779B97F4A7C15, then the two
  xor-shift-multiply mixing rounds with 0xBF58476D1CE4E5B9 and
  0x94D049BB133111EB and a final xor-shift by 31;
* a 53-bit uniform in [0, 1): (x >> 11) * 2**-53;
* the Box-Muller transform (Box and Muller, 1958): with u1 in (0, 1] and u2
  in [0, 1), z0 = sqrt(-2 ln u1) cos(2 pi u2), z1 = sqrt(-2 ln u1) sin(2 pi u2).
  Both normals of a pair are used, z0 first.

Trajectory b of a batch seeded with ``seed`` uses the stream whose initial
state is seed + b * 0xD1B54A32D192ED03 (mod 2**64).

Pinned by tests/test_oracle_rng.py (published SplitMix64 outputs, moments).
"""
import math

MASK64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15
TRAJ_STRIDE = 0xD1B54A32D192ED03


class SplitMix64:
    def __init__(self, state):
        self.state = state & MASK64

    def next_u64(self):
        self.state = (self.state + GOLDEN_GAMMA) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self):
        """53-bit uniform in [0, 1)."""
        return (self.next_u64() >> 11) * (2.0 ** -53)


class NormalStream:
    """Standard normals by Box-Muller over a SplitMix64 stream."""

    def __init__(self, seed, traj=0):
        self.gen = SplitMix64((seed + traj * TRAJ_STRIDE) & MASK64)
        self.spare = None

    def normal(self):
        if self.spare is not None:
            z, self.spare = self.spare, None
            return z
        u1 = 1.0 - self.gen.uniform()          # (0, 1]
        u2 = self.gen.uniform()                # [0, 1)
        r = math.sqrt(-2.0 * math.log(u1))
        z0 = r * math.cos(2.0 * math.pi * u2)
        z1 = r * math.sin(2.0 * math.pi * u2)
        self.spare = z1
        return z0
