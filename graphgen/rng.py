"""Counter-based random numbers: the SplitMix64 generator of Steele, Lea and Flood
("Fast splittable pseudorandom number generators", OOPSLA 2014).

The k-th output (k = 0, 1, ...) of a SplitMix64 sequence started at state ``s`` is
``mix(s + (k + 1) * GAMMA)`` with ``GAMMA = 0x9E3779B97F4A7C15`` and ``mix`` the published
64-bit finaliser (xor-shift 30, multiply, xor-shift 27, multiply, xor-shift 31). Evaluating
that expression for a tensor of counters gives a counter-based generator: any element can be
drawn independently, on any device, with integer operations only.

Tensors are torch.int64 holding the two's-complement bits of the unsigned values; additions and
multiplications wrap modulo 2^64 and right shifts are made logical with a mask.
"""

import torch

MASK64 = (1 << 64) - 1


def _as_i64(x: int) -> int:
    x &= MASK64
    return x - (1 << 64) if x >= (1 << 63) else x


GAMMA = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB
_GAMMA_I = _as_i64(GAMMA)
_MIX1_I = _as_i64(MIX1)
_MIX2_I = _as_i64(MIX2)


def srl(z: torch.Tensor, s: int) -> torch.Tensor:
    """Logical right shift of the 64-bit pattern held in an int64 tensor."""
    return (z >> s) & ((1 << (64 - s)) - 1)


def splitmix64_mix(z: torch.Tensor) -> torch.Tensor:
    """The SplitMix64 finaliser applied elementwise (a bijection on 64-bit words)."""
    z = (z ^ srl(z, 30)) * _MIX1_I
    z = (z ^ srl(z, 27)) * _MIX2_I
    return z ^ srl(z, 31)


def mix_int(z: int) -> int:
    """Python-int version of the finaliser, used for stream keys and unit tests."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * MIX1) & MASK64
    z = ((z ^ (z >> 27)) * MIX2) & MASK64
    return z ^ (z >> 31)


def splitmix64_sequence(seed: int, count: int):
    """First ``count`` outputs of a SplitMix64 sequence (Python ints; for tests)."""
    out = []
    s = seed & MASK64
    for _ in range(count):
        s = (s + GAMMA) & MASK64
        out.append(mix_int(s))
    return out


def stream_key(seed: int, *tags: int) -> int:
    """Derive an independent stream start state from a seed and integer tags."""
    k = mix_int(seed ^ 0x5851F42D4C957F2D)
    for t in tags:
        k = mix_int(k ^ mix_int(t + 0x632BE59BD9B4E019))
    return k


def draw(key: int, counter: torch.Tensor) -> torch.Tensor:
    """Element-wise counter-based draw: output number ``counter`` of the stream ``key``.

    ``counter`` is an int64 tensor of non-negative counters; the result holds 64 random bits
    per element as int64.
    """
    state = (counter + 1) * _GAMMA_I + _as_i64(key)
    return splitmix64_mix(state)


def top32(d: torch.Tensor) -> torch.Tensor:
    """Upper 32 bits of each 64-bit draw, as a non-negative int64."""
    return srl(d, 32)


def low32(d: torch.Tensor) -> torch.Tensor:
    """Lower 32 bits of each 64-bit draw, as a non-negative int64."""
    return d & 0xFFFFFFFF


def below(d: torch.Tensor, bound: int) -> torch.Tensor:
    """Map 64-bit draws to integers in [0, bound) by a 32x32-bit multiply-high (bound < 2^31)."""
    assert 0 < bound < (1 << 31)
    return (top32(d) * bound) >> 32
