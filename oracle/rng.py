"""Counter-based random numbers for the sampler.

The paper draws pixels "by multinomial sampling" without naming a generator.
Reading: every draw uses a 64-bit value from the SplitMix64 generator of
Steele, Lea and Flood ("Fast splittable pseudorandom number generators",
OOPSLA 2014): output(state) = mix(state + gamma) with gamma the odd constant
0x9E3779B97F4A7C15 and mix the 64-bit finaliser

    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    z =  z ^ (z >> 31)

used here as a stateless counter hash: each field of (seed, step, view, tile,
slot) is absorbed in turn, h <- mix(h + gamma * (field + 1)), starting from
h = seed.  Pixel slots 0..255 are hard draws, 256..511 mixed draws; the tile
pass uses tile = number of tiles and slot = the tile's index.
"""
from __future__ import annotations

MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def mix64(z: int) -> int:
    z &= MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def draw(seed: int, step: int, view: int, tile: int, slot: int) -> int:
    h = seed & MASK
    for f in (step, view, tile, slot):
        h = mix64(h + GAMMA * (f + 1))
    return h


def below(u: int, n: int) -> int:
    """floor(u * n / 2^64): a draw scaled to [0, n) by its high product bits."""
    return (u * n) >> 64
