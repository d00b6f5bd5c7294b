"""Pins of the oracle's random numbers against the published SplitMix64
sequence and closed forms (reading R8)."""
import json
import os

import pytest

import oracle

MASK = (1 << 64) - 1


def test_splitmix64_published_sequence(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "splitmix64.json")))
    for s in g["sequences"]:
        assert oracle.splitmix64_sequence(s["seed"], len(s["outputs"])) == s["outputs"]


@pytest.mark.parametrize("seed,prob,g,r,slot", [(0, 0, 0, 0, 0), (1234567, 3, 0, 0, 5),
                                                (99, 7, 0, 1, 2), (5, 1, 0, 0, 1000)])
def test_draw_is_splitmix_output_number(seed, prob, g, r, slot):
    # draw = output (ctr + 1) of SplitMix64 seeded with key, key = output
    # (prob + 1) of SplitMix64 seeded with seed; checked against the
    # sequential generator (itself pinned above).
    key = oracle.splitmix64_sequence(seed, prob + 1)[-1]
    ctr = (g << 40) | (r << 20) | slot
    assert oracle.draw(seed, prob, g, r, slot) == oracle.splitmix64_sequence(key, ctr + 1)[-1]


def test_draw_generation_bit_position():
    # g occupies bits 40.. of the counter: (g=1, r=0, slot=0) is counter 2^40,
    # which the sequential generator reaches as seed + (2^40 + 1) * gamma.
    seed, prob = 11, 2
    key = oracle.splitmix64_sequence(seed, prob + 1)[-1]
    gamma = 0x9E3779B97F4A7C15
    shifted = (key + (1 << 40) * gamma) & MASK   # state after 2^40 steps
    assert oracle.draw(seed, prob, 1, 0, 0) == oracle.splitmix64_sequence(shifted, 1)[0]
    shifted = (key + ((3 << 20) | 4) * gamma) & MASK
    assert oracle.draw(seed, prob, 0, 3, 4) == oracle.splitmix64_sequence(shifted, 1)[0]


def test_u01_closed_form():
    assert oracle.u01(0) == 0.0
    assert oracle.u01(1 << 11) == 2.0 ** -53
    assert oracle.u01(MASK) == (2.0 ** 53 - 1) / 2.0 ** 53
    assert oracle.u01(1 << 63) == 0.5


def test_uint_closed_form():
    assert oracle.uint(0, 10) == 0
    assert oracle.uint(MASK, 10) == 9
    assert oracle.uint(1 << 63, 10) == 5
    assert oracle.uint(0xFFFFFFFF_00000000, 1) == 0
    for m in (2, 3, 7, 1000):
        for hi in (0, 1, 12345, 0x7FFFFFFF, 0xFFFFFFFF):
            assert oracle.uint(hi << 32, m) == (hi * m) >> 32
