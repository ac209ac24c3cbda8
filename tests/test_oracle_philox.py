"""Pins for the oracle's Philox4x32-10 (published known-answer vectors) and
for the shot-bit convention."""
import os

import pytest

from oracle import chp
from oracle.philox import philox4x32_10, shot_bit, variant_id

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        v = [int(t, 16) for t in line.split()]
        rows.append((tuple(v[0:4]), tuple(v[4:6]), tuple(v[6:10])))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_python_kat(ctr, key, out):
    assert philox4x32_10(ctr, key) == out


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_c_kat(ctr, key, out):
    assert chp.philox_c(ctr, key) == out


def test_python_and_c_agree_on_shot_counters():
    for s in range(0, 40, 3):
        for a in (0, 5, 31, 32, 63):
            vid = variant_id(3, 2, 77)
            ctr = (a >> 5, s >> 2, vid & 0xFFFFFFFF, vid >> 32)
            key = (0x12345678, 0x9ABCDEF0)
            assert philox4x32_10(ctr, key) == chp.philox_c(ctr, key)


def test_shot_bit_layout():
    seed, vid = 0xDEADBEEF12345678, variant_id(1, 0, 5)
    for s in range(8):
        words = philox4x32_10((1, s >> 2, vid & 0xFFFFFFFF, vid >> 32),
                              (seed & 0xFFFFFFFF, seed >> 32))
        for a in (32, 40, 63):
            assert shot_bit(seed, vid, s, a) == (words[s & 3] >> (a - 32)) & 1


def test_variant_id_fields():
    assert variant_id(1, 2, 3) == (1 << 40) | (2 << 32) | 3
