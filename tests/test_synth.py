"""Seeded input generator: pinned to the published SplitMix64 outputs and to the definition of
round-to-nearest-even, independently of any GEMM code."""
import json
import os
from fractions import Fraction

import numpy as np

import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_vector():
    g = json.load(open(os.path.join(GOLD, "splitmix64_seed1234567.json")))
    # out(s, i) for i = 1..5 is words(...) with a key equal to the seed itself: check the mix
    key = np.uint64(g["seed"])
    idx = np.arange(1, 6, dtype=np.uint64)
    with np.errstate(over="ignore"):
        got = synth._mix(key + idx * synth.GAMMA)
    assert [int(x) for x in got] == [int(s) for s in g["outputs"]]


def test_words_are_counter_based_and_streams_differ():
    w = synth.words(7, 0, 0, 1000)
    assert np.array_equal(w[100:200], synth.words(7, 0, 100, 100))
    assert not np.array_equal(w[:100], synth.words(7, 1, 0, 100))
    assert not np.array_equal(w[:100], synth.words(8, 0, 0, 100))


def test_uniform_values_exact_and_in_range():
    f = synth.uniform_pm1_f32(3, 0, 200000)
    assert f.dtype == np.float32
    assert np.all(f > -1) and np.all(f < 1)
    u = (synth.words(3, 0, 0, 200000) >> np.uint64(40)).astype(np.int64)
    # f * 2^24 must be the odd integer 2u + 1 - 2^24 exactly
    assert np.array_equal((f.astype(np.float64) * 2 ** 24).astype(np.int64), 2 * u + 1 - (1 << 24))
    assert abs(float(f.mean())) < 0.01 and abs(float(f.var()) - 1 / 3) < 0.01


def _rne_by_definition(x: float) -> int:
    """Nearest BF16 to x (ties to even significand), by exact rational comparison."""
    fx = Fraction(x)
    u = np.array([x], dtype=np.float32).view(np.uint32)[0]
    lo = int(u) >> 16                       # truncation toward zero
    hi = lo + 1
    vlo = Fraction(float(synth.bf16_bits_to_f32(np.array([lo], dtype=np.uint16))[0]))
    vhi = Fraction(float(synth.bf16_bits_to_f32(np.array([hi], dtype=np.uint16))[0]))
    dlo, dhi = abs(fx - vlo), abs(vhi - fx)
    if dlo < dhi:
        return lo
    if dhi < dlo:
        return hi
    return lo if lo % 2 == 0 else hi


def test_f32_to_bf16_rne_definition():
    rng = np.random.default_rng(0)
    # every BF16 value, the FP32 values half an ulp away (ties) and one FP32 ulp either side
    base = np.arange(0, 0x7F80, 7, dtype=np.uint32) << 16      # positive finite BF16 grid
    cands = np.concatenate([base, base + 0x8000, base + 0x7FFF, base + 0x8001, base + 0x0001,
                            rng.integers(0, 0x7F7F0000, 4000).astype(np.uint32)])
    cands = np.concatenate([cands, cands | np.uint32(0x80000000)])
    x = cands.view(np.float32)
    got = synth.f32_to_bf16_bits(x)
    sample = rng.choice(x.size, 3000, replace=False)
    for t in sample:
        assert int(got[t]) == _rne_by_definition(float(x[t])), hex(int(cands[t]))


def test_bf16_widening_exact():
    h = np.arange(0, 0x7F80, dtype=np.uint16)
    f = synth.bf16_bits_to_f32(h)
    assert np.array_equal(synth.f32_to_bf16_bits(f), h)


def test_normal_moments_and_determinism():
    z = synth.normal_f32(5, 0, 400000, 1.0)
    assert abs(float(z.mean())) < 0.01
    assert abs(float(z.std()) - 1.0) < 0.01
    assert np.array_equal(z[1000:2000], synth.normal_f32(5, 0, 1000, 1.0, start=1000))
    b = synth.normal_bf16(5, 0, 100, 100, std=0.02)
    v = synth.bf16_bits_to_f32(b)
    assert 0.015 < float(v.std()) < 0.025


def test_integer_generator_exact():
    h = synth.integer_bf16(1, 0, 50, 60, -4, 4)
    v = synth.bf16_bits_to_f32(h)
    assert np.array_equal(v, np.round(v)) and v.min() == -4 and v.max() == 4
