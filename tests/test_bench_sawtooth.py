"""The fine-N sawtooth analysis of bench.py (paper Sec. 8.3, Table 13: the period of the residual
sawtooth tracks the tile width; valleys sit one N step past a multiple of the tile) on synthetic
lines whose period and valley position are known.  CPU only."""
import numpy as np
import pytest

import bench

Ns = np.arange(1, 129) * 32          # the fine-N grid: N = 32 .. 4096 step 32


def _partial_tile_line(tile, peak=900.0, ramp=True):
    """Throughput of a kernel that wastes the unused part of its last tile column: peak times
    the tile utilisation N / (ceil(N / tile) tile), on a slow ramp (wave fill)."""
    util = Ns / (np.ceil(Ns / tile) * tile)
    base = peak * (0.6 + 0.4 * Ns / Ns[-1]) if ramp else np.full(Ns.size, peak)
    return base * util


@pytest.mark.parametrize("tile", [64, 128, 256])
def test_partial_tile_sawtooth_period_and_valley(tile):
    st = bench.sawtooth(_partial_tile_line(tile), Ns, tile)
    assert st["valley_residue"] == 32 % tile           # one step past a multiple of the tile
    assert st["valley_depth"] > 0
    if tile >= 64:
        # lags are searched from 64 on: the period is the tile width (or, for a 64 tile whose
        # harmonics fall inside the search range, a multiple of it)
        assert st["period"] % tile == 0
    if tile in (128, 256):
        assert st["period"] == tile
        assert st["valleys_at_residue"] == pytest.approx(1.0)
        assert st["valley_spacing_median"] == tile


def test_sinusoid_period():
    tf = 500.0 + 20.0 * np.sin(2 * np.pi * Ns / 384.0)
    st = bench.sawtooth(tf, Ns, 128)
    assert st["period"] == 384
    assert st["period_autocorr"] > 0.5


def test_valley_residue_moves_with_the_tile_not_the_address():
    # the same line shifted by one N step moves its valleys by one step: the residue follows
    a = bench.sawtooth(_partial_tile_line(128), Ns, 128)
    tf = _partial_tile_line(128)
    shifted = np.concatenate([tf[1:], tf[-1:]])          # valley now at N mod 128 = 0
    b = bench.sawtooth(shifted, Ns, 128)
    assert (a["valley_residue"], b["valley_residue"]) == (32, 0)


def test_noise_has_no_strong_period():
    rng = np.random.default_rng(0)
    st = bench.sawtooth(500.0 + rng.normal(0, 5, Ns.size), Ns, 128)
    assert st["period_autocorr"] < 0.5


def test_ramp_texture_split():
    rng = np.random.default_rng(3)
    n = 8
    # a landscape monotone along every axis has no texture: its roughness is all ramp
    g = np.meshgrid(*[np.arange(n)] * 3, indexing="ij")
    mono = 10.0 * g[0] + 3.0 * g[1] ** 2 + np.sqrt(g[2] + 1.0)
    rt = bench.ramp_texture(mono)
    assert rt["texture_3d"] == pytest.approx(0.0, abs=1e-12)
    # ramp + texture is the roughness, line by line, on any landscape
    x = rng.uniform(0, 100, size=(n, n, n))
    rt = bench.ramp_texture(x)
    for name, axis in (("m", 0), ("n", 1), ("k", 2)):
        t = np.moveaxis(x, axis, -1)
        rough = float(np.mean(np.abs(np.diff(t, axis=-1)).sum(axis=-1) / (n - 1)))
        assert rt["ramp_" + name] + rt["texture_" + name] == pytest.approx(rough)
        assert rt["texture_" + name] >= 0
    # a zig-zag with equal end points is all texture
    z = np.zeros((1, 1, 9))
    z[..., 1::2] = 5.0
    rt = bench.ramp_texture(np.broadcast_to(z, (2, 2, 9)).copy())
    assert rt["ramp_k"] == 0.0 and rt["texture_k"] == pytest.approx(5.0)
