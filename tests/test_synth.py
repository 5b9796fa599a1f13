"""Seeded input generators: definition, determinism, slicing, moments."""
import numpy as np

import synth

M64 = (1 << 64) - 1


def mix64_py(z):
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def draw_py(key, n):
    return mix64_py((key + (n + 1) * synth.GOLDEN) & M64)


def test_splitmix64_reference_vector():
    # first output of SplitMix64 started from state 0 (published test value)
    assert synth._clib().synth_draw(0, 0) == 0xE220A8397B1DCDAF
    assert draw_py(0, 0) == 0xE220A8397B1DCDAF


def test_key_and_normals_match_definition():
    k = synth.key(1000, 7, synth.T_B)
    kp = draw_py(draw_py(draw_py(1000, 0) ^ 7, 0) ^ synth.T_B, 0)
    assert k == kp
    got = synth.normal(k, 5, 16)
    for n in range(16):
        e = 5 + n
        u1 = ((draw_py(k, 2 * e) >> 11) + 0.5) * 2.0 ** -53
        u2 = ((draw_py(k, 2 * e + 1) >> 11) + 0.5) * 2.0 ** -53
        ref = np.sqrt(-2.0 * np.log(u1)) * np.cos(6.283185307179586 * u2)
        assert abs(got[n] - ref) <= 4e-16 * max(1.0, abs(ref))


def test_three_index_slices_are_consistent():
    f = synth.random_fragment(6, 5, 7, seed=3)
    full = f.B()
    assert np.array_equal(full[2:5], f.B(2, 5))
    assert np.array_equal(full, f.B())
    flat = synth.normal(f.key_B, 0, 6 * 5 * 7).reshape(6, 5, 7) * synth.decay_scale(7, 80.0)
    assert np.array_equal(full, flat)


def test_moments_and_energy_ranges():
    x = synth.normal(synth.key(1, 2, 3), 0, 400000)
    assert abs(x.mean()) < 0.01 and abs(x.var() - 1.0) < 0.01
    eo, ev = synth.SMALL.eps()
    assert np.all(np.diff(eo) >= 0) and np.all(np.diff(ev) >= 0)
    assert eo.min() >= -20.0 and eo.max() <= -0.3 and ev.min() >= 0.1 and ev.max() <= 5.0


def test_screen_scale_and_mbe3_sizes():
    f = synth.screen_system(4000, nocc=4, nvir=3, naux=5)
    s = f.scale()
    assert s.shape == (4, 5) and np.all(s <= 0.3) and np.all(s > 0)
    sizes = synth.mbe3_sizes(40)
    kinds = [k for k, _ in sizes]
    assert kinds.count(1) == 12 and kinds.count(2) == 16 and kinds.count(3) == 12
    for kind, nocc in sizes:
        assert 5 * kind <= nocc <= 60 * kind
