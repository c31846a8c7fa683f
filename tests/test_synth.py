"""The seeded generator: per-window reproducibility and the int8 rules."""
import numpy as np

from paper_1411_0436_amd import synth


def test_window_generation_equals_whole_stream():
    spec = synth.spec_c2(n_ref=1024)
    L = synth.GEN_CHUNK
    whole = synth.generate(spec, 0, 2 * L + 300)
    parts = [synth.generate(spec, 0, 1000),
             synth.generate(spec, 1000, L + 17),
             synth.generate(spec, L + 1017, L + 300 - 1017)]
    assert np.array_equal(whole, np.concatenate(parts))


def test_deterministic_and_seed_sensitive():
    a = synth.generate(synth.spec_c1(), 0, 4096)
    b = synth.generate(synth.spec_c1(), 0, 4096)
    c = synth.generate(synth.noise_only(1, 20.0, 1), 0, 4096)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)


def test_quantise_clip_and_round_half_even():
    v = np.array([[127.6 + 0.5j], [-300.0 - 1.5j], [2.5 + 0j]])
    q = synth.quantise(v)
    assert q.dtype == np.int8
    assert q[0, 0].tolist() == [127, 0]
    assert q[1, 0].tolist() == [-127, -2]
    assert q[2, 0].tolist() == [2, 0]


def test_shapes_and_noise_level():
    x = synth.generate(synth.noise_only(2, 20.0, 3), 0, 1 << 16)
    assert x.shape == (1 << 16, 2, 2)
    p = np.mean(x.astype(float) ** 2) * 2     # E|x|^2 per polarisation
    assert abs(p - (400.0 + 1.0 / 6.0)) < 6.0


def test_exact_tone_values():
    x = synth.exact_tone(8, 1, 16, 4, 100)
    assert x[:, 0, 0].tolist() == [100, 0, -100, 0, 100, 0, -100, 0]
    assert x[:, 0, 1].tolist() == [0, 100, 0, -100, 0, 100, 0, -100]


def test_pulse_duty_cycle():
    spec = synth.StreamSpec(n_pol=1, sigma=0.0, seed=5,
                            pulse=synth.Pulse(period=1000, duty=0.05, sigma=40.0))
    x = synth.generate(spec, 0, 3000).astype(float)
    on = (np.arange(3000) % 1000) < 50
    assert np.all(x[~on] == 0)
    assert np.mean(np.abs(x[on])) > 5
